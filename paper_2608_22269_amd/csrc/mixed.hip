// Mixed-precision path.
//
// Storage: each fluid particle's position is its background cell (packed
// ix | iy << 11 | iz << 22) plus an FP32 offset inside the cell, with a Kahan
// compensation; velocity FP32 with a Kahan compensation; the potential FP64.
// The offset keeps ~2^-24 R resolution anywhere in the domain (a few 1e-10 m
// at R = h = 2.6 mm), where absolute FP32 positions would give ~6e-8 m.
//
// Pair pass: the lockstep row search of coop.h with candidate tests on FP32
// absolute positions (set membership only changes for pairs within ~1e-7 m
// of 2h, whose terms vanish like (1-q/2)^3);
// the pair vector r from cell difference and offsets in FP32; W, grad W, the
// Lax-Friedrichs, shifting and delta-SPH terms in FP32.  The correction
// matrix L, the Riemann sum S_R and the conservative sum S_C accumulate in
// FP64 from the same promoted r and grad W V, so L^-T S_R reproduces a linear
// potential to FP64 round-off whatever the FP32 rounding of r and grad W (the
// correction is kept outside the sum, Sec. 3).  The remaining sums use FP32
// partial sums per LDS chunk (<= 32 neighbours) flushed into FP64 totals.  The
// epilogue (eigenvalues, solves, branches) is the FP64 one of the FP64 path.
//
// Integrator: SSP-RK2 in its incremental form -- stage 1 adds dt*rate(q0),
// stage 2 adds (dt*rate(q1) - dt*rate(q0)) / 2, equal in exact arithmetic to
// q0/2 + (q1 + dt*rate(q1))/2 -- with Kahan-compensated FP32 adds for offsets
// and velocity, then the offset is brought back into [0, R) by moving cells.
#include "mixed.h"
#include "pair_common.h"
#include "coop.h"

namespace wb {

// waves per SIMD the register allocation targets (4 measured fastest)
#ifndef WB_MIXED_WAVES
#define WB_MIXED_WAVES 4
#endif
#define WB_MIXED_ATTR __attribute__((amdgpu_waves_per_eu(WB_MIXED_WAVES)))
constexpr int kMList = kPairList;  // kept lists share the FP64 pass's layout
constexpr int kMBatch = 4;
static_assert(kMBatch <= kRecPad, "batched candidate loads run at most kRecPad records past a run");

__device__ __forceinline__ uint32_t pack_cell(int x, int y, int z) {
  return (uint32_t)x | ((uint32_t)y << 11) | ((uint32_t)z << 22);
}
__device__ __forceinline__ int cell_x(uint32_t c) { return (int)(c & 2047u); }
__device__ __forceinline__ int cell_y(uint32_t c) { return (int)((c >> 11) & 2047u); }
__device__ __forceinline__ int cell_z(uint32_t c) { return (int)(c >> 22); }

// Kahan-compensated add of an FP64 increment to an FP32 sum; s - c is the
// represented value.
__device__ __forceinline__ void kahan_add(float &s, float &c, double d) {
  float y = (float)(d + (double)c * -1.0);
  float t = s + y;
  c = (t - s) - y;
  s = t;
}

// Position along one axis reconstructed in FP64: (lo + c R) + o, each
// operation rounded as written (no contraction), as the storage conversion
// and the field export form it.
__device__ __forceinline__ double pos_of(double lo, double R, int c, float o) {
#pragma clang fp contract(off)
  return lo + (double)c * R + (double)o;
}

// ------------------------------------------------------------ conversion

template <int DIM>
__global__ void k_to_mixed(Phys P, Grid g, FluidF64 src, int64_t n, FluidMixed dst, Scalars *sc) {
  // the offset x - (lo + c R) rounded as written (no contraction): the stored
  // state is then a plain function of the input
#pragma clang fp contract(off)
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c[3] = {0, 0, 0};
  for (int a = 0; a < DIM; ++a) {
    double x = src.x[a][i];
    int ca = cell_coord(x, g.lo[a], g.R);
    if (!(x >= g.lo[a] && x <= g.hi[a]) || ca < 0 || ca >= g.N[a]) {
      atomicOr(&sc->err, kErrDomain);
      ca = 0;
    }
    c[a] = ca;
    dst.o[a][i] = (float)(x - (g.lo[a] + (double)ca * g.R));
    dst.oc[a][i] = 0.0f;
    dst.u[a][i] = (float)src.u[a][i];
    dst.uc[a][i] = 0.0f;
    dst.dx1[a][i] = 0.0f;
    dst.du1[a][i] = 0.0f;
  }
  dst.cell[i] = pack_cell(c[0], c[1], c[2]);
  dst.phi[i] = src.phi[i];
  dst.dphi1[i] = 0.0;
  dst.m[i] = (float)src.m[i];
  dst.id[i] = src.id[i];
}

hipError_t launch_to_mixed(const Phys &P, const Grid &g, const FluidF64 &src, int64_t nf, const FluidMixed &dst,
                           Scalars *sc, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_to_mixed<2>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, g, src, nf, dst, sc);
  else
    hipLaunchKernelGGL(k_to_mixed<3>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, g, src, nf, dst, sc);
  return hipGetLastError();
}

// --------------------------------------------------------------- reorder

// Gathers the mixed state into HashID order and writes the records:
// r0 = (offset, cell bits), r1 = (U, V), phi, xa = FP32 absolute position.
template <int DIM>
__global__ void __launch_bounds__(256) k_reorder_mixed(Phys P, Grid g, const uint32_t *__restrict__ perm, int64_t n,
                                                       FluidMixed src, FluidMixed dst, MixedRec rec, int with_stage0) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  uint32_t o = perm[k];
  uint32_t c = src.cell[o];
  dst.cell[k] = c;
  float of[3] = {0.f, 0.f, 0.f}, uf[3] = {0.f, 0.f, 0.f};
  for (int a = 0; a < DIM; ++a) {
    of[a] = src.o[a][o];
    uf[a] = src.u[a][o];
    dst.o[a][k] = of[a];
    dst.oc[a][k] = src.oc[a][o];
    dst.u[a][k] = uf[a];
    dst.uc[a][k] = src.uc[a][o];
    if (with_stage0) {
      dst.dx1[a][k] = src.dx1[a][o];
      dst.du1[a][k] = src.du1[a][o];
    }
  }
  double ph = src.phi[o];
  dst.phi[k] = ph;
  float m = src.m[o];
  dst.m[k] = m;
  dst.id[k] = src.id[o];
  if (with_stage0) dst.dphi1[k] = src.dphi1[o];
  float V = (float)((double)m / (P.rho0 * exp(ph * P.inv_c02)));
  int cc[3] = {cell_x(c), cell_y(c), cell_z(c)};
  float xa[3] = {0.f, 0.f, 0.f};
  for (int a = 0; a < DIM; ++a) xa[a] = (float)pos_of(g.lo[a], g.R, cc[a], of[a]);
  rec.r0[k] = make_float4(of[0], of[1], of[2], __uint_as_float(c));
  rec.r1[k] = make_float4(uf[0], uf[1], uf[2], V);
  rec.phi[k] = ph;
  rec.xa[k] = make_float4(xa[0], xa[1], xa[2], 0.f);
}

hipError_t launch_reorder_mixed(const Phys &P, const Grid &g, const uint32_t *perm, int64_t nf, const FluidMixed &src,
                                const FluidMixed &dst, const MixedRec &rec, int with_stage0, hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_reorder_mixed<2>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, g, perm, nf, src, dst, rec,
                       with_stage0);
  else
    hipLaunchKernelGGL(k_reorder_mixed<3>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, g, perm, nf, src, dst, rec,
                       with_stage0);
  return hipGetLastError();
}

// Records of the mixed state in its current order, without a sort (second
// stage of a step that keeps the first stage's candidates).
template <int DIM>
__global__ void __launch_bounds__(256) k_refresh_mixed(Phys P, Grid g, FluidMixed f, int64_t n, MixedRec rec) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint32_t c = f.cell[k];
  float of[3] = {0.f, 0.f, 0.f}, uf[3] = {0.f, 0.f, 0.f};
  for (int a = 0; a < DIM; ++a) {
    of[a] = f.o[a][k];
    uf[a] = f.u[a][k];
  }
  const double ph = f.phi[k];
  const float V = (float)((double)f.m[k] / (P.rho0 * exp(ph * P.inv_c02)));
  const int cc[3] = {cell_x(c), cell_y(c), cell_z(c)};
  float xa[3] = {0.f, 0.f, 0.f};
  for (int a = 0; a < DIM; ++a) xa[a] = (float)pos_of(g.lo[a], g.R, cc[a], of[a]);
  rec.r0[k] = make_float4(of[0], of[1], of[2], __uint_as_float(c));
  rec.r1[k] = make_float4(uf[0], uf[1], uf[2], V);
  rec.phi[k] = ph;
  rec.xa[k] = make_float4(xa[0], xa[1], xa[2], 0.f);
}

hipError_t launch_refresh_mixed(const Phys &P, const Grid &g, const FluidMixed &f, int64_t nf, const MixedRec &rec,
                                hipStream_t s) {
  if (nf <= 0) return hipSuccess;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_refresh_mixed<2>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, g, f, nf, rec);
  else
    hipLaunchKernelGGL(k_refresh_mixed<3>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, g, f, nf, rec);
  return hipGetLastError();
}

// ---------------------------------------------------------------- mirror

// Dummy records of the mixed path (Sec. 2.4): nearest fluid particle within
// 2h by the FP32 test (ties -> lower original index); phi_d = phi_f +
// G.(x_d - x_f) with both positions in FP64; slip velocity; V_d = m_d/rho.
template <int DIM>
__global__ void __launch_bounds__(256) k_mirror_mixed(Phys P, Grid g, Dummies d, int64_t nd, MixedRec rec,
                                                      const uint32_t *__restrict__ cs_f, uint32_t nf,
                                                      const Scalars *__restrict__ sc,
                                                      const uint32_t *__restrict__ fid) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nd) return;
  const double xd = d.x[0][k], yd = d.x[1][k], zd = DIM == 3 ? d.x[2][k] : 0.0;
  const float xf = (float)xd, yf = (float)yd, zf = (float)zd;
  const float two_h2 = (float)P.two_h2;
  RowWalker w;
  walker_init<DIM>(w, g, xd, yd, zd, P.win);
  int64_t best = -1;
  uint32_t best_id = 0;
  float best_r2 = 0.f;
  auto test_run = [&](uint32_t a, uint32_t e) {
    for (uint32_t j = a; j < e; ++j) {
      float4 b = rec.xa[j];
      float dxv = b.x - xf, dyv = b.y - yf, dzv = DIM == 3 ? b.z - zf : 0.f;
      float r2 = dxv * dxv + dyv * dyv + dzv * dzv;
      if (r2 <= two_h2) {
        uint32_t jid = fid[j];
        if (best < 0 || r2 < best_r2 || (r2 == best_r2 && jid < best_id)) {
          best = j;
          best_r2 = r2;
          best_id = jid;
        }
      }
    }
  };
  // fluid runs, as in the FP64 mirror
  if (g.reach == 2) {
    constexpr int NR = DIM == 3 ? 25 : 5;
    uint32_t lo[NR], hi[NR];
    walker_fluid_runs<DIM, NR>(w, g, cs_f, lo, hi);
#pragma unroll
    for (int r = 0; r < NR; ++r) test_run(lo[r], hi[r]);
  } else {
    while (walker_next<DIM>(w, g, cs_f, cs_f, nf))
      if (w.cur < nf) test_run(w.cur, w.end);
  }
  d.src[k] = (int32_t)best;
  // static part of the record: cell and offset of the dummy
  int c[3] = {0, 0, 0};
  float of[3] = {0.f, 0.f, 0.f};
  const double xs[3] = {xd, yd, zd};
  for (int a = 0; a < DIM; ++a) {
    c[a] = cell_coord(xs[a], g.lo[a], g.R);
    of[a] = (float)(xs[a] - (g.lo[a] + (double)c[a] * g.R));
  }
  const uint32_t cb = pack_cell(c[0], c[1], c[2]);
  const uint32_t o = nf + (uint32_t)k;
  rec.r0[o] = make_float4(of[0], of[1], of[2], __uint_as_float(cb));
  rec.xa[o] = make_float4(xf, yf, zf, 0.f);
  if (best < 0) {
    rec.r1[o] = make_float4(0.f, 0.f, 0.f, 0.f);
    rec.phi[o] = d.phi_in[k];
    return;
  }
  double G[3];
  body_force(P, sc->t_rhs, G);
  const float4 f0 = rec.r0[best], f1 = rec.r1[best];
  const uint32_t fc = __float_as_uint(f0.w);
  const double xfs[3] = {pos_of(g.lo[0], g.R, cell_x(fc), f0.x), pos_of(g.lo[1], g.R, cell_y(fc), f0.y),
                         DIM == 3 ? pos_of(g.lo[2], g.R, cell_z(fc), f0.z) : 0.0};
  double gp = 0.0;
  for (int a = 0; a < DIM; ++a) gp += G[a] * (xs[a] - xfs[a]);
  const double phid = rec.phi[best] + gp;
  const float nx = (float)d.n[0][k], ny = (float)d.n[1][k], nz = DIM == 3 ? (float)d.n[2][k] : 0.f;
  // slip, relative to the body's velocity for the moving body's dummies (a
  // free body: v + omega x R (x0 - c0) at this dummy, formed in FP64)
  const bool mv = d.mov != nullptr && d.mov[k];
  double Uw[3] = {sc->body_u[0], sc->body_u[1], sc->body_u[2]};
  if (mv && sc->fb_on) {
    double q[4] = {sc->fb[3], sc->fb[4], sc->fb[5], sc->fb[6]}, R[9];
    quat_rotation(q, R);
    const double d0[3] = {d.x0[0][k] - sc->fb_c0[0], d.x0[1][k] - sc->fb_c0[1],
                          DIM == 3 ? d.x0[2][k] - sc->fb_c0[2] : 0.0};
    double dr[3];
    mat3_apply(R, d0, dr);
    free_body_point_velocity(sc->fb, dr, Uw);
  }
  const float wx = mv ? (float)Uw[0] : 0.f, wy = mv ? (float)Uw[1] : 0.f, wz = mv && DIM == 3 ? (float)Uw[2] : 0.f;
  const float un = (f1.x - wx) * nx + (f1.y - wy) * ny + (f1.z - wz) * nz;
  const float V = (float)(d.m[k] / (P.rho0 * exp(phid * P.inv_c02)));
  rec.r1[o] = make_float4(f1.x - un * nx, f1.y - un * ny, DIM == 3 ? f1.z - un * nz : 0.f, V);
  rec.phi[o] = phid;
}

hipError_t launch_mirror_mixed(const Phys &P, const Grid &g, const Dummies &d, int64_t nd, const MixedRec &rec,
                               const uint32_t *cs_f, uint32_t nf, const Scalars *sc, hipStream_t s,
                               const uint32_t *fid) {
  if (nd <= 0) return hipSuccess;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_mirror_mixed<2>, dim3(grid_for(nd)), dim3(kBlock), 0, s, P, g, d, nd, rec, cs_f, nf, sc, fid);
  else
    hipLaunchKernelGGL(k_mirror_mixed<3>, dim3(grid_for(nd)), dim3(kBlock), 0, s, P, g, d, nd, rec, cs_f, nf, sc, fid);
  return hipGetLastError();
}

// The water's force and torque on the free body's dummies from the mixed
// records, in FP64 as on the FP64 path: fluid positions rebuilt exactly from
// cell and FP32 offset, potentials in FP64, volumes from the FP32 records.
// One partial of 6 doubles per block (force, then torque about the body's
// centre), summed in a fixed tree.
template <int DIM>
__global__ void __launch_bounds__(256) k_body_force_mixed(Phys P, Grid g, Dummies d, int64_t nd, MixedRec rec,
                                                          const uint32_t *__restrict__ cs_f, uint32_t nf,
                                                          const Scalars *__restrict__ sc, double *__restrict__ part) {
  __shared__ double red[6][256];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double f[3] = {0.0, 0.0, 0.0}, tq[3] = {0.0, 0.0, 0.0};
  if (k < nd && d.mov[k] && d.src[k] >= 0) {
    const double xd = d.x[0][k], yd = d.x[1][k], zd = DIM == 3 ? d.x[2][k] : 0.0;
    const double phid = rec.phi[nf + (uint32_t)k];
    RowWalker w;
    walker_init<DIM>(w, g, xd, yd, zd, P.win);
    double a[3] = {0.0, 0.0, 0.0};
    auto sum_run = [&](uint32_t lo, uint32_t hi) {
      for (uint32_t j = lo; j < hi; ++j) {
        const float4 r0 = rec.r0[j];
        const uint32_t fc = __float_as_uint(r0.w);
        const double rx = pos_of(g.lo[0], g.R, cell_x(fc), r0.x) - xd;
        const double ry = pos_of(g.lo[1], g.R, cell_y(fc), r0.y) - yd;
        const double rz = DIM == 3 ? pos_of(g.lo[2], g.R, cell_z(fc), r0.z) - zd : 0.0;
        const double r2 = dist2_exact<DIM>(rx, ry, rz);
        if (r2 > P.two_h2) continue;
        const double t = fma(sqrt(r2), P.m_half_inv_h, 1.0);  // 1 - q/2
        const double c = (rec.phi[j] + phid) * (P.kfac * t * t * t) * (double)rec.r1[j].w;
        a[0] -= c * rx;
        a[1] -= c * ry;
        if (DIM == 3) a[2] -= c * rz;
      }
    };
    if (g.reach == 2) {
      constexpr int NR = DIM == 3 ? 25 : 5;
      uint32_t lo[NR], hi[NR];
      walker_fluid_runs<DIM, NR>(w, g, cs_f, lo, hi);
#pragma unroll
      for (int r = 0; r < NR; ++r) sum_run(lo[r], hi[r]);
    } else {
      while (walker_next<DIM>(w, g, cs_f, cs_f, nf))
        if (w.cur < nf) sum_run(w.cur, w.end);
    }
    const double m = d.m[k];
    const double arm[3] = {xd - sc->fb[0], yd - sc->fb[1], DIM == 3 ? zd - sc->fb[2] : 0.0};
    for (int c = 0; c < 3; ++c) f[c] = m * a[c];
    tq[0] = arm[1] * f[2] - arm[2] * f[1];
    tq[1] = arm[2] * f[0] - arm[0] * f[2];
    tq[2] = arm[0] * f[1] - arm[1] * f[0];
  }
  const int t = threadIdx.x;
  for (int c = 0; c < 3; ++c) {
    red[c][t] = f[c];
    red[3 + c][t] = tq[c];
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int c = 0; c < 6; ++c) red[c][t] += red[c][t + w];
    __syncthreads();
  }
  if (t < 6) part[(size_t)6 * blockIdx.x + t] = red[t][0];
}

hipError_t launch_body_force_mixed(const Phys &P, const Grid &g, const Dummies &d, int64_t nd, const MixedRec &rec,
                                   const uint32_t *cs_f, uint32_t nf, const Scalars *sc, double *part,
                                   hipStream_t s) {
  if (nd == 0) return hipSuccess;
  if (!d.mov || !part) return hipErrorInvalidValue;
  static_assert(kBlock == 256, "the block tree of the body force assumes 256 threads");
  if (P.dim == 2)
    hipLaunchKernelGGL(k_body_force_mixed<2>, dim3(grid_for(nd)), dim3(kBlock), 0, s, P, g, d, nd, rec, cs_f, nf, sc,
                       part);
  else
    hipLaunchKernelGGL(k_body_force_mixed<3>, dim3(grid_for(nd)), dim3(kBlock), 0, s, P, g, d, nd, rec, cs_f, nf, sc,
                       part);
  return hipGetLastError();
}

// -------------------------------------------------------------- pair pass

// The particle side of the mixed pair body.
struct MixedI {
  int cix, ciy, ciz;
  double Rd, oxi, oyi, ozi, phii;
  float4 a1;
  float inv_h, kfac, alpha, w0inv, c0f, pst_n;
};

__device__ __forceinline__ MixedI mixed_i(const Phys &P, const Grid &g, const float4 &a0, const float4 &a1,
                                          double phii) {
  MixedI I;
  const uint32_t ci = __float_as_uint(a0.w);
  I.cix = cell_x(ci);
  I.ciy = cell_y(ci);
  I.ciz = cell_z(ci);
  I.Rd = g.R;
  I.oxi = a0.x;
  I.oyi = a0.y;
  I.ozi = a0.z;
  I.phii = phii;
  I.a1 = a1;
  I.inv_h = (float)P.inv_h;
  I.kfac = (float)P.kfac;
  I.alpha = (float)P.alpha;
  I.w0inv = (float)P.w0inv;
  I.c0f = (float)P.c0;
  I.pst_n = (float)P.pst_n;
  return I;
}

// FP32 partial sums of one list chunk, flushed into the FP64 totals.
struct MixedChunk {
  float gsf[3], Nf[6], Pf[3], Df;
};

__device__ __forceinline__ void chunk_zero(MixedChunk &C) {
#pragma unroll
  for (int a = 0; a < 3; ++a) C.gsf[a] = C.Pf[a] = 0.f;
#pragma unroll
  for (int a = 0; a < 6; ++a) C.Nf[a] = 0.f;
  C.Df = 0.f;
}

__device__ __forceinline__ void chunk_flush(const MixedChunk &C, PairSums &S) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    S.gs[a] += C.gsf[a];
    S.Ps[a] += C.Pf[a];
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) S.N[a] += C.Nf[a];
  S.Ds += C.Df;
}

// Pair body of the mixed path for neighbour j (records b0, b1, phij).  PST4:
// the shifting exponent is 4 (two squarings); otherwise powf().
template <int DIM, bool PST4>
__device__ __forceinline__ void mixed_body(const MixedI &I, const float4 &b0, const float4 &b1, const double phij,
                                           MixedChunk &C, PairSums &S) {
  const uint32_t cj = __float_as_uint(b0.w);
  // r = (c_j - c_i) R + (o_j - o_i), formed in FP64 from the integer cell
  // difference and the promoted offsets (one rounding): the same r enters
  // L and S_R, and phi_j - phi_i of a linear potential equals G.r to FP64
  // round-off.  Its FP32 rounding feeds the FP32 part of the body.
  const double rxd = (double)(cell_x(cj) - I.cix) * I.Rd + ((double)b0.x - I.oxi);
  const double ryd = (double)(cell_y(cj) - I.ciy) * I.Rd + ((double)b0.y - I.oyi);
  const double rzd = DIM == 3 ? (double)(cell_z(cj) - I.ciz) * I.Rd + ((double)b0.z - I.ozi) : 0.0;
  const float rx = (float)rxd, ry = (float)ryd, rz = (float)rzd;
  const float r2 = rx * rx + ry * ry + rz * rz;
  S.coincident |= (r2 == 0.f);
  const float is = rsqrtf(r2);
  const float s = r2 * is;
  const float q = fminf(s * I.inv_h, 2.0f);
  const float t = 1.0f - 0.5f * q;
  const float t2 = t * t, t3 = t2 * t;
  const float wv = I.kfac * t3 * b1.w;
  const float gx = wv * rx, gy = wv * ry, gz = wv * rz;
  // FP64: L, S_R, S_C from the same FP64 r and grad W V = wv r
  const double wvd = wv;
  const double gxd = wvd * rxd, gyd = wvd * ryd, gzd = wvd * rzd;
  S.L[0] += rxd * gxd;
  S.L[1] += ryd * gyd;
  S.L[3] += rxd * gyd;
  if (DIM == 3) {
    S.L[2] += rzd * gzd;
    S.L[4] += rxd * gzd;
    S.L[5] += ryd * gzd;
  }
  const double dph = phij - I.phii;
  const float dux = b1.x - I.a1.x, duy = b1.y - I.a1.y, duz = DIM == 3 ? b1.z - I.a1.z : 0.f;
  const float dun = (dux * rx + duy * ry + duz * rz) * is;
  const double c2 = dph - (double)(I.c0f * dun);
  const double cs = phij + I.phii;
  S.SR[0] += c2 * gxd;
  S.SR[1] += c2 * gyd;
  S.SC[0] += cs * gxd;
  S.SC[1] += cs * gyd;
  if (DIM == 3) {
    S.SR[2] += c2 * gzd;
    S.SC[2] += cs * gzd;
  }
  // FP32 chunk sums
  C.gsf[0] += gx;
  C.gsf[1] += gy;
  if (DIM == 3) C.gsf[2] += gz;
  C.Nf[0] += dux * gx;
  C.Nf[1] += duy * gy;
  C.Nf[3] += dux * gy + duy * gx;
  if (DIM == 3) {
    C.Nf[2] += duz * gz;
    C.Nf[4] += dux * gz + duz * gx;
    C.Nf[5] += duy * gz + duz * gy;
  }
  C.Df += wv * (float)dph;
  const float W = I.alpha * t2 * t2 * (2.0f * q + 1.0f);
  const float wr = W * I.w0inv;
  const float wrn = PST4 ? (wr * wr) * (wr * wr) : powf(wr, I.pst_n);
  // (W / W(dx))^n grad W V; the epilogue adds grad W V times 1 / R
  C.Pf[0] += wrn * gx;
  C.Pf[1] += wrn * gy;
  if (DIM == 3) C.Pf[2] += wrn * gz;
}

// Sums of the single-precision form (SPH_FP32) that the mixed form keeps in
// FP64: the correction matrix and the potential-gradient sums, here in FP32
// over one list fill.
struct Abs32Chunk {
  float L[6], SR[3], SC[3];
};

__device__ __forceinline__ void abs32_zero(Abs32Chunk &A) {
#pragma unroll
  for (int a = 0; a < 6; ++a) A.L[a] = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) A.SR[a] = A.SC[a] = 0.f;
}

__device__ __forceinline__ void abs32_flush(const Abs32Chunk &A, PairSums &S) {
#pragma unroll
  for (int a = 0; a < 6; ++a) S.L[a] += A.L[a];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    S.SR[a] += A.SR[a];
    S.SC[a] += A.SC[a];
  }
}

// Pair body of the single-precision form, as the paper's GPU code computes
// it (Sec. 3: single precision throughout the particle interactions): r is
// the difference of the absolute FP32 positions, phi_j - phi_i that of the
// FP32 potentials, and every sum of Eq. (sph) is an FP32 sum over the list
// fill.  Only the totals over the fills and the epilogue are FP64.
template <int DIM, bool PST4>
__device__ __forceinline__ void abs32_body(const MixedI &I, const float4 &xi, const float phii, const float4 &xj,
                                           const float4 &b1, const float phij, MixedChunk &C, Abs32Chunk &A,
                                           PairSums &S) {
  const float rx = xj.x - xi.x, ry = xj.y - xi.y, rz = DIM == 3 ? xj.z - xi.z : 0.f;
  const float r2 = rx * rx + ry * ry + rz * rz;
  S.coincident |= (r2 == 0.f);
  const float is = rsqrtf(r2);
  const float s = r2 * is;
  const float q = fminf(s * I.inv_h, 2.0f);
  const float t = 1.0f - 0.5f * q;
  const float t2 = t * t, t3 = t2 * t;
  const float wv = I.kfac * t3 * b1.w;
  const float gx = wv * rx, gy = wv * ry, gz = wv * rz;
  A.L[0] += rx * gx;
  A.L[1] += ry * gy;
  A.L[3] += rx * gy;
  if (DIM == 3) {
    A.L[2] += rz * gz;
    A.L[4] += rx * gz;
    A.L[5] += ry * gz;
  }
  const float dph = phij - phii;
  const float dux = b1.x - I.a1.x, duy = b1.y - I.a1.y, duz = DIM == 3 ? b1.z - I.a1.z : 0.f;
  const float dun = (dux * rx + duy * ry + duz * rz) * is;
  const float c2 = dph - I.c0f * dun;
  const float cs = phij + phii;
  A.SR[0] += c2 * gx;
  A.SR[1] += c2 * gy;
  A.SC[0] += cs * gx;
  A.SC[1] += cs * gy;
  if (DIM == 3) {
    A.SR[2] += c2 * gz;
    A.SC[2] += cs * gz;
  }
  C.gsf[0] += gx;
  C.gsf[1] += gy;
  if (DIM == 3) C.gsf[2] += gz;
  C.Nf[0] += dux * gx;
  C.Nf[1] += duy * gy;
  C.Nf[3] += dux * gy + duy * gx;
  if (DIM == 3) {
    C.Nf[2] += duz * gz;
    C.Nf[4] += dux * gz + duz * gx;
    C.Nf[5] += duy * gz + duz * gy;
  }
  C.Df += wv * dph;
  const float W = I.alpha * t2 * t2 * (2.0f * q + 1.0f);
  const float wr = W * I.w0inv;
  const float wrn = PST4 ? (wr * wr) * (wr * wr) : powf(wr, I.pst_n);
  C.Pf[0] += wrn * gx;
  C.Pf[1] += wrn * gy;
  if (DIM == 3) C.Pf[2] += wrn * gz;
}

// The mixed pair pass with its own candidate search (FP32 test on the
// absolute FP32 positions).  ABS: the single-precision form's body.  KEEP: as for the FP64 pass -- search radius
// 2h + skin, tagged skin candidates skipped by the body, non-empty list
// fills kept in kl.
template <int DIM, bool PST4, bool KEEP, bool ABS = false>
__global__ void __launch_bounds__(256) WB_MIXED_ATTR
    k_pair_mixed(Phys P, Grid g, MixedRec rec, const uint32_t *__restrict__ cs_f, const uint32_t *__restrict__ cs_d,
                 uint32_t nf, Scalars *sc, Rates out, uint32_t *__restrict__ cand, KeptLists kl) {
  __shared__ uint32_t list[kMList][kBlock];
  const int tid = threadIdx.x;
  const uint32_t i = xcd_block(blockIdx.x, gridDim.x) * kBlock + tid;
  const bool active = i < nf;

  float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0, axa = a0;
  double phii = 0.0;
  if (active) {
    a0 = rec.r0[i];
    a1 = rec.r1[i];
    axa = rec.xa[i];
    phii = rec.phi[i];
  }
  const MixedI I = mixed_i(P, g, a0, a1, phii);
  const float two_h2 = (float)P.two_h2;
  // the kept-list work behind a run-time test (launches in this mode always
  // have a skin): compiled unconditionally it costs spilled registers
  const bool keep = KEEP && P.skin_max > 0.0;
  const double rho = keep ? P.two_h + P.skin_max : P.two_h;
  const float rho2 = keep ? (float)(rho * rho) : two_h2;
  // this lane's kept-list bookkeeping in LDS (packed chunk counts, chunks
  // so far at bit kKeptNchShift, saturating at 15): touched once per fill,
  // it holds no registers through the search
  __shared__ unsigned long long kbook[KEEP ? kBlock : 1];
  if (KEEP) kbook[tid] = 0ull;

  PairSums S;
  sums_zero(S);

  // dense pair body over the first cnt entries of this lane's list
  auto run_list = [&](int cnt) {
    if (keep) {  // copy the fill for the later right-hand sides
      const int kmax = wave_max_int(cnt);
      unsigned long long book = kbook[tid];
      const int chunk = (int)(book >> kKeptNchShift);
      const bool room = chunk < kKeepChunks;
      uint32_t *dst = kl.ent + kept_entry(i, min(chunk, kKeepChunks - 1), 0);
      // eight LDS reads in flight before their stores (read per entry, the
      // copy waited out the LDS latency once per entry)
      for (int k0 = 0; k0 < kmax; k0 += 8) {
        uint32_t e[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) e[u] = list[min(k0 + u, kMList - 1)][tid];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (room && k0 + u < cnt) dst[(size_t)(k0 + u) * 64u] = e[u];
      }
      if (cnt > 0) {
        if (room) book |= (unsigned long long)cnt << (6 * chunk);
        else sc->vovf = 1u;
        book = (book & ((1ull << kKeptNchShift) - 1ull)) | ((unsigned long long)min(chunk + 1, 15) << kKeptNchShift);
        kbook[tid] = book;
      }
    }
    MixedChunk C;
    chunk_zero(C);
    if constexpr (ABS) {
      Abs32Chunk A;
      abs32_zero(A);
      const float phif = (float)phii;
      for (int k = 0; k < cnt; ++k) {
        const uint32_t e = list[k][tid];
        if (KEEP && (e & kSkinTag)) continue;
        const uint32_t j = e;
        abs32_body<DIM, PST4>(I, axa, phif, rec.xa[j], rec.r1[j], (float)rec.phi[j], C, A, S);
        if (KEEP) S.nnb += 1;
      }
      abs32_flush(A, S);
    } else {
      for (int k = 0; k < cnt; ++k) {
        const uint32_t e = list[k][tid];
        if (KEEP && (e & kSkinTag)) continue;
        const uint32_t j = e;
        mixed_body<DIM, PST4>(I, rec.r0[j], rec.r1[j], rec.phi[j], C, S);
        if (KEEP) S.nnb += 1;
      }
    }
    chunk_flush(C, S);
    if (!KEEP) S.nnb += cnt;
  };

  // candidate search with the rows walked in lockstep by the wave
  CellPos cp;
  cp.cx = I.cix;
  cp.cy = I.ciy;
  cp.cz = DIM == 3 ? I.ciz : 0;
  cp.ux = a0.x * (float)g.invR;
  cp.uy = a0.y * (float)g.invR;
  cp.uz = DIM == 3 ? a0.z * (float)g.invR : 0.0f;
  auto load = [&](uint32_t j) { return rec.xa[j]; };
  auto near = [&](const float4 &b, uint32_t j) -> uint32_t {
    const float dx = b.x - axa.x, dy = b.y - axa.y, dz = DIM == 3 ? b.z - axa.z : 0.f;
    const float r2 = dx * dx + dy * dy + dz * dz;
    if (!KEEP) return j != i && r2 <= two_h2 ? 1u : 0u;
    return j != i && r2 <= rho2 ? (r2 <= two_h2 ? 1u : 2u) : 0u;
  };
  int cnt = 0;
  CoopWalk cw;
  coop_init(cw, g, active, (float)rho, DIM);
  for (;;) {
    const bool fin =
        coop_fill<DIM, kMList, kMBatch>(cw, g, cs_f, cs_d, nf, cp, &list[0][tid], kBlock, cnt, S.ntest, load, near);
    run_list(cnt);
    cnt = 0;
    if (fin) break;
  }
  if (keep) {
    const unsigned long long book = kbook[tid];
    const int nch = min((int)(book >> kKeptNchShift), kKeepChunks);
    kl.cnt[i] = (book & ((1ull << kKeptNchShift) - 1ull)) | ((unsigned long long)nch << kKeptNchShift);
  }
  pair_epilogue<DIM>(P, sc, out, cand, i, active, S);
}

// A right-hand side from kept candidates: the same FP32 test as the search,
// on the refreshed records, then the same body, one FP32 chunk sum per kept
// chunk.  ABS: the single-precision form's body.
template <int DIM, bool PST4, bool ABS = false>
__global__ void __launch_bounds__(256) WB_MIXED_ATTR
    k_pair_kept_mixed(Phys P, Grid g, MixedRec rec, uint32_t nf, Scalars *sc, Rates out,
                      uint32_t *__restrict__ cand, KeptLists kl) {
  __shared__ uint32_t list[kMList][kBlock];
  const int tid = threadIdx.x;
  const uint32_t i = xcd_block(blockIdx.x, gridDim.x) * kBlock + tid;
  const bool active = i < nf;
  float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0, axa = a0;
  double phii = 0.0;
  if (active) {
    a0 = rec.r0[i];
    a1 = rec.r1[i];
    axa = rec.xa[i];
    phii = rec.phi[i];
  }
  const MixedI I = mixed_i(P, g, a0, a1, phii);
  const float two_h2 = (float)P.two_h2;
  PairSums S;
  sums_zero(S);
  const unsigned long long counts = active ? kl.cnt[i] : 0ull;
  const int nch = (int)(counts >> kKeptNchShift);
  const int wch = wave_max_int(nch);
  for (int c = 0; c < wch; ++c) {
    const int cnt = c < nch ? kept_count(counts, c) : 0;
    const int kmax = wave_max_int(cnt);
    // stage the chunk in this lane's LDS column, eight loads in flight at once
    const uint32_t *src = kl.ent + kept_entry(i, c, 0);
    for (int k0 = 0; k0 < kmax; k0 += 8) {
      uint32_t e[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) e[u] = k0 + u < cnt ? src[(size_t)(k0 + u) * 64u] : 0u;
#pragma unroll
      for (int u = 0; u < 8; ++u) list[k0 + u][tid] = e[u];
    }
    MixedChunk C;
    chunk_zero(C);
    Abs32Chunk A;
    if (ABS) abs32_zero(A);
    uint32_t en = cnt > 0 ? list[0][tid] : 0u;
    for (int k = 0; k < cnt; ++k) {
      const uint32_t j = en & ~kSkinTag;
      const float4 b = rec.xa[j];
      if (k + 1 < cnt) en = list[k + 1][tid];
      const float dx = b.x - axa.x, dy = b.y - axa.y, dz = DIM == 3 ? b.z - axa.z : 0.f;
      if (dx * dx + dy * dy + dz * dz <= two_h2) {
        if constexpr (ABS)
          abs32_body<DIM, PST4>(I, axa, (float)phii, b, rec.r1[j], (float)rec.phi[j], C, A, S);
        else
          mixed_body<DIM, PST4>(I, rec.r0[j], rec.r1[j], rec.phi[j], C, S);
        S.nnb += 1;
      }
    }
    if (ABS) abs32_flush(A, S);
    chunk_flush(C, S);
    S.ntest += (uint32_t)cnt;
  }
  pair_epilogue<DIM>(P, sc, out, cand, i, active, S);
}

template <int DIM>
void launch_pair_mixed_inst(const Phys &P, const Grid &g, const MixedRec &rec, const uint32_t *cs_f,
                            const uint32_t *cs_d, uint32_t nf, Scalars *sc, const Rates &out, uint32_t *cand,
                            const KeptLists &kl, int mode, bool abs32, hipStream_t s) {
  dim3 gr(grid_for(nf)), bl(kBlock);
  const bool p4 = P.pst_n == 4.0;
  if (abs32) {
    if (mode == kPairSearch) {
      if (p4)
        hipLaunchKernelGGL((k_pair_mixed<DIM, true, false, true>), gr, bl, 0, s, P, g, rec, cs_f, cs_d, nf, sc,
                           out, cand, kl);
      else
        hipLaunchKernelGGL((k_pair_mixed<DIM, false, false, true>), gr, bl, 0, s, P, g, rec, cs_f, cs_d, nf,
                           sc, out, cand, kl);
    } else if (mode == kPairSearchKeep) {
      if (p4)
        hipLaunchKernelGGL((k_pair_mixed<DIM, true, true, true>), gr, bl, 0, s, P, g, rec, cs_f, cs_d, nf, sc,
                           out, cand, kl);
      else
        hipLaunchKernelGGL((k_pair_mixed<DIM, false, true, true>), gr, bl, 0, s, P, g, rec, cs_f, cs_d, nf, sc,
                           out, cand, kl);
    } else {
      if (p4)
        hipLaunchKernelGGL((k_pair_kept_mixed<DIM, true, true>), gr, bl, 0, s, P, g, rec, nf, sc, out, cand, kl);
      else
        hipLaunchKernelGGL((k_pair_kept_mixed<DIM, false, true>), gr, bl, 0, s, P, g, rec, nf, sc, out, cand,
                           kl);
    }
  } else if (mode == kPairSearch) {
    if (p4)
      hipLaunchKernelGGL((k_pair_mixed<DIM, true, false>), gr, bl, 0, s, P, g, rec, cs_f, cs_d, nf, sc, out,
                         cand, kl);
    else
      hipLaunchKernelGGL((k_pair_mixed<DIM, false, false>), gr, bl, 0, s, P, g, rec, cs_f, cs_d, nf, sc, out,
                         cand, kl);
  } else if (mode == kPairSearchKeep) {
    if (p4)
      hipLaunchKernelGGL((k_pair_mixed<DIM, true, true>), gr, bl, 0, s, P, g, rec, cs_f, cs_d, nf, sc, out,
                         cand, kl);
    else
      hipLaunchKernelGGL((k_pair_mixed<DIM, false, true>), gr, bl, 0, s, P, g, rec, cs_f, cs_d, nf, sc, out,
                         cand, kl);
  } else {
    if (p4)
      hipLaunchKernelGGL((k_pair_kept_mixed<DIM, true>), gr, bl, 0, s, P, g, rec, nf, sc, out, cand, kl);
    else
      hipLaunchKernelGGL((k_pair_kept_mixed<DIM, false>), gr, bl, 0, s, P, g, rec, nf, sc, out, cand, kl);
  }
}

hipError_t launch_pair_mixed(const Phys &P, const Grid &g, const MixedRec &rec, const uint32_t *cs_f,
                             const uint32_t *cs_d, uint32_t nf, Scalars *sc, const Rates &out, uint32_t *cand,
                             int mode, uint32_t *kent, unsigned long long *kcnt, hipStream_t s, bool abs32) {
  if (nf == 0) return hipSuccess;
  if (mode != kPairSearch && (!kent || !kcnt)) return hipErrorInvalidValue;
  KeptLists kl{kent, kcnt};
  if (P.dim == 2)
    launch_pair_mixed_inst<2>(P, g, rec, cs_f, cs_d, nf, sc, out, cand, kl, mode, abs32, s);
  else
    launch_pair_mixed_inst<3>(P, g, rec, cs_f, cs_d, nf, sc, out, cand, kl, mode, abs32, s);
  return hipGetLastError();
}

// ------------------------------------------------------- scan-region pass

// The scan-region test of the FP64 path (one wave per candidate) on
// positions reconstructed in FP64 from cell and offset.
template <int DIM>
__global__ void __launch_bounds__(256) k_scan_mixed(Phys P, Grid g, MixedRec rec, const uint32_t *__restrict__ cs_f,
                                                    const uint32_t *__restrict__ cs_d, uint32_t nf,
                                                    const uint32_t *__restrict__ list,
                                                    const uint32_t *__restrict__ count, Rates out, Scalars *sc) {
  __shared__ RowTables tab;
  const uint32_t total = *count;
  const int lane = (int)(threadIdx.x & 63);
  const uint32_t gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
  uint32_t nfs = 0;  // surface particles found by this wave (one atomic add at the end)
  for (uint32_t k = gw; k < total; k += nw) {
    const uint32_t i = list[k];
    const float4 a = rec.r0[i];
    const uint32_t ci = __float_as_uint(a.w);
    const double px = pos_of(g.lo[0], g.R, cell_x(ci), a.x), py = pos_of(g.lo[1], g.R, cell_y(ci), a.y),
                 pz = DIM == 3 ? pos_of(g.lo[2], g.R, cell_z(ci), a.z) : 0.0;
    const double n[3] = {out.nrm[0][i], out.nrm[1][i], DIM == 3 ? out.nrm[2][i] : 0.0};
    const double T[3] = {px + P.h * n[0], py + P.h * n[1], DIM == 3 ? pz + P.h * n[2] : 0.0};
    CellPos cp;
    cp.cx = cell_x(ci);
    cp.cy = cell_y(ci);
    cp.cz = DIM == 3 ? cell_z(ci) : 0;
    cp.ux = a.x * (float)g.invR;
    cp.uy = a.y * (float)g.invR;
    cp.uz = DIM == 3 ? a.z * (float)g.invR : 0.0f;
    int nrows;
    const uint32_t M = rows_layout<DIM>(tab, g, cp, (float)P.win, cs_f, cs_d, nf, nrows);
    bool covered = false;
    for (uint32_t c0 = 0; c0 < M && !covered; c0 += 64u) {
      bool cov = false;
      const uint32_t idx = c0 + (uint32_t)lane;
      if (idx < M) {
        const uint32_t j = record_of(tab, nrows, idx);
        if (j != i) {
          const float4 b = rec.r0[j];
          const uint32_t cj = __float_as_uint(b.w);
          const double q[3] = {pos_of(g.lo[0], g.R, cell_x(cj), b.x), pos_of(g.lo[1], g.R, cell_y(cj), b.y),
                               DIM == 3 ? pos_of(g.lo[2], g.R, cell_z(cj), b.z) : 0.0};
          const double s2 = (q[0] - px) * (q[0] - px) + (q[1] - py) * (q[1] - py) + (q[2] - pz) * (q[2] - pz);
          cov = s2 <= P.two_h2 && scan_covers<DIM>(P, q, T, n, s2);
        }
      }
      covered = __ballot(cov) != 0ull;
    }
    wave_lds_sync();  // the tables are rewritten for the next candidate
    if (lane == 0) scan_finish<DIM>(P, out, i, n, covered);
    nfs += covered ? 0u : 1u;
  }
  if (lane == 0 && nfs) atomicAdd(&sc->n_fs, nfs);
}

hipError_t launch_scan_mixed(const Phys &P, const Grid &g, const MixedRec &rec, const uint32_t *cs_f,
                             const uint32_t *cs_d, uint32_t nf, const uint32_t *list, const uint32_t *count,
                             const Rates &out, Scalars *sc, hipStream_t s) {
  if (nf == 0) return hipSuccess;
  unsigned blocks = candidate_grid(nf);
  if (P.dim == 2)
    hipLaunchKernelGGL(k_scan_mixed<2>, dim3(blocks), dim3(kBlock), 0, s, P, g, rec, cs_f, cs_d, nf, list, count, out,
                       sc);
  else
    hipLaunchKernelGGL(k_scan_mixed<3>, dim3(blocks), dim3(kBlock), 0, s, P, g, rec, cs_f, cs_d, nf, list, count, out,
                       sc);
  return hipGetLastError();
}

// ------------------------------------------------------------ integration

template <int DIM>
__global__ void __launch_bounds__(256) k_stage_mixed(Phys P, Grid g, FluidMixed f, Rates r, int64_t n,
                                                     Scalars *sc, int stage, MixedRec rec, int write_rec) {
  __shared__ double sh[kBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double u2 = 0.0;
  if (i < n) {
    const double dt = sc->dt;
    uint32_t c = f.cell[i];
    uint32_t bad = 0u;
    int cc[3] = {cell_x(c), cell_y(c), cell_z(c)};
    float of[3] = {0.f, 0.f, 0.f}, uf[3] = {0.f, 0.f, 0.f};
    for (int a = 0; a < DIM; ++a) {
      float o = f.o[a][i], oc = f.oc[a][i], u = f.u[a][i], uc = f.uc[a][i];
      // position first (uses the stage's velocity), then velocity
      const double vx = ((double)u - (double)uc + r.dus[a][i]) * dt;
      const double va = r.acc[a][i] * dt;
      if (stage == 1) {
        kahan_add(o, oc, vx);
        kahan_add(u, uc, va);
        f.dx1[a][i] = (float)vx;
        f.du1[a][i] = (float)va;
      } else {
        kahan_add(o, oc, 0.5 * (vx - (double)f.dx1[a][i]));
        kahan_add(u, uc, 0.5 * (va - (double)f.du1[a][i]));
      }
      // keep the offset inside its cell: move whole cells, subtract k R exactly
      const double ov = (double)o - (double)oc;
      if (!isfinite(ov) || !isfinite((double)u)) bad |= kErrNonFinite;
      const double kf = isfinite(ov) ? floor(ov / g.R) : 0.0;
      const int kc = (int)fmin(fmax(kf, -4096.0), 4096.0);
      if (kc != 0) {
        cc[a] += kc;
        kahan_add(o, oc, -(double)kc * g.R);
      }
      f.o[a][i] = o;
      f.oc[a][i] = oc;
      f.u[a][i] = u;
      f.uc[a][i] = uc;
      of[a] = o;
      uf[a] = u;
      u2 += (double)u * (double)u;
    }
    // a particle whose cell left the grid is an error (reported at the next
    // synchronisation); the packed fields are kept from wrapping meanwhile
    for (int a = 0; a < DIM; ++a) {
      const double xa = g.lo[a] + (double)cc[a] * g.R + ((double)of[a] - (double)f.oc[a][i]);
      if (cc[a] < 0 || cc[a] >= g.N[a] || !(xa >= g.lo[a] && xa <= g.hi[a])) bad |= kErrDomain;
    }
    for (int a = 0; a < 3; ++a) cc[a] = min(max(cc[a], 0), a == 2 ? 1023 : 2047);
    c = pack_cell(cc[0], cc[1], cc[2]);
    f.cell[i] = c;
    const double dp = r.dphi[i] * dt;
    double ph = f.phi[i];
    if (stage == 1) {
      ph += dp;
      f.dphi1[i] = dp;
    } else {
      ph += 0.5 * (dp - f.dphi1[i]);
    }
    f.phi[i] = ph;
    if (!isfinite(ph)) bad |= kErrNonFinite;
    if (bad) atomicOr(&sc->err, bad);
    if (write_rec) {  // the records of the new state, as the reorder writes them
      const float V = (float)((double)f.m[i] / (P.rho0 * exp(ph * P.inv_c02)));
      float xa[3] = {0.f, 0.f, 0.f};
      for (int a = 0; a < DIM; ++a) xa[a] = (float)pos_of(g.lo[a], g.R, cc[a], of[a]);
      rec.r0[i] = make_float4(of[0], of[1], of[2], __uint_as_float(c));
      rec.r1[i] = make_float4(uf[0], uf[1], uf[2], V);
      rec.phi[i] = ph;
      rec.xa[i] = make_float4(xa[0], xa[1], xa[2], 0.f);
    }
  }
  // max |U|^2 of the new state (the FP32 velocities, as the max-|U| kernel reads them)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) u2 = fmax(u2, __shfl_xor(u2, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = u2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = sh[0];
    for (int w = 1; w < kBlock / 64; ++w) b = fmax(b, sh[w]);
    atomicMax(&sc->umax2_bits, (unsigned long long)__double_as_longlong(b));
  }
}

hipError_t launch_stage_mixed(const Phys &P, const Grid &g, const FluidMixed &f, const Rates &r, int64_t nf,
                              Scalars *sc, int stage, hipStream_t s, const MixedRec *rec) {
  hipError_t e = launch_reset_umax(sc, s);
  if (e != hipSuccess || nf <= 0) return e;
  const MixedRec rr = rec ? *rec : MixedRec{nullptr, nullptr, nullptr, nullptr};
  if (P.dim == 2)
    hipLaunchKernelGGL(k_stage_mixed<2>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, g, f, r, nf, sc, stage, rr,
                       rec ? 1 : 0);
  else
    hipLaunchKernelGGL(k_stage_mixed<3>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, g, f, r, nf, sc, stage, rr,
                       rec ? 1 : 0);
  return hipGetLastError();
}

// ----------------------------------------------------------------- fields

template <int DIM>
__global__ void k_fields_mixed(Phys P, Grid g, FluidMixed f, int64_t n, int field, void *dst, uint32_t nout) {
#pragma clang fp contract(off)
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint32_t id = f.id[k];
  if (id >= nout) return;
  const uint32_t c = f.cell[k];
  const int cc[3] = {cell_x(c), cell_y(c), cell_z(c)};
  double *dd = (double *)dst;
  int32_t *di = (int32_t *)dst;
  switch (field) {
    case SPH_FIELD_X:
      for (int a = 0; a < DIM; ++a)
        dd[(int64_t)id * DIM + a] = g.lo[a] + (double)cc[a] * g.R + ((double)f.o[a][k] - (double)f.oc[a][k]);
      break;
    case SPH_FIELD_U:
      for (int a = 0; a < DIM; ++a) dd[(int64_t)id * DIM + a] = (double)f.u[a][k] - (double)f.uc[a][k];
      break;
    case SPH_FIELD_PHI: dd[id] = f.phi[k]; break;
    case SPH_FIELD_MASS: dd[id] = (double)f.m[k]; break;
    case SPH_FIELD_RHO: dd[id] = P.rho0 * exp(f.phi[k] * P.inv_c02); break;
    case SPH_FIELD_P: dd[id] = P.c0 * P.c0 * (P.rho0 * exp(f.phi[k] * P.inv_c02) - P.rho0); break;
    case SPH_FIELD_CELL:
      for (int a = 0; a < 3; ++a) di[(int64_t)id * 3 + a] = cc[a];
      break;
    default: break;
  }
}

hipError_t launch_fields_mixed(const Phys &P, const Grid &g, const FluidMixed &f, int64_t nf, int field, void *dst,
                               hipStream_t s, uint32_t nout) {
  if (nf <= 0) return hipSuccess;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_fields_mixed<2>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, g, f, nf, field, dst, nout);
  else
    hipLaunchKernelGGL(k_fields_mixed<3>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, g, f, nf, field, dst, nout);
  return hipGetLastError();
}

__global__ void k_dummy_fields_mixed(Phys P, MixedRec rec, int64_t nf, const uint32_t *__restrict__ did, int64_t nd,
                                     int field, void *dst, int dim, uint32_t nout) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nd) return;
  const uint32_t id = did[k];
  if (id >= nout) return;
  double *dd = (double *)dst;
  const int64_t o = nf + k;
  const double ph = rec.phi[o];
  switch (field) {
    case SPH_FIELD_U: {
      const float4 v = rec.r1[o];
      const float c[3] = {v.x, v.y, v.z};
      for (int a = 0; a < dim; ++a) dd[(int64_t)id * dim + a] = (double)c[a];
      break;
    }
    case SPH_FIELD_PHI: dd[id] = ph; break;
    case SPH_FIELD_RHO: dd[id] = P.rho0 * exp(ph * P.inv_c02); break;
    case SPH_FIELD_P: dd[id] = P.c0 * P.c0 * (P.rho0 * exp(ph * P.inv_c02) - P.rho0); break;
    default: break;
  }
}

hipError_t launch_dummy_fields_mixed(const Phys &P, const MixedRec &rec, int64_t nf, const uint32_t *did, int64_t nd,
                                     int field, void *dst, hipStream_t s, uint32_t nout) {
  if (nd <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dummy_fields_mixed, dim3(grid_for(nd)), dim3(kBlock), 0, s, P, rec, nf, did, nd, field, dst,
                     P.dim, nout);
  return hipGetLastError();
}

}  // namespace wb
