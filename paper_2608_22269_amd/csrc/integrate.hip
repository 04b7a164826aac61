// Time integration and bookkeeping kernels:
//   - fluid max |U| (atomic max on the bit pattern of a non-negative double,
//     order independent, hence deterministic) and the time-step rule of
//     Sec. 2.3 evaluated on the device, so a step never waits for the host;
//   - the two SSP-RK2 stage updates (Sec. 2.3), FP64 path;
//   - gathers from HashID order back to the caller's particle order;
//   - the input split by particle kind at set-up.
#include "common.h"
#include "kernels.h"

namespace wb {

// --------------------------------------------------------------- max |U|

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_umax(const T *__restrict__ u0, const T *__restrict__ u1,
                                              const T *__restrict__ u2, int64_t n, Scalars *sc) {
  __shared__ double sh[4];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double a = (double)u0[i], b = (double)u1[i], c = DIM == 3 ? (double)u2[i] : 0.0;
    m = fmax(m, a * a + b * b + c * c);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    atomicMax(&sc->umax2_bits, (unsigned long long)__double_as_longlong(b));
  }
}

__global__ void k_reset_umax(Scalars *sc) { sc->umax2_bits = 0ull; }

hipError_t launch_reset_umax(Scalars *sc, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_umax, dim3(1), dim3(1), 0, s, sc);
  return hipGetLastError();
}

hipError_t launch_umax(int dim, const double *const u[3], const float *const uf[3], int64_t nf, Scalars *sc,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_reset_umax, dim3(1), dim3(1), 0, s, sc);
  if (nf > 0) {
    unsigned blocks = grid_for(nf);
    if (blocks > 1024) blocks = 1024;
    if (u) {
      if (dim == 2)
        hipLaunchKernelGGL((k_umax<double, 2>), dim3(blocks), dim3(256), 0, s, u[0], u[1], u[1], nf, sc);
      else
        hipLaunchKernelGGL((k_umax<double, 3>), dim3(blocks), dim3(256), 0, s, u[0], u[1], u[2], nf, sc);
    } else {
      if (dim == 2)
        hipLaunchKernelGGL((k_umax<float, 2>), dim3(blocks), dim3(256), 0, s, uf[0], uf[1], uf[1], nf, sc);
      else
        hipLaunchKernelGGL((k_umax<float, 3>), dim3(blocks), dim3(256), 0, s, uf[0], uf[1], uf[2], nf, sc);
    }
  }
  return hipGetLastError();
}

// dt = CFL min(dx/(C0 + |U|max), dx^2/(2 nu), sqrt(2 dx/|G|max)) at the start
// of a step (Sec. 2.3); the first right-hand side is evaluated at t.
__global__ void k_dt(Phys P, Scalars *sc, double dt_override) {
  double umax = sqrt(__longlong_as_double((long long)sc->umax2_bits));
  double dt = P.dx / (P.c0 + umax);
  if (P.nu > 0.0) dt = fmin(dt, P.dx * P.dx / (2.0 * P.nu));
  if (P.gmax > 0.0) dt = fmin(dt, sqrt(2.0 * P.dx / P.gmax));
  dt *= P.cfl;
  sc->dt = dt_override > 0.0 ? dt_override : dt;
  sc->umax = umax;
  sc->t_rhs = sc->t;
}

hipError_t launch_dt(const Phys &P, Scalars *sc, double dt_override, hipStream_t s) {
  hipLaunchKernelGGL(k_dt, dim3(1), dim3(1), 0, s, P, sc, dt_override);
  return hipGetLastError();
}

// Stage bookkeeping: U_max of the stage and the time of its right-hand side
// (stage 1 at t, stage 2 at t + dt); statistics counters restart.
__global__ void k_stage_time(Scalars *sc, int stage, int mode) {
  if (sc->mode == (uint32_t)kPairKept) {  // statistics of the previous right-hand side by kind
    sc->pairs_k = sc->pairs;
    sc->tests_k = sc->tests;
  } else {
    sc->pairs_s = sc->pairs;
    sc->tests_s = sc->tests;
  }
  sc->mode = (uint32_t)mode;
  if (mode == kPairSearchKeep) {  // this right-hand side builds new kept lists
    sc->disp = 0.0;
    sc->vovf = 0u;
  }
  sc->umax = sqrt(__longlong_as_double((long long)sc->umax2_bits));
  sc->t_rhs = stage == 2 ? sc->t + sc->dt : sc->t;
  sc->n_cand = 0;
  sc->n_scan = 0;
  sc->n_fs = 0;
  sc->n_cons = 0;
  sc->n_sing = 0;
  sc->n_mlp = 0;
  sc->pairs = 0ull;
  sc->tests = 0ull;
}

hipError_t launch_stage_time(Scalars *sc, int stage, hipStream_t s, int mode) {
  hipLaunchKernelGGL(k_stage_time, dim3(1), dim3(1), 0, s, sc, stage, mode);
  return hipGetLastError();
}

// Bound on the move of every particle by the stage update just made (Sec.
// 2.3), added to sc->disp.  Stage 1: x1 - x0 = dt (U0 + dU0), |U0| <= U_max0
// and the shifting velocity is clamped to U_max0 / 2, so |x1 - x0| <= 1.5 dt
// U_max0.  Stage 2: x2 - x1 = (dt (U1 + dU1) - dt (U0 + dU0)) / 2, so
// |x2 - x1| <= 0.75 dt (U_max0 + U_max1).  The relative margin covers the
// rounding of the bound and of FP32 velocities.
__global__ void k_disp_add(Scalars *sc, int stage) {
  const double dt = sc->dt;
  if (stage == 1) {
    sc->umax1 = sc->umax;
    sc->disp += 1.5 * dt * sc->umax * (1.0 + 1e-6);
  } else {
    sc->disp += 0.75 * dt * (sc->umax1 + sc->umax) * (1.0 + 1e-6);
  }
}

hipError_t launch_disp_add(Scalars *sc, int stage, hipStream_t s) {
  hipLaunchKernelGGL(k_disp_add, dim3(1), dim3(1), 0, s, sc, stage);
  return hipGetLastError();
}

__global__ void k_set_time(Scalars *sc, double t) {
  sc->t = t;
  sc->t_rhs = t;
}

hipError_t launch_set_time(Scalars *sc, double t, hipStream_t s) {
  hipLaunchKernelGGL(k_set_time, dim3(1), dim3(1), 0, s, sc, t);
  return hipGetLastError();
}

__global__ void k_advance_time(Scalars *sc) {
  sc->t = sc->t + sc->dt;
  sc->steps += 1.0;
}

hipError_t launch_advance_time(Scalars *sc, hipStream_t s) {
  hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(1), 0, s, sc);
  return hipGetLastError();
}

// ------------------------------------------------------------ SSP-RK2, FP64
// Stage 1: phi1 = phi + dt Dphi, U1 = U + dt a, x1 = x + dt (U + dU), with
// the state of t^n read from the stage-0 arrays (the caller swaps the state
// and stage-0 arrays first, so t^n needs no copy) and stage 1 written to the
// state arrays.  Stage 2: q = 1/2 q0 + 1/2 (q1 + dt rate(q1)) for phi, U, x.
// Written without contraction, as the equations are printed.  The kernel
// also folds max |U|^2 of the new state into sc->umax2_bits (reset by the
// caller), checks the new phi and U for finiteness when asked, and writes the
// neighbour records of the new state (rec0 = (x, phi), rec1 = (U, V), as the
// reorder writes them) when rec0 is given.
template <int DIM>
__global__ void __launch_bounds__(256) k_stage_f64(Phys P, FluidF64 f, Rates r, int64_t n, Scalars *sc, int stage,
                                                   double4 *__restrict__ rec0, double4 *__restrict__ rec1,
                                                   int check) {
#pragma clang fp contract(off)
  __shared__ double sh[kBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double u2 = 0.0;
  if (i < n) {
    const double dt = sc->dt;
    double xn[3] = {0.0, 0.0, 0.0}, un[3] = {0.0, 0.0, 0.0}, pn;
    if (stage == 1) {  // the state of t^n is in the stage-0 arrays (the caller swapped them)
      pn = f.phi0[i] + dt * r.dphi[i];
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const double x = f.x0[a][i], u = f.u0[a][i];
        un[a] = u + dt * r.acc[a][i];
        xn[a] = x + dt * (u + r.dus[a][i]);
      }
    } else {
      pn = 0.5 * f.phi0[i] + 0.5 * (f.phi[i] + dt * r.dphi[i]);
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        const double u1 = f.u[a][i];
        un[a] = 0.5 * f.u0[a][i] + 0.5 * (u1 + dt * r.acc[a][i]);
        xn[a] = 0.5 * f.x0[a][i] + 0.5 * (f.x[a][i] + dt * (u1 + r.dus[a][i]));
      }
    }
    f.phi[i] = pn;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      f.u[a][i] = un[a];
      f.x[a][i] = xn[a];
    }
    u2 = un[0] * un[0] + un[1] * un[1] + un[2] * un[2];
    if (check) {
      bool ok = isfinite(pn);
      for (int a = 0; a < DIM; ++a) ok = ok && isfinite(un[a]);
      if (!ok) atomicOr(&sc->err, kErrNonFinite);
    }
    if (rec0) {
      const double V = f.m[i] / (P.rho0 * exp(pn * P.inv_c02));
      rec0[i] = make_double4(xn[0], xn[1], xn[2], pn);
      rec1[i] = make_double4(un[0], un[1], un[2], V);
    }
  }
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

hipError_t launch_stage_f64(const Phys &P, const FluidF64 &f, const Rates &r, int64_t nf, Scalars *sc, int stage,
                            hipStream_t s, double4 *rec0, double4 *rec1, int check) {
  hipLaunchKernelGGL(k_reset_umax, dim3(1), dim3(1), 0, s, sc);
  if (nf <= 0) return hipGetLastError();
  if (P.dim == 2)
    hipLaunchKernelGGL(k_stage_f64<2>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, f, r, nf, sc, stage, rec0, rec1,
                       check);
  else
    hipLaunchKernelGGL(k_stage_f64<3>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, f, r, nf, sc, stage, rec0, rec1,
                       check);
  return hipGetLastError();
}

// ---------------------------------------------------------------- gathers

__global__ void k_gather_f64(const double *__restrict__ src, const uint32_t *__restrict__ id, int64_t n,
                             double *__restrict__ dst, int stride, int comp, uint32_t nout) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && id[k] < nout) dst[(int64_t)id[k] * stride + comp] = src[k];
}

__global__ void k_gather_f32_as_f64(const float *__restrict__ src, const uint32_t *__restrict__ id, int64_t n,
                                    double *__restrict__ dst, int stride, int comp, uint32_t nout) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && id[k] < nout) dst[(int64_t)id[k] * stride + comp] = (double)src[k];
}

__global__ void k_gather_rec(const double4 *__restrict__ rec, const uint32_t *__restrict__ id, int64_t n,
                             double *__restrict__ dst, int stride, int comp, int ncomp, uint32_t nout) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || id[k] >= nout) return;
  double4 v = rec[k];
  double c[4] = {v.x, v.y, v.z, v.w};
  for (int a = 0; a < ncomp; ++a) dst[(int64_t)id[k] * stride + a] = c[comp + a];
}

__global__ void k_gather_u32_bits(const uint32_t *__restrict__ src, const uint32_t *__restrict__ id, int64_t n,
                                  int32_t *__restrict__ dst, uint32_t mask, int shift, uint32_t nout) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && id[k] < nout) dst[id[k]] = (int32_t)((src[k] & mask) >> shift);
}

__global__ void k_gather_i32(const int32_t *__restrict__ src, const uint32_t *__restrict__ id, int64_t n,
                             int32_t *__restrict__ dst, int stride, int comp, uint32_t nout) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && id[k] < nout) dst[(int64_t)id[k] * stride + comp] = src[k];
}

__global__ void k_gather_rows_f32(const float *__restrict__ src, const uint32_t *__restrict__ id, int64_t n,
                                  int width, float *__restrict__ dst, uint32_t nout) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || id[k] >= nout) return;
  for (int c = 0; c < width; ++c) dst[(int64_t)id[k] * width + c] = src[k * width + c];
}

__global__ void k_fill_f64(double *p, double v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f32(float *p, float v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <int DIM>
__global__ void k_cells_of(Grid g, const double *__restrict__ x, const double *__restrict__ y,
                           const double *__restrict__ z, const uint32_t *__restrict__ id, int64_t n,
                           int32_t *__restrict__ dst, uint32_t nout) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || id[k] >= nout) return;
  int64_t o = (int64_t)id[k] * 3;
  dst[o + 0] = cell_coord(x[k], g.lo[0], g.R);
  dst[o + 1] = cell_coord(y[k], g.lo[1], g.R);
  dst[o + 2] = DIM == 3 ? cell_coord(z[k], g.lo[2], g.R) : 0;
}

// which: 0 rho = rho0 exp(phi/C0^2); 1 p = C0^2 (rho - rho0)  (Eq. eos-water)
__global__ void k_rho_p(Phys P, const double *__restrict__ phi, const uint32_t *__restrict__ id, int64_t n,
                        double *__restrict__ dst, int which, uint32_t nout) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || id[k] >= nout) return;
  double rho = P.rho0 * exp(phi[k] * P.inv_c02);
  dst[id[k]] = which == 0 ? rho : P.c0 * P.c0 * (rho - P.rho0);
}

__global__ void k_rho_p_rec(Phys P, const double4 *__restrict__ rec, const uint32_t *__restrict__ id, int64_t n,
                            double *__restrict__ dst, int which, uint32_t nout) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || id[k] >= nout) return;
  double rho = P.rho0 * exp(rec[k].w * P.inv_c02);
  dst[id[k]] = which == 0 ? rho : P.c0 * P.c0 * (rho - P.rho0);
}

hipError_t launch_gather_f64(const double *src, const uint32_t *id, int64_t n, double *dst, int stride, int comp,
                             hipStream_t s, uint32_t nout) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_f64, dim3(grid_for(n)), dim3(kBlock), 0, s, src, id, n, dst, stride, comp, nout);
  return hipGetLastError();
}

hipError_t launch_gather_f32_as_f64(const float *src, const uint32_t *id, int64_t n, double *dst, int stride,
                                    int comp, hipStream_t s, uint32_t nout) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_f32_as_f64, dim3(grid_for(n)), dim3(kBlock), 0, s, src, id, n, dst, stride, comp, nout);
  return hipGetLastError();
}

hipError_t launch_gather_rec(const double4 *rec, const uint32_t *id, int64_t n, double *dst, int stride, int comp,
                             int ncomp, hipStream_t s, uint32_t nout) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rec, dim3(grid_for(n)), dim3(kBlock), 0, s, rec, id, n, dst, stride, comp, ncomp, nout);
  return hipGetLastError();
}

hipError_t launch_gather_u32_bits(const uint32_t *src, const uint32_t *id, int64_t n, int32_t *dst, uint32_t mask,
                                  int shift, hipStream_t s, uint32_t nout) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_u32_bits, dim3(grid_for(n)), dim3(kBlock), 0, s, src, id, n, dst, mask, shift, nout);
  return hipGetLastError();
}

hipError_t launch_gather_i32(const int32_t *src, const uint32_t *id, int64_t n, int32_t *dst, int stride, int comp,
                             hipStream_t s, uint32_t nout) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_i32, dim3(grid_for(n)), dim3(kBlock), 0, s, src, id, n, dst, stride, comp, nout);
  return hipGetLastError();
}

hipError_t launch_gather_rows_f32(const float *src, const uint32_t *id, int64_t n, int width, float *dst,
                                  hipStream_t s, uint32_t nout) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows_f32, dim3(grid_for(n)), dim3(kBlock), 0, s, src, id, n, width, dst, nout);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_cells_of(const Grid &g, int dim, const double *const x[3], const uint32_t *id, int64_t n,
                           int32_t *dst, hipStream_t s, uint32_t nout) {
  if (n <= 0) return hipSuccess;
  if (dim == 2)
    hipLaunchKernelGGL(k_cells_of<2>, dim3(grid_for(n)), dim3(kBlock), 0, s, g, x[0], x[1], x[1], id, n, dst, nout);
  else
    hipLaunchKernelGGL(k_cells_of<3>, dim3(grid_for(n)), dim3(kBlock), 0, s, g, x[0], x[1], x[2], id, n, dst, nout);
  return hipGetLastError();
}

hipError_t launch_rho_p(const Phys &P, const double *phi, const uint32_t *id, int64_t n, double *dst, int which,
                        hipStream_t s, uint32_t nout) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rho_p, dim3(grid_for(n)), dim3(kBlock), 0, s, P, phi, id, n, dst, which, nout);
  return hipGetLastError();
}

hipError_t launch_rho_p_rec(const Phys &P, const double4 *rec, const uint32_t *id, int64_t n, double *dst,
                            int which, hipStream_t s, uint32_t nout) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rho_p_rec, dim3(grid_for(n)), dim3(kBlock), 0, s, P, rec, id, n, dst, which, nout);
  return hipGetLastError();
}

// ------------------------------------------------------------------ set-up

__global__ void k_kind_flags(const uint8_t *__restrict__ kind, int64_t n, uint32_t *__restrict__ isf,
                             uint32_t *__restrict__ isd) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  isf[i] = kind[i] == 0 ? 1u : 0u;
  isd[i] = kind[i] != 0 ? 1u : 0u;
}

hipError_t launch_kind_flags(const uint8_t *kind, int64_t n, uint32_t *isf, uint32_t *isd, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kind_flags, dim3(grid_for(n)), dim3(kBlock), 0, s, kind, n, isf, isd);
  return hipGetLastError();
}

// Writes fluid rows into f (in original relative order) and dummy rows into
// d; mass == NULL -> m = rho0 exp(phi / C0^2) dx^dim.
__global__ void k_split(Phys P, int64_t n, const double *__restrict__ x, const double *__restrict__ u,
                        const double *__restrict__ phi, const double *__restrict__ mass,
                        const uint8_t *__restrict__ kind, const double *__restrict__ nrm,
                        const uint32_t *__restrict__ frank, const uint32_t *__restrict__ drank, FluidF64 f,
                        Dummies d) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int dim = P.dim;
  double vol = dim == 2 ? P.dx * P.dx : P.dx * P.dx * P.dx;
  double m = mass ? mass[i] : P.rho0 * exp(phi[i] * P.inv_c02) * vol;
  if (kind[i] == 0) {
    uint32_t k = frank[i];
    for (int a = 0; a < dim; ++a) {
      f.x[a][k] = x[i * dim + a];
      f.u[a][k] = u[i * dim + a];
    }
    f.phi[k] = phi[i];
    f.m[k] = m;
    f.id[k] = (uint32_t)i;
  } else {
    uint32_t k = drank[i];
    for (int a = 0; a < dim; ++a) {
      d.x[a][k] = x[i * dim + a];
      d.n[a][k] = nrm[i * dim + a];
    }
    d.phi_in[k] = phi[i];
    d.m[k] = m;
    d.id[k] = (uint32_t)i;
    if (d.mov) {
      d.mov[k] = kind[i] == 2 ? 1 : 0;
      for (int a = 0; a < dim; ++a) d.x0[a][k] = x[i * dim + a];
    }
    if (d.n0[0])
      for (int a = 0; a < dim; ++a) d.n0[a][k] = nrm[i * dim + a];
  }
}

hipError_t launch_split(const Phys &P, int64_t n, const double *x, const double *u, const double *phi,
                        const double *mass, const uint8_t *kind, const double *nrm, const uint32_t *frank,
                        const uint32_t *drank, FluidF64 f, Dummies d, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_split, dim3(grid_for(n)), dim3(kBlock), 0, s, P, n, x, u, phi, mass, kind, nrm, frank, drank,
                     f, d);
  return hipGetLastError();
}

__global__ void k_gather_dummies(const uint32_t *__restrict__ perm, int64_t nd, Dummies src, Dummies dst, int dim) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nd) return;
  uint32_t o = perm[k];
  for (int a = 0; a < dim; ++a) {
    dst.x[a][k] = src.x[a][o];
    dst.n[a][k] = src.n[a][o];
  }
  dst.m[k] = src.m[o];
  dst.phi_in[k] = src.phi_in[o];
  dst.id[k] = src.id[o];
  dst.src[k] = -1;
  if (src.mov) {
    dst.mov[k] = src.mov[o];
    for (int a = 0; a < dim; ++a) dst.x0[a][k] = src.x0[a][o];
  }
  if (src.n0[0])
    for (int a = 0; a < dim; ++a) dst.n0[a][k] = src.n0[a][o];
}

hipError_t launch_gather_dummies(const uint32_t *perm, int64_t nd, Dummies src, Dummies dst, int dim, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_dummies, dim3(grid_for(nd)), dim3(kBlock), 0, s, perm, nd, src, dst, dim);
  return hipGetLastError();
}

// Displacement D(t) since T_0 and velocity U(t) of the prescribed body
// motion (the ditching case of Sec. 4 gives U piecewise in time).  On piece
// k the displacement grows by the integral of a + b s from T_k to
// min(t, T_{k+1}): a (tau - T_k) + b (tau^2 - T_k^2) / 2.  Every product and
// sum is rounded as written (no contraction), so that the body's positions do
// not depend on the compiler's choice of fused operations.
__device__ void body_motion(const Body &B, double t, double D[3], double U[3]) {
#pragma clang fp contract(off)
  for (int a = 0; a < 3; ++a) D[a] = U[a] = 0.0;
  bool found = false;
  for (int k = 0; k < B.pieces; ++k) {
    const double t0 = B.T[k], t1 = B.T[k + 1];
    if (!found && t >= t0 && t <= t1) {
      for (int a = 0; a < 3; ++a) U[a] = B.a[k][a] + B.b[k][a] * t;
      found = true;
    }
    if (t > t0) {
      const double tau = t < t1 ? t : t1;
      for (int a = 0; a < 3; ++a) D[a] += B.a[k][a] * (tau - t0) + B.b[k][a] * (tau * tau - t0 * t0) / 2.0;
    }
  }
}

__global__ void k_body_move(Body B, Dummies d, int64_t nd, int dim, Scalars *sc) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double D[3], U[3];
  body_motion(B, sc->t_rhs, D, U);
  if (k == 0) {
    for (int a = 0; a < 3; ++a) {
      sc->body_x[a] = D[a];
      sc->body_u[a] = U[a];
    }
  }
  if (k >= nd || !d.mov[k]) return;
  for (int a = 0; a < dim; ++a) d.x[a][k] = d.x0[a][k] + D[a];
}

hipError_t launch_body_move(const Body &B, const Dummies &d, int64_t nd, int dim, Scalars *sc, hipStream_t s) {
  if (!d.mov) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_body_move, dim3(grid_for(std::max<int64_t>(nd, 1))), dim3(kBlock), 0, s, B, d, nd, dim, sc);
  return hipGetLastError();
}

// ------------------------------------------------------------- free body

__global__ void k_free_body_place(Dummies d, int64_t nd, int dim, Scalars *sc) {
#pragma clang fp contract(off)
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nd || !d.mov[k]) return;
  const double q[4] = {sc->fb[3], sc->fb[4], sc->fb[5], sc->fb[6]};
  double R[9];
  quat_rotation(q, R);
  double d0[3] = {0.0, 0.0, 0.0}, n0[3] = {0.0, 0.0, 0.0}, dr[3], nr[3];
  for (int a = 0; a < dim; ++a) {
    d0[a] = d.x0[a][k] - sc->fb_c0[a];
    n0[a] = d.n0[a][k];
  }
  mat3_apply(R, d0, dr);
  mat3_apply(R, n0, nr);
  for (int a = 0; a < dim; ++a) {
    d.x[a][k] = sc->fb[a] + dr[a];
    d.n[a][k] = nr[a];
  }
}

hipError_t launch_free_body_place(const Dummies &d, int64_t nd, int dim, Scalars *sc, hipStream_t s) {
  if (!d.mov || !d.n0[0]) return hipErrorInvalidValue;
  if (nd == 0) return hipSuccess;
  hipLaunchKernelGGL(k_free_body_place, dim3(grid_for(nd)), dim3(kBlock), 0, s, d, nd, dim, sc);
  return hipGetLastError();
}

// One block: thread t sums partials t, t + 1024, ... in order, then a fixed
// tree over the block; the result depends only on the partials' order.
constexpr int kBodySumThreads = 1024;
__global__ void __launch_bounds__(kBodySumThreads) k_free_body_sum(const double *__restrict__ ft, int64_t np,
                                                                    Scalars *sc) {
  __shared__ double part[6][kBodySumThreads];
  const int t = threadIdx.x;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t k = t; k < np; k += kBodySumThreads)
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] += ft[(size_t)6 * k + c];
#pragma unroll
  for (int c = 0; c < 6; ++c) part[c][t] = acc[c];
  __syncthreads();
  for (int w = kBodySumThreads / 2; w > 0; w >>= 1) {
    if (t < w)
#pragma unroll
      for (int c = 0; c < 6; ++c) part[c][t] += part[c][t + w];
    __syncthreads();
  }
  if (t < 6) sc->fbF[t] = part[t][0];
}

hipError_t launch_free_body_sum(const double *ft, int64_t np, Scalars *sc, hipStream_t s) {
  hipLaunchKernelGGL(k_free_body_sum, dim3(1), dim3(kBodySumThreads), 0, s, ft, np, sc);
  return hipGetLastError();
}

// Rates of the free body's state y = (c, q, v, omega) under the force F and
// torque T about the centre: dc/dt = v, dv/dt = F / M + G, dq/dt = (0, omega)
// q / 2 (Hamilton product, omega in the world frame), domega/dt = I_w^-1 (T -
// omega x I_w omega) with I_w = R I_body R^T (Euler's equations in the world
// frame).  2D: motion in the plane, rotation about z only.
__device__ void free_body_rates(const FreeBody &B, int dim, const double y[13], const double F[3],
                                const double T[3], const double G[3], double r[13]) {
  const double *q = y + 3, *v = y + 7, *w = y + 10;
  double R[9];
  quat_rotation(q, R);
  // I_w = R I_body R^T
  const double Ib[9] = {B.I[0], B.I[3], B.I[4], B.I[3], B.I[1], B.I[5], B.I[4], B.I[5], B.I[2]};
  double RI[9], Iw[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) RI[3 * i + j] = R[3 * i] * Ib[j] + R[3 * i + 1] * Ib[3 + j] + R[3 * i + 2] * Ib[6 + j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Iw[3 * i + j] = RI[3 * i] * R[3 * j] + RI[3 * i + 1] * R[3 * j + 1] + RI[3 * i + 2] * R[3 * j + 2];
  double Lw[3];
  mat3_apply(Iw, w, Lw);
  const double m[3] = {T[0] - (w[1] * Lw[2] - w[2] * Lw[1]), T[1] - (w[2] * Lw[0] - w[0] * Lw[2]),
                       T[2] - (w[0] * Lw[1] - w[1] * Lw[0])};
  for (int a = 0; a < 3; ++a) {
    r[a] = v[a];
    r[7 + a] = F[a] / B.mass + G[a];
  }
  if (dim == 2) {
    r[2] = r[9] = 0.0;
    r[10] = r[11] = 0.0;
    r[12] = m[2] / Iw[8];
  } else {
    // I_w^-1 m by the adjugate: I_w is symmetric positive definite
    const double c00 = Iw[4] * Iw[8] - Iw[5] * Iw[7], c01 = Iw[5] * Iw[6] - Iw[3] * Iw[8],
                 c02 = Iw[3] * Iw[7] - Iw[4] * Iw[6];
    const double c11 = Iw[0] * Iw[8] - Iw[2] * Iw[6], c12 = Iw[2] * Iw[3] - Iw[0] * Iw[5];
    const double c22 = Iw[0] * Iw[4] - Iw[1] * Iw[3];
    const double det = Iw[0] * c00 + Iw[1] * c01 + Iw[2] * c02;
    // symmetric: the cofactor matrix is its own transpose
    r[10] = (c00 * m[0] + c01 * m[1] + c02 * m[2]) / det;
    r[11] = (c01 * m[0] + c11 * m[1] + c12 * m[2]) / det;
    r[12] = (c02 * m[0] + c12 * m[1] + c22 * m[2]) / det;
  }
  // dq/dt = ((-omega . q_v), q_w omega + omega x q_v) / 2
  r[3] = -0.5 * (w[0] * q[1] + w[1] * q[2] + w[2] * q[3]);
  r[4] = 0.5 * (q[0] * w[0] + (w[1] * q[3] - w[2] * q[2]));
  r[5] = 0.5 * (q[0] * w[1] + (w[2] * q[1] - w[0] * q[3]));
  r[6] = 0.5 * (q[0] * w[2] + (w[0] * q[2] - w[1] * q[1]));
}

__global__ void k_free_body_stage(FreeBody B, Phys P, Scalars *sc, int stage) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double G[3], r[13], y[13];
  body_force(P, sc->t_rhs, G);
  for (int k = 0; k < 13; ++k) y[k] = sc->fb[k];
  free_body_rates(B, P.dim, y, sc->fbF, sc->fbF + 3, G, r);
  const double dt = sc->dt;
  if (stage == 1) {
    for (int k = 0; k < 13; ++k) {
      sc->fb0[k] = y[k];
      y[k] = y[k] + dt * r[k];
    }
  } else {
    for (int k = 0; k < 13; ++k) y[k] = 0.5 * sc->fb0[k] + 0.5 * (y[k] + dt * r[k]);
  }
  const double qn = sqrt(y[3] * y[3] + y[4] * y[4] + y[5] * y[5] + y[6] * y[6]);
  for (int k = 3; k < 7; ++k) y[k] /= qn;
  bool ok = true;
  for (int k = 0; k < 13; ++k) ok = ok && isfinite(y[k]);
  if (!ok) atomicOr(&sc->err, kErrNonFinite);
  for (int k = 0; k < 13; ++k) sc->fb[k] = y[k];
}

hipError_t launch_free_body_stage(const FreeBody &B, const Phys &P, Scalars *sc, int stage, hipStream_t s) {
  hipLaunchKernelGGL(k_free_body_stage, dim3(1), dim3(64), 0, s, B, P, sc, stage);
  return hipGetLastError();
}

}  // namespace wb
