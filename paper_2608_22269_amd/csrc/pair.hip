// Particle interaction stage, FP64 path (Sec. 2 and Sec. 3):
//   - dummy-wall mirror (Sec. 2.4, Eq. phiBn and the slip velocity);
//   - the fused pair pass: every sum of Eq. (sph) in one neighbour pass --
//     L (Eq. renorm), the Riemann sum of Eqs. (parGrad)/(lfsover) kept on the
//     right of L^T (the correction moved out of the sum, Sec. 3), the
//     conservative sum (TIC), the velocity-gradient tensor of the continuity
//     equation, the delta-SPH sum and the shifting sum -- followed by an
//     epilogue with the closed-form eigenvalues, the small solves and the
//     free-surface pre-classification;
//   - the scan-region pass over free-surface candidates;
//   - neighbour-list export for parity checks.
//
// Work mapping.  One lane per fluid particle, particles in storage (sort key)
// order.  The wave walks the cell rows of Algorithm 1 in lockstep; each lane
// compacts its in-range candidates into its own column of an LDS list (32
// entries), and whenever a list may overflow the wave runs the dense pair body
// over the lists.  Lanes of one wave belong to the same or neighbouring cells,
// so their candidate loads touch the same records, and the expensive body runs
// on real neighbours only instead of every candidate of the 3^d cells.
#include "common.h"
#include "kernels.h"
#include "pair_common.h"
#include "coop.h"

namespace wb {

// Compile-time tuning of the pair pass (values chosen by measurement on the
// 17.5M-particle sloshing tank; they change speed, never results).
#ifndef WB_PAIR_BATCH
#define WB_PAIR_BATCH 4
#endif
#ifndef WB_PAIR_UNROLL
#define WB_PAIR_UNROLL 1
#endif
// waves per SIMD the register allocation targets (4 measured fastest)
#ifndef WB_PAIR_WAVES
#define WB_PAIR_WAVES 4
#endif
// waves per SIMD of the pass from kept lists (2, 3 and 4 measured equal: its
// record gathers bound it, not latency)
#ifndef WB_KEPT_WAVES
#define WB_KEPT_WAVES 4
#endif
constexpr int kList = kPairList;       // LDS list entries per lane
constexpr int kBatch = WB_PAIR_BATCH;  // candidates fetched per search iteration
static_assert(kBatch <= kRecPad, "batched candidate loads run at most kRecPad records past a run");
#define WB_PAIR_ATTR __attribute__((amdgpu_waves_per_eu(WB_PAIR_WAVES)))

// ------------------------------------------------------------------ mirror

template <int DIM>
__global__ void __launch_bounds__(256) k_mirror_f64(Phys P, Grid g, Dummies d, int64_t nd,
                                                    const double4 *__restrict__ rec0,
                                                    const double4 *__restrict__ rec1, double4 *__restrict__ drec0,
                                                    double4 *__restrict__ drec1, const uint32_t *__restrict__ cs_f,
                                                    uint32_t nf, const Scalars *__restrict__ sc,
                                                    const uint32_t *__restrict__ fid) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nd) return;
  double xd = d.x[0][k], yd = d.x[1][k], zd = DIM == 3 ? d.x[2][k] : 0.0;
  RowWalker w;
  walker_init<DIM>(w, g, xd, yd, zd, P.win);
  int64_t best = -1;
  uint32_t best_id = 0;
  double best_r2 = 0.0;
  auto test_run = [&](uint32_t a, uint32_t e) {
    for (uint32_t j = a; j < e; ++j) {
      double4 b = rec0[j];
      double r2 = dist2_exact<DIM>(b.x - xd, b.y - yd, b.z - zd);
      if (r2 <= P.two_h2) {
        uint32_t jid = fid[j];
        if (best < 0 || r2 < best_r2 || (r2 == best_r2 && jid < best_id)) {
          best = j;
          best_r2 = r2;
          best_id = jid;
        }
      }
    }
  };
  // fluid runs only; at reach 2 the cell starts of all rows are loaded
  // together (the walk is bound by the latency of its row-by-row loads),
  // otherwise row by row (pass cs_f twice and skip the dummy runs)
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
  if (best < 0) {
    drec0[k] = make_double4(xd, yd, zd, d.phi_in[k]);
    drec1[k] = make_double4(0.0, 0.0, 0.0, 0.0);  // inactive: in no fluid's support
    return;
  }
  double G[3];
  body_force(P, sc->t_rhs, G);
  double4 f0 = rec0[best], f1 = rec1[best];
  // phi_d = phi_f + G.(x_d - x_f)        (Eq. phiBn)
  double gp = G[0] * (xd - f0.x) + G[1] * (yd - f0.y);
  if (DIM == 3) gp += G[2] * (zd - f0.z);
  double phid = f0.w + gp;
  // slip: U_d = U_f - (U_f . n_d) n_d; for the moving body relative to its
  // velocity Uw, U_d = U_f - ((U_f - Uw) . n_d) n_d (the dummy keeps the
  // wall's normal velocity)
  double nx = d.n[0][k], ny = d.n[1][k], nz = DIM == 3 ? d.n[2][k] : 0.0;
  double un;
  if (d.mov != nullptr && d.mov[k]) {
    double Uw[3] = {sc->body_u[0], sc->body_u[1], sc->body_u[2]};
    if (sc->fb_on) {
      // free body: v + omega x R (x0 - c0) at this dummy
      double q[4] = {sc->fb[3], sc->fb[4], sc->fb[5], sc->fb[6]}, R[9];
      quat_rotation(q, R);
      const double d0[3] = {d.x0[0][k] - sc->fb_c0[0], d.x0[1][k] - sc->fb_c0[1],
                            DIM == 3 ? d.x0[2][k] - sc->fb_c0[2] : 0.0};
      double dr[3];
      mat3_apply(R, d0, dr);
      free_body_point_velocity(sc->fb, dr, Uw);
    }
    un = (f1.x - Uw[0]) * nx + (f1.y - Uw[1]) * ny;
    if (DIM == 3) un += (f1.z - Uw[2]) * nz;
  } else {
    un = f1.x * nx + f1.y * ny + f1.z * nz;
  }
  double V = d.m[k] / (P.rho0 * exp(phid * P.inv_c02));
  drec0[k] = make_double4(xd, yd, zd, phid);
  drec1[k] = make_double4(f1.x - un * nx, f1.y - un * ny, DIM == 3 ? f1.z - un * nz : 0.0, V);
}

// ----------------------------------------------------------- pair pass

// Dense pair body: every sum of Eq. (sph) for neighbour j (records b0, b1) of
// particle i (records a0, a1).  PST4: the shifting exponent is 4 (the paper's
// value), evaluated as two squarings; otherwise pow().
template <int DIM, bool PST4>
__device__ __forceinline__ void pair_body_f64(const Phys &P, const double4 &a0, const double4 &a1, const double4 &b0,
                                              const double4 &b1, PairSums &S) {
  const double rx = b0.x - a0.x, ry = b0.y - a0.y, rz = DIM == 3 ? b0.z - a0.z : 0.0;
  // membership was decided by the exact test; here |r| only feeds W and K
  const double r2 = DIM == 3 ? fma(rx, rx, fma(ry, ry, rz * rz)) : fma(rx, rx, ry * ry);
  S.coincident |= (r2 == 0.0);
  const double is = rsqrt_pos(r2);
  const double s = r2 * is;
  const double t = fma(s, P.m_half_inv_h, 1.0);  // 1 - q/2
  const double t2 = t * t, t3 = t2 * t;
  const double wv = P.kfac * t3 * b1.w;  // |grad W| / |r| times V_j
  const double gx = wv * rx, gy = wv * ry, gz = wv * rz;
  // S.L = sum r (x) grad W V  (symmetric for the radial kernel)
  S.L[0] += rx * gx;
  S.L[1] += ry * gy;
  S.L[3] += rx * gy;
  if (DIM == 3) {
    S.L[2] += rz * gz;
    S.L[4] += rx * gz;
    S.L[5] += ry * gz;
  }
  S.gs[0] += gx;
  S.gs[1] += gy;
  if (DIM == 3) S.gs[2] += gz;
  const double dph = b0.w - a0.w;
  const double dux = b1.x - a1.x, duy = b1.y - a1.y, duz = DIM == 3 ? b1.z - a1.z : 0.0;
  const double dun = (dux * rx + duy * ry + duz * rz) * is;
  const double c2 = dph - P.c0 * dun;  // 2 (phi*_ij - phi_i)
  const double cs = b0.w + a0.w;        // conservative form
  S.SR[0] += c2 * gx;
  S.SR[1] += c2 * gy;
  S.SC[0] += cs * gx;
  S.SC[1] += cs * gy;
  if (DIM == 3) {
    S.SR[2] += c2 * gz;
    S.SC[2] += cs * gz;
  }
  // symmetric part of N_ab = sum (U_j - U_i)_a (grad W V)_b: S.L^-1 is
  // symmetric, so tr(S.L^-1 S.N) only sees S.N + S.N^T (packed xx yy zz xy xz yz,
  // off-diagonals hold N_ab + N_ba)
  S.N[0] += dux * gx;
  S.N[1] += duy * gy;
  S.N[3] += dux * gy + duy * gx;
  if (DIM == 3) {
    S.N[2] += duz * gz;
    S.N[4] += dux * gz + duz * gx;
    S.N[5] += duy * gz + duz * gy;
  }
  S.Ds += wv * dph;  // Phi_ij . grad W V = 2 K (phi_j - phi_i) V_j (factor 2 in the epilogue)
  // shifting: sum (W / W(dx))^n grad W V; the epilogue adds sum grad W V
  // times 1 / R, i.e. P = sum [1 + R (W / W(dx))^n] grad W V
  const double u = fma(s, P.two_inv_h, 1.0);  // 2q + 1
  const double t4u = (t2 * t2) * u;
  const double wr = P.aw0 * t4u;
  const double wrn = PST4 ? (wr * wr) * (wr * wr) : pow(wr, P.pst_n);
  S.Ps[0] += wrn * gx;
  S.Ps[1] += wrn * gy;
  if (DIM == 3) S.Ps[2] += wrn * gz;
}

// The pair pass with its own candidate search (Algorithm 1).  KEEP (the
// right-hand side that builds kept lists): the search radius grows to
// 2h + skin (P.skin_max), candidates beyond 2h enter the LDS list tagged and
// are skipped by the body, and every non-empty list fill is also copied to kl
// for the later right-hand sides; a lane with more than kKeepChunks fills
// raises sc->vovf.
template <int DIM, bool PST4, bool KEEP>
__global__ void __launch_bounds__(256) WB_PAIR_ATTR k_pair_f64(Phys P, Grid g, const double4 *__restrict__ rec0,
                                                  const double4 *__restrict__ rec1, const uint32_t *__restrict__ cs_f,
                                                  const uint32_t *__restrict__ cs_d, uint32_t nf, Scalars *sc,
                                                  Rates out, uint32_t *__restrict__ cand, KeptLists kl) {
  __shared__ uint32_t list[kList][kBlock];
  const int tid = threadIdx.x;
  const uint32_t i = xcd_block(blockIdx.x, gridDim.x) * kBlock + tid;
  const bool active = i < nf;

  double4 a0 = make_double4(0.0, 0.0, 0.0, 0.0), a1 = a0;
  if (active) {
    a0 = rec0[i];
    a1 = rec1[i];
  }
  PairSums S;
  sums_zero(S);
  // the kept-list work behind a run-time test (launches in this mode always
  // have a skin): compiled unconditionally it costs spilled registers
  const bool keep = KEEP && P.skin_max > 0.0;
  const double rho = keep ? P.two_h + P.skin_max : P.two_h;
  const double rho2 = keep ? rho * rho : P.two_h2;
  // this lane's kept-list bookkeeping in LDS (packed chunk counts, chunks
  // so far at bit kKeptNchShift, saturating at 15): touched once per fill,
  // it holds no registers through the search
  __shared__ unsigned long long kbook[KEEP ? kBlock : 1];
  if (KEEP) kbook[tid] = 0ull;

  // consume the first cnt entries of this lane's list
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
        for (int u = 0; u < 8; ++u) e[u] = list[min(k0 + u, kList - 1)][tid];
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
    // one neighbour per iteration, the next list entry read one iteration ahead
    uint32_t en = cnt > 0 ? list[0][tid] : 0u;
    for (int k = 0; k < cnt; ++k) {
      const uint32_t e = en;
      const uint32_t j = KEEP ? e & ~kSkinTag : e;
      const double4 b0 = rec0[j], b1 = rec1[j];
      if (k + 1 < cnt) en = list[k + 1][tid];
      if (!KEEP || !(e & kSkinTag)) {
        pair_body_f64<DIM, PST4>(P, a0, a1, b0, b1, S);
        if (KEEP) S.nnb += 1;
      }
    }
    if (!KEEP) S.nnb += cnt;
  };

  // candidate search with the rows walked in lockstep by the wave
  const CellPos cp = cellpos_of<DIM>(g, a0.x, a0.y, a0.z);
  int cnt = 0;
  auto load = [&](uint32_t j) { return rec0[j]; };
  auto near = [&](const double4 &b, uint32_t j) -> uint32_t {
    const double r2 = dist2_exact<DIM>(b.x - a0.x, b.y - a0.y, DIM == 3 ? b.z - a0.z : 0.0);
    if (!KEEP) return j != i && r2 <= P.two_h2 ? 1u : 0u;
    return j != i && r2 <= rho2 ? (r2 <= P.two_h2 ? 1u : 2u) : 0u;
  };
  CoopWalk cw;
  coop_init(cw, g, active, (float)rho, DIM);
  for (;;) {
    const bool fin = coop_fill<DIM, kList, kBatch>(cw, g, cs_f, cs_d, nf, cp, &list[0][tid], kBlock, cnt, S.ntest,
                                                   load, near);
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

// A right-hand side from kept candidates (no search): the records hold the
// current state in the order of the build, every kept candidate is tested
// exactly against 2h and the neighbours run the same body.  The caller uses
// the lists only while twice the bound on any particle's move since the build
// fits the skin: a pair within 2h now was within 2h + skin then, so the
// neighbour sets are those of a fresh search.
template <int DIM, bool PST4>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WB_KEPT_WAVES))) k_pair_kept_f64(Phys P, const double4 *__restrict__ rec0,
                                                                    const double4 *__restrict__ rec1, uint32_t nf,
                                                                    Scalars *sc, Rates out,
                                                                    uint32_t *__restrict__ cand, KeptLists kl) {
  __shared__ uint32_t list[kList][kBlock];
  const int tid = threadIdx.x;
  const uint32_t i = xcd_block(blockIdx.x, gridDim.x) * kBlock + tid;
  const bool active = i < nf;
  double4 a0 = make_double4(0.0, 0.0, 0.0, 0.0), a1 = a0;
  if (active) {
    a0 = rec0[i];
    a1 = rec1[i];
  }
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
    // one neighbour per iteration, the next list entry read one iteration ahead
    uint32_t en = cnt > 0 ? list[0][tid] : 0u;
    for (int k = 0; k < cnt; ++k) {
      const uint32_t j = en & ~kSkinTag;
      const double4 b0 = rec0[j], b1 = rec1[j];
      if (k + 1 < cnt) en = list[k + 1][tid];
      if (dist2_exact<DIM>(b0.x - a0.x, b0.y - a0.y, DIM == 3 ? b0.z - a0.z : 0.0) <= P.two_h2) {
        pair_body_f64<DIM, PST4>(P, a0, a1, b0, b1, S);
        S.nnb += 1;
      }
    }
    S.ntest += (uint32_t)cnt;
  }
  pair_epilogue<DIM>(P, sc, out, cand, i, active, S);
}

template <int DIM>
void launch_pair_f64_inst(const Phys &P, const Grid &g, const double4 *rec0, const double4 *rec1,
                          const uint32_t *cs_f, const uint32_t *cs_d, uint32_t nf, Scalars *sc, const Rates &out,
                          uint32_t *cand, const KeptLists &kl, int mode, hipStream_t s) {
  dim3 gr(grid_for(nf)), bl(kBlock);
  const bool p4 = P.pst_n == 4.0;
  if (mode == kPairSearch) {
    if (p4)
      hipLaunchKernelGGL((k_pair_f64<DIM, true, false>), gr, bl, 0, s, P, g, rec0, rec1, cs_f, cs_d, nf, sc, out, cand,
                         kl);
    else
      hipLaunchKernelGGL((k_pair_f64<DIM, false, false>), gr, bl, 0, s, P, g, rec0, rec1, cs_f, cs_d, nf, sc, out,
                         cand, kl);
  } else if (mode == kPairSearchKeep) {
    if (p4)
      hipLaunchKernelGGL((k_pair_f64<DIM, true, true>), gr, bl, 0, s, P, g, rec0, rec1, cs_f, cs_d, nf, sc, out, cand,
                         kl);
    else
      hipLaunchKernelGGL((k_pair_f64<DIM, false, true>), gr, bl, 0, s, P, g, rec0, rec1, cs_f, cs_d, nf, sc, out,
                         cand, kl);
  } else {
    if (p4)
      hipLaunchKernelGGL((k_pair_kept_f64<DIM, true>), gr, bl, 0, s, P, rec0, rec1, nf, sc, out, cand, kl);
    else
      hipLaunchKernelGGL((k_pair_kept_f64<DIM, false>), gr, bl, 0, s, P, rec0, rec1, nf, sc, out, cand, kl);
  }
}

hipError_t launch_pair_f64(const Phys &P, const Grid &g, const double4 *rec0, const double4 *rec1,
                           const uint32_t *cs_f, const uint32_t *cs_d, uint32_t nf, Scalars *sc, const Rates &out,
                           uint32_t *cand, int mode, uint32_t *kent, unsigned long long *kcnt, hipStream_t s) {
  if (nf == 0) return hipSuccess;
  if (mode != kPairSearch && (!kent || !kcnt)) return hipErrorInvalidValue;
  KeptLists kl{kent, kcnt};
  if (P.dim == 2)
    launch_pair_f64_inst<2>(P, g, rec0, rec1, cs_f, cs_d, nf, sc, out, cand, kl, mode, s);
  else
    launch_pair_f64_inst<3>(P, g, rec0, rec1, cs_f, cs_d, nf, sc, out, cand, kl, mode, s);
  return hipGetLastError();
}

// ---------------------------------------------------- classifier features

// The 16 classifier features of a particle from the raw sums the pair-pass
// epilogue left in its row (L, g = sum grad W V, the shifting sum P) and its
// eigenvalues, normal n and neighbour count: eigenvalues of L (3), det L,
// n.P h, neighbour count, |g| h, n.g h, tangential |g| h, n.L.n,
// tr L - n.L.n, |L^-T g| h, n.G / |G|, tangential |P| h, n.P / |P|, |P| h.
// Rows of the device-counted list (count != nullptr) or rows 0 .. n - 1.
template <int DIM>
__global__ void __launch_bounds__(256) k_features(Phys P, Rates out, const uint32_t *__restrict__ list,
                                                  const uint32_t *__restrict__ count, uint32_t n,
                                                  const Scalars *__restrict__ sc) {
  const uint32_t total = count ? *count : n;
  double G[3];
  body_force(P, sc->t_rhs, G);
  const double gg = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < total; k += gridDim.x * blockDim.x) {
    const uint32_t i = list ? list[k] : k;
    float *f = out.feat + (size_t)i * kNFeat;
    float raw[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) raw[c] = f[c];
    const double L[6] = {raw[0], raw[1], raw[2], raw[3], raw[4], raw[5]};
    const double g[3] = {raw[6], raw[7], raw[8]}, Pv[3] = {raw[9], raw[10], raw[11]};
    const double n[3] = {out.nrm[0][i], out.nrm[1][i], DIM == 3 ? out.nrm[2][i] : 0.0};
    const double Lm[3][3] = {{L[0], L[3], L[4]}, {L[3], L[1], L[5]}, {L[4], L[5], L[2]}};
    double ng = 0, gn2 = 0, nLn = 0, trL = 0, pn2 = 0, ngr = 0, nP = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      ng += n[a] * g[a];
      gn2 += g[a] * g[a];
      trL += Lm[a][a];
      pn2 += Pv[a] * Pv[a];
      nP += n[a] * Pv[a];
      ngr += n[a] * G[a];
#pragma unroll
      for (int b = 0; b < DIM; ++b) nLn += n[a] * Lm[a][b] * n[b];
    }
    double gt2 = 0, pt2 = 0;  // tangential parts by components (no cancellation)
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const double t = g[a] - ng * n[a], tp = Pv[a] - nP * n[a];
      gt2 += t * t;
      pt2 += tp * tp;
    }
    const double pm = sqrt(pn2);
    // |L^-T g| (L symmetric), or |g| where L is singular (the epilogue's rule)
    double ngv[3] = {g[0], g[1], g[2]};
    if (out.lam[0][i] > P.lambda_sing) {
      double I[6];
      inv_sym<DIM>(L, I);
      sym_mul<DIM>(I, g, ngv);
    }
    const double nn = sqrt(ngv[0] * ngv[0] + ngv[1] * ngv[1] + (DIM == 3 ? ngv[2] * ngv[2] : 0.0));
    const double detL = DIM == 2 ? L[0] * L[1] - L[3] * L[3]
                                 : L[0] * (L[1] * L[2] - L[5] * L[5]) - L[3] * (L[3] * L[2] - L[5] * L[4]) +
                                       L[4] * (L[3] * L[5] - L[1] * L[4]);
    f[0] = (float)out.lam[0][i];
    f[1] = (float)out.lam[1][i];
    f[2] = (float)(DIM == 3 ? out.lam[2][i] : out.lam[1][i]);
    f[3] = (float)detL;
    f[4] = (float)(nP * P.h);
    f[5] = (float)out.nnb[i];
    f[6] = (float)(sqrt(gn2) * P.h);
    f[7] = (float)(ng * P.h);
    f[8] = (float)(sqrt(gt2) * P.h);
    f[9] = (float)nLn;
    f[10] = (float)(trL - nLn);
    f[11] = (float)(nn * P.h);
    f[12] = (float)(gg > 0.0 ? ngr / gg : 0.0);
    f[13] = (float)(sqrt(pt2) * P.h);
    f[14] = (float)(pm > 0.0 ? nP / pm : 0.0);
    f[15] = (float)(pm * P.h);
  }
}

hipError_t launch_features(const Phys &P, const Rates &out, const uint32_t *list, const uint32_t *count, uint32_t n,
                           const Scalars *sc, hipStream_t s) {
  if (n == 0) return hipSuccess;
  unsigned blocks = grid_for(n);
  if (blocks > 2048) blocks = 2048;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_features<2>, dim3(blocks), dim3(kBlock), 0, s, P, out, list, count, n, sc);
  else
    hipLaunchKernelGGL(k_features<3>, dim3(blocks), dim3(kBlock), 0, s, P, out, list, count, n, sc);
  return hipGetLastError();
}

// --------------------------------------------------------- scan-region pass

// Candidates (lambda_lo < lambda <= lambda_hi) are on the free surface unless
// a neighbour lies in the umbrella-shaped region around T = x_i + h n: beyond
// sqrt(2) h from i within h of T, or closer than sqrt(2) h to i with
// |n.(x_j - T)| + |tangential part| < h.  One wave per candidate: the lanes
// take the candidate's rows (one row each) and then its neighbour candidates
// 64 at a time, until one covers it.  Grid-stride over the device-counted
// list, so the launch does not depend on the count.
template <int DIM>
__global__ void __launch_bounds__(256) k_scan_f64(Phys P, Grid g, const double4 *__restrict__ rec0,
                                                  const uint32_t *__restrict__ cs_f, const uint32_t *__restrict__ cs_d,
                                                  uint32_t nf, const uint32_t *__restrict__ list,
                                                  const uint32_t *__restrict__ count, Rates out, Scalars *sc) {
  __shared__ RowTables tab;
  const uint32_t total = *count;
  const int lane = (int)(threadIdx.x & 63);
  const uint32_t gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
  uint32_t nfs = 0;  // surface particles found by this wave (one atomic add at the end)
  for (uint32_t k = gw; k < total; k += nw) {
    const uint32_t i = list[k];
    const double4 a = rec0[i];
    const double n[3] = {out.nrm[0][i], out.nrm[1][i], DIM == 3 ? out.nrm[2][i] : 0.0};
    const double T[3] = {a.x + P.h * n[0], a.y + P.h * n[1], DIM == 3 ? a.z + P.h * n[2] : 0.0};
    const CellPos cp = cellpos_of<DIM>(g, a.x, a.y, a.z);
    int nrows;
    const uint32_t M = rows_layout<DIM>(tab, g, cp, (float)P.win, cs_f, cs_d, nf, nrows);
    bool covered = false;
    for (uint32_t c0 = 0; c0 < M && !covered; c0 += 64u) {
      bool cov = false;
      const uint32_t idx = c0 + (uint32_t)lane;
      if (idx < M) {
        const uint32_t j = record_of(tab, nrows, idx);
        if (j != i) {
          const double4 b = rec0[j];
          const double q[3] = {b.x, b.y, DIM == 3 ? b.z : 0.0};
          const double s2 = dist2_exact<DIM>(b.x - a.x, b.y - a.y, b.z - a.z);
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

hipError_t launch_scan_f64(const Phys &P, const Grid &g, const double4 *rec0, const uint32_t *cs_f,
                           const uint32_t *cs_d, uint32_t nf, const uint32_t *list, const uint32_t *count,
                           const Rates &out, Scalars *sc, hipStream_t s) {
  if (nf == 0) return hipSuccess;
  unsigned blocks = candidate_grid(nf);
  if (P.dim == 2)
    hipLaunchKernelGGL(k_scan_f64<2>, dim3(blocks), dim3(kBlock), 0, s, P, g, rec0, cs_f, cs_d, nf, list, count, out,
                       sc);
  else
    hipLaunchKernelGGL(k_scan_f64<3>, dim3(blocks), dim3(kBlock), 0, s, P, g, rec0, cs_f, cs_d, nf, list, count, out,
                       sc);
  return hipGetLastError();
}

// ------------------------------------------------------- neighbour export

template <int DIM>
__global__ void __launch_bounds__(256) k_nb_count(Phys P, Grid g, const double4 *__restrict__ rec0,
                                                  const uint32_t *__restrict__ cs_f, const uint32_t *__restrict__ cs_d,
                                                  uint32_t nf, const uint32_t *__restrict__ fid,
                                                  uint32_t *__restrict__ cnt, uint32_t nrows) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  double4 a = rec0[i];
  RowWalker w;
  walker_init<DIM>(w, g, a.x, a.y, a.z, P.two_h);
  uint32_t c = 0;
  while (walker_next<DIM>(w, g, cs_f, cs_d, nf)) {
    for (uint32_t j = w.cur; j < w.end; ++j) {
      if (j == i) continue;
      double4 b = rec0[j];
      if (dist2_exact<DIM>(b.x - a.x, b.y - a.y, b.z - a.z) <= P.two_h2) ++c;
    }
  }
  if (fid[i] < nrows) cnt[fid[i]] = c;
}

template <int DIM>
__global__ void __launch_bounds__(256) k_nb_fill(Phys P, Grid g, const double4 *__restrict__ rec0,
                                                 const uint32_t *__restrict__ cs_f, const uint32_t *__restrict__ cs_d,
                                                 uint32_t nf, const uint32_t *__restrict__ fid,
                                                 const uint32_t *__restrict__ did, const uint32_t *__restrict__ off,
                                                 uint32_t r0, uint32_t r1, int32_t *__restrict__ ids) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  const uint32_t row = fid[i];
  if (row < r0 || row >= r1) return;
  double4 a = rec0[i];
  RowWalker w;
  walker_init<DIM>(w, g, a.x, a.y, a.z, P.two_h);
  uint32_t o = off[row];
  while (walker_next<DIM>(w, g, cs_f, cs_d, nf)) {
    for (uint32_t j = w.cur; j < w.end; ++j) {
      if (j == i) continue;
      double4 b = rec0[j];
      if (dist2_exact<DIM>(b.x - a.x, b.y - a.y, b.z - a.z) <= P.two_h2)
        ids[o++] = (int32_t)(j < nf ? fid[j] : did[j - nf]);
    }
  }
}

__global__ void __launch_bounds__(256) k_sort_rows(const uint32_t *__restrict__ off, int64_t r0, int64_t r1,
                                                   int32_t *__restrict__ ids) {
  int64_t r = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= r1) return;
  uint32_t b = off[r], e = off[r + 1];
  for (uint32_t k = b + 1; k < e; ++k) {
    int32_t v = ids[k];
    uint32_t m = k;
    while (m > b && ids[m - 1] > v) {
      ids[m] = ids[m - 1];
      --m;
    }
    ids[m] = v;
  }
}

hipError_t launch_nb_count_f64(const Phys &P, const Grid &g, const double4 *rec0, const uint32_t *cs_f,
                               const uint32_t *cs_d, uint32_t nf, const uint32_t *fid, uint32_t *cnt, hipStream_t s,
                               uint32_t nrows) {
  if (nf == 0) return hipSuccess;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_nb_count<2>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, g, rec0, cs_f, cs_d, nf, fid, cnt,
                       nrows);
  else
    hipLaunchKernelGGL(k_nb_count<3>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, g, rec0, cs_f, cs_d, nf, fid, cnt,
                       nrows);
  return hipGetLastError();
}

hipError_t launch_nb_fill_f64(const Phys &P, const Grid &g, const double4 *rec0, const uint32_t *cs_f,
                              const uint32_t *cs_d, uint32_t nf, const uint32_t *fid, const uint32_t *did,
                              const uint32_t *off, uint32_t r0, uint32_t r1, int32_t *ids, hipStream_t s) {
  if (nf == 0) return hipSuccess;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_nb_fill<2>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, g, rec0, cs_f, cs_d, nf, fid, did, off,
                       r0, r1, ids);
  else
    hipLaunchKernelGGL(k_nb_fill<3>, dim3(grid_for(nf)), dim3(kBlock), 0, s, P, g, rec0, cs_f, cs_d, nf, fid, did, off,
                       r0, r1, ids);
  return hipGetLastError();
}

hipError_t launch_sort_rows(const uint32_t *off, int64_t r0, int64_t r1, int32_t *ids, hipStream_t s) {
  if (r1 <= r0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_rows, dim3(grid_for(r1 - r0)), dim3(kBlock), 0, s, off, r0, r1, ids);
  return hipGetLastError();
}

hipError_t launch_mirror_f64(const Phys &P, const Grid &g, const Dummies &d, int64_t nd, const double4 *rec0,
                             const double4 *rec1, double4 *drec0, double4 *drec1, const uint32_t *cs_f,
                             uint32_t nf, const Scalars *sc, hipStream_t s, const uint32_t *fid) {
  if (nd == 0) return hipSuccess;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_mirror_f64<2>, dim3(grid_for(nd)), dim3(kBlock), 0, s, P, g, d, nd, rec0, rec1, drec0, drec1,
                       cs_f, nf, sc, fid);
  else
    hipLaunchKernelGGL(k_mirror_f64<3>, dim3(grid_for(nd)), dim3(kBlock), 0, s, P, g, d, nd, rec0, rec1, drec0, drec1,
                       cs_f, nf, sc, fid);
  return hipGetLastError();
}

// ----------------------------------------------------- free body force

// Force and torque of the water on the free body: each of its dummies takes
// the conservative-form acceleration of Eq. (sph) (the branch of Sec. 2.3)
// that a dummy with mirrored potential phi_d gets from its fluid neighbours,
// a_d = -sum_i (phi_i + phi_d) grad_d W_di V_i, times its mass, and its
// moment about the body's centre.  Dummies without a mirror source (in no
// fluid particle's support) and all other rows add nothing.  Each block sums
// its rows by a fixed tree and writes one partial (6 doubles, F then the
// torque) to part[6 blockIdx.x ..]: the sums depend only on the rows' order.
template <int DIM>
__global__ void __launch_bounds__(256) k_body_force_f64(Phys P, Grid g, Dummies d, int64_t nd,
                                                        const double4 *__restrict__ rec0,
                                                        const double4 *__restrict__ rec1,
                                                        const double4 *__restrict__ drec0,
                                                        const uint32_t *__restrict__ cs_f, uint32_t nf,
                                                        const Scalars *__restrict__ sc, double *__restrict__ part) {
  __shared__ double red[6][256];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double f[3] = {0.0, 0.0, 0.0}, tq[3] = {0.0, 0.0, 0.0};
  if (k < nd && d.mov[k] && d.src[k] >= 0) {
    const double4 me = drec0[k];  // placed position and mirrored potential
    RowWalker w;
    walker_init<DIM>(w, g, me.x, me.y, me.z, P.win);
    double a[3] = {0.0, 0.0, 0.0};
    auto sum_run = [&](uint32_t lo, uint32_t hi) {
      for (uint32_t j = lo; j < hi; ++j) {
        const double4 b = rec0[j];
        const double rx = b.x - me.x, ry = b.y - me.y, rz = DIM == 3 ? b.z - me.z : 0.0;
        const double r2 = dist2_exact<DIM>(rx, ry, rz);
        if (r2 > P.two_h2) continue;
        const double t = fma(sqrt(r2), P.m_half_inv_h, 1.0);  // 1 - q/2
        const double c = (b.w + me.w) * (P.kfac * t * t * t) * rec1[j].w;
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
    const double arm[3] = {me.x - sc->fb[0], me.y - sc->fb[1], DIM == 3 ? me.z - sc->fb[2] : 0.0};
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

hipError_t launch_body_force_f64(const Phys &P, const Grid &g, const Dummies &d, int64_t nd, const double4 *rec0,
                                 const double4 *rec1, const double4 *drec0, const uint32_t *cs_f, uint32_t nf,
                                 const Scalars *sc, double *part, hipStream_t s) {
  if (nd == 0) return hipSuccess;
  if (!d.mov || !part) return hipErrorInvalidValue;
  static_assert(kBlock == 256, "the block tree of the body force assumes 256 threads");
  if (P.dim == 2)
    hipLaunchKernelGGL(k_body_force_f64<2>, dim3(grid_for(nd)), dim3(kBlock), 0, s, P, g, d, nd, rec0, rec1, drec0,
                       cs_f, nf, sc, part);
  else
    hipLaunchKernelGGL(k_body_force_f64<3>, dim3(grid_for(nd)), dim3(kBlock), 0, s, P, g, d, nd, rec0, rec1, drec0,
                       cs_f, nf, sc, part);
  return hipGetLastError();
}

}  // namespace wb
