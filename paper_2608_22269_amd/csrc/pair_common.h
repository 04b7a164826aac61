// Shared pieces of the pair passes (FP64 and mixed paths): the sums one
// particle accumulates over its neighbours and the epilogue that turns them
// into the rates of Eq. (sph) -- closed-form eigenvalues of L (Sec. 3), the
// L^T solves, the TIC / singular branch (Sec. 2.3), the continuity term, the
// delta-SPH term, the shifting velocity with its clamp, the free-surface
// pre-classification by lambda_min and the classifier features.
#pragma once

#include "common.h"

namespace wb {

__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, bool pred) {
  // wave-aggregated atomic append; returns the slot of this lane (valid if pred)
  unsigned long long mask = __ballot(pred);
  uint32_t base = 0;
  if (mask) {
    int leader = __ffsll((long long)mask) - 1;
    if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
    base = __shfl(base, leader, 64);
  }
  return base + (uint32_t)__popcll(mask & __lanemask_lt());
}

__device__ __forceinline__ void wave_count(uint32_t *counter, bool pred) {
  unsigned long long mask = __ballot(pred);
  if (mask && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)mask) - 1))
    atomicAdd(counter, (uint32_t)__popcll(mask));
}

// Candidate lists kept from a step's first stage for its second.  A lane's
// list is stored chunk by chunk, one chunk per non-empty LDS list fill of the
// pair pass (the lanes of a cell row fill together, so their chunk indices
// agree and the stores coalesce).  Each wave owns one contiguous block:
// entry k of chunk c of lane l of wave w at
// ent[((w kKeepChunks + c) kPairList + k) 64 + l].  The lane's chunk counts
// are packed into one word written once at the end of the pass, cnt[64 w + l]:
// 6 bits per chunk (c at bit 6c), the number of chunks at bit 48.
struct KeptLists {
  uint32_t *ent;
  unsigned long long *cnt;
};

constexpr int kKeptNchShift = 6 * kKeepChunks;
static_assert(kPairList < 64 && kKeptNchShift + 4 <= 64, "packed chunk counts");

__device__ __forceinline__ int kept_count(unsigned long long packed, int c) {
  return (int)((packed >> (6 * c)) & 63ull);
}
__device__ __forceinline__ size_t kept_entry(uint32_t i, int c, int k) {
  return (((size_t)(i >> 6) * kKeepChunks + (size_t)c) * kPairList + (size_t)k) * 64u + (i & 63u);
}

// Neighbour sums of one particle (FP64).  L and N are symmetric and packed
// as (xx, yy, zz, xy, xz, yz); N holds N_ab + N_ba off the diagonal.  Ps is
// sum (W / W(dx))^n grad W V (the shifting sum is gs + R Ps).
struct PairSums {
  double L[6], gs[3], SR[3], SC[3], Ps[3], N[6], Ds;
  uint32_t nnb, ntest;
  bool coincident;
};

__device__ __forceinline__ void sums_zero(PairSums &S) {
#pragma unroll
  for (int k = 0; k < 6; ++k) S.L[k] = S.N[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) S.gs[k] = S.SR[k] = S.SC[k] = S.Ps[k] = 0.0;
  S.Ds = 0.0;
  S.nnb = S.ntest = 0;
  S.coincident = false;
}

// Must be reached by every lane of the wave (wave-level atomics at the end).
template <int DIM>
__device__ __forceinline__ void pair_epilogue(const Phys &P, Scalars *sc, const Rates &out, uint32_t *cand,
                                              uint32_t i, bool active, const PairSums &S) {
  const uint32_t flags = P.flags;
  double lam[3];
  eig_sym<DIM>(S.L, lam);
  const double lmin = lam[0];
  // classifier inputs: the raw sums L, g and the shifting sum of the
  // particles in the candidate window of lambda_min (every row when the
  // features are exported), written here so that they need no registers
  // later; k_features turns them into the sixteen features
  if (((flags & SPH_F_FEATURES) || P.fs_mode == SPH_FS_LEARNED) && active &&
      ((flags & SPH_F_FEATURES) || (lmin > P.lambda_lo && lmin <= P.lambda_hi))) {
    float *f = out.feat + (size_t)i * kNFeat;
#pragma unroll
    for (int k = 0; k < 6; ++k) f[k] = (float)S.L[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      f[6 + a] = (float)S.gs[a];
      f[9 + a] = (float)(S.gs[a] + P.pst_R * S.Ps[a]);
    }
  }
  const bool singular = lmin <= P.lambda_sing;
  const bool tic = (flags & SPH_F_TIC) && lmin < P.lambda_tic;
  const bool cons = singular || tic;
  double I[6] = {0, 0, 0, 0, 0, 0};
  if (!singular) inv_sym<DIM>(S.L, I);
  double G[3];
  body_force(P, sc->t_rhs, G);
  // momentum: a = -S.L^-T S_R + G  or  -S_C + G
  double grad[3];
  if (cons) {
    grad[0] = S.SC[0];
    grad[1] = S.SC[1];
    grad[2] = S.SC[2];
  } else {
    sym_mul<DIM>(I, S.SR, grad);
  }
  // continuity: -C0^2 tr(S.L^-1 S.N) (+ delta-SPH)
  double div;
  if (singular || (tic && (flags & SPH_F_CONT_UNCORR))) {
    div = S.N[0] + S.N[1] + (DIM == 3 ? S.N[2] : 0.0);
  } else if (DIM == 2) {
    div = I[0] * S.N[0] + I[1] * S.N[1] + I[3] * S.N[3];
  } else {
    div = I[0] * S.N[0] + I[1] * S.N[1] + I[2] * S.N[2] + I[3] * S.N[3] + I[4] * S.N[4] + I[5] * S.N[5];
  }
  double dphi = -P.c0 * P.c0 * div;
  if (flags & SPH_F_DELTA) dphi += P.delta * P.h * P.c0 * (2.0 * S.Ds);
  // free-surface normal n = -S.L^-T g / |.|
  double ng[3];
  if (singular) {
    ng[0] = -S.gs[0];
    ng[1] = -S.gs[1];
    ng[2] = -S.gs[2];
  } else {
    sym_mul<DIM>(I, S.gs, ng);
    ng[0] = -ng[0];
    ng[1] = -ng[1];
    ng[2] = -ng[2];
  }
  const double nn = sqrt(ng[0] * ng[0] + ng[1] * ng[1] + (DIM == 3 ? ng[2] * ng[2] : 0.0));
  double nrm[3] = {0.0, 0.0, 0.0};
  if (nn > 0.0) {
    nrm[0] = ng[0] / nn;
    nrm[1] = ng[1] / nn;
    if (DIM == 3) nrm[2] = ng[2] / nn;
  }
  // shifting: dU* = -2 h U_max P, clamped to U_max / 2
  double dus[3] = {0.0, 0.0, 0.0};
  const double umax = sc->umax;
  if (flags & SPH_F_PST) {
    const double Pv[3] = {S.gs[0] + P.pst_R * S.Ps[0], S.gs[1] + P.pst_R * S.Ps[1], S.gs[2] + P.pst_R * S.Ps[2]};
    double ds[3] = {-2.0 * P.h * umax * Pv[0], -2.0 * P.h * umax * Pv[1], -2.0 * P.h * umax * Pv[2]};
    double dn = sqrt(ds[0] * ds[0] + ds[1] * ds[1] + (DIM == 3 ? ds[2] * ds[2] : 0.0));
    if (dn > 0.0) {
      double mag = dn < 0.5 * umax ? dn : 0.5 * umax;
      dus[0] = mag * ds[0] / dn;
      dus[1] = mag * ds[1] / dn;
      if (DIM == 3) dus[2] = mag * ds[2] / dn;
    }
  }
  // free-surface pre-classification by lambda_min
  uint32_t fl = (cons ? kFlagCons : 0u) | (singular ? kFlagSingular : 0u);
  bool is_cand = false;
  if (P.fs_mode != SPH_FS_NONE) {
    bool fs = false;
    if (lmin <= P.lambda_lo) fs = true;
    else if (lmin > P.lambda_hi) fs = false;
    else if (nn == 0.0) fs = true;
    else is_cand = true;
    if (fs) {
      fl |= kFlagFS;
      if ((flags & SPH_F_FS_PROJECT) && (flags & SPH_F_PST)) {
        double d = dus[0] * nrm[0] + dus[1] * nrm[1] + dus[2] * nrm[2];
        dus[0] -= d * nrm[0];
        dus[1] -= d * nrm[1];
        dus[2] -= d * nrm[2];
      }
    }
    if (is_cand) fl |= kFlagCand;
  }
  if (active) {
    for (int a = 0; a < DIM; ++a) {
      out.acc[a][i] = -grad[a] + G[a];
      out.dus[a][i] = dus[a];
      out.nrm[a][i] = nrm[a];
    }
    out.dphi[i] = dphi;
    out.lam[0][i] = lam[0];
    out.lam[1][i] = lam[1];
    out.lam[2][i] = lam[2];
    out.flags[i] = fl;
    out.nnb[i] = S.nnb;
    if (S.coincident) atomicOr(&sc->err, kErrNonFinite);
  }
  // candidate list and statistics (wave-aggregated atomics)
  const bool cand_l = active && is_cand;
  uint32_t slot = wave_append(&sc->n_cand, cand_l);
  if (cand_l) cand[slot] = i;
  wave_count(&sc->n_fs, active && (fl & kFlagFS));
  wave_count(&sc->n_cons, active && cons);
  wave_count(&sc->n_sing, active && singular);
  // ordered-pair and candidate-test counts
  unsigned long long pc = active ? S.nnb : 0, tc = active ? S.ntest : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    pc += __shfl_xor(pc, o, 64);
    tc += __shfl_xor(tc, o, 64);
  }
  if ((threadIdx.x & 63) == 0 && pc) atomicAdd(&sc->pairs, pc);
  if ((threadIdx.x & 63) == 0 && tc) atomicAdd(&sc->tests, tc);
}

// Scan-region test of neighbour q (squared distance s2 <= (2h)^2) for a
// candidate with normal n and T = x_i + h n.
template <int DIM>
__device__ __forceinline__ bool scan_covers(const Phys &P, const double q[3], const double T[3], const double n[3],
                                            double s2) {
  const double d0 = q[0] - T[0], d1 = q[1] - T[1], d2 = DIM == 3 ? q[2] - T[2] : 0.0;
  if (s2 >= 2.0 * P.h * P.h) return (d0 * d0 + d1 * d1 + d2 * d2) < P.h * P.h;
  const double dn = n[0] * d0 + n[1] * d1 + n[2] * d2;
  const double e0 = d0 - dn * n[0], e1 = d1 - dn * n[1], e2 = d2 - dn * n[2];
  return fabs(dn) + sqrt(e0 * e0 + e1 * e1 + e2 * e2) < P.h;
}

// Outcome of the scan-region test for candidate i: flags and the tangential
// projection of the shifting velocity at the surface (the caller counts the
// surface particles).
template <int DIM>
__device__ __forceinline__ void scan_finish(const Phys &P, const Rates &out, uint32_t i, const double n[3],
                                            bool covered) {
  uint32_t fl = out.flags[i] | kFlagByScan;
  if (!covered) {
    fl |= kFlagFS;
    if ((P.flags & SPH_F_FS_PROJECT) && (P.flags & SPH_F_PST)) {
      const double u0 = out.dus[0][i], u1 = out.dus[1][i], u2 = DIM == 3 ? out.dus[2][i] : 0.0;
      const double d = u0 * n[0] + u1 * n[1] + u2 * n[2];
      out.dus[0][i] = u0 - d * n[0];
      out.dus[1][i] = u1 - d * n[1];
      if (DIM == 3) out.dus[2][i] = u2 - d * n[2];
    }
  }
  out.flags[i] = fl;
}

}  // namespace wb
