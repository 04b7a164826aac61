// Host launchers of the device kernels, grouped by translation unit.
#pragma once

#include "common.h"

namespace wb {

struct SortScratch {
  uint32_t *key, *slot, *count, *scan_tmp;
};

// grid.hip
hipError_t launch_sort_keys(const Grid &g, int dim, const double *x, const double *y, const double *z,
                            const uint32_t *packed_cell, int64_t n, const uint32_t *id, SortScratch &ss,
                            uint32_t *start, uint32_t *perm, Scalars *sc, hipStream_t s);
hipError_t launch_reorder_f64(const Phys &P, const uint32_t *perm, int64_t n, const FluidF64 &src,
                              const FluidF64 &dst, double4 *rec0, double4 *rec1, int with_stage0, hipStream_t s);
// records of the FP64 state in its current order (no sort)
hipError_t launch_refresh_f64(const Phys &P, const FluidF64 &f, int64_t n, double4 *rec0, double4 *rec1,
                              hipStream_t s);

// Dummy wall particles, sorted by (cell, original index): once, or at every
// right-hand side when a body moves.
struct Dummies {
  double *x[3], *n[3], *m, *phi_in;
  uint32_t *id;
  int32_t *src;  // sorted fluid index of the mirror source, -1 if inactive
  // with a moving body only (else null): positions at the body's reference
  // time (or pose) and 1 for the body's dummies (kind 2)
  double *x0[3];
  uint8_t *mov;
  // with a free body only (else null): normals in the reference pose
  double *n0[3];
};

// Constants of the free body: mass, inertia tensor about the centre in the
// body frame (xx yy zz xy xz yz).
struct FreeBody {
  double mass;
  double I[6];
};

// Prescribed motion of the body (Sec. 4, aircraft ditching): velocity a_k +
// b_k t on piece k (T_k <= t <= T_{k+1}), zero outside [T_0, T_K].
struct Body {
  int pieces;
  double T[5];
  double a[4][3], b[4][3];
};

// pair.hip
hipError_t launch_mirror_f64(const Phys &P, const Grid &g, const Dummies &d, int64_t nd, const double4 *rec0,
                             const double4 *rec1, double4 *drec0, double4 *drec1, const uint32_t *cs_f,
                             uint32_t nf, const Scalars *sc, hipStream_t s, const uint32_t *fid);
// Force and torque (F, then the torque about sc->fb's centre) of the water on
// the free body's dummies after the mirror, one partial of 6 doubles per
// block of kBlock dummy rows (part: 6 grid_for(nd) doubles).
hipError_t launch_body_force_f64(const Phys &P, const Grid &g, const Dummies &d, int64_t nd, const double4 *rec0,
                                 const double4 *rec1, const double4 *drec0, const uint32_t *cs_f, uint32_t nf,
                                 const Scalars *sc, double *part, hipStream_t s);
// pair pass modes: own search; own search keeping its candidate lists for the
// step's second stage (kept lists kent, sized for kKeepChunks list fills of
// kPairList entries per lane of the launch, and kcnt, one word of packed
// chunk counts per lane); a right-hand side from the kept lists
constexpr int kPairSearch = 0, kPairSearchKeep = 1, kPairKept = 2;
hipError_t launch_pair_f64(const Phys &P, const Grid &g, const double4 *rec0, const double4 *rec1,
                           const uint32_t *cs_f, const uint32_t *cs_d, uint32_t nf, Scalars *sc, const Rates &out,
                           uint32_t *cand, int mode, uint32_t *kent, unsigned long long *kcnt,
                           hipStream_t s);
// classifier features from the raw sums of the pair-pass epilogue, for the
// rows of a device-counted list (count != nullptr) or rows 0 .. n - 1
hipError_t launch_features(const Phys &P, const Rates &out, const uint32_t *list, const uint32_t *count, uint32_t n,
                           const Scalars *sc, hipStream_t s);
hipError_t launch_scan_f64(const Phys &P, const Grid &g, const double4 *rec0, const uint32_t *cs_f,
                           const uint32_t *cs_d, uint32_t nf, const uint32_t *list, const uint32_t *count,
                           const Rates &out, Scalars *sc, hipStream_t s);
hipError_t launch_nb_count_f64(const Phys &P, const Grid &g, const double4 *rec0, const uint32_t *cs_f,
                               const uint32_t *cs_d, uint32_t nf, const uint32_t *fid, uint32_t *cnt, hipStream_t s,
                               uint32_t nrows);
hipError_t launch_nb_fill_f64(const Phys &P, const Grid &g, const double4 *rec0, const uint32_t *cs_f,
                              const uint32_t *cs_d, uint32_t nf, const uint32_t *fid, const uint32_t *did,
                              const uint32_t *off, uint32_t r0, uint32_t r1, int32_t *ids, hipStream_t s);
hipError_t launch_sort_rows(const uint32_t *off, int64_t r0, int64_t r1, int32_t *ids, hipStream_t s);

// integrate.hip
hipError_t launch_umax(int dim, const double *const u[3], const float *const uf[3], int64_t nf, Scalars *sc,
                       hipStream_t s);
hipError_t launch_dt(const Phys &P, Scalars *sc, double dt_override, hipStream_t s);
// stage bookkeeping; mode: the right-hand side's pair-pass mode (kPairSearch,
// kPairSearchKeep: it builds new kept lists, kPairKept)
hipError_t launch_stage_time(Scalars *sc, int stage, hipStream_t s, int mode = 0);
// adds the bound on a particle's move by the stage update just made to sc->disp
hipError_t launch_disp_add(Scalars *sc, int stage, hipStream_t s);
// clears sc->umax2_bits (before a kernel that folds max |U|^2 into it)
hipError_t launch_reset_umax(Scalars *sc, hipStream_t s);
// SSP-RK2 stage update (FP64; stage 1 reads t^n from the stage-0 arrays,
// which the caller has swapped with the state arrays); also max |U|^2 of the new state into
// sc->umax2_bits (reset here), a finiteness check of phi and U (check != 0)
// and the neighbour records of the new state (rec0 != nullptr)
hipError_t launch_stage_f64(const Phys &P, const FluidF64 &f, const Rates &r, int64_t nf, Scalars *sc, int stage,
                            hipStream_t s, double4 *rec0 = nullptr, double4 *rec1 = nullptr, int check = 0);
hipError_t launch_advance_time(Scalars *sc, hipStream_t s);
hipError_t launch_set_time(Scalars *sc, double t, hipStream_t s);
hipError_t launch_gather_f64(const double *src, const uint32_t *id, int64_t n, double *dst, int stride, int comp,
                             hipStream_t s, uint32_t nout);
hipError_t launch_gather_f32_as_f64(const float *src, const uint32_t *id, int64_t n, double *dst, int stride,
                                    int comp, hipStream_t s, uint32_t nout);
hipError_t launch_gather_rec(const double4 *rec, const uint32_t *id, int64_t n, double *dst, int stride,
                             int comp, int ncomp, hipStream_t s, uint32_t nout);
hipError_t launch_gather_u32_bits(const uint32_t *src, const uint32_t *id, int64_t n, int32_t *dst,
                                  uint32_t mask, int shift, hipStream_t s, uint32_t nout);
hipError_t launch_gather_i32(const int32_t *src, const uint32_t *id, int64_t n, int32_t *dst, int stride,
                             int comp, hipStream_t s, uint32_t nout);
hipError_t launch_gather_rows_f32(const float *src, const uint32_t *id, int64_t n, int width, float *dst,
                                  hipStream_t s, uint32_t nout);
hipError_t launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t s);
hipError_t launch_cells_of(const Grid &g, int dim, const double *const x[3], const uint32_t *id, int64_t n,
                           int32_t *dst, hipStream_t s, uint32_t nout);
hipError_t launch_rho_p(const Phys &P, const double *phi, const uint32_t *id, int64_t n, double *dst, int which,
                        hipStream_t s, uint32_t nout);
hipError_t launch_rho_p_rec(const Phys &P, const double4 *rec, const uint32_t *id, int64_t n, double *dst,
                            int which, hipStream_t s, uint32_t nout);

// Setup: split the caller's particles by kind.
hipError_t launch_split(const Phys &P, int64_t n, const double *x, const double *u, const double *phi,
                        const double *mass, const uint8_t *kind, const double *nrm, const uint32_t *fluid_rank,
                        const uint32_t *dummy_rank, FluidF64 f, Dummies d, hipStream_t s);
hipError_t launch_kind_flags(const uint8_t *kind, int64_t n, uint32_t *is_fluid, uint32_t *is_dummy,
                             hipStream_t s);
hipError_t launch_gather_dummies(const uint32_t *perm, int64_t nd, Dummies src, Dummies dst, int dim,
                                 hipStream_t s);
// Moves the body's dummies to their positions of time sc->t_rhs (x0 + D(t))
// and stores D and the body velocity in sc->body_x / sc->body_u.
hipError_t launch_body_move(const Body &B, const Dummies &d, int64_t nd, int dim, Scalars *sc, hipStream_t s);
// Puts the free body's dummies at the pose of sc->fb: x = c + R (x0 - c0),
// n = R n0.
hipError_t launch_free_body_place(const Dummies &d, int64_t nd, int dim, Scalars *sc, hipStream_t s);
// Sums np partials of 6 doubles (force, torque) into sc->fbF in a fixed
// order (one block).
hipError_t launch_free_body_sum(const double *ft, int64_t np, Scalars *sc, hipStream_t s);
// SSP-RK2 stage of the free body's state from the force and torque of the
// right-hand side just evaluated (stage 1 keeps the state of t^n in sc->fb0).
hipError_t launch_free_body_stage(const FreeBody &B, const Phys &P, Scalars *sc, int stage, hipStream_t s);

}  // namespace wb
