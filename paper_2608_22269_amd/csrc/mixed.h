// Mixed-precision path: positions as an integer cell plus an FP32 offset
// inside the cell, FP32 pair evaluation, FP64 accumulation of the
// correction matrix and of the potential-gradient sums.
#pragma once

#include "common.h"
#include "kernels.h"

namespace wb {

// Neighbour-facing records of the mixed path (fluid rows then dummy rows):
// r0 = (offset x, y, z, packed cell as float bits), r1 = (u, v, w, V) in FP32,
// phi in FP64, xa = FP32 absolute position (candidate tests only).
struct MixedRec {
  float4 *r0, *r1, *xa;
  double *phi;
};

hipError_t launch_to_mixed(const Phys &P, const Grid &g, const FluidF64 &src, int64_t nf, const FluidMixed &dst,
                           Scalars *sc, hipStream_t s);
hipError_t launch_reorder_mixed(const Phys &P, const Grid &g, const uint32_t *perm, int64_t nf,
                                const FluidMixed &src, const FluidMixed &dst, const MixedRec &rec, int with_stage0,
                                hipStream_t s);
hipError_t launch_mirror_mixed(const Phys &P, const Grid &g, const Dummies &d, int64_t nd, const MixedRec &rec,
                               const uint32_t *cs_f, uint32_t nf, const Scalars *sc, hipStream_t s,
                               const uint32_t *fid);
// The free body's force and torque partials from the mixed records (as
// launch_body_force_f64).
hipError_t launch_body_force_mixed(const Phys &P, const Grid &g, const Dummies &d, int64_t nd, const MixedRec &rec,
                                   const uint32_t *cs_f, uint32_t nf, const Scalars *sc, double *part,
                                   hipStream_t s);
// modes and kept lists as for launch_pair_f64; abs32: the single-precision
// form of the pair sums (SPH_FP32)
hipError_t launch_pair_mixed(const Phys &P, const Grid &g, const MixedRec &rec, const uint32_t *cs_f,
                             const uint32_t *cs_d, uint32_t nf, Scalars *sc, const Rates &out, uint32_t *cand,
                             int mode, uint32_t *kent, unsigned long long *kcnt, hipStream_t s,
                             bool abs32 = false);
// records of the mixed state in its current order (no sort)
hipError_t launch_refresh_mixed(const Phys &P, const Grid &g, const FluidMixed &f, int64_t nf, const MixedRec &rec,
                                hipStream_t s);
hipError_t launch_scan_mixed(const Phys &P, const Grid &g, const MixedRec &rec, const uint32_t *cs_f,
                             const uint32_t *cs_d, uint32_t nf, const uint32_t *list, const uint32_t *count,
                             const Rates &out, Scalars *sc, hipStream_t s);
// SSP-RK2 stage update of the mixed state; also max |U|^2 of the new state
// into sc->umax2_bits (reset here) and, when rec is given, the neighbour
// records of the new state
hipError_t launch_stage_mixed(const Phys &P, const Grid &g, const FluidMixed &f, const Rates &r, int64_t nf,
                              Scalars *sc, int stage, hipStream_t s, const MixedRec *rec = nullptr);
// state fields of the fluid rows (x, u, phi, rho, p, mass, cell) in original order
hipError_t launch_fields_mixed(const Phys &P, const Grid &g, const FluidMixed &f, int64_t nf, int field, void *dst,
                               hipStream_t s, uint32_t nout);
// dummy rows of u, phi, rho, p from the mixed records
hipError_t launch_dummy_fields_mixed(const Phys &P, const MixedRec &rec, int64_t nf, const uint32_t *did, int64_t nd,
                                     int field, void *dst, hipStream_t s, uint32_t nout);

}  // namespace wb
