#include "mixed.h"
namespace wb {
hipError_t launch_to_mixed(const Phys &, const Grid &, const FluidF64 &, int64_t, const FluidMixed &, Scalars *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_reorder_mixed(const Phys &, const Grid &, const uint32_t *, int64_t, const FluidMixed &, const FluidMixed &, const MixedRec &, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_mirror_mixed(const Phys &, const Grid &, const Dummies &, int64_t, const MixedRec &, const uint32_t *, uint32_t, const Scalars *, hipStream_t, const uint32_t *) { return hipErrorNotSupported; }
hipError_t launch_pair_mixed(const Phys &, const Grid &, const MixedRec &, const uint32_t *, const uint32_t *, uint32_t, Scalars *, const Rates &, uint32_t *, bool, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_scan_mixed(const Phys &, const Grid &, const MixedRec &, const uint32_t *, const uint32_t *, uint32_t, const uint32_t *, const uint32_t *, const Rates &, Scalars *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_stage_mixed(const Phys &, const Grid &, const FluidMixed &, const Rates &, int64_t, const Scalars *, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_fields_mixed(const Phys &, const Grid &, const FluidMixed &, int64_t, int, void *, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_dummy_fields_mixed(const Phys &, const MixedRec &, int64_t, const uint32_t *, int64_t, int, void *, hipStream_t) { return hipErrorNotSupported; }
}
