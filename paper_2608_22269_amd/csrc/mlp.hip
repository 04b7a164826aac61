#include "mlp.h"
#include "wbsph.h"
namespace wb {
hipError_t launch_classify(const Classifier &, const Rates &, const uint32_t *, const uint32_t *, uint32_t *, Scalars *, const Phys &, uint32_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_mlp_infer(const float *, const float *, const float *, const float *, const uint32_t *, const uint32_t *, int64_t, float *, hipStream_t) { return hipErrorNotSupported; }
}

extern "C" {
sph_status sph_set_classifier(sph_ctx *, const float *, int64_t, const float *, const float *, float) { return SPH_EUNSUPPORTED; }
size_t sph_mlp_workspace_bytes(int64_t) { return 0; }
sph_status sph_mlp_create(int64_t, const float *, const float *, const float *, void *, size_t, void *, sph_mlp **) { return SPH_EUNSUPPORTED; }
void sph_mlp_destroy(sph_mlp *) {}
sph_status sph_mlp_forward(sph_mlp *, const float *, int64_t, float *) { return SPH_EUNSUPPORTED; }
sph_status sph_mlp_loss_grad(sph_mlp *, const float *, const float *, const float *, int64_t, float *, float *) { return SPH_EUNSUPPORTED; }
sph_status sph_mlp_adam(sph_mlp *, float, float, float, float) { return SPH_EUNSUPPORTED; }
sph_status sph_mlp_train_epoch(sph_mlp *, const float *, const float *, const float *, const int32_t *, int64_t, int64_t, float, float *) { return SPH_EUNSUPPORTED; }
sph_status sph_mlp_get_params(sph_mlp *, float *, int32_t) { return SPH_EUNSUPPORTED; }
sph_status sph_mlp_infer_bf16(const float *, const float *, const float *, const float *, int64_t, float *, void *) { return SPH_EUNSUPPORTED; }
}
