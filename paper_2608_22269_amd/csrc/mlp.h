// Learned free-surface classifier: 16 features -> 64 -> 64 -> 1 with GELU
// (tanh form); FP32 training kernels and BF16 MFMA inference.
#pragma once

#include "common.h"

namespace wb {

constexpr int kMlpIn = 16, kMlpHid = 64;
constexpr int kMlpParams = kMlpIn * kMlpHid + kMlpHid + kMlpHid * kMlpHid + kMlpHid + kMlpHid + 1;  // 5313

struct Classifier {
  float *w;      // flat FP32 parameters (W1 b1 W2 b2 W3 b3)
  float *mean;   // 16
  float *std;    // 16
  float margin;  // |logit| < margin -> exact fallback
};

// Classifies the candidates listed in cand[0..*n_cand) from their feature
// rows; confident ones get their free-surface flag (and the shifting
// projection), the rest are appended to fallback (count in sc->n_scan).
hipError_t launch_classify(const Classifier &c, const Rates &r, const uint32_t *cand, const uint32_t *n_cand,
                           uint32_t *fallback, Scalars *sc, const Phys &P, uint32_t nf, float *lgbuf, hipStream_t s);

// Stateless BF16 MFMA inference over n feature rows.
hipError_t launch_mlp_infer(const float *w, const float *mean, const float *std, const float *X,
                            const uint32_t *rows, const uint32_t *nrows_dev, int64_t n, float *logits,
                            hipStream_t s);

}  // namespace wb
