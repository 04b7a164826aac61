// Learned free-surface classifier: a per-particle MLP 16 -> 64 -> 64 -> 1
// with GELU (tanh form), trained on labels the exact scan-region criterion
// produces, used for the particles lambda_min alone cannot decide.
//
// Training (FP32, hand-written): forward with stored activations (one wave
// per row, one lane per hidden unit), weighted binary cross-entropy on the
// logit, backward pass, parameter gradients as fixed-order batch reductions
// (deterministic), Adam with bias correction.
//
// Inference (BF16 MFMA, FP32 accumulate): one wave handles 16 rows per
// iteration; layer 1 is a 16x16x32 bf16 MFMA per 16-unit tile with K = 16
// zero-padded to 32, layer 2 two MFMAs per tile (K = 64), biases and GELU in
// FP32 between layers (the activations move from the accumulator layout to
// the operand layout through LDS), layer 3 a FP32 dot product reduced across
// the 16 lanes that share a row.  Weights stay in registers for the whole
// (persistent, grid-stride) kernel.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "mlp.h"
#include "pair_common.h"
#include "wbsph.h"

namespace wb {

// flat parameter layout
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpIn * kMlpHid;
constexpr int kOffW2 = kOffB1 + kMlpHid;
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid;
constexpr int kOffB3 = kOffW3 + kMlpHid;
static_assert(kOffB3 + 1 == kMlpParams, "parameter layout");

__device__ __forceinline__ float gelu_f(float z) {
  const float c = 0.7978845608028654f;  // sqrt(2 / pi)
  return 0.5f * z * (1.0f + tanhf(c * (z + 0.044715f * z * z * z)));
}

// GELU (tanh form) for BF16 inference: 0.5 z (1 + tanh u) = z / (1 + e^{-2u})
// with u = sqrt(2/pi) (z + 0.044715 z^3), on the hardware exp2 and
// reciprocal (relative error ~1e-6, far below the BF16 rounding of the
// activations).  Saturates correctly: e -> inf gives 0, e -> 0 gives z.
__device__ __forceinline__ float gelu_fast(float z) {
  const float k = -2.0f * 0.7978845608028654f * 1.4426950408889634f;  // -2 sqrt(2/pi) log2(e)
  const float kc = k * 0.044715f;                                       // folded into the cubic term
  const float e = __builtin_amdgcn_exp2f(z * fmaf(kc, z * z, k));
  return z * __builtin_amdgcn_rcpf(1.0f + e);
}

__device__ __forceinline__ float gelu_grad_f(float z) {
  const float c = 0.7978845608028654f;
  const float th = tanhf(c * (z + 0.044715f * z * z * z));
  return 0.5f * (1.0f + th) + 0.5f * z * (1.0f - th * th) * c * (1.0f + 3.0f * 0.044715f * z * z);
}

// ------------------------------------------------------------- training

// Forward for rows[b] = perm ? perm[off + b] : off + b.  blockDim = 256 = four
// rows, one wave per row, lane = hidden unit.  Stores standardised input,
// pre-activations and activations for the backward pass; logit to s[b].
__global__ void __launch_bounds__(256) k_mlp_fwd(const float *__restrict__ w, const float *__restrict__ mean,
                                                 const float *__restrict__ std, const float *__restrict__ X,
                                                 const int32_t *__restrict__ perm, int64_t off, int64_t B,
                                                 float *__restrict__ xs, float *__restrict__ z1,
                                                 float *__restrict__ z2, float *__restrict__ a2,
                                                 float *__restrict__ s) {
  __shared__ float sx[4][kMlpIn];
  __shared__ float sa1[4][kMlpHid];
  const int lane = threadIdx.x & 63, r = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * 4 + r;
  const bool on = b < B;
  const int64_t row = on ? (perm ? (int64_t)perm[off + b] : off + b) : 0;
  if (on && lane < kMlpIn) {
    float v = (X[row * kMlpIn + lane] - mean[lane]) / std[lane];
    sx[r][lane] = v;
    xs[b * kMlpIn + lane] = v;
  }
  __syncthreads();
  float z = w[kOffB1 + lane];
  for (int i = 0; i < kMlpIn; ++i) z += sx[r][i] * w[kOffW1 + i * kMlpHid + lane];
  if (on) z1[b * kMlpHid + lane] = z;
  sa1[r][lane] = gelu_f(z);
  __syncthreads();
  float y = w[kOffB2 + lane];
  for (int k = 0; k < kMlpHid; ++k) y += sa1[r][k] * w[kOffW2 + k * kMlpHid + lane];
  const float act = gelu_f(y);
  if (on) {
    z2[b * kMlpHid + lane] = y;
    a2[b * kMlpHid + lane] = act;
  }
  float p = act * w[kOffW3 + lane];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
  if (on && lane == 0) s[b] = p + w[kOffB3];
}

// dL/ds for the weighted mean BCE and the per-row loss terms.
__global__ void k_mlp_loss(const float *__restrict__ s, const float *__restrict__ y, const float *__restrict__ wt,
                           const int32_t *__restrict__ perm, int64_t off, int64_t B, float *__restrict__ ds,
                           float *__restrict__ lrow) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int64_t row = perm ? (int64_t)perm[off + b] : off + b;
  const float sv = s[b], yv = y[row], wv = wt ? wt[row] : 1.0f;
  const float sig = 1.0f / (1.0f + expf(-sv));
  ds[b] = wv * (sig - yv) / (float)B;
  lrow[b] = wv * (fmaxf(sv, 0.0f) - sv * yv + log1pf(expf(-fabsf(sv))));
}

// Backward through layers 3 and 2 per row: dz2 = ds W3 gelu'(z2); then
// dz1 = (dz2 W2^T) gelu'(z1).  One wave per row.
__global__ void __launch_bounds__(256) k_mlp_bwd_rows(const float *__restrict__ w, const float *__restrict__ z1,
                                                      const float *__restrict__ z2, const float *__restrict__ ds,
                                                      int64_t B, float *__restrict__ dz1, float *__restrict__ dz2) {
  __shared__ float sd[4][kMlpHid];
  const int lane = threadIdx.x & 63, r = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * 4 + r;
  const bool on = b < B;
  float d2 = 0.0f;
  if (on) d2 = ds[b] * w[kOffW3 + lane] * gelu_grad_f(z2[b * kMlpHid + lane]);
  sd[r][lane] = d2;
  __syncthreads();
  if (!on) return;
  dz2[b * kMlpHid + lane] = d2;
  float a = 0.0f;
  for (int k = 0; k < kMlpHid; ++k) a += sd[r][k] * w[kOffW2 + lane * kMlpHid + k];
  dz1[b * kMlpHid + lane] = a * gelu_grad_f(z1[b * kMlpHid + lane]);
}

// Parameter gradients: one thread per parameter, a fixed-order loop over the
// batch (deterministic).  a1 is recomputed from z1.
__global__ void __launch_bounds__(256) k_mlp_param_grad(const float *__restrict__ xs, const float *__restrict__ z1,
                                                        const float *__restrict__ a2, const float *__restrict__ ds,
                                                        const float *__restrict__ dz1, const float *__restrict__ dz2,
                                                        int64_t B, float *__restrict__ g) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  float acc = 0.0f;
  if (p < kOffB1) {  // W1[i, o]
    const int i = p / kMlpHid, o = p % kMlpHid;
    for (int64_t b = 0; b < B; ++b) acc += xs[b * kMlpIn + i] * dz1[b * kMlpHid + o];
  } else if (p < kOffW2) {  // b1[o]
    const int o = p - kOffB1;
    for (int64_t b = 0; b < B; ++b) acc += dz1[b * kMlpHid + o];
  } else if (p < kOffB2) {  // W2[k, o]
    const int q = p - kOffW2, k = q / kMlpHid, o = q % kMlpHid;
    for (int64_t b = 0; b < B; ++b) acc += gelu_f(z1[b * kMlpHid + k]) * dz2[b * kMlpHid + o];
  } else if (p < kOffW3) {  // b2[o]
    const int o = p - kOffB2;
    for (int64_t b = 0; b < B; ++b) acc += dz2[b * kMlpHid + o];
  } else if (p < kOffB3) {  // W3[k]
    const int k = p - kOffW3;
    for (int64_t b = 0; b < B; ++b) acc += a2[b * kMlpHid + k] * ds[b];
  } else {  // b3
    for (int64_t b = 0; b < B; ++b) acc += ds[b];
  }
  g[p] = acc;
}

// Fixed-order sum of the row losses divided by B.
__global__ void __launch_bounds__(256) k_mlp_loss_sum(const float *__restrict__ lrow, int64_t B, float *__restrict__ out) {
  __shared__ float sh[256];
  float a = 0.0f;
  for (int64_t b = threadIdx.x; b < B; b += 256) a += lrow[b];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0] / (float)B;
}

__global__ void k_mlp_loss_acc(const float *loss, float *acc, int reset) {
  *acc = (reset ? 0.0f : *acc) + *loss;
}

__global__ void k_mlp_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                           float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.0f - b1) * gp;
  const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  w[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// --------------------------------------------------------- BF16 inference

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

// One wave per 16-row tile (grid-stride over tiles).  rows: optional index
// list (feature row r of output k is rows[k]); nrows_dev: optional device
// count overriding n.
__global__ void __launch_bounds__(256) k_mlp_infer_bf16(const float *__restrict__ w, const float *__restrict__ mean,
                                                        const float *__restrict__ std, const float *__restrict__ X,
                                                        const uint32_t *__restrict__ rows,
                                                        const uint32_t *__restrict__ nrows_dev, int64_t n,
                                                        float *__restrict__ logits) {
  __shared__ __bf16 act[4][16][kMlpHid + 8];  // per wave: 16 rows x 64 (+pad)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;  // MFMA lane coordinates
  const int64_t total = nrows_dev ? (int64_t)(*nrows_dev) : n;
  const int64_t ntiles = (total + 15) / 16;
  const int64_t wave_id = (int64_t)blockIdx.x * 4 + wv;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  // waves without a tile leave before loading the weights (the grid is sized
  // for the largest possible count; the device count may be far smaller)
  if (wave_id >= ntiles) return;

  // B operands (weights) in registers: B[k][n] for n = col + 16 t,
  // k = 8 grp + e (+ 32 kb).  Layer 1 has K = 16: groups 2, 3 hold zeros.
  bf16x8 w1b[4], w2b[4][2];
  float b1c[4], b2c[4], w3c[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int nn = col + 16 * t;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 8 * grp + e;
      w1b[t][e] = to_bf16(k < kMlpIn ? w[kOffW1 + k * kMlpHid + nn] : 0.0f);
      w2b[t][0][e] = to_bf16(w[kOffW2 + k * kMlpHid + nn]);
      w2b[t][1][e] = to_bf16(w[kOffW2 + (k + 32) * kMlpHid + nn]);
    }
    b1c[t] = w[kOffB1 + nn];
    b2c[t] = w[kOffB2 + nn];
    w3c[t] = w[kOffW3 + nn];
  }
  const float b3 = w[kOffB3];
  float mu[8], isd[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k = 8 * grp + e;
    mu[e] = k < kMlpIn ? mean[k] : 0.0f;
    isd[e] = k < kMlpIn ? 1.0f / std[k] : 0.0f;
  }

  for (int64_t tile = wave_id; tile < ntiles; tile += nwaves) {
    const int64_t r0 = tile * 16;
    // A operand of layer 1: row = col, k = 8 grp + e (features 0..15)
    const int64_t rr = r0 + col;
    const bool rv = rr < total;
    const int64_t src = rv ? (rows ? (int64_t)rows[rr] : rr) : 0;
    bf16x8 xa;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 8 * grp + e;
      float v = (rv && k < kMlpIn) ? (X[src * kMlpIn + k] - mu[e]) * isd[e] : 0.0f;
      xa[e] = to_bf16(v);
    }
    // layer 1 -> GELU -> LDS (row-major 16 x 64)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa, w1b[t], acc, 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; ++j) act[wv][4 * grp + j][col + 16 * t] = to_bf16(gelu_fast(acc[j] + b1c[t]));
    }
    // hand the tile to the other lanes of this wave through LDS
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // A operands of layer 2: row = col, k = 8 grp + e (+32)
    bf16x8 h0, h1;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      h0[e] = act[wv][col][8 * grp + e];
      h1[e] = act[wv][col][32 + 8 * grp + e];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h0, w2b[t][0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h1, w2b[t][1], acc, 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; ++j) part[j] += gelu_fast(acc[j] + b2c[t]) * w3c[t];
    }
    // layer 3: reduce over the 16 lanes (columns) sharing rows 4 grp + j
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) part[j] += __shfl_xor(part[j], o, 16);
    }
    if (col == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t r = r0 + 4 * grp + j;
        if (r < total) logits[r] = part[j] + b3;
      }
    }
  }
}

hipError_t launch_mlp_infer(const float *w, const float *mean, const float *std, const float *X, const uint32_t *rows,
                            const uint32_t *nrows_dev, int64_t n, float *logits, hipStream_t s) {
  int64_t tiles = (n + 15) / 16;
  int64_t blocks = (tiles + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_mlp_infer_bf16, dim3((unsigned)blocks), dim3(256), 0, s, w, mean, std, X, rows, nrows_dev, n,
                     logits);
  return hipGetLastError();
}

// ---------------------------------------------------- classify candidates

// Candidates' features are the rows feat[cand[k] * 16]; logit k belongs to
// particle cand[k].  Decide: logit >= margin -> surface, <= -margin ->
// interior, otherwise append to the fallback list for the scan pass.
template <int DIM>
__global__ void __launch_bounds__(256) k_decide(Phys P, Rates out, const uint32_t *__restrict__ cand,
                                                const uint32_t *__restrict__ n_cand, const float *__restrict__ lg,
                                                float margin, uint32_t *__restrict__ fallback, Scalars *sc) {
  const uint32_t total = *n_cand;
  const uint32_t stride = gridDim.x * blockDim.x;
  // every lane runs the same number of iterations (wave-level atomics inside)
  const uint32_t iters = (total + stride - 1) / stride;
  for (uint32_t it = 0; it < iters; ++it) {
    const uint32_t k = it * stride + blockIdx.x * blockDim.x + threadIdx.x;
    const bool on = k < total;
    uint32_t i = 0;
    float l = 0.0f;
    bool fb = false, fs = false;
    if (on) {
      i = cand[k];
      l = lg[k];
      out.logit[i] = l;
      fb = fabsf(l) < margin;
      fs = !fb && l > 0.0f;
    }
    const uint32_t slot = wave_append(&sc->n_scan, on && fb);
    if (on && fb) fallback[slot] = i;
    wave_count(&sc->n_mlp, on && !fb);
    if (on && !fb) {
      uint32_t fl = out.flags[i] | kFlagByMLP;
      if (fs) {
        fl |= kFlagFS;
        if ((P.flags & SPH_F_FS_PROJECT) && (P.flags & SPH_F_PST)) {
          const double n0 = out.nrm[0][i], n1 = out.nrm[1][i], n2 = DIM == 3 ? out.nrm[2][i] : 0.0;
          double u0 = out.dus[0][i], u1 = out.dus[1][i], u2 = DIM == 3 ? out.dus[2][i] : 0.0;
          double d = u0 * n0 + u1 * n1 + u2 * n2;
          out.dus[0][i] = u0 - d * n0;
          out.dus[1][i] = u1 - d * n1;
          if (DIM == 3) out.dus[2][i] = u2 - d * n2;
        }
      }
      out.flags[i] = fl;
    }
    wave_count(&sc->n_fs, on && fs);
  }
}

hipError_t launch_classify(const Classifier &c, const Rates &r, const uint32_t *cand, const uint32_t *n_cand,
                           uint32_t *fallback, Scalars *sc, const Phys &P, uint32_t nf, float *lgbuf, hipStream_t s) {
  if (nf == 0) return hipSuccess;
  hipError_t e = launch_mlp_infer(c.w, c.mean, c.std, r.feat, cand, n_cand, nf, lgbuf, s);
  if (e != hipSuccess) return e;
  unsigned db = grid_for(nf);
  if (db > 1024) db = 1024;
  if (P.dim == 2)
    hipLaunchKernelGGL(k_decide<2>, dim3(db), dim3(256), 0, s, P, r, cand, n_cand, lgbuf, c.margin, fallback, sc);
  else
    hipLaunchKernelGGL(k_decide<3>, dim3(db), dim3(256), 0, s, P, r, cand, n_cand, lgbuf, c.margin, fallback, sc);
  return hipGetLastError();
}

}  // namespace wb

// ====================================================================== ABI

using namespace wb;

struct sph_mlp {
  int64_t max_batch;
  hipStream_t s;
  float *w, *g, *m, *v, *mean, *std;
  float *xs, *z1, *z2, *a2, *sv, *ds, *dz1, *dz2, *lrow, *loss, *loss_acc;
  int64_t step;
};

namespace {

size_t mlp_carve(sph_mlp *m, uintptr_t base, int64_t B) {
  uintptr_t off = 0;
  auto take = [&](int64_t count) {
    off = (off + 255) & ~(uintptr_t)255;
    float *p = base ? reinterpret_cast<float *>(base + off) : nullptr;
    off += (uintptr_t)(count > 0 ? count : 1) * sizeof(float);
    return p;
  };
  m->w = take(kMlpParams);
  m->g = take(kMlpParams);
  m->m = take(kMlpParams);
  m->v = take(kMlpParams);
  m->mean = take(kMlpIn);
  m->std = take(kMlpIn);
  m->xs = take(B * kMlpIn);
  m->z1 = take(B * kMlpHid);
  m->z2 = take(B * kMlpHid);
  m->a2 = take(B * kMlpHid);
  m->sv = take(B);
  m->ds = take(B);
  m->dz1 = take(B * kMlpHid);
  m->dz2 = take(B * kMlpHid);
  m->lrow = take(B);
  m->loss = take(1);
  m->loss_acc = take(1);
  return off + 256;
}

hipError_t mlp_loss_grad(sph_mlp *m, const float *X, const float *y, const float *w, const int32_t *perm, int64_t off,
                         int64_t B) {
  hipStream_t s = m->s;
  const unsigned rb = (unsigned)((B + 3) / 4);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(rb), dim3(256), 0, s, m->w, m->mean, m->std, X, perm, off, B, m->xs, m->z1, m->z2,
                     m->a2, m->sv);
  hipLaunchKernelGGL(k_mlp_loss, dim3(grid_for(B)), dim3(256), 0, s, m->sv, y, w, perm, off, B, m->ds, m->lrow);
  hipLaunchKernelGGL(k_mlp_bwd_rows, dim3(rb), dim3(256), 0, s, m->w, m->z1, m->z2, m->ds, B, m->dz1, m->dz2);
  hipLaunchKernelGGL(k_mlp_param_grad, dim3(grid_for(kMlpParams)), dim3(256), 0, s, m->xs, m->z1, m->a2, m->ds, m->dz1,
                     m->dz2, B, m->g);
  hipLaunchKernelGGL(k_mlp_loss_sum, dim3(1), dim3(256), 0, s, m->lrow, B, m->loss);
  return hipGetLastError();
}

hipError_t mlp_adam(sph_mlp *m, float lr, float b1, float b2, float eps) {
  m->step += 1;
  const float c1 = 1.0f - std::pow(b1, (float)m->step);
  const float c2 = 1.0f - std::pow(b2, (float)m->step);
  hipLaunchKernelGGL(k_mlp_adam, dim3(grid_for(kMlpParams)), dim3(256), 0, m->s, m->w, m->g, m->m, m->v, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

}  // namespace

// Scratch of sph_mlp_forward_noalloc: the activations k_mlp_fwd stores
// (standardised input, both pre-activations, the second activation) for up
// to SPH_MLP_NOALLOC_MAX_ROWS rows, in a fixed device array (each device
// that runs the library holds its own copy).  Host code never passes the
// array's name to a kernel: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and kept.
static __device__ __align__(256) float scratch[(size_t)SPH_MLP_NOALLOC_MAX_ROWS * (kMlpIn + 3 * kMlpHid)];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kScratchDevices] = {};

// Device address of the current device's scratch array.
sph_status noalloc_scratch(float **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return SPH_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return SPH_EHIP;
    g_scratch_ptr[dev] = static_cast<float *>(p);
  }
  *out = g_scratch_ptr[dev];
  return SPH_OK;
}

}  // namespace

extern "C" {

size_t sph_mlp_workspace_bytes(int64_t max_batch) {
  if (max_batch <= 0 || max_batch > (1 << 24)) return 0;
  sph_mlp m;
  return mlp_carve(&m, 0, max_batch);
}

sph_status sph_mlp_create(int64_t max_batch, const float *params0, const float *mean, const float *std, void *workspace,
                          size_t ws_bytes, void *hip_stream, sph_mlp **out) {
  if (!out || !params0 || !mean || !std) return SPH_EINVAL;
  *out = nullptr;
  size_t need = sph_mlp_workspace_bytes(max_batch);
  if (need == 0) return SPH_EINVAL;
  if (!workspace || ((uintptr_t)workspace % 256) != 0 || ws_bytes < need) return SPH_EWORKSPACE;
  for (int k = 0; k < kMlpIn; ++k)
    if (!(std[k] > 0.0f) || !std::isfinite(mean[k])) return SPH_EINVAL;
  sph_mlp *m = new sph_mlp();
  m->max_batch = max_batch;
  m->s = (hipStream_t)hip_stream;
  m->step = 0;
  mlp_carve(m, (uintptr_t)workspace, max_batch);
  hipError_t e = hipMemcpyAsync(m->w, params0, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, m->s);
  if (e == hipSuccess) e = hipMemcpyAsync(m->mean, mean, sizeof(float) * kMlpIn, hipMemcpyHostToDevice, m->s);
  if (e == hipSuccess) e = hipMemcpyAsync(m->std, std, sizeof(float) * kMlpIn, hipMemcpyHostToDevice, m->s);
  if (e == hipSuccess) e = hipMemsetAsync(m->m, 0, sizeof(float) * kMlpParams, m->s);
  if (e == hipSuccess) e = hipMemsetAsync(m->v, 0, sizeof(float) * kMlpParams, m->s);
  if (e == hipSuccess) e = hipStreamSynchronize(m->s);
  if (e != hipSuccess) {
    delete m;
    return SPH_EHIP;
  }
  *out = m;
  return SPH_OK;
}

void sph_mlp_destroy(sph_mlp *m) { delete m; }

sph_status sph_mlp_forward(sph_mlp *m, const float *X, int64_t B, float *logits) {
  if (!m || !X || !logits || B < 0 || B > m->max_batch) return SPH_EINVAL;
  if (B == 0) return SPH_OK;
  const unsigned rb = (unsigned)((B + 3) / 4);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(rb), dim3(256), 0, m->s, m->w, m->mean, m->std, X, (const int32_t *)nullptr,
                     (int64_t)0, B, m->xs, m->z1, m->z2, m->a2, logits);
  return hipGetLastError() == hipSuccess ? SPH_OK : SPH_EHIP;
}

sph_status sph_mlp_loss_grad(sph_mlp *m, const float *X, const float *y, const float *w, int64_t B, float *loss,
                             float *grad) {
  if (!m || !X || !y || B <= 0 || B > m->max_batch) return SPH_EINVAL;
  hipError_t e = mlp_loss_grad(m, X, y, w, nullptr, 0, B);
  if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToDevice, m->s);
  if (e == hipSuccess && grad)
    e = hipMemcpyAsync(grad, m->g, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice, m->s);
  return e == hipSuccess ? SPH_OK : SPH_EHIP;
}

sph_status sph_mlp_adam(sph_mlp *m, float lr, float beta1, float beta2, float eps) {
  if (!m || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0)) return SPH_EINVAL;
  return mlp_adam(m, lr, beta1, beta2, eps) == hipSuccess ? SPH_OK : SPH_EHIP;
}

sph_status sph_mlp_train_epoch(sph_mlp *m, const float *X, const float *y, const float *w, const int32_t *perm,
                               int64_t n, int64_t batch, float lr, float *mean_loss) {
  if (!m || !X || !y || !perm || n <= 0 || batch <= 0 || batch > m->max_batch || !(lr > 0)) return SPH_EINVAL;
  // the batch losses accumulate on the device; one synchronisation at the end
  int64_t nb = 0;
  for (int64_t off = 0; off < n; off += batch) {
    const int64_t B = std::min(batch, n - off);
    hipError_t e = mlp_loss_grad(m, X, y, w, perm, off, B);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_mlp_loss_acc, dim3(1), dim3(1), 0, m->s, m->loss, m->loss_acc, nb == 0 ? 1 : 0);
      e = mlp_adam(m, lr, 0.9f, 0.999f, 1e-8f);
    }
    if (e != hipSuccess) return SPH_EHIP;
    ++nb;
  }
  if (mean_loss) {
    float l = 0.0f;
    if (hipMemcpyAsync(&l, m->loss_acc, sizeof(float), hipMemcpyDeviceToHost, m->s) != hipSuccess ||
        hipStreamSynchronize(m->s) != hipSuccess)
      return SPH_EHIP;
    *mean_loss = l / (float)nb;
  }
  return SPH_OK;
}

sph_status sph_mlp_get_params(sph_mlp *m, float *out, int32_t out_on_device) {
  if (!m || !out) return SPH_EINVAL;
  hipError_t e = hipMemcpyAsync(out, m->w, sizeof(float) * kMlpParams,
                                out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, m->s);
  if (e == hipSuccess && !out_on_device) e = hipStreamSynchronize(m->s);
  return e == hipSuccess ? SPH_OK : SPH_EHIP;
}

sph_status sph_mlp_forward_noalloc(const float *params, const float *mean, const float *std, const float *X,
                                   int64_t B, float *logits, void *hip_stream) {
  if (!params || !mean || !std || !X || !logits || B < 0 || B > SPH_MLP_NOALLOC_MAX_ROWS) return SPH_EINVAL;
  if (B == 0) return SPH_OK;
  float *sp = nullptr;
  if (noalloc_scratch(&sp) != SPH_OK) return SPH_EHIP;
  float *xs = sp;
  float *z1 = xs + (size_t)SPH_MLP_NOALLOC_MAX_ROWS * kMlpIn;
  float *z2 = z1 + (size_t)SPH_MLP_NOALLOC_MAX_ROWS * kMlpHid;
  float *a2 = z2 + (size_t)SPH_MLP_NOALLOC_MAX_ROWS * kMlpHid;
  const unsigned rb = (unsigned)((B + 3) / 4);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(rb), dim3(256), 0, (hipStream_t)hip_stream, params, mean, std, X,
                     (const int32_t *)nullptr, (int64_t)0, B, xs, z1, z2, a2, logits);
  return hipGetLastError() == hipSuccess ? SPH_OK : SPH_EHIP;
}

sph_status sph_mlp_infer_bf16(const float *params, const float *mean, const float *std, const float *X, int64_t n,
                              float *logits, void *hip_stream) {
  if (!params || !mean || !std || !X || !logits || n < 0) return SPH_EINVAL;
  if (n == 0) return SPH_OK;
  return launch_mlp_infer(params, mean, std, X, nullptr, nullptr, n, logits, (hipStream_t)hip_stream) == hipSuccess
             ? SPH_OK
             : SPH_EHIP;
}

}  // extern "C"
