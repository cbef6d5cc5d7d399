// Kernels of the learned initial-guess proposer: a 3-layer tanh network
// (59 -> 64 -> 64 -> 11) trained in FP32 with Adam and run in BF16 for
// inference.  One block of 64 threads per sample; thread j owns neuron j.
//
// Loss per sample (exact, from the Gram form of the residual of a mix of
// converged solutions): L(y) = 1 + 2 h.(m*y) + (m*y).G.(m*y), mean over the
// batch.  Per-sample gradients go to a buffer and are summed over samples in a
// fixed order by the update kernel (deterministic), which also applies Adam.
#include <hip/hip_bf16.h>

#include "mlp.h"

namespace ndtm {
namespace {

constexpr int NF = kMlpNFeat, WD = kMlpWidth, KO = kMlpKMax;
constexpr int OFF_W1 = 0, OFF_B1 = WD * NF, OFF_W2 = OFF_B1 + WD, OFF_B2 = OFF_W2 + WD * WD, OFF_W3 = OFF_B2 + WD,
              OFF_B3 = OFF_W3 + KO * WD;
static_assert(OFF_B3 + KO == kMlpNParam, "parameter layout");

template <bool GRAD>
__global__ __launch_bounds__(64) void mlp_sample_k(const float* __restrict__ Wt, const float* __restrict__ feat,
                                                   const float* __restrict__ mask, const float* __restrict__ G,
                                                   const float* __restrict__ h, int B, float* y_out, float* loss_out,
                                                   float* gbuf) {
  const int s = blockIdx.x, j = threadIdx.x;
  __shared__ float f[NF], h1[WD], h2[WD], ym[KO], dy[KO], dz2[WD], dz1[WD], lj[KO];
  for (int k = j; k < NF; k += WD) f[k] = feat[(size_t)s * NF + k];
  __syncthreads();
  float z = Wt[OFF_B1 + j];
  for (int k = 0; k < NF; ++k) z += Wt[OFF_W1 + j * NF + k] * f[k];
  h1[j] = tanhf(z);
  __syncthreads();
  z = Wt[OFF_B2 + j];
  for (int k = 0; k < WD; ++k) z += Wt[OFF_W2 + j * WD + k] * h1[k];
  h2[j] = tanhf(z);
  __syncthreads();
  if (j < KO) {
    float y = Wt[OFF_B3 + j];
    for (int k = 0; k < WD; ++k) y += Wt[OFF_W3 + j * WD + k] * h2[k];
    if (y_out) y_out[(size_t)s * KO + j] = y;
    ym[j] = mask[(size_t)s * KO + j] * y;
  }
  __syncthreads();
  if (j < KO) {
    const float* Gs = G + (size_t)s * KO * KO;
    float gy = 0.f;
    for (int k = 0; k < KO; ++k) gy += Gs[j * KO + k] * ym[k];
    const float hj = h[(size_t)s * KO + j];
    dy[j] = 2.f * mask[(size_t)s * KO + j] * (hj + gy) / (float)B;
    lj[j] = (2.f * hj + gy) * ym[j];
  }
  __syncthreads();
  if (j == 0 && loss_out) {
    float L = 1.f;
    for (int k = 0; k < KO; ++k) L += lj[k];
    loss_out[s] = L;
  }
  if (!GRAD) return;
  float* g = gbuf + (size_t)s * kMlpNParam;
  // layer 3
  for (int o = 0; o < KO; ++o) g[OFF_W3 + o * WD + j] = dy[o] * h2[j];
  if (j < KO) g[OFF_B3 + j] = dy[j];
  float dh = 0.f;
  for (int o = 0; o < KO; ++o) dh += Wt[OFF_W3 + o * WD + j] * dy[o];
  dz2[j] = dh * (1.f - h2[j] * h2[j]);
  __syncthreads();
  // layer 2
  for (int k = 0; k < WD; ++k) g[OFF_W2 + j * WD + k] = dz2[j] * h1[k];
  g[OFF_B2 + j] = dz2[j];
  dh = 0.f;
  for (int o = 0; o < WD; ++o) dh += Wt[OFF_W2 + o * WD + j] * dz2[o];
  dz1[j] = dh * (1.f - h1[j] * h1[j]);
  __syncthreads();
  // layer 1
  for (int k = 0; k < NF; ++k) g[OFF_W1 + j * NF + k] = dz1[j] * f[k];
  g[OFF_B1 + j] = dz1[j];
}

// sums the per-sample gradients (fixed sample order) and applies one Adam step
// (bias-corrected, step t >= 1); with adam == 0 it only writes the gradient.
__global__ void mlp_update_k(float* Wt, float* m, float* v, const float* gbuf, int B, float* gout, int adam,
                             float lr, int t) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpNParam) return;
  float g = 0.f;
  for (int s = 0; s < B; ++s) g += gbuf[(size_t)s * kMlpNParam + p];
  if (gout) gout[p] = g;
  if (!adam) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mm = b1 * m[p] + (1.f - b1) * g;
  const float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float mh = mm / (1.f - powf(b1, (float)t));
  const float vh = vv / (1.f - powf(b2, (float)t));
  Wt[p] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void mlp_mean_k(const float* loss, int B, float* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < B; ++i) s += loss[i];
    *dst = s / (float)B;
  }
}

__global__ void mlp_to_bf16_k(const float* W, __hip_bfloat16* Wb) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kMlpNParam) Wb[p] = __float2bfloat16(W[p]);
}

__device__ __forceinline__ float bfr(float x) { return __bfloat162float(__float2bfloat16(x)); }

// BF16 inference: weights, inputs and activations stored in BF16, FP32 accumulation.
__global__ __launch_bounds__(64) void mlp_infer_bf16_k(const __hip_bfloat16* __restrict__ Wb,
                                                       const float* __restrict__ feat, float* y_out) {
  const int s = blockIdx.x, j = threadIdx.x;
  __shared__ float f[NF], h1[WD], h2[WD];
  for (int k = j; k < NF; k += WD) f[k] = bfr(feat[(size_t)s * NF + k]);
  __syncthreads();
  float z = __bfloat162float(Wb[OFF_B1 + j]);
  for (int k = 0; k < NF; ++k) z += __bfloat162float(Wb[OFF_W1 + j * NF + k]) * f[k];
  h1[j] = bfr(tanhf(z));
  __syncthreads();
  z = __bfloat162float(Wb[OFF_B2 + j]);
  for (int k = 0; k < WD; ++k) z += __bfloat162float(Wb[OFF_W2 + j * WD + k]) * h1[k];
  h2[j] = bfr(tanhf(z));
  __syncthreads();
  if (j < KO) {
    float y = __bfloat162float(Wb[OFF_B3 + j]);
    for (int k = 0; k < WD; ++k) y += __bfloat162float(Wb[OFF_W3 + j * WD + k]) * h2[k];
    y_out[(size_t)s * KO + j] = y;
  }
}

}  // namespace

void mlp_forward_fp32(const float* W, const float* feat, const float* mask, const float* G, const float* h, int B,
                      float* y_out, float* loss_out, hipStream_t st) {
  hipLaunchKernelGGL(mlp_sample_k<false>, dim3(B), dim3(64), 0, st, W, feat, mask, G, h, B, y_out, loss_out,
                     (float*)nullptr);
}

void mlp_grad_step(float* W, float* m, float* v, const float* feat, const float* mask, const float* G,
                   const float* h, int B, float* loss_out, float* gbuf, float* gout, int adam, float lr, int t,
                   float* mean_dst, hipStream_t st) {
  hipLaunchKernelGGL(mlp_sample_k<true>, dim3(B), dim3(64), 0, st, (const float*)W, feat, mask, G, h, B,
                     (float*)nullptr, loss_out, gbuf);
  if (mean_dst) hipLaunchKernelGGL(mlp_mean_k, dim3(1), dim3(64), 0, st, (const float*)loss_out, B, mean_dst);
  hipLaunchKernelGGL(mlp_update_k, dim3((kMlpNParam + 255) / 256), dim3(256), 0, st, W, m, v, (const float*)gbuf, B,
                     gout, adam, lr, t);
}

void mlp_make_bf16(const float* W, void* Wb, hipStream_t st) {
  hipLaunchKernelGGL(mlp_to_bf16_k, dim3((kMlpNParam + 255) / 256), dim3(256), 0, st, W,
                     static_cast<__hip_bfloat16*>(Wb));
}

void mlp_infer_bf16(const void* Wb, const float* feat, int B, float* y_out, hipStream_t st) {
  hipLaunchKernelGGL(mlp_infer_bf16_k, dim3(B), dim3(64), 0, st, static_cast<const __hip_bfloat16*>(Wb), feat,
                     y_out);
}

}  // namespace ndtm
