// Learned initial-guess proposer: sizes, parameter layout and kernel launchers.
#pragma once

#include "ndtm_internal.h"

namespace ndtm {

constexpr int kMlpNFeat = 59;   // 11 slots x 5 + 4 global features
constexpr int kMlpWidth = 64;
constexpr int kMlpKMax = 11;    // at most 11 converged solutions mixed
// flat FP32 parameters: W1 (64x59), b1, W2 (64x64), b2, W3 (11x64), b3, row-major
constexpr int kMlpNParam = kMlpWidth * kMlpNFeat + kMlpWidth + kMlpWidth * kMlpWidth + kMlpWidth +
                           kMlpKMax * kMlpWidth + kMlpKMax;

void mlp_forward_fp32(const float* W, const float* feat, const float* mask, const float* G, const float* h, int B,
                      float* y_out, float* loss_out, hipStream_t st);
// per-sample forward/backward, deterministic gradient sum (into gout if not null),
// optional Adam step t with learning rate lr; mean loss before the step into mean_dst
void mlp_grad_step(float* W, float* m, float* v, const float* feat, const float* mask, const float* G,
                   const float* h, int B, float* loss_out, float* gbuf, float* gout, int adam, float lr, int t,
                   float* mean_dst, hipStream_t st);
void mlp_make_bf16(const float* W, void* Wb, hipStream_t st);
void mlp_infer_bf16(const void* Wb, const float* feat, int B, float* y_out, hipStream_t st);

}  // namespace ndtm
