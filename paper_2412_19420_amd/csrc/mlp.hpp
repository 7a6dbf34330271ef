// Cost model layout and launchers (k_mlp.hip).
#pragma once

#include "internal.hpp"

namespace bm {

constexpr int MLP_IN = 8;
constexpr int MLP_H = 64;
constexpr int MLP_W1 = 0;                          // [8][64]
constexpr int MLP_B1 = MLP_W1 + MLP_IN * MLP_H;    // [64]
constexpr int MLP_W2 = MLP_B1 + MLP_H;             // [64][64]
constexpr int MLP_B2 = MLP_W2 + MLP_H * MLP_H;     // [64]
constexpr int MLP_W3 = MLP_B2 + MLP_H;             // [64]
constexpr int MLP_B3 = MLP_W3 + MLP_H;             // [1]
constexpr int MLP_PARAMS = MLP_B3 + 1;             // 4801
constexpr int MLP_R = 64;                          // rows per workgroup in the gradient kernel

void launch_mlp_forward(const float* X, uint64_t rows, const uint16_t* wbf, const float* norm,
                        float* out, hipStream_t s);
// grad += d/dparams of scale * sum_{r in [r0, r1)} (f(x_r) - y_r)^2; loss += that sum
void launch_mlp_grad(const float* X, const float* Y, uint64_t r0, uint64_t r1, float scale,
                     const uint16_t* wbf, const float* norm, float* grad, float* loss, hipStream_t s);
void launch_mlp_adam(float* master, float* m, float* v, const float* grad, uint16_t* wbf, float lr,
                     uint64_t step, hipStream_t s);
void launch_mlp_round(const float* master, uint16_t* wbf, hipStream_t s);

}  // namespace bm
