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
// Workgroup slots (each MLP_PARAMS + 1 floats) the gradient of `rows` rows uses.
uint32_t mlp_grad_slots(uint64_t rows);
// grad = d/dparams of scale * sum_{r in [r0, r1)} (f(x_r) - y_r)^2 (overwritten);
// *loss += that sum.  partial: mlp_grad_slots(r1 - r0) * (MLP_PARAMS + 1) floats.
// Deterministic: no atomics, fixed summation order.
void launch_mlp_grad(const float* X, const float* Y, uint64_t r0, uint64_t r1, float scale,
                     const uint16_t* wbf, const float* norm, float* partial, float* grad, float* loss,
                     hipStream_t s);
// One Adam step with step number *step_base + step_add.
void launch_mlp_adam(float* master, float* m, float* v, const float* grad, uint16_t* wbf, float lr,
                     const uint32_t* step_base, uint32_t step_add, hipStream_t s);
// losses[ctr[0]] = *acc / batches; ctr[0] += 1; ctr[1] += batches; *acc = 0.
void launch_mlp_epoch_end(float* acc, float* losses, uint32_t* ctr, uint32_t batches, hipStream_t s);
void launch_mlp_round(const float* master, uint16_t* wbf, hipStream_t s);

}  // namespace bm
