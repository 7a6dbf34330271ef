// Cost model of the scheduler: an 8 -> 64 -> 64 -> 1 perceptron with ReLU,
// BF16 weights and FP32 accumulation, trained with Adam on an FP32 master copy.
// It predicts log2(1 + candidates in a subtree) from 8 features of a prefix
// class and is used only to order subtree tasks; it never changes a result.
//
// Parameter layout (4,801 values): W1[8][64], b1[64], W2[64][64], b2[64],
// W3[64], b3.  Inputs are standardised with a per-feature mean and 1/std kept
// in the model.
#include "internal.hpp"
#include "mlp.hpp"

namespace bm {

namespace {

constexpr int kThreads = 256;

uint32_t grid_for(uint64_t work, uint32_t per_block, uint32_t cap = 65535) {
  uint64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline void load_weights(const uint16_t* __restrict__ wbf, float* w) {
  for (int i = threadIdx.x; i < MLP_PARAMS; i += blockDim.x) w[i] = bf16_to_f32(wbf[i]);
}

// Forward pass of one row; h1 and z2 optional outputs.
__device__ inline float forward_row(const float* w, const float* x, float* h1, float* z2) {
  const float* W1 = w + MLP_W1;
  const float* b1 = w + MLP_B1;
  const float* W2 = w + MLP_W2;
  const float* b2 = w + MLP_B2;
  const float* W3 = w + MLP_W3;
#pragma unroll 4
  for (int j = 0; j < MLP_H; ++j) {
    float a = b1[j];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) a = fmaf(x[i], W1[i * MLP_H + j], a);
    h1[j] = fmaxf(a, 0.f);
  }
  float out = w[MLP_B3];
  for (int j = 0; j < MLP_H; ++j) {
    float a = b2[j];
#pragma unroll 8
    for (int i = 0; i < MLP_H; ++i) a = fmaf(h1[i], W2[i * MLP_H + j], a);
    if (z2) z2[j] = a;
    out = fmaf(fmaxf(a, 0.f), W3[j], out);
  }
  return out;
}

__global__ __launch_bounds__(kThreads) void k_mlp_forward(const float* __restrict__ X, uint64_t rows,
                                                          const uint16_t* __restrict__ wbf,
                                                          const float* __restrict__ norm,
                                                          float* __restrict__ out) {
  __shared__ float w[MLP_PARAMS];
  __shared__ float nm[2 * MLP_IN];
  load_weights(wbf, w);
  if (threadIdx.x < 2 * MLP_IN) nm[threadIdx.x] = norm[threadIdx.x];
  __syncthreads();
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < rows;
       r += (uint64_t)gridDim.x * blockDim.x) {
    float x[MLP_IN], h1[MLP_H];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) x[i] = (X[r * MLP_IN + i] - nm[i]) * nm[MLP_IN + i];
    out[r] = forward_row(w, x, h1, nullptr);
  }
}

// Gradient of sum_r (out_r - y_r)^2 * scale over a block of MLP_R rows:
// per-row backpropagation by one wavefront, then the parameter sums over the
// block's rows by all threads, added atomically into grad.
__global__ __launch_bounds__(kThreads) void k_mlp_grad(const float* __restrict__ X,
                                                       const float* __restrict__ Y, uint64_t r0,
                                                       uint64_t r1, float scale,
                                                       const uint16_t* __restrict__ wbf,
                                                       const float* __restrict__ norm,
                                                       float* __restrict__ grad,
                                                       float* __restrict__ loss) {
  __shared__ float w[MLP_PARAMS];
  __shared__ float nm[2 * MLP_IN];
  __shared__ float sX[MLP_R][MLP_IN];
  __shared__ float sH1[MLP_R][MLP_H + 1];  // padded: conflict-free per-row access
  __shared__ float sH2[MLP_R][MLP_H + 1];  // padded: conflict-free per-row access
  __shared__ float sD2[MLP_R][MLP_H + 1];  // padded: conflict-free per-row access
  __shared__ float sD1[MLP_R][MLP_H + 1];  // padded: conflict-free per-row access
  __shared__ float sDo[MLP_R];
  __shared__ float sL[MLP_R];
  load_weights(wbf, w);
  if (threadIdx.x < 2 * MLP_IN) nm[threadIdx.x] = norm[threadIdx.x];
  __syncthreads();
  for (uint64_t b0 = r0 + (uint64_t)blockIdx.x * MLP_R; b0 < r1; b0 += (uint64_t)gridDim.x * MLP_R) {
    const int nr = (int)min<uint64_t>(MLP_R, r1 - b0);
    if (threadIdx.x < MLP_R) {
      const int t = threadIdx.x;
      float* h1 = sH1[t];
      float* d2 = sD2[t];
      float* d1 = sD1[t];
      if (t < nr) {
        const uint64_t r = b0 + t;
        float x[MLP_IN], z2[MLP_H];
#pragma unroll
        for (int i = 0; i < MLP_IN; ++i) {
          x[i] = (X[r * MLP_IN + i] - nm[i]) * nm[MLP_IN + i];
          sX[t][i] = x[i];
        }
        const float out = forward_row(w, x, h1, z2);
        const float err = out - Y[r];
        const float dout = 2.f * err * scale;
        sDo[t] = dout;
        sL[t] = err * err * scale;
        for (int j = 0; j < MLP_H; ++j) {
          sH2[t][j] = fmaxf(z2[j], 0.f);
          d2[j] = z2[j] > 0.f ? dout * w[MLP_W3 + j] : 0.f;
        }
        for (int i = 0; i < MLP_H; ++i) {
          float a = 0.f;
#pragma unroll 8
          for (int j = 0; j < MLP_H; ++j) a = fmaf(w[MLP_W2 + i * MLP_H + j], d2[j], a);
          d1[i] = h1[i] > 0.f ? a : 0.f;
        }
      } else {
        for (int i = 0; i < MLP_IN; ++i) sX[t][i] = 0.f;
        for (int j = 0; j < MLP_H; ++j) {
          h1[j] = 0.f;
          sH2[t][j] = 0.f;
          d2[j] = 0.f;
          d1[j] = 0.f;
        }
        sDo[t] = 0.f;
        sL[t] = 0.f;
      }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < MLP_PARAMS; p += blockDim.x) {
      float g = 0.f;
      if (p < MLP_B1) {  // W1[i][j]
        const int i = p / MLP_H, j = p % MLP_H;
        for (int r = 0; r < MLP_R; ++r) g = fmaf(sX[r][i], sD1[r][j], g);
      } else if (p < MLP_W2) {  // b1[j]
        const int j = p - MLP_B1;
        for (int r = 0; r < MLP_R; ++r) g += sD1[r][j];
      } else if (p < MLP_B2) {  // W2[i][j]
        const int q = p - MLP_W2, i = q / MLP_H, j = q % MLP_H;
        for (int r = 0; r < MLP_R; ++r) g = fmaf(sH1[r][i], sD2[r][j], g);
      } else if (p < MLP_W3) {  // b2[j]
        const int j = p - MLP_B2;
        for (int r = 0; r < MLP_R; ++r) g += sD2[r][j];
      } else if (p < MLP_B3) {  // W3[j]
        const int j = p - MLP_W3;
        for (int r = 0; r < MLP_R; ++r) g = fmaf(sDo[r], sH2[r][j], g);
      } else {  // b3
        for (int r = 0; r < MLP_R; ++r) g += sDo[r];
      }
      if (g != 0.f) atomicAdd(&grad[p], g);
    }
    if (threadIdx.x == 0) {
      float l = 0.f;
      for (int r = 0; r < MLP_R; ++r) l += sL[r];
      atomicAdd(loss, l);
    }
    __syncthreads();
  }
}

__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

// Adam on the FP32 master copy, then the BF16 weights are rounded from it.
__global__ void k_mlp_adam(float* __restrict__ master, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ grad, uint16_t* __restrict__ wbf, float lr,
                           float b1, float b2, float eps, float c1, float c2) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < MLP_PARAMS; p += gridDim.x * blockDim.x) {
    const float g = grad[p];
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float w = master[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    master[p] = w;
    wbf[p] = f32_to_bf16_rne(w);
  }
}

__global__ void k_mlp_round(const float* __restrict__ master, uint16_t* __restrict__ wbf) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < MLP_PARAMS; p += gridDim.x * blockDim.x)
    wbf[p] = f32_to_bf16_rne(master[p]);
}

}  // namespace

void launch_mlp_forward(const float* X, uint64_t rows, const uint16_t* wbf, const float* norm,
                        float* out, hipStream_t s) {
  if (rows == 0) return;
  k_mlp_forward<<<grid_for(rows, kThreads, 4096), kThreads, 0, s>>>(X, rows, wbf, norm, out);
  BM_LAUNCH_CHECK();
}

void launch_mlp_grad(const float* X, const float* Y, uint64_t r0, uint64_t r1, float scale,
                     const uint16_t* wbf, const float* norm, float* grad, float* loss, hipStream_t s) {
  if (r1 <= r0) return;
  k_mlp_grad<<<grid_for(r1 - r0, MLP_R, 1024), kThreads, 0, s>>>(X, Y, r0, r1, scale, wbf, norm,
                                                                  grad, loss);
  BM_LAUNCH_CHECK();
}

void launch_mlp_adam(float* master, float* m, float* v, const float* grad, uint16_t* wbf, float lr,
                     uint64_t step, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  k_mlp_adam<<<grid_for(MLP_PARAMS, kThreads), kThreads, 0, s>>>(master, m, v, grad, wbf, lr, b1, b2,
                                                                  eps, c1, c2);
  BM_LAUNCH_CHECK();
}

void launch_mlp_round(const float* master, uint16_t* wbf, hipStream_t s) {
  k_mlp_round<<<grid_for(MLP_PARAMS, kThreads), kThreads, 0, s>>>(master, wbf);
  BM_LAUNCH_CHECK();
}

}  // namespace bm
