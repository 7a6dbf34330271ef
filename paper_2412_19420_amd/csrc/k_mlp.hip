// Cost model of the scheduler: an 8 -> 64 -> 64 -> 1 perceptron with ReLU,
// BF16 weights and FP32 accumulation, trained with Adam on an FP32 master copy.
// It predicts log2(1 + column words streamed for a subtree) from 8 features of
// a prefix class and is used only to order subtree tasks; it never changes a
// result.
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

// Inference on blocks of MLP_R rows: four threads per row, each computing 16
// hidden units of both layers from activations staged in LDS (no per-thread
// arrays, so nothing spills), then a 4-lane sum of the output layer.
__global__ __launch_bounds__(kThreads) void k_mlp_forward(const float* __restrict__ X, uint64_t rows,
                                                          const uint16_t* __restrict__ wbf,
                                                          const float* __restrict__ norm,
                                                          float* __restrict__ out) {
  static_assert(kThreads == 4 * MLP_R, "four threads per row");
  __shared__ float w[MLP_PARAMS];
  __shared__ float nm[2 * MLP_IN];
  __shared__ float sX[MLP_R][MLP_IN + 1];
  __shared__ float sH1[MLP_R][MLP_H + 1];
  load_weights(wbf, w);
  if (threadIdx.x < 2 * MLP_IN) nm[threadIdx.x] = norm[threadIdx.x];
  const int r = threadIdx.x >> 2, part = threadIdx.x & 3, c0 = part * 16;
  for (uint64_t b0 = (uint64_t)blockIdx.x * MLP_R; b0 < rows; b0 += (uint64_t)gridDim.x * MLP_R) {
    __syncthreads();
    for (int e = threadIdx.x; e < MLP_R * MLP_IN; e += kThreads) {
      const int rr = e / MLP_IN, i = e % MLP_IN;
      const uint64_t g = b0 + rr;
      sX[rr][i] = g < rows ? (X[g * MLP_IN + i] - nm[i]) * nm[MLP_IN + i] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      float a = w[MLP_B1 + c0 + j];
#pragma unroll
      for (int i = 0; i < MLP_IN; ++i) a = fmaf(sX[r][i], w[MLP_W1 + i * MLP_H + c0 + j], a);
      sH1[r][c0 + j] = fmaxf(a, 0.f);
    }
    __syncthreads();
    float acc[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = w[MLP_B2 + c0 + j];
    for (int i = 0; i < MLP_H; ++i) {
      const float h = sH1[r][i];
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] = fmaf(h, w[MLP_W2 + i * MLP_H + c0 + j], acc[j]);
    }
    float o = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) o = fmaf(fmaxf(acc[j], 0.f), w[MLP_W3 + c0 + j], o);
    o += __shfl_xor(o, 1);
    o += __shfl_xor(o, 2);
    const uint64_t g = b0 + r;
    if (part == 0 && g < rows) out[g] = o + w[MLP_B3];
  }
}

// Gradient of scale * sum_r (out_r - y_r)^2 over rows [r0, r1): each workgroup
// takes chunks of MLP_R rows (per-row backpropagation by one wavefront, then
// the parameter sums over the chunk by all threads) and accumulates into its
// own slot partial[blockIdx.x][0..MLP_PARAMS] (the last entry is the loss);
// every slot entry has one owning thread, so there are no atomics and the
// result does not depend on scheduling.
__global__ __launch_bounds__(kThreads) void k_mlp_grad(const float* __restrict__ X,
                                                       const float* __restrict__ Y, uint64_t r0,
                                                       uint64_t r1, float scale,
                                                       const uint16_t* __restrict__ wbf,
                                                       const float* __restrict__ norm,
                                                       float* __restrict__ partial) {
  __shared__ float w[MLP_PARAMS];
  __shared__ float nm[2 * MLP_IN];
  __shared__ float sX[MLP_R][MLP_IN];
  __shared__ float sH1[MLP_R][MLP_H + 1];  // padded: conflict-free per-row access
  __shared__ float sH2[MLP_R][MLP_H + 1];  // padded: conflict-free per-row access
  __shared__ float sD2[MLP_R][MLP_H + 1];  // padded: conflict-free per-row access
  __shared__ float sD1[MLP_R][MLP_H + 1];  // padded: conflict-free per-row access
  __shared__ float sDo[MLP_R];
  __shared__ float sL[MLP_R];
  float* slot = partial + (uint64_t)blockIdx.x * (MLP_PARAMS + 1);
  load_weights(wbf, w);
  if (threadIdx.x < 2 * MLP_IN) nm[threadIdx.x] = norm[threadIdx.x];
  for (int p = threadIdx.x; p <= MLP_PARAMS; p += blockDim.x) slot[p] = 0.f;
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
      slot[p] += g;
    }
    if (threadIdx.x == (MLP_PARAMS % kThreads)) {  // the owner of slot[MLP_PARAMS]
      float l = 0.f;
      for (int r = 0; r < MLP_R; ++r) l += sL[r];
      slot[MLP_PARAMS] += l;
    }
    __syncthreads();
  }
}

// grad[p] = sum over workgroup slots in slot order; *loss += the summed loss.
__global__ void k_mlp_reduce(const float* __restrict__ partial, uint32_t nslots,
                             float* __restrict__ grad, float* __restrict__ loss) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p <= MLP_PARAMS; p += gridDim.x * blockDim.x) {
    float g = 0.f;
    for (uint32_t b = 0; b < nslots; ++b) g += partial[(uint64_t)b * (MLP_PARAMS + 1) + p];
    if (p < MLP_PARAMS) grad[p] = g;
    else *loss += g;
  }
}

// Per-epoch bookkeeping on the device (so an epoch can be replayed as a graph):
// losses[*epoch] = *acc / batches, then the epoch and Adam step counters advance.
__global__ void k_mlp_epoch_end(float* __restrict__ acc, float* __restrict__ losses,
                                uint32_t* __restrict__ ctr, uint32_t batches) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    losses[ctr[0]] = *acc / (float)batches;
    ctr[0] += 1;
    ctr[1] += batches;
    *acc = 0.f;
  }
}

__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

// Adam on the FP32 master copy, then the BF16 weights are rounded from it.
// The step number is *step_base + step_add (a device counter, so replays of a
// captured epoch use the right bias corrections).
__global__ void k_mlp_adam(float* __restrict__ master, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ grad, uint16_t* __restrict__ wbf, float lr,
                           float b1, float b2, float eps, const uint32_t* __restrict__ step_base,
                           uint32_t step_add) {
  const float t = (float)(*step_base + step_add);
  const float c1 = 1.f - powf(b1, t), c2 = 1.f - powf(b2, t);
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
  k_mlp_forward<<<grid_for(rows, MLP_R, 2048), kThreads, 0, s>>>(X, rows, wbf, norm, out);
  BM_LAUNCH_CHECK();
}

uint32_t mlp_grad_slots(uint64_t rows) { return grid_for(rows, MLP_R, 1024); }

void launch_mlp_grad(const float* X, const float* Y, uint64_t r0, uint64_t r1, float scale,
                     const uint16_t* wbf, const float* norm, float* partial, float* grad, float* loss,
                     hipStream_t s) {
  if (r1 <= r0) return;
  const uint32_t g = mlp_grad_slots(r1 - r0);
  k_mlp_grad<<<g, kThreads, 0, s>>>(X, Y, r0, r1, scale, wbf, norm, partial);
  BM_LAUNCH_CHECK();
  k_mlp_reduce<<<grid_for(MLP_PARAMS + 1, kThreads), kThreads, 0, s>>>(partial, g, grad, loss);
  BM_LAUNCH_CHECK();
}

void launch_mlp_adam(float* master, float* m, float* v, const float* grad, uint16_t* wbf, float lr,
                     const uint32_t* step_base, uint32_t step_add, hipStream_t s) {
  k_mlp_adam<<<grid_for(MLP_PARAMS, kThreads), kThreads, 0, s>>>(master, m, v, grad, wbf, lr, 0.9f,
                                                                  0.999f, 1e-8f, step_base, step_add);
  BM_LAUNCH_CHECK();
}

void launch_mlp_epoch_end(float* acc, float* losses, uint32_t* ctr, uint32_t batches, hipStream_t s) {
  k_mlp_epoch_end<<<1, 64, 0, s>>>(acc, losses, ctr, batches);
  BM_LAUNCH_CHECK();
}

void launch_mlp_round(const float* master, uint16_t* wbf, hipStream_t s) {
  k_mlp_round<<<grid_for(MLP_PARAMS, kThreads), kThreads, 0, s>>>(master, wbf);
  BM_LAUNCH_CHECK();
}

}  // namespace bm
