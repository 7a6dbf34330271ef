// Pair supports of a prefix class as a masked Gram matrix on int8 MFMA.
//
// For a class with prefix P (tidset t(P), the AND of P's columns) and children
// c_0..c_{q-1}, the support of P + {c_i, c_l} is
//     S = sum_rows t(P)[r] & M[r, c_i] & M[r, c_l]
// (Eq. 2, with the prefix's columns ANDed in first as the method prescribes
// for longer itemsets).  Over all pairs this is the Gram matrix
// X^T X of the 0/1 matrix X[r, i] = t(P)[r] & M[r, c_i]; for the root class
// (P empty) it is the pair-support matrix A^T A itself.  With 0/1 entries the
// products are exact in int8 x int8 -> int32 (supports < 2^31).
//
// Kernel shape (gfx950, wave64):
//   * one workgroup = 4 waves computes a 128 x 128 output tile of the class's
//     triangle over a range of words; waves own 64 x 64 sub-tiles, each a 2 x 2
//     grid of v_mfma_i32_32x32x32_i8 accumulators;
//   * the bit panels of both tile sides are staged through LDS 16 words
//     (1024 transactions) at a time, with the prefix mask ANDed in on the way,
//     and the next stage's global loads are issued before the current stage's
//     MFMAs (software pipelining);
//   * bits are expanded to int8 in registers right before each MFMA: the lane's
//     32-bit half-word v yields four dwords (v >> d) & 0x01010101, so each
//     byte holds one transaction bit.  A and B fragments use the identical
//     bit -> (lane, byte) map, so every transaction meets itself in the K sum;
//   * the accumulated tile is added atomically into the class's triangle
//     (integer adds: exact and independent of the order of word splits).
#include "internal.hpp"

namespace bm {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int T = GRAM_TILE;     // 128
constexpr int KW = GRAM_KW;      // 16 words per stage
constexpr int LDW = 2 * KW + 1;  // dwords per column row in LDS (odd stride: conflict-free reads)

__device__ __forceinline__ v4i expand4(uint32_t v, int d0) {
  v4i r;
  r[0] = (int)((v >> (d0 + 0)) & 0x01010101u);
  r[1] = (int)((v >> (d0 + 1)) & 0x01010101u);
  r[2] = (int)((v >> (d0 + 2)) & 0x01010101u);
  r[3] = (int)((v >> (d0 + 3)) & 0x01010101u);
  return r;
}

__global__ __launch_bounds__(256) void k_gram_mfma(ClassArgs a) {
  __shared__ uint32_t sA[T * LDW];
  __shared__ uint32_t sB[T * LDW];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int sub = tid & 7;     // 16-byte slot of a column's 128-byte stage slice
  const int cslot = tid >> 3;  // column slot 0..31
  const uint64_t ntasks = *a.ntasks;

  for (uint64_t t = blockIdx.x; t < ntasks; t += gridDim.x) {
    const Task task = a.tasks[t];
    const ClassDesc cd = a.cls[task.cls];
    const DbInfo db = a.dbs[cd.db];
    const uint64_t Wp = db.Wp;
    const uint32_t q = cd.q;
    const uint32_t I0 = (uint32_t)task.bi * T, L0 = (uint32_t)task.bl * T;
    const bool diag = task.bi == task.bl;
    const int nload = diag ? 4 : 8;

    // base pointers of the columns this thread stages (nullptr = zero column)
    const uint64_t* colp[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const uint32_t idx = ((p >> 2) ? L0 : I0) + cslot + 32 * (p & 3);
      colp[p] = nullptr;
      if (p < nload && idx < q) {
        const uint32_t item = a.child_item[cd.child0 + idx];
        const uint32_t col = db.f1 ? db.f1[item] : item;
        colp[p] = db.B + (uint64_t)col * Wp + 2 * sub;
      }
    }
    const uint32_t* pre = a.pre_cols + cd.pre_off;
    const uint32_t pre_len = cd.pre_len;

    uint4 reg[8];
    uint64_t m0 = ~0ull, m1 = ~0ull;
    auto load_stage = [&](uint32_t w) {
      m0 = ~0ull;
      m1 = ~0ull;
      for (uint32_t j = 0; j < pre_len; ++j) {
        const uint4 x = *reinterpret_cast<const uint4*>(db.B + (uint64_t)pre[j] * Wp + w + 2 * sub);
        m0 &= (uint64_t)x.x | ((uint64_t)x.y << 32);
        m1 &= (uint64_t)x.z | ((uint64_t)x.w << 32);
      }
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        if (colp[p]) reg[p] = *reinterpret_cast<const uint4*>(colp[p] + w);
        else reg[p] = make_uint4(0, 0, 0, 0);
      }
    };

    v16i acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

    const uint32_t nst = (task.w1 - task.w0) / KW;
    if (nst) load_stage(task.w0);
    for (uint32_t s = 0; s < nst; ++s) {
      __syncthreads();  // previous stage (or task) finished reading LDS
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        if (p < nload) {
          uint32_t* dst = ((p >> 2) ? sB : sA) + (cslot + 32 * (p & 3)) * LDW + 4 * sub;
          const uint64_t x0 = ((uint64_t)reg[p].x | ((uint64_t)reg[p].y << 32)) & m0;
          const uint64_t x1 = ((uint64_t)reg[p].z | ((uint64_t)reg[p].w << 32)) & m1;
          dst[0] = (uint32_t)x0;
          dst[1] = (uint32_t)(x0 >> 32);
          dst[2] = (uint32_t)x1;
          dst[3] = (uint32_t)(x1 >> 32);
        }
      }
      __syncthreads();
      if (s + 1 < nst) load_stage(task.w0 + (s + 1) * KW);

      const uint32_t* pa = sA + (wr * 64 + (lane & 31)) * LDW + (lane >> 5);
      const uint32_t* pb = (diag ? sA : sB) + (wc * 64 + (lane & 31)) * LDW + (lane >> 5);
#pragma unroll 4
      for (int w = 0; w < KW; ++w) {
        const uint32_t va0 = pa[2 * w], va1 = pa[32 * LDW + 2 * w];
        const uint32_t vb0 = pb[2 * w], vb1 = pb[32 * LDW + 2 * w];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const v4i A0 = expand4(va0, 4 * e), A1 = expand4(va1, 4 * e);
          const v4i B0 = expand4(vb0, 4 * e), B1 = expand4(vb1, 4 * e);
          acc[0][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A0, B0, acc[0][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A0, B1, acc[0][1], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A1, B0, acc[1][0], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A1, B1, acc[1][1], 0, 0, 0);
        }
      }
    }

    // 32x32 accumulator layout: lane holds column (lane & 31); register r holds
    // row 8*(r/4) + 4*(lane/32) + (r%4).
    uint32_t* tri = a.tri + cd.tri_off;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const uint32_t gi = I0 + wr * 64 + rb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const uint32_t gl = L0 + wc * 64 + cb * 32 + (lane & 31);
          const int v = acc[rb][cb][r];
          if (gi < gl && gl < q && v) atomicAdd(tri + tri_index(gi, gl, q), (uint32_t)v);
        }
  }
}

}  // namespace

void launch_gram_mfma(const ClassArgs& a, uint32_t grid, hipStream_t s) {
  if (grid == 0) return;
  k_gram_mfma<<<grid, 256, 0, s>>>(a);
  BM_LAUNCH_CHECK();
}

}  // namespace bm
