// Pair supports of big prefix classes (at least mfma_big_children children)
// as masked Gram tiles on MFMA, 256 x 256 block pairs split into 128-row
// halves.  The contraction, the operand forms (FP4 bit planes or int8 bytes)
// and the staging follow the 128-tile kernel in k_gram_mfma.hip; this kernel
// only changes the tile shape per wave.
#include <type_traits>

#include "internal.hpp"

namespace bm {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));


__device__ __forceinline__ v4i expand4(uint32_t v, int d0) {
  v4i r;
  r[0] = (int)((v >> (d0 + 0)) & 0x01010101u);
  r[1] = (int)((v >> (d0 + 1)) & 0x01010101u);
  r[2] = (int)((v >> (d0 + 2)) & 0x01010101u);
  r[3] = (int)((v >> (d0 + 3)) & 0x01010101u);
  return r;
}

// FP4 (e2m1) form.  The e2m1 codes 0001, 0010 and 0100 are the values 0.5, 1
// and 2, so one AND turns a 32-bit half-word v into eight FP4 elements that
// each hold one transaction bit: plane 0 = v & 0x11111111 (bits 0, 4, .., 28
// as 0.5), plane 1 = v & 0x22222222 (bits 1, 5, .. as 1), plane 2 =
// v & 0x44444444 (as 2); plane 3 (bits 3, 7, ..) would land on the sign bit,
// so it is shifted first: (v >> 2) & 0x22222222 (as 1).  One
// v_mfma_scale_f32_32x32x64_f8f6f4 takes one plane of four consecutive words
// (a lane's four operand dwords), and its E8M0 block scales (2, 1, 1/2, 1 on
// both operands) make every product of two set bits exactly 1.0; four MFMAs,
// one per plane, cover the four words.  A and B use the identical bit ->
// (lane, element) map, so every transaction meets itself in the K sum.  FP32
// holds every integer up to 2^24 exactly, so a task's sums are exact while its
// counts stay at most 2^24 -- the task word split is capped at
// GRAM_FP4_MAX_WORDS for that.
__device__ __forceinline__ uint32_t fp4_plane(uint32_t v, int pl) {
  return pl == 0 ? (v & 0x11111111u)
       : pl == 1 ? (v & 0x22222222u)
       : pl == 2 ? (v & 0x44444444u)
                 : ((v >> 2) & 0x22222222u);
}
__device__ __forceinline__ int fp4_plane_scale(int pl) {  // E8M0: 2^(e - 127)
  return pl == 0 ? 128 : pl == 2 ? 126 : 127;
}

// Big classes: 256 x 256 block pairs, each as two tasks of 128 rows x 256
// columns, one workgroup of 4 waves per task.  A wave owns 64 x 128 (2 x 4
// accumulators of 32 x 32, 128 registers), so per word it builds 6 operand
// rows for 8 MFMAs (the 128-tile kernel: 4 rows for 4), and two workgroups
// share a CU as in the 128-tile kernel.  On a diagonal block pair the 128 rows
// are a slice of the 256 staged columns, so only the column side is staged,
// and a wave whose block lies wholly below the diagonal skips its MFMAs.
constexpr int BR = GRAM_TILE_BIG / 2;  // 128 rows per task
constexpr int BC = GRAM_TILE_BIG;      // 256 columns
constexpr int BKW = 8;                 // words per stage
constexpr int BLDW = 2 * BKW + 1;      // dwords per staged column row (odd: conflict-free reads)
constexpr int BSUBS = BKW / 2;         // 16-byte slots per column per stage
constexpr int BCSL = 256 / BSUBS;      // columns staged per pass (64)
constexpr int BNSC = BC / BCSL;        // passes for the columns (4)
constexpr int BNSR = BR / BCSL;        // passes for the rows (2)

template <bool F4>
__device__ __forceinline__ void gram_tiles_big(const ClassArgs& a, uint32_t* sR, uint32_t* sC) {
  static_assert(GRAM_KW % BKW == 0, "stages must tile the task word ranges");
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;  // rows wr*64 .. +63, columns wc*128 .. +127
  const int sub = tid % BSUBS;
  const int cslot = tid / BSUBS;
  const uint64_t ntasks = *a.ntasks;
  constexpr int NP = BNSC + BNSR;

  for (uint64_t t = blockIdx.x; t < ntasks; t += gridDim.x) {
    const Task task = a.tasks[t];
    const ClassDesc cd = a.cls[task.cls];
    const DbInfo db = class_view(cd, a.dbs, a.views);
    const uint64_t Wp = db.Wp;
    const uint32_t q = cd.q;
    const uint32_t half = task.bi & 1u;
    const uint32_t I0 = (uint32_t)task.bi * BR, L0 = (uint32_t)task.bl * BC;
    const bool diag = (uint32_t)(task.bi >> 1) == (uint32_t)task.bl;
    // no pair to count: every row of the wave's block exceeds every column
    // (below the diagonal), or its rows or columns lie past the last child
    const bool skip = I0 + wr * 64 >= L0 + wc * 128 + 128 || I0 + wr * 64 >= q || L0 + wc * 128 >= q;

    // passes 0..3 stage the 256 columns, passes 4..5 the 128 rows (not on a
    // diagonal block pair); nullptr = zero column
    const uint64_t* colp[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const uint32_t idx = (p < BNSC ? L0 + BCSL * p : I0 + BCSL * (p - BNSC)) + cslot;
      colp[p] = nullptr;
      if ((p < BNSC || !diag) && idx < q) {
        const uint32_t item = a.child_item[cd.child0 + idx];
        const uint32_t col = class_col(cd, db, idx, item);
        colp[p] = db.B + (uint64_t)col * Wp + 2 * sub;
      }
    }
    const uint32_t* pre = a.pre_cols + cd.pre_off;
    const uint32_t pre_len = cd.proj ? 0u : cd.pre_len;  // a view has the prefix applied

    uint4 reg[NP];
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
      for (int p = 0; p < NP; ++p) {
        if (colp[p]) reg[p] = *reinterpret_cast<const uint4*>(colp[p] + w);
        else reg[p] = make_uint4(0, 0, 0, 0);
      }
    };

    using Acc = typename std::conditional<F4, v16f, v16i>::type;
    Acc acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

    const uint32_t nst = (task.w1 - task.w0) / BKW;
    if (nst) load_stage(task.w0);
    for (uint32_t s = 0; s < nst; ++s) {
      __syncthreads();  // previous stage (or task) finished reading LDS
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        if (p < BNSC || !diag) {
          uint32_t* dst = (p < BNSC ? sC + (cslot + BCSL * p) * BLDW
                                    : sR + (cslot + BCSL * (p - BNSC)) * BLDW) + 4 * sub;
          uint4 v = reg[p];
          // the prefix mask once per pair: on the rows, or on the columns of a
          // diagonal block pair (whose rows are read from them)
          if (pre_len && (diag ? p < BNSC : p >= BNSC)) {
            v.x &= (uint32_t)m0;
            v.y &= (uint32_t)(m0 >> 32);
            v.z &= (uint32_t)m1;
            v.w &= (uint32_t)(m1 >> 32);
          }
          dst[0] = v.x;
          dst[1] = v.y;
          dst[2] = v.z;
          dst[3] = v.w;
        }
      }
      __syncthreads();
      if (s + 1 < nst) load_stage(task.w0 + (s + 1) * BKW);
      if (skip) continue;

      const uint32_t* pa = (diag ? sC + half * BR * BLDW : sR) + (wr * 64 + (lane & 31)) * BLDW +
                           (lane >> 5);
      const uint32_t* pb = sC + (wc * 128 + (lane & 31)) * BLDW + (lane >> 5);
      if constexpr (F4) {
#pragma unroll
        for (int w4 = 0; w4 < BKW; w4 += 4) {
          uint32_t va[2][4], vb[4][4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
#pragma unroll
            for (int i = 0; i < 2; ++i) va[i][j] = pa[i * 32 * BLDW + 2 * (w4 + j)];
#pragma unroll
            for (int i = 0; i < 4; ++i) vb[i][j] = pb[i * 32 * BLDW + 2 * (w4 + j)];
          }
#pragma unroll
          for (int pl = 0; pl < 4; ++pl) {
            v8i A[2], B[4];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
#pragma unroll
              for (int j = 0; j < 4; ++j) A[i][j] = (int)fp4_plane(va[i][j], pl);
              A[i][4] = A[i][5] = A[i][6] = A[i][7] = 0;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
#pragma unroll
              for (int j = 0; j < 4; ++j) B[i][j] = (int)fp4_plane(vb[i][j], pl);
              B[i][4] = B[i][5] = B[i][6] = B[i][7] = 0;
            }
            const int sc = fp4_plane_scale(pl);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                    A[i], B[j], acc[i][j], 4, 4, 0, sc, 0, sc);
          }
        }
      } else {
#pragma unroll
        for (int w = 0; w < BKW; ++w) {
          uint32_t va[2], vb[4];
#pragma unroll
          for (int i = 0; i < 2; ++i) va[i] = pa[i * 32 * BLDW + 2 * w];
#pragma unroll
          for (int i = 0; i < 4; ++i) vb[i] = pb[i * 32 * BLDW + 2 * w];
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            v4i A[2], B[4];
#pragma unroll
            for (int i = 0; i < 2; ++i) A[i] = expand4(va[i], 4 * e);
#pragma unroll
            for (int i = 0; i < 4; ++i) B[i] = expand4(vb[i], 4 * e);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[i], B[j], acc[i][j], 0, 0, 0);
          }
        }
      }
    }
    if (skip) continue;

    uint32_t* tri = a.tri + cd.tri_off;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const uint32_t gi = I0 + wr * 64 + rb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const uint32_t gl = L0 + wc * 128 + cb * 32 + (lane & 31);
          uint32_t v;
          if constexpr (F4) v = __float2uint_rn(acc[rb][cb][r]);
          else v = (uint32_t)acc[rb][cb][r];
          if (gi < gl && gl < q && v) atomicAdd(tri + tri_index(gi, gl, q), v);
        }
  }
}

// two workgroups per CU: at most 256 registers per lane
template <bool F4>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_gram_mfma_big(ClassArgs a) {
  __shared__ uint32_t sR[BR * BLDW];
  __shared__ uint32_t sC[BC * BLDW];
  gram_tiles_big<F4>(a, sR, sC);
}

}  // namespace

void launch_gram_mfma_big(const ClassArgs& a, uint32_t grid, bool fp4, hipStream_t s) {
  if (grid == 0) return;
  if (fp4) k_gram_mfma_big<true><<<grid, 256, 0, s>>>(a);
  else k_gram_mfma_big<false><<<grid, 256, 0, s>>>(a);
  BM_LAUNCH_CHECK();
}

}  // namespace bm
