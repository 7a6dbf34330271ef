// Pair supports of a prefix class as a masked Gram matrix on MFMA.
//
// For a class with prefix P (tidset t(P), the AND of P's columns) and children
// c_0..c_{q-1}, the support of P + {c_i, c_l} is
//     S = sum_rows t(P)[r] & M[r, c_i] & M[r, c_l]
// (Eq. 2, with the prefix's columns ANDed in first as the method prescribes
// for longer itemsets).  Over all pairs this is the Gram matrix
// X^T X of the 0/1 matrix X[r, i] = t(P)[r] & M[r, c_i]; for the root class
// (P empty) it is the pair-support matrix A^T A itself.  With 0/1 entries the
// products are exact, in FP4 x FP4 -> FP32 (the default form, below) or in
// int8 x int8 -> int32.
//
// Kernel shape (gfx950, wave64):
//   * one workgroup = 4 waves computes a 128 x 128 output tile of the class's
//     triangle over a range of words; waves own 64 x 64 sub-tiles, each a 2 x 2
//     grid of 32 x 32 MFMA accumulators;
//   * the bit panels of both tile sides are staged through LDS 16 words
//     (1024 transactions) at a time, with the prefix mask ANDed into the A
//     side on the way (t & a_i & b_l needs it once; a diagonal tile reads its
//     masked A panel for both sides),
//     and the next stage's global loads are issued before the current stage's
//     MFMAs (software pipelining);
//   * bits become MFMA operands in registers right before each MFMA (FP4
//     bit planes, or for int8 the lane's 32-bit half-word v yields four dwords
//     (v >> d) & 0x01010101, one transaction bit per byte).  A and B fragments
//     use the identical bit -> (lane, element) map, so every transaction meets
//     itself in the K sum;
//   * the accumulated tile is added atomically into the class's triangle
//     (integer adds: exact and independent of the order of word splits).
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

// One LDS stage of the FP4 form for one wave (NB = 2: 2 x 2 accumulators of
// 32 x 32).  pa / pb point at the wave's first A row block and first B column
// block (lane's row, half-word).  MODE 0: an off-diagonal tile -- A blocks
// 0, 1 against B blocks 0, 1.  On a diagonal tile (A and B the same panel)
// the 10 useful blocks of the 4 x 4 are shared out so that no wave does more
// than three products or builds more than three operand rows:
//   MODE 1 (waves on the diagonal): its two blocks against themselves,
//     (0,0), (0,1), (1,1), with B taken from A's operands;
//   MODE 2 (the two off-diagonal waves): one A block against B blocks 0, 1.
template <int MODE, int KW, int LDW>
__device__ __forceinline__ void fp4_stage(const uint32_t* pa, const uint32_t* pb,
                                          v16f (&acc)[2][2]) {
  constexpr int NA = MODE == 2 ? 1 : 2;  // A row blocks this wave builds
  constexpr bool BSAME = MODE == 1;      // B operands are A's
  // fully unrolled, so the next group's plane masks overlap this group's MFMAs
#pragma unroll
  for (int w4 = 0; w4 < KW; w4 += 4) {
    uint32_t va[2][4], vb[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        va[i][j] = i < NA ? pa[i * 32 * LDW + 2 * (w4 + j)] : 0u;
        vb[i][j] = BSAME ? 0u : pb[i * 32 * LDW + 2 * (w4 + j)];
      }
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) {
      v8i A[2], B[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          A[i][j] = i < NA ? (int)fp4_plane(va[i][j], pl) : 0;
          B[i][j] = BSAME ? 0 : (int)fp4_plane(vb[i][j], pl);
        }
        A[i][4] = A[i][5] = A[i][6] = A[i][7] = 0;
        B[i][4] = B[i][5] = B[i][6] = B[i][7] = 0;
      }
      const int sc = fp4_plane_scale(pl);  // format 4 = e2m1 for both operands
      if constexpr (MODE == 0) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[i], B[j], acc[i][j], 4,
                                                                        4, 0, sc, 0, sc);
      } else if constexpr (MODE == 1) {
        acc[0][0] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[0], A[0], acc[0][0], 4, 4, 0,
                                                                    sc, 0, sc);
        acc[0][1] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[0], A[1], acc[0][1], 4, 4, 0,
                                                                    sc, 0, sc);
        acc[1][1] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[1], A[1], acc[1][1], 4, 4, 0,
                                                                    sc, 0, sc);
      } else {
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[0][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A[0], B[j], acc[0][j], 4, 4,
                                                                      0, sc, 0, sc);
      }
    }
  }
}

// NB = 32x32 accumulator blocks per wave side: NB = 2 gives 64x64 per wave and
// a 128x128 workgroup tile of 4 waves.
// KW = words per LDS stage (a divisor of GRAM_KW, so stages tile every task).
template <int NB, int KW, bool F4>
__device__ __forceinline__ void gram_tiles(const ClassArgs& a, uint32_t* sA, uint32_t* sB) {
  static_assert(GRAM_KW % KW == 0, "stages must tile the task word ranges");
  constexpr int T = 64 * NB;         // workgroup tile (children per side)
  constexpr int LDW = 2 * KW + 1;    // dwords per column row in LDS (odd stride: conflict-free reads)
  constexpr int SUBS = KW / 2;       // 16-byte slots per column per stage
  constexpr int CSL = 256 / SUBS;    // columns staged per pass of the workgroup
  constexpr int NS = T / CSL;        // column slots per side staged by each thread
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int sub = tid % SUBS;   // 16-byte slot of a column's stage slice
  const int cslot = tid / SUBS; // column slot 0..CSL-1
  const uint64_t ntasks = *a.ntasks;

  for (uint64_t t = blockIdx.x; t < ntasks; t += gridDim.x) {
    const Task task = a.tasks[t];
    const ClassDesc cd = a.cls[task.cls];
    const DbInfo db = class_view(cd, a.dbs, a.views);
    const uint64_t Wp = db.Wp;
    const uint32_t q = cd.q;
    const uint32_t I0 = (uint32_t)task.bi * T, L0 = (uint32_t)task.bl * T;
    const bool diag = task.bi == task.bl;
    // the wave's first A row block and first B column block (32-wide blocks
    // of the tile): FP4 diagonal tiles share their useful blocks out by mode
    const int mode = (F4 && diag) ? (wr == wc ? 1 : 2) : 0;
    const int rb0 = mode == 2 ? wr : NB * wr;
    const int cb0 = mode == 2 ? NB : NB * wc;
    const int nload = diag ? NS : 2 * NS;

    // base pointers of the columns this thread stages (nullptr = zero column)
    const uint64_t* colp[2 * NS];
#pragma unroll
    for (int p = 0; p < 2 * NS; ++p) {
      const uint32_t idx = ((p >= NS) ? L0 : I0) + cslot + CSL * (p % NS);
      colp[p] = nullptr;
      if (p < nload && idx < q) {
        const uint32_t item = a.child_item[cd.child0 + idx];
        const uint32_t col = class_col(cd, db, idx, item);
        colp[p] = db.B + (uint64_t)col * Wp + 2 * sub;
      }
    }
    const uint32_t* pre = a.pre_cols + cd.pre_off;
    const uint32_t pre_len = cd.proj ? 0u : cd.pre_len;  // a view has the prefix applied

    uint4 reg[2 * NS];
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
      for (int p = 0; p < 2 * NS; ++p) {
        if (colp[p]) reg[p] = *reinterpret_cast<const uint4*>(colp[p] + w);
        else reg[p] = make_uint4(0, 0, 0, 0);
      }
    };

    using Acc = typename std::conditional<F4, v16f, v16i>::type;
    Acc acc[NB][NB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

    const uint32_t nst = (task.w1 - task.w0) / KW;
    if (nst) load_stage(task.w0);
    for (uint32_t s = 0; s < nst; ++s) {
      __syncthreads();  // previous stage (or task) finished reading LDS
#pragma unroll
      for (int p = 0; p < 2 * NS; ++p) {
        if (p < nload) {
          uint32_t* dst = ((p >= NS) ? sB : sA) + (cslot + CSL * (p % NS)) * LDW + 4 * sub;
          uint4 v = reg[p];
          if (pre_len && p < NS) {  // the prefix mask on the A side only: t & a_i & b_l
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
      if (s + 1 < nst) load_stage(task.w0 + (s + 1) * KW);

      const uint32_t* pa = sA + (rb0 * 32 + (lane & 31)) * LDW + (lane >> 5);
      const uint32_t* pb = (diag ? sA : sB) + (cb0 * 32 + (lane & 31)) * LDW + (lane >> 5);
      if constexpr (F4) {
        static_assert(NB == 2, "the FP4 stage is written for 2 x 2 accumulators per wave");
        // a wave in its MFMA section outranks the other workgroup's staging
        // waves for issue slots (measured 3% faster on the dense root class)
        __builtin_amdgcn_s_setprio(3);
        if (mode == 0) fp4_stage<0, KW, LDW>(pa, pb, acc);
        else if (mode == 1) fp4_stage<1, KW, LDW>(pa, pb, acc);
        else fp4_stage<2, KW, LDW>(pa, pb, acc);
        __builtin_amdgcn_s_setprio(0);
      } else {
#pragma unroll(NB == 2 ? KW : 1)
        for (int w = 0; w < KW; ++w) {
          uint32_t va[NB], vb[NB];
#pragma unroll
          for (int i = 0; i < NB; ++i) {
            va[i] = pa[i * 32 * LDW + 2 * w];
            vb[i] = pb[i * 32 * LDW + 2 * w];
          }
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            v4i A[NB], B[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
              A[i] = expand4(va[i], 4 * e);
              B[i] = expand4(vb[i], 4 * e);
            }
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
              for (int j = 0; j < NB; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[i], B[j], acc[i][j], 0, 0, 0);
          }
        }
      }
    }

    // 32x32 accumulator layout: lane holds column (lane & 31); register r holds
    // row 8*(r/4) + 4*(lane/32) + (r%4).
    uint32_t* tri = a.tri + cd.tri_off;
#pragma unroll
    for (int rb = 0; rb < NB; ++rb)
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const uint32_t gi = I0 + (rb0 + rb) * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const uint32_t gl = L0 + (cb0 + cb) * 32 + (lane & 31);
          uint32_t v;
          if constexpr (F4) v = __float2uint_rn(acc[rb][cb][r]);  // exact integer counts
          else v = (uint32_t)acc[rb][cb][r];
          if (gi < gl && gl < q && v) atomicAdd(tri + tri_index(gi, gl, q), v);
        }
  }
}

template <bool F4>
// Two workgroups per CU (two waves per SIMD): the register budget is capped
// at 256 so the three stage variants do not push the kernel to one wave.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_gram_mfma(ClassArgs a) {
  constexpr int KW = 16;
  __shared__ uint32_t sA[GRAM_TILE * (2 * KW + 1)];
  __shared__ uint32_t sB[GRAM_TILE * (2 * KW + 1)];
  gram_tiles<2, KW, F4>(a, sA, sB);
}

}  // namespace

void launch_gram_mfma(const ClassArgs& a, uint32_t grid, bool fp4, hipStream_t s) {
  if (grid == 0) return;
  if (fp4) k_gram_mfma<true><<<grid, 256, 0, s>>>(a);
  else k_gram_mfma<false><<<grid, 256, 0, s>>>(a);
  BM_LAUNCH_CHECK();
}


}  // namespace bm
