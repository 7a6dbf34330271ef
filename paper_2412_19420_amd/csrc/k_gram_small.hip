// Pair supports of mid-size prefix classes (more children than the small-class
// limit, fewer than mfma_min_children) as 32 x 32 masked Gram tiles on MFMA.
//
// A class's candidate supports are sum_rows t(P) & M[:, c_i] & M[:, c_l] (Eq. 2
// with the prefix columns ANDed in first), i.e. the Gram matrix of the 0/1
// matrix X[r, i] = t(P)[r] & M[r, c_i].  For a few dozen children one 32 x 32
// MFMA tile covers a whole block pair, and a single wave evaluates it:
//   * each wave owns one task (block pair of 32 children, word range) -- four
//     independent tasks per workgroup and no workgroup barriers;
//   * a wave stages 16 words of its (up to 64) columns at a time through its
//     own LDS slice: 8 lanes per column read its 128 contiguous bytes, the
//     prefix mask is ANDed into the A side only (t & a_i & b_l needs it once),
//     and the next stage's loads are issued before this stage's MFMAs.  A
//     diagonal block pair has only its 32 columns to stage, so it takes 32
//     words per stage in the same slice: a class of at most 32 children is
//     one diagonal task per word range, and its loads in flight double;
//   * lane (r, h) then reads half-word h of row r's words from LDS;
//   * FP4 form: the 32-bit half-word v becomes nibbles (v >> d) & 0x11111111
//     (e2m1 0.5), one v_mfma_f32_32x32x64_f8f6f4 per 64 transactions; the word
//     split of a task keeps its counts below 2^24, where FP32 sums of quarters
//     are exact.  int8 form: bytes (v >> d) & 0x01010101, two
//     v_mfma_i32_32x32x32_i8 per 64 transactions.
// Against the LDS-blocked AND+popcount kernel this trades ~31 VALU
// instructions per word of a 32-child block (496 AND+popcount pairs) for 7
// VALU instructions and one MFMA.
#include <type_traits>

#include "internal.hpp"

namespace bm {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int SB = GRAM_SMALL_TILE;  // 32 children per block

__device__ __forceinline__ v8i fp4_of(uint32_t v) {
  return v8i{(int)(v & 0x11111111u), (int)((v >> 1) & 0x11111111u), (int)((v >> 2) & 0x11111111u),
             (int)((v >> 3) & 0x11111111u), 0, 0, 0, 0};
}
__device__ __forceinline__ v4i i8_of(uint32_t v, int d0) {
  return v4i{(int)((v >> d0) & 0x01010101u), (int)((v >> (d0 + 1)) & 0x01010101u),
             (int)((v >> (d0 + 2)) & 0x01010101u), (int)((v >> (d0 + 3)) & 0x01010101u)};
}

// Orders one wave's LDS writes before its own later reads (and reads before
// later writes): a wave's LDS operations complete in issue order once the
// counters are drained, and the fence keeps the compiler from moving them.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

constexpr int SKW = 16;                // words per stage of a two-block task
constexpr int SPRE = 4;                // prefix columns whose loads are issued with a stage's
constexpr int SLD = 2 * SKW + 1;       // dwords per staged column row (odd: conflict-free reads)
constexpr int DKW = 2 * SKW;           // a diagonal task (one block) stages twice the words
constexpr int DLD = 2 * DKW + 1;
static_assert(GRAM_SMALL_KW % DKW == 0, "stages must tile the task word ranges");
static_assert(SB * DLD <= 2 * SB * SLD, "a diagonal stage fits the wave's slice");

// One task of one wave.  DIAG: the block pair is a diagonal block (bi == bl),
// so only its 32 columns are staged, DKW words at a time in the whole slice
// (twice the bytes in flight per stage); else both blocks, SKW words each.
template <bool F4, bool DIAG>
__device__ __forceinline__ void small_task(const ClassArgs& a, const Task& task, uint32_t* xa,
                                           uint32_t* xb, int lane) {
  constexpr int KW = DIAG ? DKW : SKW;
  constexpr int LD = DIAG ? DLD : SLD;
  const int r = lane & 31, h = lane >> 5;
  const int sc = lane >> 3, sl = lane & 7;  // staging: column sc + 8 (p & 3), 16-byte slot sl
  const ClassDesc cd = a.cls[task.cls];
  const DbInfo db = class_view(cd, a.dbs, a.views);
  const uint64_t Wp = db.Wp;
  const uint32_t q = cd.q;
  const uint32_t I0 = (uint32_t)task.bi * SB, L0 = (uint32_t)task.bl * SB;
  // staged columns of this lane, p = 0..7: DIAG -- the block's column sc + 8 (p & 3),
  // words 16 (p >> 2) + 2 sl of the stage; else A side p < 4, B side p >= 4
  const uint64_t* colp[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const uint32_t idx = ((!DIAG && p >= 4) ? L0 : I0) + sc + 8 * (p & 3);
    colp[p] = nullptr;
    if (idx < q) {
      const uint32_t item = a.child_item[cd.child0 + idx];
      colp[p] = db.B + (uint64_t)class_col(cd, db, idx, item) * Wp + 2 * sl +
                (DIAG ? SKW * (p >> 2) : 0);
    }
  }
  const uint32_t* pre = a.pre_cols + cd.pre_off;
  const uint32_t pre_len = cd.proj ? 0u : cd.pre_len;  // a view has the prefix applied
  // The first SPRE prefix columns are addressed once per task, and their
  // chunks of a stage are loaded together with the stage's column chunks and
  // ANDed only when the stage is written to LDS, so a stage costs one round
  // trip to memory whatever the prefix length up to SPRE.  Columns beyond
  // SPRE (prefixes of more than SPRE items) are ANDed in as they arrive.
  constexpr int NU = DIAG ? 2 : 1;
  const uint64_t* pcol[SPRE];
#pragma unroll
  for (int j = 0; j < SPRE; ++j)
    pcol[j] = (uint32_t)j < pre_len ? db.B + (uint64_t)load_global_u32(pre + j) * Wp + 2 * sl
                                    : nullptr;

  uint4 reg[8];
  uint4 pch[SPRE][NU];  // the stage's prefix chunks
  uint4 msk[NU];        // the AND of the prefix columns beyond SPRE
  auto load_stage = [&](uint32_t w) {
#pragma unroll
    for (int u = 0; u < NU; ++u) msk[u] = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (uint32_t j = SPRE; j < pre_len; ++j) {
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const uint4 v = load_global16(db.B + (uint64_t)load_global_u32(pre + j) * Wp + w +
                                      2 * sl + SKW * u);
        msk[u].x &= v.x;
        msk[u].y &= v.y;
        msk[u].z &= v.z;
        msk[u].w &= v.w;
      }
    }
#pragma unroll
    for (int j = 0; j < SPRE; ++j)
#pragma unroll
      for (int u = 0; u < NU; ++u)
        pch[j][u] = pcol[j] ? load_global16(pcol[j] + w + SKW * u) : make_uint4(~0u, ~0u, ~0u, ~0u);
#pragma unroll
    for (int p = 0; p < 8; ++p)
      reg[p] = colp[p] ? load_global16(colp[p] + w) : make_uint4(0, 0, 0, 0);
  };

  using Acc = typename std::conditional<F4, v16f, v16i>::type;
  Acc acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0;

  const uint32_t nst = (task.w1 - task.w0) / KW;
  if (nst) load_stage(task.w0);
  for (uint32_t s = 0; s < nst; ++s) {
    wave_lds_sync();  // this wave finished reading the previous stage
#pragma unroll
    for (int u = 0; u < NU; ++u)
#pragma unroll
      for (int j = 0; j < SPRE; ++j) {
        msk[u].x &= pch[j][u].x;
        msk[u].y &= pch[j][u].y;
        msk[u].z &= pch[j][u].z;
        msk[u].w &= pch[j][u].w;
      }
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      // the prefix mask goes into the A side only: t & a_i & b_l needs it once
      const bool m = DIAG || p < 4;
      const uint4 mk = msk[DIAG ? (p >> 2) : 0];
      uint32_t* dst = ((!DIAG && p >= 4) ? xb : xa) + (sc + 8 * (p & 3)) * LD + 4 * sl +
                      (DIAG ? 2 * SKW * (p >> 2) : 0);
      const uint4 v = reg[p];
      dst[0] = m ? v.x & mk.x : v.x;
      dst[1] = m ? v.y & mk.y : v.y;
      dst[2] = m ? v.z & mk.z : v.z;
      dst[3] = m ? v.w & mk.w : v.w;
    }
    wave_lds_sync();
    if (s + 1 < nst) load_stage(task.w0 + (s + 1) * KW);
    const uint32_t* ra = xa + r * LD + h;
    const uint32_t* rb = (DIAG ? xa : xb) + r * LD + h;
#pragma unroll
    for (int w = 0; w < KW; ++w) {
      const uint32_t va = ra[2 * w];
      if constexpr (F4) {
        const v8i A = fp4_of(va);
        const v8i B = DIAG ? A : fp4_of(rb[2 * w]);
        // format 4 = e2m1 for both operands, no scaling
        acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, B, acc, 4, 4, 0, 0, 0, 0);
      } else {
        const uint32_t vb = DIAG ? va : rb[2 * w];
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          const v4i A = i8_of(va, 4 * d);
          const v4i B = DIAG ? A : i8_of(vb, 4 * d);
          acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B, acc, 0, 0, 0);
        }
      }
    }
  }

  // 32x32 accumulator layout: lane holds column (lane & 31); register i
  // holds row 8*(i/4) + 4*(lane/32) + (i%4).
  uint32_t* tri = a.tri + cd.tri_off;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const uint32_t gi = I0 + 8 * (i >> 2) + 4 * h + (i & 3);
    const uint32_t gl = L0 + r;
    uint32_t v;
    if constexpr (F4) v = __float2uint_rn(acc[i] * 4.0f);  // exact: quarters
    else v = (uint32_t)acc[i];
    if (gi < gl && gl < q && v) atomicAdd(tri + tri_index(gi, gl, q), v);
  }
}

template <bool F4>
__global__ __launch_bounds__(256) void k_gram_small(ClassArgs a) {
  __shared__ uint32_t sX[4][2 * SB * SLD];  // per wave: A rows then B rows (or one diagonal block)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t* xa = sX[wave];
  uint32_t* xb = sX[wave] + SB * SLD;
  const uint64_t ntasks = *a.ntasks;
  for (uint64_t t = (uint64_t)blockIdx.x * 4 + wave; t < ntasks; t += (uint64_t)gridDim.x * 4) {
    const Task task = a.tasks[t];
    if (task.bi == task.bl) small_task<F4, true>(a, task, xa, xb, lane);
    else small_task<F4, false>(a, task, xa, xb, lane);
  }
}

}  // namespace

void launch_gram_small(const ClassArgs& a, uint32_t grid, bool fp4, hipStream_t s) {
  if (grid == 0) return;
  if (fp4) k_gram_small<true><<<grid, 256, 0, s>>>(a);
  else k_gram_small<false><<<grid, 256, 0, s>>>(a);
  BM_LAUNCH_CHECK();
}

}  // namespace bm
