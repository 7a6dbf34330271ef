// Pieces shared by the FP4 Gram kernels (k_gram_mfma.hip: 128 x 128 tiles,
// k_gram_big.hip: 256 x 256 tiles).
#pragma once

#include "internal.hpp"

namespace bm {

typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// FP4 (e2m1) form.  The e2m1 codes 0001, 0010 and 0100 are the values 0.5, 1
// and 2, so one AND turns a 32-bit half-word v into eight FP4 elements that
// each hold one transaction bit: plane 0 = v & 0x11111111 (bits 0, 4, .., 28
// as 0.5), plane 1 = v & 0x22222222 (bits 1, 5, .. as 1), plane 2 =
// v & 0x44444444 (as 2); plane 3 (bits 3, 7, ..) would land on the sign bit,
// so it is shifted first: (v >> 2) & 0x22222222 (as 1).  One
// v_mfma_scale_f32_32x32x64_f8f6f4 takes one plane of a lane's four operand
// dwords, and its E8M0 block scales (2, 1, 1/2, 1 on both operands) make every
// product of two set bits exactly 1.0; four MFMAs, one per plane, cover the
// four dwords.  A and B use the identical bit -> (lane, element) map, so every
// transaction meets itself in the K sum.  FP32 holds every integer up to 2^24
// exactly, so a task's sums are exact while its counts stay at most 2^24 --
// the task word split is capped at GRAM_FP4_MAX_WORDS for that.
__device__ __forceinline__ uint32_t fp4_plane(uint32_t v, int pl) {
  return pl == 0 ? (v & 0x11111111u)
       : pl == 1 ? (v & 0x22222222u)
       : pl == 2 ? (v & 0x44444444u)
                 : ((v >> 2) & 0x22222222u);
}
__device__ __forceinline__ int fp4_plane_scale(int pl) {  // E8M0: 2^(e - 127)
  return pl == 0 ? 128 : pl == 2 ? 126 : 127;
}
// acc += A B^T over one plane (format 4 = e2m1 for both operands)
__device__ __forceinline__ v16f fp4_mfma(const v8i& A, const v8i& B, const v16f& acc, int sc) {
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, B, acc, 4, 4, 0, sc, 0, sc);
}

// Direct-to-LDS staging.  Each stage (DKW = 16 words = 128 bytes of every
// panel column) travels from global memory into LDS with
// global_load_lds_dwordx4, bypassing registers, into one of two buffers: the
// loads of stage s + 1 fly while stage s is multiplied, so a stage costs one
// barrier and no staging instructions beyond the loads themselves.  The two
// buffers are distinct LDS arrays and the stage loop is unrolled by two, so
// the compiler sees that the reads of one buffer need not wait for the loads
// into the other.
//
// LDS layout: a column's 128 bytes are eight 16-byte chunks; chunk c of the
// column in panel row r sits in slot c ^ (r & 7) of that row (XOR swizzle).
// A load instruction moves 64 chunks into 1 KiB of consecutive LDS (lane L to
// byte 16 L), so lane L fetches the chunk that belongs in slot L % 8 of row
// L / 8 of its group of eight rows.  The operand reads take one chunk per lane
// per 32-row block (lane l: row l % 32, chunk 2 g + l / 32 for word group g),
// and the swizzle spreads any eight consecutive rows over all 32 banks.
//
// The operand map: lane l's four dwords for word group g are chunk
// 2 g + l / 32 (words 4 g + 2 (l / 32), +1) of its row (A) or column (B); A and
// B use the same map.
//
// The prefix mask t(P) of a stage is ANDed into the A operands as they are
// built.  It lives in LDS as eight chunks per stage in three rotating rows: a
// row is set to all ones two stages ahead, the prefix columns of its stage are
// ANDed in (ds_and, by the threads that loaded them) during the stage before,
// and it is read during its own stage.
constexpr int DKW = 16;        // words per stage
constexpr int DCH = DKW / 2;   // 16-byte chunks per column per stage
static_assert(GRAM_KW % DKW == 0, "stages must tile the task word ranges");

// Chunk pch of the stage at word w of this thread's prefix columns j =
// pj0, pj0 + stride, ... (stride = threads / 8; pm holds column pj0's chunk,
// loaded earlier), ANDed into mask row `row`.
__device__ __forceinline__ void fp4_mask_and(uint4 pm, const uint64_t* B, uint64_t Wp,
                                             const uint32_t* pre, uint32_t pre_len, uint32_t pj0,
                                             uint32_t pch, uint32_t w, uint4* row,
                                             uint32_t stride) {
  for (uint32_t j = pj0 + stride; j < pre_len; j += stride) {  // prefixes longer than stride
    const uint4 x = load_global16(B + (uint64_t)pre[j] * Wp + w + 2 * pch);
    pm.x &= x.x;
    pm.y &= x.y;
    pm.z &= x.z;
    pm.w &= x.w;
  }
  uint32_t* r = reinterpret_cast<uint32_t*>(row + pch);
  atomicAnd(r + 0, pm.x);
  atomicAnd(r + 1, pm.y);
  atomicAnd(r + 2, pm.z);
  atomicAnd(r + 3, pm.w);
}

// Stage 0's mask row in full (threads 0..7, one chunk each, before the first
// barrier).
__device__ __forceinline__ uint4 fp4_mask_full(const uint64_t* B, uint64_t Wp,
                                               const uint32_t* pre, uint32_t pre_len, uint32_t w,
                                               uint32_t ch) {
  uint4 r = make_uint4(~0u, ~0u, ~0u, ~0u);
  for (uint32_t j = 0; j < pre_len; ++j) {
    const uint4 x = load_global16(B + (uint64_t)pre[j] * Wp + w + 2 * ch);
    r.x &= x.x;
    r.y &= x.y;
    r.z &= x.z;
    r.w &= x.w;
  }
  return r;
}

// Balanced split of a launch's work (stream-K).  The tasks' costs laid end to
// end (P: exclusive prefix sums, n + 1 entries) are cut into gridDim.x
// ranges, one per workgroup; the workgroup of range [u0, u1) runs, of each
// task whose cost span meets it, the stages whose first cost unit lies in the
// range.  Every stage runs exactly once, every workgroup gets its share of the
// cost (up to one stage at each end), and partial tasks add their partial
// sums atomically like whole ones.
//
// SKEW (a grid of two workgroups per CU): the first half of the grid is
// dispatched first, one workgroup per CU, and wins its CU's issue
// arbitration against the workgroup that joins it (2.6 against 3.2 us per
// stage in a per-workgroup timeline), so the shares are 11 : 9 between the
// halves; the slower one speeds up once the faster has finished.  Only the
// running time depends on this; the split stays exact for any placement.
struct SkRange {
  uint64_t u0, u1;  // this workgroup's cost range
  uint64_t i;       // the last task with P[i] <= u0
};
__device__ __forceinline__ uint64_t sk_share(uint64_t b, uint64_t G, bool skew) {
  if (!skew) return b;
  const uint64_t h = G / 2;  // weights 11 (first half), 9 (second half)
  return b < h ? 11 * b : 11 * h + 9 * (b - h);
}
// Called by every thread of the workgroup (it synchronises): the last i in
// [0, n] with P[i] <= u0, by rounds of blockDim.x-way sampling.
template <bool SKEW>
__device__ __forceinline__ SkRange sk_range(const uint64_t* P, uint64_t n) {
  SkRange r;
  const uint64_t C = P[n];
  const uint64_t G = gridDim.x, b = blockIdx.x;
  const uint64_t WT = sk_share(G, G, SKEW);
  r.u0 = (uint64_t)((unsigned __int128)C * sk_share(b, G, SKEW) / WT);
  r.u1 = (uint64_t)((unsigned __int128)C * sk_share(b + 1, G, SKEW) / WT);
  const uint64_t k = threadIdx.x, nt = blockDim.x;
  uint64_t lo = 0, hi = n;  // P[lo] <= u0 (P[0] = 0); the answer lies in [lo, hi]
  while (hi > lo) {
    const uint64_t m = hi - lo;  // candidates lo + 1 .. hi
    if (m <= nt) {
      const int t = k < m && P[lo + 1 + k] <= r.u0;
      lo += (uint64_t)__syncthreads_count(t);  // the true ones are a prefix
      break;
    }
    const uint64_t idx = lo + (k + 1) * m / nt;  // the last thread samples hi
    const uint64_t c = (uint64_t)__syncthreads_count(P[idx] <= r.u0);
    const uint64_t nlo = c ? lo + c * m / nt : lo;
    const uint64_t nhi = c < nt ? lo + (c + 1) * m / nt - 1 : hi;
    lo = nlo;
    hi = nhi;
  }
  r.i = lo;
  return r;
}
// The stages [s_lo, s_hi) of a task with cost span [base, end) and cost wt per
// stage that belong to the range [u0, u1); false if none.
__device__ __forceinline__ bool sk_stages(uint64_t base, uint64_t end, const SkRange& r,
                                          uint32_t wt, uint32_t& s_lo, uint32_t& s_hi) {
  const uint64_t lo = r.u0 > base ? r.u0 - base : 0;
  const uint64_t hi = (r.u1 < end ? r.u1 : end) - base;
  s_lo = (uint32_t)((lo + wt - 1) / wt);
  s_hi = (uint32_t)((hi + wt - 1) / wt);
  return s_lo < s_hi;
}

}  // namespace bm
