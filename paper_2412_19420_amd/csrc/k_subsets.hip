// Whole subtrees of small prefix classes by subset counting, for databases
// whose columns are too long for one workgroup to walk a subtree.
//
// The supports the recursion of the method needs below a class with prefix P
// and children c_0..c_{q-1} are all of the form
//     supp(P + {c_i : i in S}) = sum_words popcount(t(P) & AND_{i in S} col(c_i))
// for subsets S of the children (Eq. 2 with the prefix columns ANDed in first,
// applied to longer itemsets).  With q <= SUBSET_Q every such subset fits in
// 2^q counters, so one pass over the columns (two or four for q = 7, 8)
// counts them all:
//   * k_subset_count: a workgroup takes one word range of one class; each
//     thread ANDs its words of the prefix and child columns along a
//     depth-first walk of the subset lattice (one AND per subset, from its
//     parent's value) and popcounts every subset of two or more children into
//     its own register counter; the counters are reduced over the workgroup
//     and added atomically into the class's counter block;
//   * k_subset_emit: one wave per class turns the counters into the
//     subtree's frequent itemsets.  A subset is frequent when its count meets
//     the threshold (every subset of a frequent set is frequent, so this is
//     exactly the set the class-by-class recursion reaches).  The nodes are
//     written to the subtree arena with each node's frequent extensions as one
//     contiguous block, the format the depth-first kernel writes, so the same
//     merge produces the canonical output.  Candidate and frequent counts per
//     length are those of the recursion: a node with e >= 2 frequent
//     extensions forms a class of e(e-1)/2 candidates.
#include "internal.hpp"
#include "levels.hpp"
#include "dfs.hpp"

namespace bm {

namespace {

constexpr int LQ = SUBSET_LAT;  // children walked in registers per pass
constexpr int LN = 1 << LQ;     // counters per pass
constexpr int SQ = SUBSET_Q;    // most children of a task
constexpr int SN = 1 << SQ;     // counters per task
constexpr int kCountThreads = 256;
constexpr uint32_t kMaxPairs = 511;  // word pairs per thread: 16-bit counters hold 511 * 128
constexpr int kEmitWaves = 4;  // tasks per emit workgroup

// Visits every subset that extends MASK by columns L.. (each exactly once, by
// the step that adds its highest child); x = t(P) & the pass's fixed columns &
// the columns of MASK.  all: count single children too (the pass's fixed
// children already make them sets of two or more).  Counters are 16-bit
// halves of acc (mask m in half m & 1 of acc[m >> 1]), which frees registers
// for a fourth wave per SIMD; a thread adds at most 128 per word pair, and
// the host keeps a task's word range to at most kMaxPairs pairs per thread.
template <int L, int MASK>
__device__ __forceinline__ void subsets_from(const uint64_t (&c0)[LQ], const uint64_t (&c1)[LQ],
                                             uint64_t x0, uint64_t x1, int q, bool all,
                                             uint32_t (&acc)[LN / 2]) {
  if constexpr (L < LQ) {
    if (L < q) {
      constexpr int M2 = MASK | (1 << L);
      const uint64_t y0 = x0 & c0[L], y1 = x1 & c1[L];
      if (MASK != 0 || all)
        acc[M2 >> 1] += (uint32_t)(__popcll(y0) + __popcll(y1)) << (16 * (M2 & 1));
      subsets_from<L + 1, M2>(c0, c1, y0, y1, q, all, acc);
      subsets_from<L + 1, MASK>(c0, c1, x0, x1, q, all, acc);
    }
  }
}

// Block b counts pass b / (ntasks * splits) of word range b % splits of task
// (b / splits) % ntasks (the host picks splits so that a range holds at most
// kCountThreads * kMaxPairs word pairs).  Pass-major order keeps consecutive
// blocks -- which the dispatcher sends to different XCDs -- on real work.  A task of more than LQ children runs
// one pass per subset g of its children LQ.. ("fixed" in that pass): the pass
// ANDs them into the prefix mask and walks the first LQ children, so counter
// g << LQ | mask holds the set g + mask.  Each pass is a workgroup of its own,
// so the few long tasks do not trail the launch; blocks of passes a task does
// not need exit at once.
__global__ __launch_bounds__(kCountThreads) void k_subset_count(DfsArgs a,
                                                                uint32_t* __restrict__ counts,
                                                                uint32_t splits) {
  __shared__ uint32_t s_red[kCountThreads / 64][LN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t per_pass = a.ntasks * splits;
  const uint32_t g = blockIdx.x / per_pass, b = blockIdx.x % per_pass;
  const uint32_t t = b / splits, sp = b % splits;
  const DfsTask tk = a.tasks[t];
  const int q = (int)tk.q;  // 2 <= q <= SQ
  const int ql = min(q, LQ), nfix = q - ql;
  if (g >= (1u << nfix)) return;  // this task needs fewer passes than the launch holds
  const DbInfo db = a.dbs[tk.db];
  const uint32_t W = (uint32_t)db.W;
  // even word ranges: the 16-byte loads at even words stay inside the padded column
  const uint32_t len = ((W + splits - 1) / splits + 1) & ~1u;
  const uint32_t w0 = sp * len;
  const uint32_t w1 = min(W, w0 + len);
  const uint32_t* lit = a.lv_item[tk.level];
  const uint64_t* col[SQ];
#pragma unroll
  for (int i = 0; i < SQ; ++i) {
    uint32_t c = 0;
    if (i < q) {
      const uint32_t it = lit[tk.child0 + i];
      c = db.f1 ? db.f1[it] : it;
    }
    col[i] = db.B + (uint64_t)c * db.Wp;
  }
  const uint32_t* pre = a.step_pre[tk.level] + tk.pre_off;
  const uint32_t pre_len = tk.pre_len;
  const uint64_t* pc[PREFIX_REG];
#pragma unroll
  for (int j = 0; j < PREFIX_REG; ++j)
    pc[j] = (uint32_t)j < pre_len ? db.B + (uint64_t)load_global_u32(pre + j) * db.Wp : nullptr;
  {
    const int gpop = __popc(g);
    uint32_t acc[LN / 2];
#pragma unroll
    for (int j = 0; j < LN / 2; ++j) acc[j] = 0;
    uint32_t acc0 = 0;  // the fixed children alone (a set of two when gpop == 2)
    for (uint32_t w = w0 + 2 * tid; w < w1; w += 2 * kCountThreads) {
      uint64_t m0 = ~0ull, m1 = (w + 1 < w1) ? ~0ull : 0ull;
      prefix_and(pc, db.B, db.Wp, pre, pre_len, w, m0, m1);
#pragma unroll
      for (int i = 0; i < SQ - LQ; ++i)
        if ((g >> i) & 1) {
          const uint4 x = load_global16(col[LQ + i] + w);
          m0 &= (uint64_t)x.x | ((uint64_t)x.y << 32);
          m1 &= (uint64_t)x.z | ((uint64_t)x.w << 32);
        }
      uint64_t c0[LQ], c1[LQ];
#pragma unroll
      for (int i = 0; i < LQ; ++i) {
        c0[i] = 0;
        c1[i] = 0;
        if (i < ql) {
          const uint4 v = load_global16(col[i] + w);
          c0[i] = (uint64_t)v.x | ((uint64_t)v.y << 32);
          c1[i] = (uint64_t)v.z | ((uint64_t)v.w << 32);
        }
      }
      subsets_from<0, 0>(c0, c1, m0, m1, ql, gpop > 0, acc);
      if (gpop >= 2) acc0 += (uint32_t)(__popcll(m0) + __popcll(m1));
    }
#pragma unroll
    for (int mask = 0; mask < LN; ++mask) {
      if (__builtin_popcount(mask) + gpop < 2 || mask >= (1 << ql)) continue;
      uint32_t v = mask == 0 ? acc0 : (acc[mask >> 1] >> (16 * (mask & 1))) & 0xffffu;
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) s_red[wave][mask] = v;
    }
    __syncthreads();
    if (tid < (1 << ql) && __popc(tid) + gpop >= 2) {
      uint32_t v = 0;
#pragma unroll
      for (int j = 0; j < kCountThreads / 64; ++j) v += s_red[j][tid];
      if (v) atomicAdd(counts + (uint64_t)t * SN + ((uint32_t)g << LQ | tid), v);
    }
  }
}

// Orders one wave's LDS writes before its own later reads: a wave's LDS
// operations complete in issue order, and the fence keeps the compiler from
// moving them across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Wave per task: frequent subsets -> arena nodes, links and statistics.
// Lane l owns masks l, l + 64, ...  The arena order is breadth-first: by
// number of children, then lexicographically by child tuple, which for masks
// of one size is descending order of the bit-reversed mask.  In that order a
// node's frequent extensions are consecutive, so every node's children form
// one block, the format the depth-first kernel writes.
__global__ __launch_bounds__(64 * kEmitWaves) void k_subset_emit(DfsArgs a,
                                                                 const uint32_t* __restrict__ counts) {
  constexpr int MPL = SN / 64;  // masks per lane
  __shared__ uint32_t s_cnt[kEmitWaves][SN];
  __shared__ uint32_t s_fr[kEmitWaves][SN];   // mask is a frequent set (single children: 1)
  __shared__ uint32_t s_pos[kEmitWaves][SN];  // arena slot of a frequent mask of >= 2 children
  __shared__ unsigned long long s_cand[BM_MAX_LEVELS + 1], s_freq[BM_MAX_LEVELS + 1];
  __shared__ unsigned long long s_words;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = tid; j <= BM_MAX_LEVELS; j += 64 * kEmitWaves) {
    s_cand[j] = 0;
    s_freq[j] = 0;
  }
  if (tid == 0) s_words = 0;
  __syncthreads();
  const uint32_t t = blockIdx.x * kEmitWaves + wave;
  if (t < a.ntasks) {  // uniform over the wave
    const DfsTask tk = a.tasks[t];
    const DbInfo db = a.dbs[tk.db];
    const uint32_t q = tk.q, level = tk.level, minsup = db.minsup;
    const uint32_t nsub = 1u << q;
    uint32_t* cnt = s_cnt[wave];
    uint32_t* fr = s_fr[wave];
    uint32_t* pos = s_pos[wave];
#pragma unroll
    for (int k = 0; k < MPL; ++k) {
      const uint32_t m = lane + 64 * k;
      const uint32_t c = m < nsub ? counts[(uint64_t)t * SN + m] : 0u;
      const int j = __popc(m);
      cnt[m] = c;
      fr[m] = (m < nsub && (j == 1 || (j >= 2 && c >= minsup))) ? 1u : 0u;
    }
    wave_lds_sync();
    // per owned mask: frequent sets of 2..j-1 children before it, and of j
    // children ordered before it; also the totals
    uint32_t before[MPL], rank[MPL], mj[MPL], mbr[MPL];
#pragma unroll
    for (int k = 0; k < MPL; ++k) {
      const uint32_t m = lane + 64 * k;
      before[k] = 0;
      rank[k] = 0;
      mj[k] = (uint32_t)__popc(m);
      mbr[k] = __brev(m) >> (32 - q);
    }
    uint32_t total = 0, maxj = 1;
    for (uint32_t m2 = 3; m2 < nsub; ++m2) {
      const uint32_t j2 = (uint32_t)__popc(m2);
      if (j2 < 2 || !fr[m2]) continue;
      total += 1;
      maxj = max(maxj, j2);
      const uint32_t br2 = __brev(m2) >> (32 - q);
#pragma unroll
      for (int k = 0; k < MPL; ++k) {
        before[k] += j2 < mj[k] ? 1u : 0u;
        rank[k] += (j2 == mj[k] && br2 > mbr[k]) ? 1u : 0u;
      }
    }
    bool ok = level + maxj - 1 <= BM_MAX_LEVELS;  // itemsets of level + j - 1 items
    if (!ok && lane == 0) atomicOr(a.flags, DFS_TOO_LONG);
    uint32_t base = 0;
    if (ok && total) {
      if (lane == 0) base = atomicAdd(a.arena_count, total);
      base = __shfl(base, 0);
      if (base + total > a.arena_cap) {
        if (lane == 0) atomicOr(a.flags, DFS_OVERFLOW);
        ok = false;
      }
    }
    if (ok) {
#pragma unroll
      for (int k = 0; k < MPL; ++k) {
        const uint32_t m = lane + 64 * k;
        if (m < nsub && mj[k] >= 2 && fr[m]) pos[m] = base + before[k] + rank[k];
      }
      wave_lds_sync();
      const uint32_t* lit = a.lv_item[tk.level] + tk.child0;
      unsigned long long words = 0;
#pragma unroll
      for (int k = 0; k < MPL; ++k) {
        const uint32_t m = lane + 64 * k;
        if (m == 0 || m >= nsub || !fr[m]) continue;
        const uint32_t j = mj[k], hb = 31u - (uint32_t)__clz(m);
        uint32_t ext = 0;
        for (uint32_t l = hb + 1; l < q; ++l)
          if (fr[m | (1u << l)]) ext |= 1u << l;
        const uint32_t ne = (uint32_t)__popc(ext);
        const uint32_t first = ne ? pos[m | (1u << (__ffs(ext) - 1))] : 0u;
        if (j == 1) {
          a.ls_first[level][tk.child0 + hb] = first;
          a.ls_count[level][tk.child0 + hb] = ne;
        } else {
          ArenaNode an;
          an.item = lit[hb];
          an.supp = cnt[m];
          an.first = first;
          an.count = ne;
          a.arena[pos[m]] = an;
          atomicAdd(&s_freq[level + j - 1], 1ull);
        }
        if (ne >= 2) {  // this node's class: its extensions paired
          if (level + j + 1 <= BM_MAX_LEVELS)
            atomicAdd(&s_cand[level + j + 1], (unsigned long long)ne * (ne - 1) / 2);
          words += (unsigned long long)(tk.pre_len + j + ne) * db.W;
        }
      }
      for (int off = 32; off > 0; off >>= 1) words += __shfl_xor(words, off);
      if (lane == 0) {
        const unsigned long long read = (unsigned long long)(tk.pre_len + q) * db.W;
        if (level + 1 <= BM_MAX_LEVELS)
          atomicAdd(&s_cand[level + 1], (unsigned long long)q * (q - 1) / 2);
        if (a.task_cost) a.task_cost[t] = (float)(words + read);
        atomicAdd(&s_words, read);
      }
    }
  }
  __syncthreads();
  for (int j = tid; j <= BM_MAX_LEVELS; j += 64 * kEmitWaves) {
    if (s_cand[j]) atomicAdd(&a.level_cand[j], s_cand[j]);
    if (s_freq[j]) atomicAdd(&a.level_freq[j], s_freq[j]);
  }
  if (tid == 0 && s_words) atomicAdd(a.words_read, s_words);
}

}  // namespace

uint32_t subset_min_splits(uint64_t W) {
  const uint64_t per = 2ull * kCountThreads * kMaxPairs;  // words per range at most
  return (uint32_t)((W + per - 1) / per);
}

void launch_subset_count(const DfsArgs& a, uint32_t* counts, uint32_t splits, uint32_t max_q,
                         hipStream_t s) {
  if (a.ntasks == 0) return;
  if (max_q < 2 || max_q > (uint32_t)SQ) fail(BM_ERR_INVALID_ARG, "subset tasks of %u children", max_q);
  const uint32_t passes = max_q > (uint32_t)LQ ? 1u << (max_q - LQ) : 1u;
  const uint64_t grid = (uint64_t)a.ntasks * splits * passes;
  if (splits == 0 || grid > 0x7fffffffull) fail(BM_ERR_UNSUPPORTED, "too many subset-count blocks");
  k_subset_count<<<(uint32_t)grid, kCountThreads, 0, s>>>(a, counts, splits);
  BM_LAUNCH_CHECK();
}

void launch_subset_emit(const DfsArgs& a, const uint32_t* counts, hipStream_t s) {
  if (a.ntasks == 0) return;
  k_subset_emit<<<(a.ntasks + kEmitWaves - 1) / kEmitWaves, 64 * kEmitWaves, 0, s>>>(a, counts);
  BM_LAUNCH_CHECK();
}

}  // namespace bm
