// Frequent-itemset extraction (Eq. 3) and the recursive extension of frequent
// prefixes, level by level, for one or many databases at once, plus the
// canonical-order output.
//
// Level k holds the frequent k-itemsets of all databases of the call, database
// by database and lexicographically within one, as records (parent index in
// level k-1, last item, support, database); the children of a node are
// contiguous in level k+1.  A step turns level k into level k+1:
//   * classes: the level-k nodes grouped by parent.  A parent with q >= 2
//     frequent children forms a prefix class whose candidates are the q(q-1)/2
//     pairs of children; supports land in the step's triangle buffer, class by
//     class, row by row -- which is exactly lexicographic order of the
//     candidate itemsets;
//   * each node's entries of its triangle row that meet its database's
//     minsup are counted (a lane per node for short rows, the whole wave for
//     long ones); an exclusive scan over the nodes gives each node's first
//     child in level k+1, and in-row ranks place the children after it, so the
//     next level comes out already sorted;
//   * a node with c >= 2 frequent children becomes a class of the next step.
#include "internal.hpp"
#include <algorithm>

#include "levels.hpp"
#include "dfs.hpp"

namespace bm {

namespace {

constexpr int kThreads = 256;

uint32_t grid_for(uint64_t work, uint32_t per_block, uint32_t cap = 65535) {
  uint64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

// Database of a global index, given the exclusive prefix `base` (size ndb+1).
__device__ inline uint32_t db_of(const uint64_t* __restrict__ base, uint32_t ndb, uint64_t g) {
  uint32_t lo = 0, hi = ndb;  // base[lo] <= g < base[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (base[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// Frequent single items of every database (Eq. 3): flag item j of database d.
__global__ void k_f1_flags(const DbInfo* __restrict__ dbs, uint32_t ndb,
                           const uint64_t* __restrict__ item_base, uint64_t total,
                           uint32_t* __restrict__ flags) {
  for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < total;
       g += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t d = db_of(item_base, ndb, g);
    const uint64_t j = g - item_base[d];
    flags[g] = dbs[d].colsum[j] >= dbs[d].minsup ? 1u : 0u;
  }
}

__global__ void k_f1_fill(const uint32_t* __restrict__ flags, const uint64_t* __restrict__ pos,
                          uint32_t ndb, const uint64_t* __restrict__ item_base, uint64_t total,
                          uint32_t* __restrict__ f1) {
  for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < total;
       g += (uint64_t)gridDim.x * blockDim.x) {
    if (flags[g]) {
      const uint32_t d = db_of(item_base, ndb, g);
      f1[pos[g]] = (uint32_t)(g - item_base[d]);
    }
  }
}

// Level 1: every frequent item is a node whose parent is its database's root.
__global__ void k_init_level1(DbInfo* __restrict__ dbs, uint32_t ndb,
                              const uint64_t* __restrict__ f1_base, uint64_t n1,
                              const uint32_t* __restrict__ f1, uint32_t* __restrict__ item,
                              uint32_t* __restrict__ parent, uint32_t* __restrict__ supp,
                              uint32_t* __restrict__ ndbv) {
  // each database's table entry gets its slice of the frequent-item list (no
  // thread of this kernel reads that field)
  for (uint64_t d = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; d < ndb;
       d += (uint64_t)gridDim.x * blockDim.x)
    dbs[d].f1 = f1 + f1_base[d];
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n1;
       x += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t d = db_of(f1_base, ndb, x);
    item[x] = (uint32_t)(x - f1_base[d]);
    parent[x] = d;
    supp[x] = dbs[d].colsum[f1[x]];
    ndbv[x] = d;
  }
}

__global__ void k_gather_idx(const uint64_t* __restrict__ arr, const uint64_t* __restrict__ idx,
                             uint32_t k, uint64_t* __restrict__ out, uint64_t* __restrict__ out2) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const uint64_t v = arr[idx[i]];
    out[i] = v;
    if (out2) out2[i] = v;
  }
}

__device__ inline uint32_t mfma_pairs(uint32_t q, uint32_t tile = GRAM_TILE) {
  const uint32_t nb = (q + tile - 1) / tile;
  return nb * (nb + 1) / 2;
}
__device__ inline uint32_t andpop_pairs(uint32_t q, uint32_t block = AP_BLOCK) {
  const uint32_t nb = (q + block - 1) / block;
  // the diagonal block of a lone last child holds no pair
  return nb * (nb + 1) / 2 - ((q % block) == 1 ? 1u : 0u);
}

// Rows of at most this many entries are counted (and written out) by one
// lane, longer ones by a whole wave.
constexpr uint32_t NODE_LANE_ROW = 16;

}  // namespace

// Nodes per wave of the node-count and next-level kernels: up to 64 (one per
// lane) when rows are short, fewer as rows grow (a long row takes the whole
// wave, node after node), and few enough that the level still spreads over
// about 2,048 waves.
uint32_t node_batch(uint64_t n, uint64_t tri_total) {
  const uint64_t avg = n ? tri_total / n : 0;
  const uint64_t units = std::max<uint64_t>(1, (avg + NODE_LANE_ROW - 1) / NODE_LANE_ROW);
  uint64_t b = std::max<uint64_t>(1, 64 / units);
  b = std::min<uint64_t>(b, std::max<uint64_t>(1, n / 2048));
  return (uint32_t)b;
}

namespace {

// loc[base + idx] += v for a run-time idx < n, with constant indices only, so
// the counters stay in registers (a run-time index would put them in scratch)
__device__ __forceinline__ void loc_add(unsigned long long (&loc)[NC_COUNT], int base, int idx,
                                        int n, unsigned long long v) {
#pragma unroll
  for (int j = 0; j < 5; ++j)
    if (j < n && j == idx) loc[base + j] += v;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int j) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, j);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), j);
  return ((uint64_t)hi << 32) | lo;
}

// Per node of level k: number of frequent children, and what it contributes
// to the next step if it becomes a class.  Also accumulates per-step totals
// (candidates, columns read, classes per kernel) for the statistics, and the
// next step's task-count bounds.
__global__ __launch_bounds__(kThreads) void k_node_counts(
    uint64_t n, uint32_t nb, uint32_t k, const uint32_t* __restrict__ parent,
    const int32_t* __restrict__ pcls, const ClassDesc* __restrict__ cls,
    const DbInfo* __restrict__ dbs, const uint32_t* __restrict__ tri, uint32_t mfma_min_q,
    uint32_t big_q, uint32_t small_on,
    uint32_t tiny_q, uint32_t* __restrict__ cnt, uint32_t* __restrict__ is_cls,
    uint64_t* __restrict__ tri_sz, unsigned long long* __restrict__ st,
    const uint32_t* __restrict__ supp, uint32_t proj_on, uint32_t* __restrict__ pflag,
    uint32_t* __restrict__ prows, uint64_t* __restrict__ pwords) {
  __shared__ unsigned long long s_st[NC_COUNT];
  if (threadIdx.x < NC_COUNT) s_st[threadIdx.x] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  unsigned long long loc[NC_COUNT];
#pragma unroll
  for (int j = 0; j < NC_COUNT; ++j) loc[j] = 0;
  // a node's frequent extensions are the entries of its row of its class's
  // triangle that meet the class's threshold.  Nodes go to waves nb at a
  // time: each lane fetches its own node's class, database and row, so the
  // chain of dependent loads is paid once per nb nodes; a row of at most
  // NODE_LANE_ROW entries is then counted by its lane, a longer one by the
  // whole wave, one such node after another.
  const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t i0 = wave * nb; i0 < n; i0 += nwaves * nb) {
    const uint64_t i = i0 + lane;
    const bool mine = (uint32_t)lane < nb && i < n;
    uint64_t n_db = 0, w_db = 0, rs = 0, len = 0;
    uint32_t minsup = 0;
    if (mine) {
      const int32_t c = pcls[parent[i]];
      if (c >= 0) {
        const ClassDesc cd = cls[c];
        n_db = dbs[cd.db].n;
        w_db = dbs[cd.db].W;
        const uint64_t li = i - cd.child0;
        if (li + 1 < cd.q) {
          rs = cd.tri_off + tri_index(li, li + 1, cd.q);
          len = cd.q - li - 1;
          minsup = dbs[cd.db].minsup;
        }
      }
    }
    uint32_t kc = 0;
    if (len <= NODE_LANE_ROW) {  // the lane's own row: its loads in flight together
      uint32_t v[NODE_LANE_ROW];
#pragma unroll
      for (uint32_t u = 0; u < NODE_LANE_ROW; ++u) v[u] = u < len ? tri[rs + u] : 0u;
#pragma unroll
      for (uint32_t u = 0; u < NODE_LANE_ROW; ++u) kc += (u < len && v[u] >= minsup) ? 1u : 0u;
    }
    for (uint64_t lm = __ballot(len > NODE_LANE_ROW); lm; lm &= lm - 1) {
      const int j = __builtin_ctzll(lm);
      const uint64_t rj = readlane64(rs, j), lj = readlane64(len, j);
      const uint32_t mj = (uint32_t)__builtin_amdgcn_readlane((int)minsup, j);
      // sixteen 64-entry chunks per pass: their loads are in flight together
      // (a level-1 row is as long as the number of frequent items)
      uint32_t sum = 0;
      for (uint64_t t0 = 0; t0 < lj; t0 += 1024) {
        uint32_t v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const uint64_t t = t0 + 64 * u + lane;
          v[u] = t < lj ? tri[rj + t] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const bool f = t0 + 64 * u + lane < lj && v[u] >= mj;
          sum += (uint32_t)__popcll(__ballot(f));
        }
      }
      if (lane == j) kc = sum;
    }
    if (mine) {
      cnt[i] = kc;
      const bool cl = kc >= 2;
      const int kind = cl ? class_kind(kc, mfma_min_q, big_q, small_on, tiny_q) : -1;
      const uint64_t tsz = cl ? (uint64_t)kc * (kc - 1) / 2 : 0ull;
      is_cls[i] = cl ? 1u : 0u;
      tri_sz[i] = tsz;
      bool pj = false;
      if (proj_on) {
        // the class's prefix is this node's itemset: its support is the node's
        const uint32_t sp = supp[i];
        pj = cl && project_class(kind, kc, sp, n_db, proj_on);
        pflag[i] = pj ? 1u : 0u;
        prows[i] = pj ? sp : 0u;
        pwords[i] = pj ? (uint64_t)kc * view_padded_words(sp) : 0ull;
        if (pj) {
          const int b = kind == 3 ? NC_PJ_CAND_B - NC_PJ_CAND_M : 0;
          loc_add(loc, NC_PJ_CAND_M, b, 3, tsz);
          loc_add(loc, NC_PJ_WORK_M, b, 3, (unsigned long long)sp * tsz);
          loc[NC_PJ_COLS] += kc;
        }
      }
      if (cl) {
        // a narrow tail's candidates and 32-wide block pairs go to the 32-wide kernel
        const bool tail = kind == 0 && small_on && !pj && gram_tail(kc);
        const uint64_t qm = tail ? gram_tail_q(kc) : kc;
        const uint64_t tm_sz = tail ? qm * (qm - 1) / 2 : tsz;
        loc_add(loc, ST_CAND_M, kind, 5, tm_sz);
        loc_add(loc, ST_COLS_M, kind, 5, kc + k);
        loc_add(loc, ST_CLS_M, kind, 5, 1);
        if (tail) {
          loc[ST_CAND_S] += tsz - tm_sz;
          loc[ST_COLS_S] += kc + k;
          // in 16-wide units, like a mid-size class's pairs: four per 32-wide pair
          loc[NC_PAIRS_V] += 4ull * gram_tail_pairs(kc);
          loc[NC_PAIRS_VW] += 4ull * gram_tail_pairs(kc) * w_db;
        }
        // 16-wide block pairs: also a bound on a mid-size class's 32-wide ones
        if (kind == 0) loc[NC_PAIRS_M] += mfma_pairs(kc);
        else if (kind == 3) loc[NC_PAIRS_B] += mfma_pairs(kc, GRAM_TILE_BIG);
        else if (kind == 1 || kind == 4) {
          loc[NC_PAIRS_V] += andpop_pairs(kc);
          loc[NC_PAIRS_VW] += (unsigned long long)andpop_pairs(kc) * w_db;
        }
        else loc[NC_TINY] += 1;
      }
    }
  }
  // the wave's sums, one LDS atomic per counter
#pragma unroll
  for (int j = 0; j < NC_COUNT; ++j) {
    unsigned long long x = loc[j];
    if (__ballot(x != 0)) {
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
      if (lane == 0) atomicAdd(&s_st[j], x);
    }
  }
  __syncthreads();
  if (threadIdx.x < NC_COUNT && s_st[threadIdx.x]) atomicAdd(&st[threadIdx.x], s_st[threadIdx.x]);
}

// The nodes' frequent extensions written into the next level, nb nodes per
// wave as in the node-count kernel: a short row by its node's lane, a long
// one by the whole wave.  Threads [t0, t0 + nt) of a launch take part.
__device__ inline void fill_level_body(const LevelPost& a, uint64_t t0, uint64_t nt) {
  const int lane = threadIdx.x & 63;
  const uint64_t wave0 = t0 >> 6;
  const uint64_t nwaves = nt >> 6;
  const uint32_t nb = a.nb;
  for (uint64_t i0 = wave0 * nb; i0 < a.n; i0 += nwaves * nb) {
    const uint64_t i = i0 + lane;
    uint64_t rs = 0, len = 0, base = 0, ci = 0;  // row, its length, first slot, first child
    uint32_t minsup = 0, db = 0;
    if ((uint32_t)lane < nb && i < a.n) {
      const int32_t c = a.pcls[a.parent[i]];
      if (c >= 0) {
        const ClassDesc cd = a.cls[c];
        const uint64_t li = i - cd.child0;
        if (li + 1 < cd.q) {
          rs = cd.tri_off + tri_index(li, li + 1, cd.q);
          len = cd.q - li - 1;
          minsup = a.dbs[cd.db].minsup;
          base = a.child_start[i];  // the node's children, in row order
          ci = cd.child0 + li + 1;
          db = cd.db;
        }
      }
    }
    if (len <= NODE_LANE_ROW) {
      uint32_t v[NODE_LANE_ROW];
#pragma unroll
      for (uint32_t u = 0; u < NODE_LANE_ROW; ++u) v[u] = u < len ? a.tri[rs + u] : 0u;
#pragma unroll
      for (uint32_t u = 0; u < NODE_LANE_ROW; ++u) {
        if (u < len && v[u] >= minsup) {
          a.nitem[base] = a.child_item[ci + u];
          a.nparent[base] = (uint32_t)i;
          a.nsupp[base] = v[u];
          a.ndbv[base] = db;
          ++base;
        }
      }
    }
    for (uint64_t lm = __ballot(len > NODE_LANE_ROW); lm; lm &= lm - 1) {
      const int j = __builtin_ctzll(lm);
      const uint64_t rj = readlane64(rs, j), lj = readlane64(len, j), cj = readlane64(ci, j);
      uint64_t bj = readlane64(base, j);
      const uint32_t mj = (uint32_t)__builtin_amdgcn_readlane((int)minsup, j);
      const uint32_t dj = (uint32_t)__builtin_amdgcn_readlane((int)db, j);
      const uint32_t ij = (uint32_t)(i0 + (uint64_t)j);
      for (uint64_t t0 = 0; t0 < lj; t0 += 64) {
        const uint64_t t = t0 + lane;
        const uint32_t v = t < lj ? a.tri[rj + t] : 0u;
        const bool f = t < lj && v >= mj;
        const uint64_t m = __ballot(f);
        if (f) {
          const uint64_t pos = bj + (uint64_t)__popcll(m & ((1ull << lane) - 1));
          a.nitem[pos] = a.child_item[cj + t];
          a.nparent[pos] = ij;
          a.nsupp[pos] = v;
          a.ndbv[pos] = dj;
        }
        bj += (uint64_t)__popcll(m);
      }
    }
  }
}

// Task records of one class: block pairs (bi <= bl, row-major) x word splits.
// Lanes stride over the class's tasks.
__device__ void write_tasks(uint32_t ci, uint32_t q, uint32_t npairs, uint32_t block,
                            uint32_t nsplit, uint32_t split_len, uint32_t wend, Task* out,
                            int lane, int nl) {
  const uint32_t nb = (q + block - 1) / block;
  const uint64_t total = (uint64_t)npairs * nsplit;
  for (uint64_t t = lane; t < total; t += nl) {
    uint32_t tp = (uint32_t)(t / nsplit);
    const uint32_t sp = (uint32_t)(t % nsplit);
    uint32_t bi = 0;
    while (tp >= nb - bi) {
      tp -= nb - bi;
      ++bi;
    }
    Task k;
    k.cls = ci;
    k.bi = (uint16_t)bi;
    k.bl = (uint16_t)(bi + tp);
    k.w0 = sp * split_len;
    k.w1 = min(wend, (sp + 1) * split_len);
    out[t] = k;
  }
}

// Word range each kernel covers for a database: MFMA stages need multiples of 16.
__device__ inline uint32_t wend_of(const DbInfo& d, int kind) {
  const uint64_t W = d.W ? d.W : 1;
  if (is_mfma_kind(kind)) return (uint32_t)((W + GRAM_KW - 1) / GRAM_KW * GRAM_KW);
  if (kind == 4) return (uint32_t)((W + GRAM_SMALL_KW - 1) / GRAM_SMALL_KW * GRAM_SMALL_KW);
  return (uint32_t)W;
}

struct ClassWork {
  int kind;
  uint32_t npairs, nsplit, split, block, wend;
  uint32_t qm;                                  // children the kernel's tasks cover
  uint32_t npairs_s, nsplit_s, split_s, wend_s;  // a kind-0 class's narrow tail (32-wide)
};

__device__ inline ClassWork class_work(const ClassDesc& cd, const DbInfo& d, uint32_t mfma_min_q,
                                       const TaskGeom& geo) {
  ClassWork w;
  w.kind = class_kind(cd.q, mfma_min_q, geo.big_q, geo.small_on, geo.tiny_q);
  w.wend = wend_of(d, w.kind);
  w.qm = cd.q;
  w.npairs_s = w.nsplit_s = w.split_s = w.wend_s = 0;
  if (w.kind == 0) {
    if (geo.small_on && !cd.proj && gram_tail(cd.q)) {  // (a projected class keeps its tail)
      w.qm = gram_tail_q(cd.q);
      w.npairs_s = gram_tail_pairs(cd.q);
      w.split_s = geo.split_s;
      w.wend_s = wend_of(d, 4);
      w.nsplit_s = (w.wend_s + w.split_s - 1) / w.split_s;
    }
    w.npairs = mfma_pairs(w.qm);
    w.split = geo.split_m;
    w.block = GRAM_TILE;
  } else if (w.kind == 3) {  // 256 x 256 block pairs
    w.npairs = mfma_pairs(cd.q, GRAM_TILE_BIG);
    w.split = geo.split_b;
    w.block = GRAM_TILE_BIG;
  } else if (w.kind == 4) {
    w.npairs = andpop_pairs(cd.q, GRAM_SMALL_TILE);
    w.split = geo.split_s;
    w.block = GRAM_SMALL_TILE;
  } else if (w.kind == 1) {
    w.npairs = andpop_pairs(cd.q);
    w.split = geo.split_v;
    w.block = AP_BLOCK;
  } else {
    w.npairs = 1;
    w.split = geo.split_t;
    w.block = TINY_Q;
  }
  w.nsplit = (w.wend + w.split - 1) / w.split;
  return w;
}

// Number of tasks of each class, per kernel.  With dfs set, every small class
// becomes one depth-first subtree task instead of level-synchronous tasks.
__global__ void k_class_task_counts(const ClassDesc* __restrict__ cls, uint64_t ncls,
                                    const DbInfo* __restrict__ dbs,
                                    const DbInfo* __restrict__ views, uint32_t mfma_min_q,
                                    TaskGeom geo, uint32_t dfs, uint32_t* __restrict__ cm,
                                    uint32_t* __restrict__ cv, uint32_t* __restrict__ ct,
                                    uint32_t* __restrict__ cb, uint32_t* __restrict__ cs) {
  for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < ncls;
       c += (uint64_t)gridDim.x * blockDim.x) {
    const ClassDesc cd = cls[c];
    const ClassWork w = class_work(cd, class_view(cd, dbs, views), mfma_min_q, geo);
    const uint32_t nt = w.npairs * w.nsplit;
    cm[c] = w.kind == 0 ? nt : 0u;
    cv[c] = w.kind == 1 ? nt : 0u;
    ct[c] = w.kind == 2 ? (dfs ? 1u : nt) : 0u;
    cb[c] = w.kind == 3 ? nt : 0u;
    cs[c] = (w.kind == 4 ? nt : 0u) + w.npairs_s * w.nsplit_s;
  }
}

__global__ void k_task_costs(const Task* __restrict__ tasks, const uint64_t* __restrict__ ntasks,
                             uint64_t ub, uint32_t w_off, uint32_t w_diag,
                             uint32_t* __restrict__ cost) {
  const uint64_t n = *ntasks;
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < ub;
       t += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t c = 0;
    if (t < n) {
      const Task k = tasks[t];
      c = (k.w1 - k.w0) / GRAM_KW * (k.bi == k.bl ? w_diag : w_off);
    }
    cost[t] = c;
  }
}

// Workgroup per class: write its tasks at the scanned offsets (with dfs set, small
// classes become depth-first subtree tasks whose children are level `level`).
__global__ void k_write_class_tasks(const ClassDesc* __restrict__ cls, uint64_t ncls,
                                    const DbInfo* __restrict__ dbs,
                                    const DbInfo* __restrict__ views, uint32_t mfma_min_q,
                                    TaskGeom geo, const uint64_t* __restrict__ om,
                                    const uint64_t* __restrict__ ov, const uint64_t* __restrict__ ot,
                                    Task* __restrict__ tm, Task* __restrict__ tv,
                                    Task* __restrict__ tt, DfsTask* __restrict__ dt,
                                    uint32_t level, const uint64_t* __restrict__ ob,
                                    Task* __restrict__ tb, const uint64_t* __restrict__ os,
                                    Task* __restrict__ ts) {
  // a workgroup per class: a big class has thousands of tasks
  const int lane = threadIdx.x;
  for (uint64_t c = blockIdx.x; c < ncls; c += gridDim.x) {
    const ClassDesc cd = cls[c];
    const ClassWork w = class_work(cd, class_view(cd, dbs, views), mfma_min_q, geo);
    if (w.kind == 2 && dt) {
      if (lane == 0) {
        DfsTask k;
        k.db = cd.db;
        k.level = level;
        k.child0 = cd.child0;
        k.q = cd.q;
        k.pre_off = cd.pre_off;
        k.pre_len = cd.pre_len;
        dt[ot[c]] = k;
      }
      continue;
    }
    Task* out = w.kind == 0 ? tm + om[c]
                : w.kind == 1 ? tv + ov[c]
                : w.kind == 2 ? tt + ot[c]
                : w.kind == 3 ? tb + ob[c]
                              : ts + os[c];
    write_tasks((uint32_t)c, w.qm, w.npairs, w.block, w.nsplit, w.split, w.wend, out, lane,
                (int)blockDim.x);
    if (w.npairs_s) {  // the narrow tail: 32-wide row blocks 0 .. tb against block tb
      const uint32_t tb32 = w.npairs_s - 1;
      const uint64_t total = (uint64_t)w.npairs_s * w.nsplit_s;
      Task* os_out = ts + os[c];
      for (uint64_t t = lane; t < total; t += blockDim.x) {
        const uint32_t p = (uint32_t)(t / w.nsplit_s), sp = (uint32_t)(t % w.nsplit_s);
        Task k;
        k.cls = (uint32_t)c;
        k.bi = (uint16_t)p;
        k.bl = (uint16_t)tb32;
        k.w0 = sp * w.split_s;
        k.w1 = min(w.wend_s, (sp + 1) * w.split_s);
        os_out[t] = k;
      }
    }
  }
}

// A node of level k with >= 2 frequent children becomes a class of the next
// step, whose prefix is the node's itemset.
__device__ inline void fill_classes_body(const LevelPost& a, uint64_t t0, uint64_t nt) {
  const uint32_t k = a.k;
  for (uint64_t i = t0; i < a.n; i += nt) {
    const uint32_t q = a.cnt[i];
    if (q < 2) {
      a.pcls_out[i] = -1;
      continue;
    }
    const uint32_t ci = (uint32_t)a.cls_pos[i];
    a.pcls_out[i] = (int32_t)ci;
    const uint32_t d = a.node_db[i];
    ClassDesc cd;
    cd.tri_off = a.tri_off[i];
    cd.child0 = (uint32_t)a.child_start[i];
    cd.q = q;
    cd.pre_off = ci * k;
    cd.pre_len = k;
    cd.db = d;
    cd.proj = 0;
    DbInfo view = a.dbs[d];
    if (a.views && a.pflag[i]) {
      // the projected view: the children's columns over the prefix's rows,
      // written by the projection kernels before the step's class kernels
      const uint32_t slot = (uint32_t)a.pslot[i];
      const uint64_t sp = a.nodesupp[i];
      cd.proj = slot + 1;
      view.B = a.vbuf + a.pword_off[i];
      view.Wp = view_padded_words(sp);
      view.W = view_words(sp);
      view.n = sp;
      view.f1 = nullptr;
      view.m = q;
      a.views[slot] = view;
      ProjWork pw;
      pw.row_off = a.prow_off[i];
      pw.cls = ci;
      pw.pad = 0;
      a.pwork[slot] = pw;
    }
    a.ocls[ci] = cd;
    {
      const ClassWork w = class_work(cd, view, a.mfma_min_q, a.geo);
      const uint32_t nt = w.npairs * w.nsplit;
      a.cm[ci] = w.kind == 0 ? nt : 0u;
      a.cv[ci] = w.kind == 1 ? nt : 0u;
      a.ct[ci] = w.kind == 2 ? (a.dfs ? 1u : nt) : 0u;
      a.cb[ci] = w.kind == 3 ? nt : 0u;
      a.cs[ci] = (w.kind == 4 ? nt : 0u) + w.npairs_s * w.nsplit_s;
    }
    const uint32_t* f1 = a.dbs[d].f1;
    uint64_t x = i;
    for (int lev = (int)k; lev >= 1; --lev) {
      a.opre[(uint64_t)ci * k + (k - lev)] = f1[a.lv.item[lev][x]];
      x = a.lv.parent[lev][x];
    }
  }
}

// The work between two level steps that depends only on the finished counts,
// in one launch: blocks [0, b_level) write the next level, blocks
// [b_level, b_level + b_cls) the next step's classes (when ocls is set) and
// the remaining blocks zero the next step's support triangle.
__global__ __launch_bounds__(kThreads) void k_level_post(LevelPost a) {
  const uint32_t b = blockIdx.x;
  if (b < a.b_level) {
    fill_level_body(a, (uint64_t)b * kThreads + threadIdx.x, (uint64_t)a.b_level * kThreads);
  } else if (b < a.b_level + a.b_cls) {
    fill_classes_body(a, (uint64_t)(b - a.b_level) * kThreads + threadIdx.x,
                      (uint64_t)a.b_cls * kThreads);
  } else {
    const uint32_t nb = gridDim.x - a.b_level - a.b_cls;
    for (uint64_t i = (uint64_t)(b - a.b_level - a.b_cls) * kThreads + threadIdx.x; i < a.nz;
         i += (uint64_t)nb * kThreads)
      a.ztri[i] = 0u;
  }
}

// ---------------------------------------------------------------- output

// Canonical output in one pass.  Each level's nodes are stored in the
// lexicographic order of their itemsets (children contiguous, in parent
// order), so the depth-first rank of a level-k node v among all itemsets is a
// sum over levels: for every shallower level j, the index of v's level-j
// ancestor plus one (that ancestor and every node before it come first); at
// level k, v's own index; for every deeper level, the index of v's first
// level-j descendant slot (all level-j nodes below earlier level-k nodes come
// first), found by following the child-start arrays down.  The item offset is
// the same sum with each level's count weighted by its itemset length.  With
// no scan over subtree sizes, every node is placed independently.
//
// Threads past the F itemsets compute, for each database d (and d = N), the
// first level-k node of d on every level -- the descendants of d's first
// frequent item, followed down the same way -- and from those the first
// itemset and first item id of d's slice of the output.
__global__ __launch_bounds__(kThreads) void k_emit_all(EmitArgs a, uint64_t F) {
  const uint32_t K = a.K;
  const uint64_t total = F + a.N + 1;
  for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < total;
       g += (uint64_t)gridDim.x * blockDim.x) {
    if (g < F) {
      uint32_t k = 1;
      while (a.base[k + 1] <= g) ++k;
      const uint64_t i = g - a.base[k];
      uint64_t pos = i, ioff = (uint64_t)k * i, x = i;
      for (uint32_t j = k; j < K; ++j) {
        x = a.cstart[j][x];
        pos += x;
        ioff += (uint64_t)(j + 1) * x;
      }
      uint64_t y = i;
      for (uint32_t j = k; j >= 2; --j) {
        y = a.parent[j][y];
        pos += y + 1;
        ioff += (uint64_t)(j - 1) * (y + 1);
      }
      a.o_off[pos] = ioff;
      a.o_supp[pos] = a.supp[k][i];
      const uint32_t* f1 = a.dbs[a.node_db[k][i]].f1;
      y = i;
      for (uint32_t j = k; j >= 1; --j) {
        a.o_items[ioff + j - 1] = f1[a.item[j][y]];
        if (j > 1) y = a.parent[j][y];
      }
    } else {
      const uint32_t d = (uint32_t)(g - F);
      const uint64_t rows = (uint64_t)a.N + 1;
      uint64_t x = a.first_root[d];
      uint64_t fs = x, is = x;
      a.bounds[rows + d] = x;
      for (uint32_t j = 1; j < K; ++j) {
        x = a.cstart[j][x];
        a.bounds[(uint64_t)(j + 1) * rows + d] = x;
        fs += x;
        is += (uint64_t)(j + 1) * x;
      }
      a.slices[d] = fs;
      a.slices[rows + d] = is;
      if (d == a.N) a.o_off[F] = is;
    }
  }
}

__global__ void k_rebase(const uint64_t* __restrict__ src, uint64_t n, uint64_t base,
                         uint64_t* __restrict__ dst) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i] - base;
}

__global__ void k_expand_pairs(uint32_t k, const uint32_t* __restrict__ items,
                               const uint32_t* __restrict__ colsum, const uint32_t* __restrict__ tri,
                               uint32_t* __restrict__ out) {
  const uint64_t total = (uint64_t)k * k;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t a = e / k, b = e % k;
    uint32_t v;
    if (a == b) v = colsum[items[a]];
    else v = tri[a < b ? tri_index(a, b, k) : tri_index(b, a, k)];
    out[e] = v;
  }
}

struct Words64 {
  uint32_t w[kWriteWordsMax];
};

__global__ void k_write_words(uint32_t* __restrict__ dst, Words64 v, uint32_t n) {
  const uint32_t i = threadIdx.x;
  if (i < n) dst[i] = v.w[i];
}

__global__ void k_iota_u32(uint32_t* __restrict__ dst, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    dst[i] = i;
}

}  // namespace

void launch_write_words(uint32_t* dst, const uint32_t* words, uint32_t n, hipStream_t s) {
  if (n == 0) return;
  Words64 v{};
  for (uint32_t i = 0; i < n; ++i) v.w[i] = words[i];
  k_write_words<<<1, kWriteWordsMax, 0, s>>>(dst, v, n);
  BM_LAUNCH_CHECK();
}

void launch_iota_u32(uint32_t* dst, uint32_t n, hipStream_t s) {
  if (n == 0) return;
  k_iota_u32<<<grid_for(n, kThreads), kThreads, 0, s>>>(dst, n);
  BM_LAUNCH_CHECK();
}

void launch_f1_flags(const DbInfo* dbs, uint32_t ndb, const uint64_t* item_base, uint64_t total,
                     uint32_t* flags, hipStream_t s) {
  if (total == 0) return;
  k_f1_flags<<<grid_for(total, kThreads), kThreads, 0, s>>>(dbs, ndb, item_base, total, flags);
  BM_LAUNCH_CHECK();
}

void launch_f1_fill(const uint32_t* flags, const uint64_t* pos, uint32_t ndb,
                    const uint64_t* item_base, uint64_t total, uint32_t* f1, hipStream_t s) {
  if (total == 0) return;
  k_f1_fill<<<grid_for(total, kThreads), kThreads, 0, s>>>(flags, pos, ndb, item_base, total, f1);
  BM_LAUNCH_CHECK();
}

void launch_init_level1(DbInfo* dbs, uint32_t ndb, const uint64_t* f1_base, uint64_t n1,
                        const uint32_t* f1, uint32_t* item, uint32_t* parent, uint32_t* supp,
                        uint32_t* ndbv, hipStream_t s) {
  if (n1 == 0 && ndb == 0) return;
  k_init_level1<<<grid_for(std::max<uint64_t>(n1, ndb), kThreads), kThreads, 0, s>>>(
      dbs, ndb, f1_base, n1, f1, item, parent, supp, ndbv);
  BM_LAUNCH_CHECK();
}

void launch_gather_idx(const uint64_t* arr, const uint64_t* idx, uint32_t k, uint64_t* out,
                       uint64_t* out2, hipStream_t s) {
  if (k == 0) return;
  k_gather_idx<<<grid_for(k, kThreads), kThreads, 0, s>>>(arr, idx, k, out, out2);
  BM_LAUNCH_CHECK();
}


void launch_node_counts(uint64_t n, uint32_t nb, uint32_t k, const uint32_t* parent,
                        const int32_t* pcls, const ClassDesc* cls, const DbInfo* dbs,
                        const uint32_t* tri, uint32_t mfma_min_q, uint32_t big_q, uint32_t small_on,
                        uint32_t tiny_q, uint32_t* cnt, uint32_t* is_cls, uint64_t* tri_sz,
                        unsigned long long* st, const uint32_t* supp, uint32_t proj_on,
                        uint32_t* pflag, uint32_t* prows, uint64_t* pwords, hipStream_t s) {
  if (n == 0) return;
  if (nb == 0 || nb > 64) fail(BM_ERR_INVALID_ARG, "node batch %u outside 1..64", nb);
  // at most 1,024 workgroups: each ends with a few device-wide atomic adds
  // on the same counters, and with 4,096 of them those serialised (T40-style
  // level steps 0.46 ms per mine call, against 0.40 with 1,024 and 0.41 with
  // 256; 256 cost the batch of 256 databases 9% on this kernel)
  k_node_counts<<<grid_for((n + nb - 1) / nb, kThreads / 64, 1024), kThreads, 0, s>>>(
      n, nb, k, parent, pcls, cls, dbs, tri, mfma_min_q, big_q, small_on, tiny_q, cnt, is_cls,
      tri_sz, st, supp, proj_on, pflag, prows, pwords);
  BM_LAUNCH_CHECK();
}

void launch_level_post(LevelPost a, hipStream_t s) {
  if (a.n == 0) return;
  if (a.nb == 0 || a.nb > 64) fail(BM_ERR_INVALID_ARG, "node batch %u outside 1..64", a.nb);
  a.b_level = grid_for((a.n + a.nb - 1) / a.nb * 64, kThreads);
  a.b_cls = a.ocls ? grid_for(a.n, kThreads) : 0u;
  const uint32_t bz = a.nz ? grid_for(a.nz, kThreads, 16384) : 0u;
  k_level_post<<<a.b_level + a.b_cls + bz, kThreads, 0, s>>>(a);
  BM_LAUNCH_CHECK();
}

void launch_class_task_counts(const ClassDesc* cls, uint64_t ncls, const DbInfo* dbs,
                              const DbInfo* views, uint32_t mfma_min_q, const TaskGeom& geo,
                              bool dfs, uint32_t* cm, uint32_t* cv, uint32_t* ct, uint32_t* cb,
                              uint32_t* cs, hipStream_t s) {
  if (ncls == 0) return;
  k_class_task_counts<<<grid_for(ncls, kThreads), kThreads, 0, s>>>(cls, ncls, dbs, views,
                                                                     mfma_min_q, geo,
                                                                     dfs ? 1u : 0u, cm, cv, ct, cb,
                                                                     cs);
  BM_LAUNCH_CHECK();
}

void launch_write_class_tasks(const ClassDesc* cls, uint64_t ncls, const DbInfo* dbs,
                              const DbInfo* views, uint32_t mfma_min_q, const TaskGeom& geo,
                              const uint64_t* om,
                              const uint64_t* ov, const uint64_t* ot, Task* tm, Task* tv, Task* tt,
                              DfsTask* dt, uint32_t level, const uint64_t* ob, Task* tb,
                              const uint64_t* os, Task* ts, hipStream_t s) {
  if (ncls == 0) return;
  k_write_class_tasks<<<grid_for(ncls, 1), kThreads, 0, s>>>(
      cls, ncls, dbs, views, mfma_min_q, geo, om, ov, ot, tm, tv, tt, dt, level, ob, tb, os, ts);
  BM_LAUNCH_CHECK();
}

void launch_task_costs(const Task* tasks, const uint64_t* ntasks, uint64_t ub, uint32_t w_off,
                       uint32_t w_diag, uint32_t* cost, hipStream_t s) {
  if (ub == 0) return;
  k_task_costs<<<grid_for(ub, kThreads), kThreads, 0, s>>>(tasks, ntasks, ub, w_off, w_diag, cost);
  BM_LAUNCH_CHECK();
}

void launch_emit_all(const EmitArgs& a, uint64_t F, hipStream_t s) {
  k_emit_all<<<grid_for(F + a.N + 1, kThreads), kThreads, 0, s>>>(a, F);
  BM_LAUNCH_CHECK();
}

void launch_rebase(const uint64_t* src, uint64_t n, uint64_t base, uint64_t* dst, hipStream_t s) {
  if (n == 0) return;
  k_rebase<<<grid_for(n, kThreads), kThreads, 0, s>>>(src, n, base, dst);
  BM_LAUNCH_CHECK();
}

void launch_expand_pairs(uint32_t k, const uint32_t* items, const uint32_t* colsum,
                         const uint32_t* tri, uint32_t* out, hipStream_t s) {
  const uint64_t total = (uint64_t)k * k;
  if (total == 0) return;
  k_expand_pairs<<<grid_for(total, kThreads), kThreads, 0, s>>>(k, items, colsum, tri, out);
  BM_LAUNCH_CHECK();
}

}  // namespace bm
