// Persistent depth-first mining of small prefix classes, fed from a device
// work queue, and the merge of its output with the level-synchronous levels.
//
// A prefix class with at most TINY_Q frequent children only has small classes
// below it (a child's class holds a subset of its later siblings), so its
// whole subtree is mined by one workgroup:
//   * workgroups pop subtree tasks from a queue (an atomic head over an order
//     array: plain order, or longest-predicted-first from the cost model);
//   * each workgroup keeps a private stack of classes in LDS.  Evaluating a
//     class streams the prefix columns and the child columns once, ANDs them
//     word by word and popcounts every child pair (the sequential AND of the
//     method), reduces the pair counts across the workgroup, then records the
//     frequent extensions of every child in an output arena and pushes the
//     children that have two or more of them as new classes;
//   * a workgroup exits when its stack is empty and the queue is exhausted --
//     no workgroup ever waits for another, so the kernel always drains.
// The arena links every node to its block of children; reconstruction merges
// those blocks with the level-synchronous levels into final levels in
// canonical order.
#include "internal.hpp"
#include "levels.hpp"
#include "dfs.hpp"

namespace bm {

namespace {

constexpr int kThreads = 256;  // helper kernels
constexpr int TQ = TINY_Q;
constexpr int TNP = TQ * (TQ - 1) / 2;
constexpr int SCAP = 32;  // stack entries: <= 6 + 5 + ... + 1 pending classes

uint32_t grid_for(uint64_t work, uint32_t per_block, uint32_t cap = 65535) {
  uint64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

struct Entry {
  uint32_t pre_len;              // prefix length; children are itemsets of length pre_len + 1
  uint32_t q;                    // children
  uint32_t ls_level;             // != 0: children are level-synchronous nodes of this level
  uint32_t db;
  uint32_t item[TQ];             // frequent-item index of each child
  uint32_t node[TQ];             // child's node: level-synchronous index or arena index
  uint32_t pre[BM_MAX_LEVELS];   // prefix column ids
};

__device__ inline int pair_slot(int i, int l) { return i * (2 * TQ - i - 1) / 2 + (l - i - 1); }

// Inclusive sum over the first TQ lanes of a wavefront (other lanes pass 0).
__device__ inline uint32_t lane_scan(uint32_t x, int lane) {
#pragma unroll
  for (int off = 1; off < TQ; off <<= 1) {
    const uint32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  return x;
}

// Per-worker bookkeeping kept in LDS and written by one lane only: level
// statistics are summed locally and flushed once at exit, and arena space is
// reserved ARENA_CHUNK nodes at a time, so the classes of a subtree touch no
// device-wide counter (about a hundred thousand classes would otherwise
// serialise on a handful of addresses).
constexpr uint32_t ARENA_CHUNK = 256;

struct WorkerStats {
  unsigned long long cand[BM_MAX_LEVELS + 1];
  unsigned long long freq[BM_MAX_LEVELS + 1];
  unsigned long long words;
  uint32_t next, end;  // free arena range reserved by this worker
};

__device__ inline void ws_init(WorkerStats& w, int lane, int nl) {
  for (int j = lane; j <= BM_MAX_LEVELS; j += nl) {
    w.cand[j] = 0;
    w.freq[j] = 0;
  }
  if (lane == 0) {
    w.words = 0;
    w.next = 0;
    w.end = 0;
  }
}

__device__ inline void ws_flush(const WorkerStats& w, const DfsArgs& a, int lane, int nl) {
  for (int j = lane; j <= BM_MAX_LEVELS; j += nl) {
    if (w.cand[j]) atomicAdd(&a.level_cand[j], w.cand[j]);
    if (w.freq[j]) atomicAdd(&a.level_freq[j], w.freq[j]);
  }
  if (lane == 0 && w.words) atomicAdd(a.words_read, w.words);
}

// Arena block of `total` nodes for one class, from the worker's reserved range
// (a new range when it runs out).  false: the arena is full (the call retries
// with a bigger one; the reservation counter tells the host how big).
__device__ inline bool ws_alloc(WorkerStats& w, const DfsArgs& a, uint32_t total, uint32_t* base) {
  if (w.next + total > w.end) {
    const uint32_t want = total > ARENA_CHUNK ? total : ARENA_CHUNK;
    const uint32_t b = atomicAdd(a.arena_count, want);
    if (b + want > a.arena_cap) return false;
    w.next = b;
    w.end = b + want;
  }
  *base = w.next;
  w.next += total;
  return true;
}

template <int NT>
__global__ __launch_bounds__(NT) void k_dfs(DfsArgs a) {
  constexpr int NW = NT / 64;
  __shared__ Entry s_stack[SCAP];
  __shared__ Entry s_cur;
  __shared__ int s_sp;
  __shared__ uint32_t s_task;
  __shared__ uint32_t s_red[NW][TNP];
  __shared__ uint32_t s_cnt[TNP];
  __shared__ unsigned long long s_task_cost;  // column words streamed by the current task
  __shared__ int s_done;
  __shared__ WorkerStats s_ws;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) {
    s_sp = 0;
    s_done = 0;
  }
  ws_init(s_ws, tid, NT);
  __syncthreads();
  for (;;) {
    // ---- next class: from the stack, else a new task from the queue
    if (tid == 0) {
      if (s_sp == 0) {
        const uint32_t t = atomicAdd(a.queue_head, 1u);
        if (t >= (a.ntasks_dev ? *a.ntasks_dev : a.ntasks)) {
          s_done = 1;
        } else {
          const uint32_t ti = a.order ? a.order[t] : t;
          s_task = ti;
          s_task_cost = 0;
          const DfsTask tk = a.tasks[ti];
          Entry& e = s_stack[0];
          e.pre_len = tk.pre_len;
          e.q = tk.q;
          e.ls_level = tk.level;
          e.db = tk.db;
          const uint32_t* lit = a.lv_item[tk.level];
          for (uint32_t i = 0; i < TQ; ++i) {
            e.item[i] = i < tk.q ? lit[tk.child0 + i] : 0u;
            e.node[i] = tk.child0 + i;
          }
          const uint32_t* pre = a.step_pre[tk.level] + tk.pre_off;
          for (uint32_t j = 0; j < tk.pre_len; ++j) e.pre[j] = pre[j];
          s_sp = 1;
        }
      }
      if (!s_done) {
        s_sp -= 1;
        s_cur = s_stack[s_sp];
      }
    }
    __syncthreads();
    if (s_done) {
      ws_flush(s_ws, a, tid, NT);
      break;
    }

    // ---- evaluate every child pair of the class over all words
    const Entry& c = s_cur;
    const DbInfo db = a.dbs[c.db];
    const int q = (int)c.q;
    const uint64_t* col[TQ];
#pragma unroll
    for (int i = 0; i < TQ; ++i)
      col[i] = db.B + (uint64_t)(i < q ? db.f1[c.item[i]] : 0u) * db.Wp;
    uint32_t acc[TNP];
#pragma unroll
    for (int p = 0; p < TNP; ++p) acc[p] = 0;
    const uint32_t W = (uint32_t)db.W;
    const uint32_t pre_len = c.pre_len;
    const uint64_t* pc[PREFIX_REG];
#pragma unroll
    for (int j = 0; j < PREFIX_REG; ++j)
      pc[j] = (uint32_t)j < pre_len ? db.B + (uint64_t)c.pre[j] * db.Wp : nullptr;
    // two words per thread: columns are padded to a multiple of 64 words, so
    // the 16-byte load at an even word stays inside the column
    for (uint32_t w = 2 * tid; w < W; w += 2 * NT) {
      uint64_t m0 = ~0ull, m1 = (w + 1 < W) ? ~0ull : 0ull;
      prefix_and(pc, db.B, db.Wp, c.pre, pre_len, w, m0, m1);
      uint64_t x0[TQ], x1[TQ];
#pragma unroll
      for (int i = 0; i < TQ; ++i) {
        x0[i] = 0;
        x1[i] = 0;
        if (i < q) {
          const uint4 v = load_global16(col[i] + w);
          x0[i] = ((uint64_t)v.x | ((uint64_t)v.y << 32)) & m0;
          x1[i] = ((uint64_t)v.z | ((uint64_t)v.w << 32)) & m1;
        }
      }
      int p = 0;
#pragma unroll
      for (int i = 0; i < TQ; ++i)
#pragma unroll
        for (int l = i + 1; l < TQ; ++l, ++p)
          if (l < q) acc[p] += (uint32_t)(__popcll(x0[i] & x0[l]) + __popcll(x1[i] & x1[l]));
    }
#pragma unroll
    for (int p = 0; p < TNP; ++p) {
      uint32_t v = acc[p];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) s_red[wave][p] = v;
    }
    __syncthreads();
    if (tid < TNP) {
      uint32_t v = 0;
#pragma unroll
      for (int j = 0; j < NW; ++j) v += s_red[j][tid];
      s_cnt[tid] = v;
    }
    __syncthreads();

    // ---- record frequent extensions (lane i of wave 0 handles child i), push
    // the children that form classes
    if (wave == 0) {
      const int i = lane;
      const uint32_t minsup = db.minsup;
      const uint32_t len = c.pre_len + 2;  // length of the candidate itemsets
      uint32_t mask = 0;                   // bit l: extension of child i by sibling l is frequent
      if (i < q)
        for (int l = i + 1; l < q; ++l)
          if (s_cnt[pair_slot(i, l)] >= minsup) mask |= 1u << l;
      const uint32_t nf = (uint32_t)__popc(mask);
      const uint32_t incl = lane_scan(i < TQ ? nf : 0u, lane);
      const uint32_t total = __shfl(incl, TQ - 1);
      uint32_t base = 0, ok = total > 0 ? 1u : 0u;
      if (lane == 0) {
        const uint64_t ncand = (uint64_t)q * (q - 1) / 2;
        const unsigned long long words = (unsigned long long)(c.pre_len + q) * db.W;
        s_task_cost += words;
        if (len <= BM_MAX_LEVELS) s_ws.cand[len] += ncand;
        s_ws.words += words;
        if (total) {
          if (len > BM_MAX_LEVELS) {
            atomicOr(a.flags, DFS_TOO_LONG);
            ok = 0;
          } else if (!ws_alloc(s_ws, a, total, &base)) {
            atomicOr(a.flags, DFS_OVERFLOW);
            ok = 0;
          } else {
            s_ws.freq[len] += total;
          }
        }
      }
      base = __shfl(base, 0);
      ok = __shfl(ok, 0);
      const uint32_t cnt = ok ? nf : 0u;
      const uint32_t first = base + incl - nf;
      const int sp0 = s_sp;
      const uint32_t push = (i < q && cnt >= 2) ? 1u : 0u;
      const uint32_t pincl = lane_scan(i < TQ ? push : 0u, lane);
      const uint32_t npush = __shfl(pincl, TQ - 1);
      if (i < q) {
        uint32_t mm = ok ? mask : 0u;
        for (uint32_t r = 0; mm; ++r) {
          const int l = __ffs(mm) - 1;
          mm &= mm - 1;
          ArenaNode an;
          an.item = c.item[l];
          an.supp = s_cnt[pair_slot(i, l)];
          an.first = 0;
          an.count = 0;
          a.arena[first + r] = an;
        }
        // link the child's block of children
        if (c.ls_level) {
          a.ls_first[c.ls_level][c.node[i]] = first;
          a.ls_count[c.ls_level][c.node[i]] = cnt;
        } else {
          a.arena[c.node[i]].first = first;
          a.arena[c.node[i]].count = cnt;
        }
        if (push) {
          const int slot = sp0 + (int)(pincl - 1);
          if (slot < SCAP) {
            Entry& e = s_stack[slot];
            e.pre_len = c.pre_len + 1;
            e.q = cnt;
            e.ls_level = 0;
            e.db = c.db;
            for (uint32_t j = 0; j < c.pre_len; ++j) e.pre[j] = c.pre[j];
            e.pre[c.pre_len] = db.f1[c.item[i]];
            uint32_t m2 = mask;
            for (uint32_t r = 0; r < TQ; ++r) {
              uint32_t it = 0;
              if (m2) {
                it = c.item[__ffs(m2) - 1];
                m2 &= m2 - 1;
              }
              e.item[r] = it;
              e.node[r] = first + r;
            }
          } else {
            atomicOr(a.flags, DFS_STACK);
          }
        }
      }
      if (lane == 0) {
        const int sp = min(sp0 + (int)npush, SCAP);
        s_sp = sp;
        if (sp == 0 && a.task_cost) a.task_cost[s_task] = (float)s_task_cost;
      }
    }
    __syncthreads();
  }
}

// Orders one wave's LDS writes before its own later reads (and reads before
// later writes): a wave's LDS operations are performed in issue order, and the
// fence keeps the compiler from moving them across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

constexpr int WSCAP = 24;  // stack entries per wave: <= 6 + 5 + ... + 1 pending classes

// Depth-first subtrees with one stack per wave.  The class evaluation is the
// workgroup kernel's, shrunk to a wave: 64 lanes stream two words each per
// step, the 28 pair counts are reduced by a transposing butterfly (lane 2p
// ends up with pair p after 32 shuffles), and lane i records child i.  No
// workgroup barrier is ever taken, so four waves per workgroup mine four
// subtrees independently.  Three workgroups per CU: 144 VGPRs and no spills
// (the 128-VGPR bound of four spilled 12 registers and measured 5% slower on
// the batch of 256 databases).
__global__ __launch_bounds__(256, 3) void k_dfs_wave(DfsArgs a) {
  __shared__ Entry s_stack[4][WSCAP];
  __shared__ uint32_t s_pre[4][BM_MAX_LEVELS];
  __shared__ WorkerStats s_ws[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  Entry* stk = s_stack[wv];
  uint32_t* cpre = s_pre[wv];
  WorkerStats& ws = s_ws[wv];
  ws_init(ws, lane, 64);
  wave_lds_sync();
  const uint32_t ntasks = a.ntasks_dev ? *a.ntasks_dev : a.ntasks;
  int sp = 0;                    // wave-uniform
  uint32_t task = 0;
  unsigned long long tcost = 0;  // column words streamed by the current task
  for (;;) {
    uint32_t pre_len, q, ls_level, dbi, my_item = 0, my_node = 0;
    if (sp == 0) {
      uint32_t t = 0;
      if (lane == 0) t = atomicAdd(a.queue_head, 1u);
      t = __shfl(t, 0);
      if (t >= ntasks) {
        wave_lds_sync();
        ws_flush(ws, a, lane, 64);
        break;
      }
      task = a.order ? a.order[t] : t;
      tcost = 0;
      const DfsTask tk = a.tasks[task];
      pre_len = tk.pre_len;
      q = tk.q;
      ls_level = tk.level;
      dbi = tk.db;
      if (lane < (int)q) {
        my_item = a.lv_item[tk.level][tk.child0 + lane];
        my_node = tk.child0 + lane;
      }
      const uint32_t* pre = a.step_pre[tk.level] + tk.pre_off;
      if (lane < (int)pre_len) cpre[lane] = pre[lane];
    } else {
      sp -= 1;
      const Entry& e = stk[sp];
      pre_len = e.pre_len;
      q = e.q;
      ls_level = e.ls_level;
      dbi = e.db;
      if (lane < TQ) {
        my_item = e.item[lane];
        my_node = e.node[lane];
      }
      wave_lds_sync();  // every lane has read the entry before cpre is rewritten
      if (lane < (int)pre_len) cpre[lane] = e.pre[lane];
    }
    wave_lds_sync();

    // ---- evaluate every child pair over all words
    const DbInfo db = a.dbs[dbi];
    const unsigned long long mycol =
        lane < (int)q ? (unsigned long long)db.f1[my_item] * db.Wp : 0ull;
    const uint64_t* col[TQ];
#pragma unroll
    for (int i = 0; i < TQ; ++i) col[i] = db.B + __shfl(mycol, i);
    uint32_t acc[TNP];
#pragma unroll
    for (int p = 0; p < TNP; ++p) acc[p] = 0;
    const uint32_t W = (uint32_t)db.W;
    const int qi = (int)q;
    const uint64_t* pc[PREFIX_REG];
#pragma unroll
    for (int j = 0; j < PREFIX_REG; ++j)
      pc[j] = (uint32_t)j < pre_len ? db.B + (uint64_t)cpre[j] * db.Wp : nullptr;
    for (uint32_t w = 2 * lane; w < W; w += 128) {
      uint64_t m0 = ~0ull, m1 = (w + 1 < W) ? ~0ull : 0ull;
      prefix_and(pc, db.B, db.Wp, cpre, pre_len, w, m0, m1);
      uint64_t x0[TQ], x1[TQ];
#pragma unroll
      for (int i = 0; i < TQ; ++i) {
        x0[i] = 0;
        x1[i] = 0;
        if (i < qi) {
          const uint4 v = load_global16(col[i] + w);
          x0[i] = ((uint64_t)v.x | ((uint64_t)v.y << 32)) & m0;
          x1[i] = ((uint64_t)v.z | ((uint64_t)v.w << 32)) & m1;
        }
      }
      int p = 0;
#pragma unroll
      for (int i = 0; i < TQ; ++i)
#pragma unroll
        for (int l = i + 1; l < TQ; ++l, ++p)
          if (l < qi) acc[p] += (uint32_t)(__popcll(x0[i] & x0[l]) + __popcll(x1[i] & x1[l]));
    }
    // transposing reduction: after the step with distance d a lane keeps the
    // half of its values selected by (lane & d) and adds its partner's copy
    uint32_t v[32];
#pragma unroll
    for (int p = 0; p < 32; ++p) v[p] = p < TNP ? acc[p] : 0u;
#pragma unroll
    for (int d = 32, n = 16; d >= 2; d >>= 1, n >>= 1) {
      const bool up = (lane & d) != 0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (k < n) {
          const uint32_t send = up ? v[k] : v[k + n];
          const uint32_t keep = up ? v[k + n] : v[k];
          v[k] = keep + __shfl_xor(send, d);
        }
      }
    }
    const uint32_t pair_total = v[0] + __shfl_xor(v[0], 1);  // lanes 2p, 2p+1: pair p

    // ---- record frequent extensions (lane i: child i), push new classes
    const uint32_t minsup = db.minsup;
    const uint32_t len = pre_len + 2;
    uint32_t cnt_l[TQ], item_l[TQ];
    uint32_t mask = 0;
#pragma unroll
    for (int l = 0; l < TQ; ++l) {
      item_l[l] = __shfl(my_item, l);
      const int src = (lane < l) ? 2 * pair_slot(lane, l) : 0;
      cnt_l[l] = __shfl(pair_total, src);
      if (lane < l && l < qi && cnt_l[l] >= minsup) mask |= 1u << l;
    }
    const int i = lane;
    const uint32_t nf = (uint32_t)__popc(mask);
    const uint32_t incl = lane_scan(i < TQ ? nf : 0u, lane);
    const uint32_t total = __shfl(incl, TQ - 1);
    uint32_t base = 0, ok = total > 0 ? 1u : 0u;
    if (lane == 0) {
      const uint64_t ncand = (uint64_t)q * (q - 1) / 2;
      const unsigned long long words = (unsigned long long)(pre_len + q) * db.W;
      if (len <= BM_MAX_LEVELS) ws.cand[len] += ncand;
      ws.words += words;
      if (total) {
        if (len > BM_MAX_LEVELS) {
          atomicOr(a.flags, DFS_TOO_LONG);
          ok = 0;
        } else if (!ws_alloc(ws, a, total, &base)) {
          atomicOr(a.flags, DFS_OVERFLOW);
          ok = 0;
        } else {
          ws.freq[len] += total;
        }
      }
    }
    tcost += (unsigned long long)(pre_len + q) * db.W;
    base = __shfl(base, 0);
    ok = __shfl(ok, 0);
    const uint32_t cnt = ok ? nf : 0u;
    const uint32_t first = base + incl - nf;
    const uint32_t push = (i < qi && cnt >= 2) ? 1u : 0u;
    const uint32_t pincl = lane_scan(i < TQ ? push : 0u, lane);
    const uint32_t npush = __shfl(pincl, TQ - 1);
    wave_lds_sync();  // cpre fully read by the word loop before entries copy it
    if (i < qi) {
      if (ok) {
        uint32_t r = 0;
#pragma unroll
        for (int l = 0; l < TQ; ++l) {
          if ((mask >> l) & 1u) {
            ArenaNode an;
            an.item = item_l[l];
            an.supp = cnt_l[l];
            an.first = 0;
            an.count = 0;
            a.arena[first + r] = an;
            ++r;
          }
        }
      }
      if (ls_level) {
        a.ls_first[ls_level][my_node] = first;
        a.ls_count[ls_level][my_node] = cnt;
      } else {
        a.arena[my_node].first = first;
        a.arena[my_node].count = cnt;
      }
      if (push) {
        const int slot = sp + (int)(pincl - 1);
        if (slot < WSCAP) {
          Entry& e = stk[slot];
          e.pre_len = pre_len + 1;
          e.q = cnt;
          e.ls_level = 0;
          e.db = dbi;
          for (uint32_t j = 0; j < pre_len; ++j) e.pre[j] = cpre[j];
          e.pre[pre_len] = db.f1[my_item];
          uint32_t r = 0;
#pragma unroll
          for (int l = 0; l < TQ; ++l) {
            if ((mask >> l) & 1u) {
              e.item[r] = item_l[l];
              ++r;
            }
          }
          for (uint32_t k = 0; k < TQ; ++k) {
            if (k >= r) e.item[k] = 0u;
            e.node[k] = first + k;
          }
        } else {
          atomicOr(a.flags, DFS_STACK);
        }
      }
    }
    sp = min(sp + (int)npush, WSCAP);
    if (sp == 0 && lane == 0 && a.task_cost) a.task_cost[task] = (float)tcost;
    wave_lds_sync();
  }
}

}  // namespace

}  // namespace bm

namespace bm {

namespace {

// log2 of a positive count, 0 for zero.
__device__ inline float lg(float x) { return x > 0.f ? __log2f(x) : 0.f; }

__global__ void k_dfs_features(FeatArgs a) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < a.ntasks; t += gridDim.x * blockDim.x) {
    const DfsTask tk = a.tasks[t];
    const DbInfo db = a.dbs[tk.db];
    const uint32_t* sup = a.lv_supp[tk.level];
    float sp = (float)db.n;
    if (tk.level > 1) sp = (float)a.lv_supp[tk.level - 1][a.lv_parent[tk.level][tk.child0]];
    float mlog = 0.f, mx = 0.f, mean = 0.f;
    for (uint32_t i = 0; i < tk.q; ++i) {
      const float s = (float)sup[tk.child0 + i];
      mlog += lg(s);
      const float r = sp > 0.f ? s / sp : 0.f;
      mx = fmaxf(mx, r);
      mean += r;
    }
    const float q = (float)tk.q;
    float* f = a.feats + (uint64_t)t * 8;
    f[0] = (float)tk.level;
    f[1] = lg(sp);
    f[2] = lg(1.f + q);
    f[3] = mlog / q;
    f[4] = mx;
    f[5] = mean / q;
    f[6] = lg((float)db.minsup);
    f[7] = lg((float)(db.W ? db.W : 1));
  }
}

constexpr int kBuckets = 256;

__device__ inline uint32_t bucket_of(float key) {
  // descending order: larger predicted cost -> smaller bucket index
  int b = (int)(key * 8.0f);
  b = b < 0 ? 0 : (b > kBuckets - 1 ? kBuckets - 1 : b);
  return (uint32_t)(kBuckets - 1 - b);
}

// Counting sort of tasks by bucket, descending predicted cost.  Per-workgroup
// LDS counts keep global atomics to one per (workgroup, bucket): the keys of
// many tasks fall into a handful of buckets.
__global__ void k_bucket_hist(const float* __restrict__ key, uint32_t n, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kBuckets];
  for (int b = threadIdx.x; b < kBuckets; b += blockDim.x) h[b] = 0;
  __syncthreads();
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    atomicAdd(&h[bucket_of(key[t])], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < kBuckets; b += blockDim.x)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// Each workgroup takes a contiguous chunk: count its tasks per bucket, reserve
// a range of each bucket with one atomic, then place the tasks.
__global__ void k_bucket_scatter(const float* __restrict__ key, uint32_t n, uint32_t chunk,
                                 unsigned long long* __restrict__ cursor, uint32_t* __restrict__ order) {
  __shared__ uint32_t cnt[kBuckets];
  __shared__ unsigned long long base[kBuckets];
  const uint32_t c0 = blockIdx.x * chunk, c1 = min(n, c0 + chunk);
  for (int b = threadIdx.x; b < kBuckets; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  for (uint32_t t = c0 + threadIdx.x; t < c1; t += blockDim.x) atomicAdd(&cnt[bucket_of(key[t])], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < kBuckets; b += blockDim.x) {
    base[b] = cnt[b] ? atomicAdd(&cursor[b], (unsigned long long)cnt[b]) : 0ull;
    cnt[b] = 0;
  }
  __syncthreads();
  for (uint32_t t = c0 + threadIdx.x; t < c1; t += blockDim.x) {
    const uint32_t b = bucket_of(key[t]);
    order[base[b] + atomicAdd(&cnt[b], 1u)] = t;
  }
}

__global__ void k_dfs_short_flags(const DfsTask* __restrict__ tasks, const DbInfo* __restrict__ dbs,
                                  const uint32_t* __restrict__ order, uint32_t n, uint32_t max_words,
                                  uint32_t* __restrict__ flags) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const uint32_t ti = order ? order[t] : t;
    flags[t] = dbs[tasks[ti].db].W <= max_words ? 1u : 0u;
  }
}

__global__ void k_dfs_split(const uint32_t* __restrict__ order, uint32_t n,
                            const uint32_t* __restrict__ flags, const uint64_t* __restrict__ pos,
                            uint32_t* __restrict__ short_, uint32_t* __restrict__ long_,
                            uint32_t* __restrict__ counts) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t <= n; t += gridDim.x * blockDim.x) {
    if (t == n) {
      counts[0] = (uint32_t)pos[n];
      counts[1] = n - (uint32_t)pos[n];
    } else {
      const uint32_t ti = order ? order[t] : t;
      if (flags[t]) short_[pos[t]] = ti;
      else long_[t - pos[t]] = ti;
    }
  }
}

__device__ inline void source_of_ls(uint64_t i, const uint64_t* cstart, const uint32_t* ls_first,
                                    const uint32_t* ls_count, uint32_t* kind, uint32_t* first,
                                    uint32_t* count) {
  *kind = SRC_NONE;
  *first = 0;
  *count = 0;
  if (cstart) {
    const uint64_t a = cstart[i], b = cstart[i + 1];
    if (b > a) {
      *kind = SRC_LS;
      *first = (uint32_t)a;
      *count = (uint32_t)(b - a);
      return;
    }
  }
  if (ls_count && ls_count[i]) {
    *kind = SRC_ARENA;
    *first = ls_first[i];
    *count = ls_count[i];
  }
}

__global__ void k_fin_level1(uint64_t n, const uint32_t* __restrict__ item,
                             const uint32_t* __restrict__ parent, const uint32_t* __restrict__ supp,
                             const uint32_t* __restrict__ db, const uint64_t* __restrict__ cstart,
                             const uint32_t* __restrict__ ls_first, const uint32_t* __restrict__ ls_count,
                             uint32_t* __restrict__ fitem, uint32_t* __restrict__ fparent,
                             uint32_t* __restrict__ fsupp, uint32_t* __restrict__ fdb,
                             uint32_t* __restrict__ skind, uint32_t* __restrict__ sfirst,
                             uint32_t* __restrict__ scount) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    fitem[i] = item[i];
    fparent[i] = parent[i];
    fsupp[i] = supp[i];
    fdb[i] = db[i];
    source_of_ls(i, cstart, ls_first, ls_count, &skind[i], &sfirst[i], &scount[i]);
  }
}

// Wave per node of final level k: copy its children (from the level-synchronous
// level k+1 or from the arena) to their places in final level k+1.
__global__ void k_fin_gather(uint64_t n, const uint32_t* __restrict__ fdb,
                             const uint32_t* __restrict__ skind, const uint32_t* __restrict__ sfirst,
                             const uint32_t* __restrict__ scount, const uint64_t* __restrict__ fcstart,
                             const uint32_t* __restrict__ ls_item, const uint32_t* __restrict__ ls_supp,
                             const uint32_t* __restrict__ ls_db, const uint64_t* __restrict__ ls_cstart,
                             const uint32_t* __restrict__ ls_first, const uint32_t* __restrict__ ls_count,
                             const ArenaNode* __restrict__ arena, uint32_t* __restrict__ nitem,
                             uint32_t* __restrict__ nparent, uint32_t* __restrict__ nsupp,
                             uint32_t* __restrict__ ndb, uint32_t* __restrict__ nkind,
                             uint32_t* __restrict__ nfirst, uint32_t* __restrict__ ncount) {
  const int lane = threadIdx.x & 63;
  const uint64_t wave0 = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t y = wave0; y < n; y += nwaves) {
    const uint32_t kind = skind[y], first = sfirst[y], count = scount[y];
    if (kind == SRC_NONE) continue;
    const uint64_t base = fcstart[y];
    for (uint32_t j = lane; j < count; j += 64) {
      const uint64_t o = base + j;
      nparent[o] = (uint32_t)y;
      if (kind == SRC_LS) {
        const uint64_t c = (uint64_t)first + j;
        nitem[o] = ls_item[c];
        nsupp[o] = ls_supp[c];
        ndb[o] = ls_db[c];
        source_of_ls(c, ls_cstart, ls_first, ls_count, &nkind[o], &nfirst[o], &ncount[o]);
      } else {
        const ArenaNode an = arena[(uint64_t)first + j];
        nitem[o] = an.item;
        nsupp[o] = an.supp;
        ndb[o] = fdb[y];
        nkind[o] = an.count ? SRC_ARENA : SRC_NONE;
        nfirst[o] = an.first;
        ncount[o] = an.count;
      }
    }
  }
}

}  // namespace

void launch_dfs(const DfsArgs& a, uint32_t threads, uint32_t grid, hipStream_t s) {
  if (a.ntasks == 0 || grid == 0) return;
  if (threads == 1024) k_dfs<1024><<<grid, 1024, 0, s>>>(a);
  else if (threads == 512) k_dfs<512><<<grid, 512, 0, s>>>(a);
  else k_dfs<256><<<grid, 256, 0, s>>>(a);
  BM_LAUNCH_CHECK();
}

void launch_dfs_wave(const DfsArgs& a, uint32_t grid, hipStream_t s) {
  if (grid == 0) return;
  k_dfs_wave<<<grid, 256, 0, s>>>(a);
  BM_LAUNCH_CHECK();
}

void launch_dfs_short_flags(const DfsTask* tasks, const DbInfo* dbs, const uint32_t* order,
                            uint32_t n, uint32_t max_words, uint32_t* flags, hipStream_t s) {
  if (n == 0) return;
  k_dfs_short_flags<<<grid_for(n, kThreads), kThreads, 0, s>>>(tasks, dbs, order, n, max_words,
                                                               flags);
  BM_LAUNCH_CHECK();
}

void launch_dfs_split(const uint32_t* order, uint32_t n, const uint32_t* flags, const uint64_t* pos,
                      uint32_t* short_, uint32_t* long_, uint32_t* counts, hipStream_t s) {
  k_dfs_split<<<grid_for(n + 1, kThreads), kThreads, 0, s>>>(order, n, flags, pos, short_, long_,
                                                             counts);
  BM_LAUNCH_CHECK();
}

void launch_dfs_features(const FeatArgs& a, hipStream_t s) {
  if (a.ntasks == 0) return;
  k_dfs_features<<<grid_for(a.ntasks, kThreads), kThreads, 0, s>>>(a);
  BM_LAUNCH_CHECK();
}

void launch_order_by_key(const float* key, uint32_t n, uint32_t* hist, uint64_t* hist_off,
                         uint32_t* order, hipStream_t s) {
  if (n == 0) return;
  launch_fill_u32(hist, 0, kBuckets, s);
  k_bucket_hist<<<grid_for(n, 4 * kThreads, 1024), kThreads, 0, s>>>(key, n, hist);
  BM_LAUNCH_CHECK();
  ScanMulti sm{};
  sm.in[0] = hist;
  sm.is64[0] = 0;
  sm.out[0] = hist_off;
  if (!scan_multi_single(sm, 1, kBuckets, s)) fail(BM_ERR_DEVICE, "bucket scan");
  const uint32_t g = grid_for(n, 4 * kThreads, 1024);
  const uint32_t chunk = (n + g - 1) / g;
  k_bucket_scatter<<<g, kThreads, 0, s>>>(key, n, chunk,
                                          reinterpret_cast<unsigned long long*>(hist_off), order);
  BM_LAUNCH_CHECK();
}

void launch_fin_level1(uint64_t n, const uint32_t* item, const uint32_t* parent, const uint32_t* supp,
                       const uint32_t* db, const uint64_t* cstart, const uint32_t* ls_first,
                       const uint32_t* ls_count, uint32_t* fitem, uint32_t* fparent, uint32_t* fsupp,
                       uint32_t* fdb, uint32_t* skind, uint32_t* sfirst, uint32_t* scount,
                       hipStream_t s) {
  if (n == 0) return;
  k_fin_level1<<<grid_for(n, kThreads), kThreads, 0, s>>>(n, item, parent, supp, db, cstart, ls_first,
                                                           ls_count, fitem, fparent, fsupp, fdb, skind,
                                                           sfirst, scount);
  BM_LAUNCH_CHECK();
}

void launch_fin_gather(uint64_t n, const uint32_t* fdb, const uint32_t* skind, const uint32_t* sfirst,
                       const uint32_t* scount, const uint64_t* fcstart, const uint32_t* ls_item,
                       const uint32_t* ls_supp, const uint32_t* ls_db, const uint64_t* ls_cstart,
                       const uint32_t* ls_first, const uint32_t* ls_count, const ArenaNode* arena,
                       uint32_t* nitem, uint32_t* nparent, uint32_t* nsupp, uint32_t* ndb,
                       uint32_t* nkind, uint32_t* nfirst, uint32_t* ncount, hipStream_t s) {
  if (n == 0) return;
  k_fin_gather<<<grid_for(n * 64, kThreads), kThreads, 0, s>>>(
      n, fdb, skind, sfirst, scount, fcstart, ls_item, ls_supp, ls_db, ls_cstart, ls_first, ls_count,
      arena, nitem, nparent, nsupp, ndb, nkind, nfirst, ncount);
  BM_LAUNCH_CHECK();
}

}  // namespace bm
