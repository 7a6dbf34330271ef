// Matrix construction, pair supports and the level-synchronous miner.
//
// bm_build (Section III, matrix construction, Eq. 1) validates the CSR on the
// device, packs it into column bitsets and counts every column (Eq. 3's
// column aggregation).  Mining extends frequent prefixes level by level (the
// paper's recursive mining by sequential column ANDs), for one database or a
// whole batch at once:
//   level 1: frequent single items (column popcounts >= minsup);
//   level 2: all pairs of frequent items -- the Gram matrix A^T A on MFMA
//            (FP4 form by default, int8 on request; AND+popcount when there
//            are few items);
//   level k+1: every prefix class of level k (nodes sharing a parent) evaluates
//            its q(q-1)/2 sibling pairs, big classes as a masked Gram matrix on
//            128- or 256-wide MFMA tiles, mid-size ones on 32-wide MFMA tiles,
//            small ones with AND+popcount;
// small classes can instead be finished whole: by subset counting when columns
// are long, or by the depth-first kernel from a work queue when asked for; the
// output of those subtrees is merged into the canonical order with the rest.
// One host sync per level reads back the next level's sizes -- for the whole
// batch.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <cmath>
#include <memory>
#include <mutex>
#include <vector>

#include "dfs.hpp"
#include "handles.hpp"
#include "levels.hpp"
#include "mlp.hpp"
#include "rules.hpp"

namespace bm {

namespace {

// Temporaries of one call are returned to the pool only after the call has
// synchronised its stream, so no other stream can reuse a block while this
// call's kernels may still touch it.
struct Scope {
  hipStream_t s;
  std::vector<void*> held;
};
thread_local Scope* t_scope = nullptr;

// While set, temporaries are carved from a fixed device region instead of the
// pool (the allocation-free entry point): bump allocation, 256-byte aligned,
// nothing returned, a request past the end is an error.
struct StaticArena {
  char* base;
  size_t cap;
  size_t used;
};
thread_local StaticArena* t_arena = nullptr;

void* arena_take(size_t bytes) {
  StaticArena& a = *t_arena;
  const size_t at = (a.used + 255) & ~size_t(255);
  if (at + bytes > a.cap)
    fail(BM_ERR_UNSUPPORTED, "the call needs more than the %zu bytes of static scratch", a.cap);
  a.used = at + bytes;
  return a.base + at;
}

template <class T>
struct TBuf {  // temporary device buffer bound to the current call scope
  T* p = nullptr;
  size_t n = 0;
  TBuf() = default;
  TBuf(size_t count, hipStream_t s) { alloc(count, s); }
  void alloc(size_t count, hipStream_t s) {
    n = count;
    if (t_arena) {
      p = count ? static_cast<T*>(arena_take(count * sizeof(T))) : nullptr;
      return;
    }
    p = count ? static_cast<T*>(dalloc(count * sizeof(T), s)) : nullptr;
    if (p) t_scope->held.push_back(p);
  }
  T* get() const { return p; }
};

// Page-locked staging for a call's small host <-> device transfers: copies
// between device memory and pinned host memory run as plain asynchronous DMA,
// where pageable memory would go through the runtime's bounce buffers at every
// level's synchronisation.  Buffers are bump-allocated per thread, kept for
// the life of the process, and recycled when the outermost call scope has
// synchronised its stream.
struct PinnedPool {
  std::vector<std::pair<char*, size_t>> bufs;
  std::vector<char*> dev;  // device address of each buffer (kernels may write there)
  size_t cur = 0, used = 0;
};
thread_local PinnedPool t_pin;
thread_local int t_depth = 0;

void* pinned(size_t bytes) {
  bytes = (bytes + 63) & ~size_t(63);
  for (;;) {
    if (t_pin.cur < t_pin.bufs.size()) {
      if (t_pin.used + bytes <= t_pin.bufs[t_pin.cur].second) {
        void* p = t_pin.bufs[t_pin.cur].first + t_pin.used;
        t_pin.used += bytes;
        return p;
      }
      if (t_pin.cur + 1 < t_pin.bufs.size()) {
        ++t_pin.cur;
        t_pin.used = 0;
        continue;
      }
    }
    const size_t last = t_pin.bufs.empty() ? 0 : t_pin.bufs.back().second;
    const size_t sz = std::max<size_t>({bytes, size_t(1) << 20, 2 * last});
    void* p = nullptr;
    BM_HIP(hipHostMalloc(&p, sz, hipHostMallocDefault));
    void* d = nullptr;
    BM_HIP(hipHostGetDevicePointer(&d, p, 0));
    t_pin.bufs.push_back({static_cast<char*>(p), sz});
    t_pin.dev.push_back(static_cast<char*>(d));
    t_pin.cur = t_pin.bufs.size() - 1;
    t_pin.used = 0;
  }
}

template <class T>
T* pinned_array(size_t n) {
  return static_cast<T*>(pinned(std::max<size_t>(1, n) * sizeof(T)));
}

// Device address of a staging-pool pointer: a kernel writes its small results
// straight into host memory, which the host reads after synchronising the
// stream (no copy launch).
template <class T>
T* mapped(T* host) {
  const char* h = reinterpret_cast<const char*>(host);
  for (size_t b = 0; b < t_pin.bufs.size(); ++b) {
    const char* base = t_pin.bufs[b].first;
    if (h >= base && h < base + t_pin.bufs[b].second)
      return reinterpret_cast<T*>(t_pin.dev[b] + (h - base));
  }
  fail(BM_ERR_DEVICE, "pointer outside the staging pool");
}

class CallScope {
 public:
  explicit CallScope(hipStream_t s) : sc_{s, {}} {
    prev_ = t_scope;
    t_scope = &sc_;
    ++t_depth;
  }
  ~CallScope() {
    (void)hipStreamSynchronize(sc_.s);
    for (void* p : sc_.held) dfree(p, sc_.s);
    t_scope = prev_;
    if (--t_depth == 0) {  // nothing of this thread's calls is in flight any more
      t_pin.cur = 0;
      t_pin.used = 0;
    }
  }

 private:
  Scope sc_;
  Scope* prev_;
};

template <class T>
T read_back(const T* dev, hipStream_t s) {
  if (t_arena) {  // no staging pool: one small copy into the caller's stack
    T v{};
    BM_HIP(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    BM_HIP(hipStreamSynchronize(s));
    return v;
  }
  T* v = pinned_array<T>(1);
  BM_HIP(hipMemcpyAsync(v, dev, sizeof(T), hipMemcpyDeviceToHost, s));
  BM_HIP(hipStreamSynchronize(s));
  return *v;
}

// Host -> device copy of a small host array through pinned staging (the
// staging copy lives until the call's scope has synchronised).
template <class T>
void upload(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return;
  if (t_arena) {  // no staging pool: small tables travel as kernel arguments
    static_assert(sizeof(T) % 4 == 0, "tables are whole 32-bit words");
    const size_t words = src.size() * sizeof(T) / 4;
    if (words > kWriteWordsMax) fail(BM_ERR_UNSUPPORTED, "table too large for static scratch mode");
    launch_write_words(reinterpret_cast<uint32_t*>(dst),
                       reinterpret_cast<const uint32_t*>(src.data()), (uint32_t)words, s);
    return;
  }
  T* st = pinned_array<T>(src.size());
  std::memcpy(st, src.data(), src.size() * sizeof(T));
  BM_HIP(hipMemcpyAsync(dst, st, src.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Up to this length one workgroup scans an array in a single launch (a few
// looped chunks); longer arrays take the three-launch tiled scan.
constexpr uint64_t kOneLaunchScan = 16384;

// Exclusive scans of sm's count arrays of length n (out[j][n] = total), with
// sm's totals option.
void scan_arrays(const ScanMulti& sm, int count, uint64_t n, hipStream_t s) {
  if (n <= kOneLaunchScan && scan_multi_single(sm, count, n, s)) return;
  {
    TBuf<uint64_t> tmp(scan_tiles_tmp_words(count, n), s);
    if (scan_multi_tiles(sm, count, n, tmp.get(), s)) return;
  }
  // more than 2^18 tiles: one recursive block scan per array
  TBuf<uint64_t> tmp(scan_tmp_words(n), s);
  for (int j = 0; j < count; ++j) {
    if (sm.is64[j]) scan_u64(static_cast<const uint64_t*>(sm.in[j]), sm.out[j], n, tmp.get(), s);
    else scan_u32_to_u64(static_cast<const uint32_t*>(sm.in[j]), sm.out[j], n, tmp.get(), s);
  }
  if (sm.tot) {
    GatherU64 g{};
    for (int j = 0; j < count; ++j) g.src[j] = sm.out[j] + n;
    for (uint32_t e = 0; e < sm.nextra; ++e) g.src[count + e] = sm.extra + e;
    launch_gather_u64(g, count + (int)sm.nextra, sm.tot, s);
  }
}

void scan32(const uint32_t* in, uint64_t* out, uint64_t n, hipStream_t s) {
  ScanMulti sm{};
  sm.in[0] = in;
  sm.out[0] = out;
  scan_arrays(sm, 1, n, s);
}
void scan64(const uint64_t* in, uint64_t* out, uint64_t n, hipStream_t s) {
  ScanMulti sm{};
  sm.in[0] = in;
  sm.is64[0] = 1;
  sm.out[0] = out;
  scan_arrays(sm, 1, n, s);
}
// Scan of up to 8 same-length arrays (is64[j]: element type of in[j]).
void scan_many(const void* const* in, const bool* is64, uint64_t* const* out, int count, uint64_t n,
               hipStream_t s) {
  ScanMulti sm{};
  for (int j = 0; j < count; ++j) {
    sm.in[j] = in[j];
    sm.is64[j] = is64[j] ? 1u : 0u;
    sm.out[j] = out[j];
  }
  scan_arrays(sm, count, n, s);
}

// scan_many that also writes the totals to tot[0..count) and then
// extra[0..nextra) to tot[count..] (tot may be mapped host memory).
void scan_many_tot(const void* const* in, const bool* is64, uint64_t* const* out, int count,
                   uint64_t n, uint64_t* tot, const uint64_t* extra, uint32_t nextra,
                   hipStream_t s) {
  ScanMulti sm{};
  for (int j = 0; j < count; ++j) {
    sm.in[j] = in[j];
    sm.is64[j] = is64[j] ? 1u : 0u;
    sm.out[j] = out[j];
  }
  sm.tot = tot;
  sm.extra = extra;
  sm.nextra = nextra;
  scan_arrays(sm, count, n, s);
}

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
uint64_t round_up(uint64_t a, uint64_t b) { return ceil_div(a, b) * b; }

// Word-split lengths for a step: enough tasks to fill the chip, not shorter
// than a minimum that keeps per-task overheads small.
TaskGeom make_geom(uint64_t Wmax, uint64_t pairs_m, uint64_t pairs_v, uint64_t pairs_vw,
                   uint64_t classes_t, const Tuning& tu) {
  const uint64_t target = (uint64_t)cu_count() * 8;
  const uint64_t W = std::max<uint64_t>(1, Wmax);
  TaskGeom g{};
  auto pick = [&](uint64_t units, uint64_t min_len, uint64_t align, uint64_t per_wg = 1) {
    if (tu.split_words) return round_up(tu.split_words, align);
    uint64_t ns = units ? ceil_div(target * per_wg, units) : 1;
    ns = std::min<uint64_t>(ns, std::max<uint64_t>(1, W / min_len));
    return round_up(ceil_div(W, ns), align);
  };
  // The FP4 Gram kernels split each launch's stages evenly over their
  // workgroups by cost, whatever the task lengths, so their tasks are whole
  // block pairs (up to the FP4 word cap below): every task boundary a
  // workgroup crosses costs a flush of 16K (128-wide) or 64K (256-wide)
  // atomic adds.  The int8 form deals tasks out round-robin: enough of them
  // to fill the chip, at least 1,024 words each (the flush paid twice over
  // below that).
  const uint32_t whole = (uint32_t)round_up(W, GRAM_KW);
  g.split_m = tu.split_words ? (uint32_t)round_up(tu.split_words, GRAM_KW)
              : tu.mfma_fp4  ? whole
                             : (uint32_t)pick(pairs_m, 1024, GRAM_KW);
  g.split_v = (uint32_t)pick(pairs_v, 512, 1);
  g.split_t = (uint32_t)pick(classes_t, 2048, 64);  // tiny-class loads read 4-word groups
  g.split_b = tu.split_words ? (uint32_t)round_up(tu.split_words, GRAM_KW) : whole;
  // 32-wide block pairs number about a quarter of the 16-wide ones, and each
  // is one wave's task: two per workgroup slot (measured 8% faster on the
  // T40-style workload than four, and no slower on the dense one).  The
  // length comes from the pairs weighted by their databases' words, so that
  // in a batch of unequal databases the long ones are split as finely as the
  // short ones' whole ranges (one database: the same as splitting W evenly).
  if (tu.split_words || pairs_vw == 0) {
    g.split_s = (uint32_t)pick((pairs_v + 3) / 4, 128, GRAM_SMALL_KW, 2);
  } else {
    const uint64_t len = ceil_div((pairs_vw + 3) / 4, target * 2);
    g.split_s = (uint32_t)round_up(std::min<uint64_t>(W, std::max<uint64_t>(len, 128)), GRAM_SMALL_KW);
  }
  g.big_q = tu.mfma_big_q;
  g.small_on = tu.mfma_small ? 1u : 0u;
  g.tiny_q = tu.tiny_q;
  if (tu.mfma_fp4) {  // keep every MFMA task's counts below 2^24
    g.split_m = std::min<uint32_t>(g.split_m, GRAM_FP4_MAX_WORDS);
    g.split_b = std::min<uint32_t>(g.split_b, GRAM_FP4_MAX_WORDS);
    g.split_s = std::min<uint32_t>(g.split_s, GRAM_FP4_MAX_WORDS);
  }
  return g;
}

// Device-side work of one level step.
struct StepWork {
  uint64_t ncls = 0;
  bool prefixed = true;  // some class may have a prefix (the FP4 Gram kernels then apply masks)
  TBuf<ClassDesc> cls;
  TBuf<uint32_t> pre;
  TBuf<Task> tm, tv, tt, tb, ts;
  uint64_t ub_m = 0, ub_v = 0, ub_t = 0, ub_b = 0, ub_s = 0;  // task-count upper bounds (host)
  TBuf<uint64_t> om, ov, ot, ob, os;  // task offsets per class (+ total at [ncls])
  TBuf<uint64_t> pcm, pcb;  // FP4 Gram kernels: prefix sums of the task costs (tm, tb)
  TBuf<uint32_t> tri;
  uint64_t T = 0;
  uint64_t st[ST_COUNT] = {};
  TBuf<DfsTask> dt;  // small classes handed to the depth-first kernel
  uint64_t ndt = 0;
  TBuf<uint32_t> ccount[5];   // tasks per class per kind (128, LDS, tiny, 256, 32-wide)
  bool counts_ready = false;  // ccount already written (by the previous step's post kernel)
  // projected classes (written by the previous step's post kernel)
  uint64_t nproj = 0, proj_rows = 0, proj_words = 0, proj_cols = 0;
  TBuf<DbInfo> views;
  TBuf<ProjWork> pwork;
  TBuf<uint64_t> vbuf;
  double pj_cand[2] = {0, 0}, pj_work[2] = {0, 0};  // 128-wide, 256-wide projected classes
};

// Task lists of a step's classes: counts per class on the device, scanned
// offsets, then the records.  The kernels read the totals from device memory;
// the host only sizes buffers from upper bounds.
void prepare_tasks(StepWork& w, const DbInfo* ddb, uint64_t Wmax, uint64_t pairs_m, uint64_t pairs_b,
                   uint64_t pairs_v, uint64_t pairs_vw, uint64_t classes_t, const Tuning& tu,
                   bool dfs, uint32_t level, hipStream_t s) {
  const TaskGeom g = make_geom(Wmax, pairs_m, pairs_v, pairs_vw, classes_t, tu);
  const uint64_t Wm = round_up(std::max<uint64_t>(1, Wmax), GRAM_KW);
  w.ub_m = pairs_m * ceil_div(Wm, g.split_m);
  w.ub_b = pairs_b * ceil_div(Wm, g.split_b);
  w.ub_v = tu.mfma_small ? 0 : pairs_v * ceil_div(std::max<uint64_t>(1, Wmax), g.split_v);
  w.ub_s = tu.mfma_small ? pairs_v * ceil_div(round_up(std::max<uint64_t>(1, Wmax), GRAM_SMALL_KW),
                                              g.split_s)
                         : 0;
  w.ub_t = dfs ? 0 : classes_t * ceil_div(std::max<uint64_t>(1, Wmax), g.split_t);
  if (dfs) {
    w.ndt = classes_t;
    w.dt.alloc(classes_t, s);
  }
  if (!w.counts_ready) {  // else the previous step's k_level_post wrote them
    for (auto& c : w.ccount) c.alloc(w.ncls, s);
    launch_class_task_counts(w.cls.get(), w.ncls, ddb, w.views.get(), tu.mfma_min_q, g, dfs,
                             w.ccount[0].get(),
                             w.ccount[1].get(), w.ccount[2].get(), w.ccount[3].get(),
                             w.ccount[4].get(), s);
  }
  w.om.alloc(w.ncls + 1, s);
  w.ov.alloc(w.ncls + 1, s);
  w.ot.alloc(w.ncls + 1, s);
  w.ob.alloc(w.ncls + 1, s);
  w.os.alloc(w.ncls + 1, s);
  const void* in[5] = {w.ccount[0].get(), w.ccount[1].get(), w.ccount[2].get(), w.ccount[3].get(),
                       w.ccount[4].get()};
  const bool is64[5] = {false, false, false, false, false};
  uint64_t* out[5] = {w.om.get(), w.ov.get(), w.ot.get(), w.ob.get(), w.os.get()};
  scan_many(in, is64, out, 5, w.ncls, s);
  w.tm.alloc(w.ub_m, s);
  w.tv.alloc(w.ub_v, s);
  w.tt.alloc(w.ub_t, s);
  w.tb.alloc(w.ub_b, s);
  w.ts.alloc(w.ub_s, s);
  launch_write_class_tasks(w.cls.get(), w.ncls, ddb, w.views.get(), tu.mfma_min_q, g, w.om.get(),
                           w.ov.get(),
                           w.ot.get(), w.tm.get(), w.tv.get(), w.tt.get(), dfs ? w.dt.get() : nullptr,
                           level, w.ob.get(), w.tb.get(), w.os.get(), w.ts.get(), s);
  if (tu.mfma_fp4) {  // the FP4 Gram kernels split their launch's stages evenly by cost
    auto costs = [&](const Task* t, const uint64_t* nt, uint64_t ub, uint32_t w_off,
                     uint32_t w_diag, TBuf<uint64_t>& P) {
      if (!ub) return;
      TBuf<uint32_t> c(ub, s);
      launch_task_costs(t, nt, ub, w_off, w_diag, c.get(), s);
      P.alloc(ub + 1, s);
      const void* cin[1] = {c.get()};
      const bool c64[1] = {false};
      uint64_t* cout[1] = {P.get()};
      scan_many(cin, c64, cout, 1, ub, s);
    };
    costs(w.tm.get(), w.om.get() + w.ncls, w.ub_m, GRAM_COST_OFF, GRAM_COST_DIAG, w.pcm);
    costs(w.tb.get(), w.ob.get() + w.ncls, w.ub_b, GRAM_BIG_COST_OFF, GRAM_BIG_COST_DIAG, w.pcb);
  }
}

// Views of the step's projected classes: each child column compressed by its
// class's prefix tidset.
void project_views(StepWork& w, const DbInfo* ddb, const uint32_t* child_item, uint64_t Wmax,
                   double nW, KTimer& tm, hipStream_t s) {
  const uint32_t np = (uint32_t)w.nproj;
  const uint64_t nc = (uint64_t)np * view_chunks(Wmax);
  tm.begin(BM_K_PROJECT);
  TBuf<uint32_t> cnt(nc, s);
  TBuf<uint64_t> off(nc + 1, s);
  launch_fill_u64(w.vbuf.get(), 0, w.proj_words, s);
  launch_project_count(w.pwork.get(), np, w.cls.get(), ddb, w.pre.get(), Wmax, cnt.get(), s);
  scan32(cnt.get(), off.get(), nc, s);
  launch_project_compact(w.pwork.get(), np, w.cls.get(), ddb, w.views.get(), w.pre.get(),
                         child_item, Wmax, off.get(), s);
  // algorithmic bytes: the children's columns read once, the views written
  tm.end(8.0 * nW * (double)w.proj_cols + 8.0 * (double)w.proj_words, 0.0);
}

void run_class_kernels(const DbInfo* ddb, const uint32_t* child_item, const StepWork& w,
                       const Tuning& tu, double nW, double nN, KTimer& tm, hipStream_t s) {
  ClassArgs a{ddb, child_item, w.cls.get(), w.pre.get(), w.views.get(), nullptr, nullptr,
              w.tri.get()};
  const uint64_t ncu = (uint64_t)cu_count();
  // algorithmic ops of a projected class: 2 supp(P) per candidate pair
  auto gram_ops = [&](int kind, int pj) {
    return 2.0 * (((double)w.st[ST_CAND_M + kind] - w.pj_cand[pj]) * nN + w.pj_work[pj]);
  };
  if (w.ub_b && w.st[ST_CLS_B]) {
    a.tasks = w.tb.get();
    a.ntasks = w.ob.get() + w.ncls;
    a.tcost = w.pcb.get();
    tm.begin(BM_K_GRAM_MFMA_BIG);
    // one workgroup per CU, each with an equal share of the stages
    launch_gram_mfma_big(a, (uint32_t)ncu, w.prefixed, s);
    tm.end(8.0 * nW * (double)w.st[ST_COLS_B], gram_ops(3, 1));
  }
  if (w.ub_m && w.st[ST_CLS_M]) {
    a.tasks = w.tm.get();
    a.ntasks = w.om.get() + w.ncls;
    a.tcost = w.pcm.get();
    tm.begin(BM_K_GRAM_MFMA);
    // FP4: two workgroups per CU (all resident at once), each with an equal
    // share of the stages; int8: a grid-stride loop over the tasks
    launch_gram_mfma(a, tu.mfma_fp4 ? (uint32_t)(ncu * 2)
                                    : (uint32_t)std::min<uint64_t>(w.ub_m, ncu * 4),
                     tu.mfma_fp4, w.prefixed, s);
    tm.end(8.0 * nW * (double)w.st[ST_COLS_M], gram_ops(0, 0));
  }
  if (w.ub_s && (w.st[ST_CLS_S] || w.st[ST_CAND_S])) {  // mid-size classes or narrow tails
    a.tasks = w.ts.get();
    a.ntasks = w.os.get() + w.ncls;
    tm.begin(BM_K_GRAM_SMALL);
    launch_gram_small(a, (uint32_t)std::min<uint64_t>((w.ub_s + 3) / 4, ncu * 8), tu.mfma_fp4, s);
    tm.end(8.0 * nW * (double)w.st[ST_COLS_S], 2.0 * (double)w.st[ST_CAND_S] * nN);
  }
  if (w.ub_v && w.st[ST_CLS_V]) {
    a.tasks = w.tv.get();
    a.ntasks = w.ov.get() + w.ncls;
    tm.begin(BM_K_ANDPOP);
    launch_andpop(a, tu.andpop_chunk, (uint32_t)std::min<uint64_t>(w.ub_v, ncu * 8), s);
    tm.end(8.0 * nW * (double)w.st[ST_COLS_V], (double)w.st[ST_CAND_V] * nW);
  }
  if (w.ub_t) {
    a.tasks = w.tt.get();
    a.ntasks = w.ot.get() + w.ncls;
    tm.begin(BM_K_ANDPOP_REG);
    launch_andpop_reg(a, (uint32_t)std::min<uint64_t>(w.ub_t, ncu * 8), s);
    tm.end(8.0 * nW * (double)w.st[ST_COLS_T], (double)w.st[ST_CAND_T] * nW);
  }
}

// Classes given on the host (the roots of each database, or an explicit
// column list): records, a zeroed triangle buffer and the task lists.
void host_classes(StepWork& w, const std::vector<ClassDesc>& hc, const DbInfo* ddb,
                  const DbInfo* hdb, uint64_t Wmax, const Tuning& tu, bool dfs, hipStream_t s) {
  w.ncls = hc.size();
  w.prefixed = false;
  for (const auto& c : hc) w.prefixed |= c.pre_len > 0;
  w.cls.alloc(w.ncls, s);
  upload(w.cls.get(), hc, s);
  w.pre.alloc(1, s);
  launch_fill_u32(w.pre.get(), 0, 1, s);
  uint64_t pm = 0, pb = 0, pv = 0, pvw = 0, ct = 0;  // pvw: pv weighted by the databases' words
  w.T = 0;
  for (const auto& c : hc) {
    const uint64_t tsz = (uint64_t)c.q * (c.q - 1) / 2;
    w.T += tsz;
    const int kind =
        class_kind(c.q, tu.mfma_min_q, tu.mfma_big_q, tu.mfma_small ? 1u : 0u, tu.tiny_q);
    // a narrow tail's candidates and 32-wide block pairs go to the 32-wide kernel
    const bool tail = kind == 0 && tu.mfma_small && gram_tail(c.q);
    const uint64_t qm = tail ? gram_tail_q(c.q) : c.q;
    const uint64_t tm_sz = tail ? qm * (qm - 1) / 2 : tsz;
    if (kind == 0) pm += host_mfma_pairs(c.q);
    else if (kind == 3) pb += host_mfma_pairs(c.q, GRAM_TILE_BIG);
    else if (kind == 1 || kind == 4) {
      pv += host_andpop_pairs(c.q);
      pvw += (uint64_t)host_andpop_pairs(c.q) * hdb[c.db].W;
    } else ct += 1;
    if (tail) {
      pv += 4ull * gram_tail_pairs(c.q);  // in 16-wide units: four per 32-wide pair
      pvw += 4ull * gram_tail_pairs(c.q) * hdb[c.db].W;
      w.st[ST_CAND_S] += tsz - tm_sz;
      w.st[ST_COLS_S] += c.q;
    }
    w.st[ST_CAND_M + kind] += tm_sz;
    w.st[ST_COLS_M + kind] += c.q;
    w.st[ST_CLS_M + kind] += 1;
  }
  w.tri.alloc(w.T, s);
  launch_fill_u32(w.tri.get(), 0, w.T, s);
  prepare_tasks(w, ddb, Wmax, pm, pb, pv, pvw, ct, tu, dfs, 1, s);
}

struct Level {
  uint64_t n = 0;
  TBuf<uint32_t> item, parent, supp, db;
  TBuf<uint64_t> cstart;  // n + 1, child ranges in the next level
};

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

Tuning tuning_from(const bm_options* opt) {
  Tuning t;
  if (!opt) return t;
  if (opt->mfma_min_children) t.mfma_min_q = std::max<uint32_t>(2, opt->mfma_min_children);
  if (opt->andpop_chunk_words) {
    if (opt->andpop_chunk_words != 128 && opt->andpop_chunk_words != 256)
      fail(BM_ERR_INVALID_ARG, "andpop_chunk_words must be 128 or 256");
    t.andpop_chunk = opt->andpop_chunk_words;
  }
  if (opt->split_words) {
    if (opt->split_words % 64) fail(BM_ERR_INVALID_ARG, "split_words must be a multiple of 64");
    t.split_words = opt->split_words;
  }
  if (opt->dfs_threads) {
    if (opt->dfs_threads != 256 && opt->dfs_threads != 512 && opt->dfs_threads != 1024)
      fail(BM_ERR_INVALID_ARG, "dfs_threads must be 256, 512 or 1024");
    t.dfs_threads = opt->dfs_threads;
  }
  if (opt->dfs_max_words) t.dfs_max_words = opt->dfs_max_words;
  if (opt->dfs_wave_max_words) t.dfs_wave_words = opt->dfs_wave_max_words;
  if (opt->flags & BM_FLAG_DFS_BLOCK_ONLY) t.dfs_wave_words = 0;
  if (opt->mfma_big_children) t.mfma_big_q = std::max<uint32_t>(2, opt->mfma_big_children);
  if (opt->flags & BM_FLAG_LEVELSYNC) t.dfs = false;
  if (opt->subset_max_children) {
    if (opt->subset_max_children > (uint32_t)SUBSET_Q)
      fail(BM_ERR_INVALID_ARG, "subset_max_children must be at most %d", SUBSET_Q);
    t.subset_q = opt->subset_max_children == 1 ? 0u : opt->subset_max_children;
  }
  t.arena_nodes = opt->dfs_arena_nodes;
  if (opt->project_gain) t.project_gain = opt->project_gain;
  if (opt->flags & BM_FLAG_NO_PROJECT) t.project_gain = 0;
  if (opt->flags & BM_FLAG_FP4_MFMA) t.mfma_fp4 = true;
  if (opt->flags & BM_FLAG_INT8_MFMA) t.mfma_fp4 = false;
  if (!t.mfma_fp4) t.mfma_big_q = 0xffffffffu;  // the 256-wide kernel has the FP4 form only
  if (opt->flags & BM_FLAG_NO_MFMA) {
    t.mfma_min_q = 0xffffffffu;
    t.mfma_small = false;
  }
  if (opt->flags & BM_FLAG_ALL_MFMA) t.mfma_min_q = 2;
  return t;
}

// ------------------------------------------------------------------ build

bm_db* build_db(const uint64_t* row_ptr, const uint32_t* col_idx, uint64_t n, uint32_t m,
                hipStream_t s) {
  if (!row_ptr) fail(BM_ERR_INVALID_ARG, "row_ptr is NULL");
  if (n >= (1ull << 31)) fail(BM_ERR_UNSUPPORTED, "n_tx = %llu >= 2^31", (unsigned long long)n);
  std::unique_ptr<bm_db> db(new bm_db);
  CallScope scope(s);  // declared after db: on failure it synchronises before db is freed
  BM_HIP(hipGetDevice(&db->device));
  db->n = n;
  db->m = m;
  db->W = (n + 63) / 64;
  db->Wp = padded_words(n);
  const bool rp_dev = is_device_ptr(row_ptr);
  const bool ci_host = col_idx && !is_device_ptr(col_idx);
  const bool tiled = pack_tiled_ok(m, db->Wp);
  const double words = (double)m * (double)db->Wp;
  if (words * 8.0 > 1.0e15) fail(BM_ERR_UNSUPPORTED, "bitset matrix too large");
  // nnz is needed on the host only to copy host item ids or for the untiled
  // path; the tiled kernel reads it, and checks row_ptr, on the device
  uint64_t nnz = 0;
  if (!rp_dev || !tiled || ci_host) {
    uint64_t rp0 = 0;
    if (rp_dev) {
      uint64_t* h = pinned_array<uint64_t>(2);
      BM_HIP(hipMemcpyAsync(h, row_ptr, 8, hipMemcpyDeviceToHost, s));
      BM_HIP(hipMemcpyAsync(h + 1, row_ptr + n, 8, hipMemcpyDeviceToHost, s));
      BM_HIP(hipStreamSynchronize(s));
      rp0 = h[0];
      nnz = h[1];
    } else {
      rp0 = row_ptr[0];
      nnz = row_ptr[n];
    }
    if (rp0 != 0) fail(BM_ERR_CSR, "row_ptr[0] = %llu, expected 0", (unsigned long long)rp0);
    if (nnz > 0 && !col_idx) fail(BM_ERR_INVALID_ARG, "col_idx is NULL but row_ptr[n] = %llu",
                                  (unsigned long long)nnz);
  }

  const uint64_t* d_rp = row_ptr;
  TBuf<uint64_t> rp_copy;
  if (!rp_dev) {
    rp_copy.alloc(n + 1, s);
    BM_HIP(hipMemcpyAsync(rp_copy.get(), row_ptr, (n + 1) * 8, hipMemcpyHostToDevice, s));
    d_rp = rp_copy.get();
  }
  const uint32_t* d_ci = col_idx;
  TBuf<uint32_t> ci_copy;
  if (nnz > 0 && ci_host) {
    ci_copy.alloc(nnz, s);
    BM_HIP(hipMemcpyAsync(ci_copy.get(), col_idx, nnz * 4, hipMemcpyHostToDevice, s));
    d_ci = ci_copy.get();
  }
  TBuf<uint32_t> err(1, s);
  launch_fill_u32(err.get(), 0, 1, s);
  db->B.reset((size_t)m * db->Wp, s);
  db->colsum.reset(m, s);
  if (tiled) {
    launch_fill_u32(db->colsum.get(), 0, m, s);
    launch_pack_tiled(d_rp, d_ci, n, m, db->B.get(), db->Wp, db->colsum.get(), err.get(), s);
  } else if (m > 0) {
    launch_fill_u32(db->colsum.get(), 0, m, s);
    launch_validate(d_rp, d_ci, n, nnz, m, err.get(), s);
    const uint32_t e0 = read_back(err.get(), s);
    if (e0 & 1u) fail(BM_ERR_CSR, "row_ptr is not non-decreasing");
    if (e0 & 2u) fail(BM_ERR_CSR, "an item id is >= n_items (%u)", m);
    launch_fill_u64(db->B.get(), 0, (uint64_t)m * db->Wp, s);
    launch_pack(d_rp, d_ci, n, db->B.get(), db->Wp, s);
    launch_colsum(db->B.get(), db->Wp, m, db->colsum.get(), s);
  } else {
    launch_validate(d_rp, d_ci, n, nnz, m, err.get(), s);
  }
  const uint32_t e = read_back(err.get(), s);
  if (e & 8u) fail(BM_ERR_CSR, "row_ptr[0] is not 0");
  if (e & 4u) fail(BM_ERR_INVALID_ARG, "col_idx is NULL but row_ptr[n] > 0");
  if (e & 1u) fail(BM_ERR_CSR, "row_ptr is not non-decreasing");
  if (e & 2u) fail(BM_ERR_CSR, "an item id is >= n_items (%u)", m);
  return db.release();
}

// Batched construction: every database whose item count the tiled kernel
// handles is validated and packed for the whole batch at once: a pre-pass
// reads each nnz into host memory, then one grid packs the tiles of the
// sparse databases and one those of the dense (two synchronisations in all);
// the others are built one by one.  All or nothing: on any failure no handle
// is returned.
std::vector<bm_db*> build_many(uint32_t count, const uint64_t* const* row_ptrs,
                               const uint32_t* const* col_idxs, const uint64_t* ns,
                               const uint32_t* ms, hipStream_t s) {
  std::vector<std::unique_ptr<bm_db>> dbs(count);
  {
    CallScope scope(s);  // after dbs: on failure it synchronises before they are freed
    std::vector<PackJob> jobs;
    std::vector<uint32_t> job_db;
    std::vector<uint32_t> single;
    for (uint32_t d = 0; d < count; ++d) {
      const uint64_t n = ns[d];
      const uint32_t m = ms[d];
      if (!row_ptrs[d]) fail(BM_ERR_INVALID_ARG, "database %u: row_ptr is NULL", d);
      if (n >= (1ull << 31))
        fail(BM_ERR_UNSUPPORTED, "database %u: n_tx = %llu >= 2^31", d, (unsigned long long)n);
      const uint64_t Wp = padded_words(n);
      if ((double)m * (double)Wp * 8.0 > 1.0e15)
        fail(BM_ERR_UNSUPPORTED, "database %u: bitset matrix too large", d);
      if (!pack_tiled_ok(m, Wp)) {
        single.push_back(d);
        continue;
      }
      auto db = std::make_unique<bm_db>();
      BM_HIP(hipGetDevice(&db->device));
      db->n = n;
      db->m = m;
      db->W = (n + 63) / 64;
      db->Wp = Wp;
      PackJob jb{};
      jb.rp = row_ptrs[d];
      jb.ci = col_idxs ? col_idxs[d] : nullptr;
      if (!is_device_ptr(jb.rp)) {
        const uint64_t nnz = row_ptrs[d][n];
        TBuf<uint64_t> rp(n + 1, s);
        BM_HIP(hipMemcpyAsync(rp.get(), row_ptrs[d], (n + 1) * 8, hipMemcpyHostToDevice, s));
        jb.rp = rp.get();
        if (nnz > 0 && jb.ci && !is_device_ptr(jb.ci)) {
          TBuf<uint32_t> ci(nnz, s);
          BM_HIP(hipMemcpyAsync(ci.get(), col_idxs[d], nnz * 4, hipMemcpyHostToDevice, s));
          jb.ci = ci.get();
        }
      } else if (jb.ci && !is_device_ptr(jb.ci)) {
        fail(BM_ERR_INVALID_ARG, "database %u: row_ptr on the device but col_idx on the host", d);
      }
      db->B.reset((size_t)m * Wp, s);
      db->colsum.reset(m, s);
      jb.n = n;
      jb.m = m;
      jb.B = db->B.get();
      jb.Wp = Wp;
      jb.colsum = db->colsum.get();
      jobs.push_back(jb);
      job_db.push_back(d);
      dbs[d] = std::move(db);
    }
    const uint32_t nj = (uint32_t)jobs.size();
    if (nj) {
      TBuf<PackJob> djobs(nj, s);
      TBuf<uint32_t> derr(nj, s);
      upload(djobs.get(), jobs, s);
      uint64_t* hnnz = pinned_array<uint64_t>(nj);
      launch_build_multi_pre(djobs.get(), nj, derr.get(), mapped(hnnz), s);
      BM_HIP(hipStreamSynchronize(s));
      // Split the tiles by kind: [sparse starts | dense starts | sparse ids | dense ids].
      std::vector<uint32_t> kid[2];
      std::vector<uint64_t> kst[2] = {{0}, {0}};
      for (uint32_t j = 0; j < nj; ++j) {
        const int k = pack_sparse(hnnz[j], jobs[j].n) ? 0 : 1;
        kid[k].push_back(j);
        kst[k].push_back(kst[k].back() + pack_blocks(jobs[j].Wp));
      }
      std::vector<uint64_t> tab(kst[0]);
      tab.insert(tab.end(), kst[1].begin(), kst[1].end());
      const size_t id_at = tab.size();
      tab.resize(id_at + (nj + 1) / 2, 0);
      uint32_t* ids = reinterpret_cast<uint32_t*>(tab.data() + id_at);
      std::copy(kid[0].begin(), kid[0].end(), ids);
      std::copy(kid[1].begin(), kid[1].end(), ids + kid[0].size());
      TBuf<uint64_t> dtab(tab.size(), s);
      upload(dtab.get(), tab, s);
      const uint32_t* did = reinterpret_cast<const uint32_t*>(dtab.get() + id_at);
      launch_pack_multi(djobs.get(), true, did, (uint32_t)kid[0].size(), dtab.get(),
                        kst[0].back(), derr.get(), s);
      launch_pack_multi(djobs.get(), false, did + kid[0].size(), (uint32_t)kid[1].size(),
                        dtab.get() + kst[0].size(), kst[1].back(), derr.get(), s);
      uint32_t* herr = pinned_array<uint32_t>(nj);
      BM_HIP(hipMemcpyAsync(herr, derr.get(), nj * 4, hipMemcpyDeviceToHost, s));
      BM_HIP(hipStreamSynchronize(s));
      for (uint32_t j = 0; j < nj; ++j) {
        const uint32_t e = herr[j], d = job_db[j];
        if (e & 8u) fail(BM_ERR_CSR, "database %u: row_ptr[0] is not 0", d);
        if (e & 4u) fail(BM_ERR_INVALID_ARG, "database %u: col_idx is NULL but row_ptr[n] > 0", d);
        if (e & 1u) fail(BM_ERR_CSR, "database %u: row_ptr is not non-decreasing", d);
        if (e & 2u) fail(BM_ERR_CSR, "database %u: an item id is >= n_items (%u)", d, ms[d]);
      }
    }
    for (uint32_t d : single) {
      try {
        dbs[d].reset(build_db(row_ptrs[d], col_idxs ? col_idxs[d] : nullptr, ns[d], ms[d], s));
      } catch (const Error& e) {
        fail(e.status, "database %u: %s", d, e.msg.c_str());
      }
    }
  }
  std::vector<bm_db*> out(count);
  for (uint32_t d = 0; d < count; ++d) out[d] = dbs[d].release();
  return out;
}

// ------------------------------------------------------------------ pairs

namespace {

// Pair supports of k items.  static_scratch: every temporary comes from the
// static region (items and out must then be device memory, and nothing is
// allocated).
void pair_support_impl(const bm_db* db, const uint32_t* items, uint32_t k, uint32_t* out,
                       hipStream_t s, bool static_scratch) {
  if (k == 0) return;
  if (!out) fail(BM_ERR_INVALID_ARG, "out is NULL");
  if (!items && k != db->m) fail(BM_ERR_INVALID_ARG, "items == NULL requires k == n_items");
  CallScope scope(s);
  TBuf<uint32_t> d_items(k, s);
  std::vector<uint32_t> h_items;
  if (!items) {
    if (static_scratch) {
      launch_iota_u32(d_items.get(), k, s);
    } else {
      h_items.resize(k);
      for (uint32_t i = 0; i < k; ++i) h_items[i] = i;
      upload(d_items.get(), h_items, s);
    }
  } else if (is_device_ptr(items)) {
    BM_HIP(hipMemcpyAsync(d_items.get(), items, (size_t)k * 4, hipMemcpyDeviceToDevice, s));
    TBuf<uint32_t> err(1, s);
    launch_fill_u32(err.get(), 0, 1, s);
    launch_validate(nullptr, d_items.get(), 0, k, db->m, err.get(), s);
    if (read_back(err.get(), s)) fail(BM_ERR_INVALID_ARG, "an item id is >= n_items");
  } else {
    for (uint32_t i = 0; i < k; ++i)
      if (items[i] >= db->m) fail(BM_ERR_INVALID_ARG, "items[%u] = %u >= n_items", i, items[i]);
    h_items.assign(items, items + k);
    upload(d_items.get(), h_items, s);
  }
  const Tuning tu;
  std::vector<DbInfo> hdb(1);
  hdb[0] = DbInfo{db->B.get(), db->Wp, db->W, db->n, nullptr, db->colsum.get(), 1, db->m};
  TBuf<DbInfo> ddb(1, s);
  upload(ddb.get(), hdb, s);
  StepWork w;
  std::vector<ClassDesc> hc;
  if (k >= 2) {
    hc.push_back(ClassDesc{0, 0, k, 0, 0, 0, 0});
    host_classes(w, hc, ddb.get(), hdb.data(), db->W, tu, false, s);
    KTimer tm(0u, s);
    run_class_kernels(ddb.get(), d_items.get(), w, tu, (double)db->W, (double)db->n, tm, s);
  }
  const bool out_dev = is_device_ptr(out);
  TBuf<uint32_t> d_out;
  uint32_t* dst = out;
  if (!out_dev) {
    d_out.alloc((size_t)k * k, s);
    dst = d_out.get();
  }
  launch_expand_pairs(k, d_items.get(), db->colsum.get(), w.tri.get(), dst, s);
  if (!out_dev)
    BM_HIP(hipMemcpyAsync(out, dst, (size_t)k * k * 4, hipMemcpyDeviceToHost, s));
  BM_HIP(hipStreamSynchronize(s));
}

// The allocation-free variant's scratch: one copy per GPU, held until the
// process ends.  Its host-side name is a stand-in, not a device address: host
// code only ever uses the address hipGetSymbolAddress returns for the current
// device.
constexpr size_t kScratchBytes = size_t(16) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_of_current_device() {
  int dev = 0;
  BM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(BM_ERR_UNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    BM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(BM_ERR_DEVICE, "no device address for the static scratch");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

void pair_support(const bm_db* db, const uint32_t* items, uint32_t k, uint32_t* out,
                  hipStream_t s) {
  pair_support_impl(db, items, k, out, s, false);
}

void pair_support_noalloc(const bm_db* db, const uint32_t* items, uint32_t k, uint32_t* out,
                          hipStream_t s) {
  if (k > kNoAllocMaxItems)
    fail(BM_ERR_UNSUPPORTED, "k = %u exceeds the allocation-free limit of %u items", k,
         kNoAllocMaxItems);
  if (k == 0) return;
  if (!out || !is_device_ptr(out))
    fail(BM_ERR_INVALID_ARG, "out must be device memory in the allocation-free call");
  if (items && !is_device_ptr(items))
    fail(BM_ERR_INVALID_ARG, "items must be device memory (or NULL) in the allocation-free call");
  StaticArena arena{static_cast<char*>(scratch_of_current_device()), kScratchBytes, 0};
  struct Restore {
    ~Restore() { t_arena = nullptr; }
  } restore;
  t_arena = &arena;
  pair_support_impl(db, items, k, out, s, true);
}

// ------------------------------------------------------------------ out of core

namespace {

// The blocks of a host CSR: block b holds transactions [b R, min(n, (b+1) R)),
// packed into the database handle's one matrix of m columns x Wp words (every
// block the same shape: the last one's missing rows are zero bits).  Loading
// copies the block's row offsets (rebased to 0) and item ids to the device and
// packs them, adding the block's column popcounts into `colsum`.
class HostBlocks : public BlockSource {
 public:
  HostBlocks(const uint64_t* rp, const uint32_t* ci, uint64_t n, uint32_t m, uint64_t R,
             bm_db* db, hipStream_t s)
      : rp_(rp), ci_(ci), n_(n), m_(m), R_(R), db_(db) {
    nb_ = n ? (n + R - 1) / R : 0;
    uint64_t most = 0;
    for (uint64_t b = 0; b < nb_; ++b) {
      const uint64_t b0 = b * R, b1 = std::min(n, b0 + R);
      most = std::max(most, rp[b1] - rp[b0]);
    }
    d_rp_.reset(R + 1, s);
    d_raw_.reset(R + 1, s);
    d_ci_.reset(std::max<uint64_t>(most, 1), s);
    err_.reset(1, s);
    scratch_sum_.reset(std::max<uint32_t>(m, 1), s);
    tiled_ = pack_tiled_ok(m, db->Wp);
  }
  uint64_t blocks() const override { return nb_; }
  uint32_t* err() const { return err_.get(); }
  // load into the matrix, the popcounts going to colsum (the database's own
  // in the first pass, a scratch array afterwards)
  void load_to(uint64_t b, uint32_t* colsum, hipStream_t s) {
    if (b == cur_) return;  // already in place (a database of one block)
    const uint64_t b0 = b * R_, b1 = std::min(n_, b0 + R_), rows = b1 - b0;
    const uint64_t base = rp_[b0];
    if (rp_[b1] < base) fail(BM_ERR_CSR, "row_ptr is not non-decreasing");
    const uint64_t nnz = rp_[b1] - base;
    // the block's row offsets, rebased to 0 on the device; the pack checks
    // their order and clamps every range to the block's nnz item ids
    BM_HIP(hipMemcpyAsync(d_raw_.get(), rp_ + b0, (rows + 1) * 8, hipMemcpyHostToDevice, s));
    if (nnz) BM_HIP(hipMemcpyAsync(d_ci_.get(), ci_ + base, nnz * 4, hipMemcpyHostToDevice, s));
    launch_rebase(d_raw_.get(), rows + 1, base, d_rp_.get(), s);
    uint64_t* B = db_->B.get();
    if (tiled_) {
      launch_pack_tiled(d_rp_.get(), d_ci_.get(), rows, m_, B, db_->Wp, colsum, err_.get(), s);
    } else {
      // the atomic pack trusts its ranges: check them first
      launch_validate(d_rp_.get(), d_ci_.get(), rows, nnz, m_, err_.get(), s);
      const uint32_t e = read_back(err_.get(), s);
      if (e & 1u) fail(BM_ERR_CSR, "row_ptr is not non-decreasing");
      if (e & 2u) fail(BM_ERR_CSR, "an item id is >= n_items (%u)", m_);
      launch_fill_u64(B, 0, (uint64_t)m_ * db_->Wp, s);
      launch_pack(d_rp_.get(), d_ci_.get(), rows, B, db_->Wp, s);
      launch_colsum(B, db_->Wp, m_, colsum, s);
    }
    cur_ = b;
  }
  void load(uint64_t b, hipStream_t s) override { load_to(b, scratch_sum_.get(), s); }

 private:
  const uint64_t* rp_;
  const uint32_t* ci_;
  uint64_t n_;
  uint32_t m_;
  uint64_t R_, nb_ = 0;
  bm_db* db_;
  bool tiled_ = true;
  uint64_t cur_ = ~0ull;
  DBuf<uint64_t> d_rp_, d_raw_;
  DBuf<uint32_t> d_ci_, err_, scratch_sum_;
};

}  // namespace

bm_result* mine_blocked(const uint64_t* row_ptr, const uint32_t* col_idx, uint64_t n, uint32_t m,
                        uint32_t minsup, uint64_t block_rows, const bm_options* opt, hipStream_t s) {
  if (!row_ptr) fail(BM_ERR_INVALID_ARG, "row_ptr is NULL");
  if (is_device_ptr(row_ptr) || (col_idx && is_device_ptr(col_idx)))
    fail(BM_ERR_INVALID_ARG, "blocked mining reads the transactions from host memory");
  if (minsup == 0) fail(BM_ERR_INVALID_ARG, "minsup must be >= 1");
  if (block_rows == 0) fail(BM_ERR_INVALID_ARG, "block_rows must be >= 1");
  if (n >= (1ull << 31)) fail(BM_ERR_UNSUPPORTED, "n_tx = %llu >= 2^31", (unsigned long long)n);
  if (row_ptr[0] != 0) fail(BM_ERR_CSR, "row_ptr[0] = %llu, expected 0",
                            (unsigned long long)row_ptr[0]);
  if (row_ptr[n] > 0 && !col_idx)
    fail(BM_ERR_INVALID_ARG, "col_idx is NULL but row_ptr[n] = %llu", (unsigned long long)row_ptr[n]);
  const uint64_t R = std::min<uint64_t>(block_rows, std::max<uint64_t>(n, 1));
  auto db = std::make_unique<bm_db>();
  BM_HIP(hipGetDevice(&db->device));
  db->n = n;
  db->m = m;
  db->Wp = padded_words(R);
  db->W = (R + 63) / 64;  // every block spans the same words; tasks are built once per step
  db->B.reset((size_t)m * db->Wp, s);
  db->colsum.reset(m, s);
  std::unique_ptr<HostBlocks> src;
  {
    CallScope scope(s);  // synchronises before anything above is freed on failure
    src.reset(new HostBlocks(row_ptr, col_idx, n, m, R, db.get(), s));
    if (m > 0) launch_fill_u32(db->colsum.get(), 0, m, s);
    launch_fill_u32(src->err(), 0, 1, s);
    // first pass: the single-item supports, summed over the blocks
    for (uint64_t b = 0; b < src->blocks() && m > 0; ++b) src->load_to(b, db->colsum.get(), s);
    const uint32_t e = read_back(src->err(), s);
    if (e & 1u) fail(BM_ERR_CSR, "row_ptr is not non-decreasing");
    if (e & 2u) fail(BM_ERR_CSR, "an item id is >= n_items (%u)", m);
  }
  // level by level (no whole-column subtree phases) and no projected views:
  // every kernel then sees only the block in the matrix
  bm_options o{};
  if (opt) o = *opt;
  o.flags |= BM_FLAG_LEVELSYNC | BM_FLAG_NO_PROJECT;
  o.flags &= ~(BM_FLAG_TRACE | BM_FLAG_DEPTH_FIRST);
  const bm_db* dp = db.get();
  auto r = mine_many(&dp, &minsup, 1, nullptr, &o, s, src.get());
  r[0]->n_tx = n;
  return r[0];
}

// ------------------------------------------------------------------ mining

std::vector<bm_result*> mine_many(const bm_db* const* dbs, const uint32_t* minsups, uint32_t N,
                                  const bm_model* sched, const bm_options* opt, hipStream_t s,
                                  BlockSource* blocks) {
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t d = 0; d < N; ++d)
    if (minsups[d] == 0) fail(BM_ERR_INVALID_ARG, "minsup of database %u must be >= 1", d);
  Tuning tu = tuning_from(opt);
  const uint32_t flags = opt ? opt->flags : 0u;
  int device = 0;
  BM_HIP(hipGetDevice(&device));
  auto store = std::make_shared<ResultStore>();
  bm_stats st{};
  st.mfma_form = tu.mfma_fp4 ? 1u : 0u;
  // the support-counting kernels; the rest only without BM_FLAG_TIMING_MAIN
  constexpr uint32_t kMainKinds = (1u << BM_K_BUILD) | (1u << BM_K_GRAM_MFMA) |
                                  (1u << BM_K_GRAM_MFMA_BIG) | (1u << BM_K_GRAM_SMALL) |
                                  (1u << BM_K_PROJECT) |
                                  (1u << BM_K_ANDPOP) | (1u << BM_K_ANDPOP_REG) | (1u << BM_K_DFS);
  KTimer tm(!(flags & BM_FLAG_TIMING) ? 0u
            : (flags & BM_FLAG_TIMING_MAIN) ? kMainKinds
                                            : (1u << BM_K_COUNT) - 1u,
            s);
  std::vector<uint64_t> Fs(N + 1, 0), Is(N + 1, 0);
  std::vector<std::vector<uint64_t>> per_level;  // [k] -> first node of each database (N+1)
  uint32_t K = 0;
  {
    CallScope scope(s);
    // ---- database table
    std::vector<DbInfo> hdb(N);
    std::vector<uint64_t> item_base(N + 1, 0);
    uint64_t Wmax = 1;
    double sumW = 0, sumN = 0;
    for (uint32_t d = 0; d < N; ++d) {
      const bm_db* b = dbs[d];
      const bool live = b && b->n > 0 && b->m > 0 && minsups[d] <= b->n;
      hdb[d] = DbInfo{};
      if (b) hdb[d] = DbInfo{b->B.get(), b->Wp, b->W, b->n, nullptr, b->colsum.get(), minsups[d],
                             live ? b->m : 0u};
      item_base[d + 1] = item_base[d] + hdb[d].m;
      if (live) {
        Wmax = std::max<uint64_t>(Wmax, b->W);
        sumW += (double)b->W;
        sumN += (double)b->n;
      }
    }
    const double nW = N ? sumW / N : 0, nN = N ? sumN / N : 0;  // per-database means for work counts
    // Long columns: small subtrees by subset counting (one workgroup would walk
    // a whole subtree, so the depth-first kernel is slow there).  Short
    // columns: level by level, where the subtree phase's fixed costs (merge,
    // read-back) measured more than it saves, unless the depth-first phase is
    // asked for -- by the flag, a cost model to order its queue, or a trace
    // of its tasks.
    if (tu.dfs && Wmax > tu.dfs_max_words) {
      tu.dfs = tu.subset_q >= 2;
      tu.subsets = tu.dfs;
      if (tu.subsets) tu.tiny_q = tu.subset_q;
    } else if (tu.dfs) {
      tu.dfs = sched != nullptr || (flags & (BM_FLAG_DEPTH_FIRST | BM_FLAG_TRACE)) != 0;
    }
    // the database table and the item bases in one upload
    static_assert(sizeof(DbInfo) % 8 == 0, "DbInfo is a whole number of words");
    const size_t tab_words = std::max<uint32_t>(N, 1) * (sizeof(DbInfo) / 8);
    TBuf<uint64_t> tables(tab_words + N + 1, s);
    {
      uint64_t* st_h = pinned_array<uint64_t>(tab_words + N + 1);
      std::memcpy(st_h, hdb.data(), N * sizeof(DbInfo));
      std::memcpy(st_h + tab_words, item_base.data(), (N + 1) * 8);
      BM_HIP(hipMemcpyAsync(tables.get(), st_h, (tab_words + N + 1) * 8, hipMemcpyHostToDevice, s));
    }
    DbInfo* const ddb_p = reinterpret_cast<DbInfo*>(tables.get());
    const uint64_t* const dibase_p = tables.get() + tab_words;
    const uint64_t total_items = item_base[N];

    // ---- frequent single items of every database
    std::vector<uint64_t> f1_base(N + 1, 0);
    TBuf<uint64_t> dfb(N + 1, s);
    TBuf<uint32_t> f1;
    std::vector<Level> L(1);
    if (total_items > 0) {
      tm.begin(BM_K_LEVEL);
      TBuf<uint32_t> fl(total_items, s);
      TBuf<uint64_t> pos(total_items + 1, s);
      launch_f1_flags(ddb_p, N, dibase_p, total_items, fl.get(), s);
      scan32(fl.get(), pos.get(), total_items, s);
      uint64_t* pf1 = pinned_array<uint64_t>(N + 1);
      launch_gather_idx(pos.get(), dibase_p, N + 1, dfb.get(), mapped(pf1), s);
      tm.end();
      BM_HIP(hipStreamSynchronize(s));
      std::copy(pf1, pf1 + N + 1, f1_base.begin());
      st.host_syncs++;
      const uint64_t M1 = f1_base[N];
      if (M1 > 0) {
        tm.begin(BM_K_LEVEL);
        f1.alloc(M1, s);
        launch_f1_fill(fl.get(), pos.get(), N, dibase_p, total_items, f1.get(), s);
        L.emplace_back();
        L[1].n = M1;
        L[1].item.alloc(M1, s);
        L[1].parent.alloc(M1, s);
        L[1].supp.alloc(M1, s);
        L[1].db.alloc(M1, s);
        launch_init_level1(ddb_p, N, dfb.get(), M1, f1.get(), L[1].item.get(), L[1].parent.get(),
                           L[1].supp.get(), L[1].db.get(), s);
        tm.end();
      }
    }
    st.n_frequent_items = (uint32_t)std::min<uint64_t>(f1_base[N], 0xffffffffu);
    if (f1_base[N]) st.frequent[1] = f1_base[N];

    // ---- level steps
    struct Part {
      const DfsTask* p;
      uint64_t n;
    };
    std::vector<Part> parts;                            // depth-first tasks of each step
    std::vector<const uint32_t*> step_pre(BM_MAX_LEVELS + 2, nullptr);
    std::vector<ClassDesc> roots;
    std::vector<int32_t> hpcls(std::max<uint32_t>(N, 1), -1);
    uint64_t tri_off = 0;
    for (uint32_t d = 0; d < N; ++d) {
      const uint64_t q = f1_base[d + 1] - f1_base[d];
      if (q >= 2) {
        hpcls[d] = (int32_t)roots.size();
        roots.push_back(ClassDesc{tri_off, (uint32_t)f1_base[d], (uint32_t)q, 0, 0, d, 0});
        tri_off += q * (q - 1) / 2;
      }
    }
    if (!roots.empty()) {
      // per-step statistics counters of every level step, zeroed once
      TBuf<unsigned long long> step_stats((size_t)(BM_MAX_LEVELS + 2) * NC_COUNT, s);
      launch_fill_u64(reinterpret_cast<uint64_t*>(step_stats.get()), 0,
                      (uint64_t)(BM_MAX_LEVELS + 2) * NC_COUNT, s);
      TBuf<int32_t> pcls_prev(hpcls.size(), s);
      upload(pcls_prev.get(), hpcls, s);
      auto w = std::make_unique<StepWork>();
      host_classes(*w, roots, ddb_p, hdb.data(), Wmax, tu, tu.dfs, s);
      uint32_t k = 1;
      for (;;) {
        const uint64_t nk = L[k].n;
        const uint64_t ls_cand = w->T - (tu.dfs ? w->st[ST_CAND_T] : 0);
        st.candidates[k + 1] += ls_cand;
        st.candidates_total += ls_cand;
        if (w->ndt) parts.push_back({w->dt.get(), w->ndt});
        step_pre[k] = w->pre.get();
        st.classes_mfma += w->st[ST_CLS_M] + w->st[ST_CLS_B] + w->st[ST_CLS_S];
        st.classes_andpop += w->st[ST_CLS_V] + w->st[ST_CLS_T];
        // every class of this step is a deferred subtree: no level-synchronous
        // level k + 1, so neither node counts nor a synchronisation are needed
        if (ls_cand == 0) break;
        if (blocks) {
          // out of core: every row block in turn, the supports summed over blocks
          for (uint64_t b = 0; b < blocks->blocks(); ++b) {
            blocks->load(b, s);
            run_class_kernels(ddb_p, L[k].item.get(), *w, tu, nW, nN, tm, s);
          }
        } else {
          if (w->nproj) project_views(*w, ddb_p, L[k].item.get(), Wmax, nW, tm, s);
          run_class_kernels(ddb_p, L[k].item.get(), *w, tu, nW, nN, tm, s);
        }

        tm.begin(BM_K_LEVEL);
        // each node counts the frequent entries of its triangle row (the
        // step's statistics counters were zeroed at the start of the call)
        unsigned long long* dst = step_stats.get() + (size_t)k * NC_COUNT;
        uint64_t* dst64 = reinterpret_cast<uint64_t*>(dst);
        TBuf<uint32_t> cnt(nk, s), iscls(nk, s);
        TBuf<uint64_t> trisz(nk, s);
        // projected classes of the next step: flags, row-list and view sizes per node
        const bool proj = tu.project_gain != 0;
        TBuf<uint32_t> pflag, prows;
        TBuf<uint64_t> pwords;
        if (proj) {
          pflag.alloc(nk, s);
          prows.alloc(nk, s);
          pwords.alloc(nk, s);
        }
        const uint32_t nb = node_batch(nk, w->T);
        launch_node_counts(nk, nb, k, L[k].parent.get(), pcls_prev.get(), w->cls.get(), ddb_p,
                           w->tri.get(), tu.mfma_min_q, tu.mfma_big_q, tu.mfma_small ? 1u : 0u,
                           tu.tiny_q, cnt.get(), iscls.get(), trisz.get(), dst,
                           L[k].supp.get(), proj ? tu.project_gain : 0u, pflag.get(), prows.get(),
                           pwords.get(),
                           s);
        L[k].cstart.alloc(nk + 1, s);
        TBuf<uint64_t> clspos(nk + 1, s), trioff(nk + 1, s);
        TBuf<uint64_t> pslot, prow_off, pword_off;
        if (proj) {
          pslot.alloc(nk + 1, s);
          prow_off.alloc(nk + 1, s);
          pword_off.alloc(nk + 1, s);
        }
        const void* ins[6] = {cnt.get(), iscls.get(), trisz.get(), pflag.get(), prows.get(),
                              pwords.get()};
        const bool is64[6] = {false, false, true, false, false, true};
        uint64_t* outs[6] = {L[k].cstart.get(), clspos.get(), trioff.get(), pslot.get(),
                             prow_off.get(), pword_off.get()};
        const int nscan = proj ? 6 : 3;
        // totals: next level size, classes, candidates (and projected classes,
        // their rows and view words); then the counters
        uint64_t* tot = pinned_array<uint64_t>(6 + NC_COUNT);
        scan_many_tot(ins, is64, outs, nscan, nk, mapped(tot), dst64, NC_COUNT, s);
        tm.end();
        BM_HIP(hipStreamSynchronize(s));
        st.host_syncs++;
        const uint64_t n_next = tot[0], ncls = tot[1], Tn = tot[2];
        const uint64_t* stt = tot + nscan;  // the step counters
        const uint64_t PM = stt[NC_PAIRS_M], PB = stt[NC_PAIRS_B], PV = stt[NC_PAIRS_V],
                       PVW = stt[NC_PAIRS_VW],
                       PT = stt[NC_TINY];
        if (n_next == 0) break;
        if (k + 1 > BM_MAX_LEVELS)
          fail(BM_ERR_UNSUPPORTED, "frequent itemsets longer than %d items", BM_MAX_LEVELS);
        if (n_next > 0xffffffffull) fail(BM_ERR_UNSUPPORTED, "more than 2^32 itemsets of one length");
        L.emplace_back();
        Level& Ln = L[k + 1];
        Ln.n = n_next;
        Ln.item.alloc(n_next, s);
        Ln.parent.alloc(n_next, s);
        Ln.supp.alloc(n_next, s);
        Ln.db.alloc(n_next, s);
        tm.begin(BM_K_LEVEL);
        LevelPost lp{};
        lp.n = nk;
        lp.nb = nb;
        lp.parent = L[k].parent.get();
        lp.pcls = pcls_prev.get();
        lp.cls = w->cls.get();
        lp.dbs = ddb_p;
        lp.child_item = L[k].item.get();
        lp.tri = w->tri.get();
        lp.child_start = L[k].cstart.get();
        lp.nitem = Ln.item.get();
        lp.nparent = Ln.parent.get();
        lp.nsupp = Ln.supp.get();
        lp.ndbv = Ln.db.get();
        st.frequent[k + 1] = n_next;
        if (ncls == 0) {
          launch_level_post(lp, s);
          tm.end();
          k += 1;
          break;
        }
        auto nw = std::make_unique<StepWork>();
        nw->ncls = ncls;
        nw->cls.alloc(ncls, s);
        nw->pre.alloc(ncls * k, s);
        TBuf<int32_t> pcls_k(nk, s);
        nw->T = Tn;
        nw->tri.alloc(Tn, s);
        for (int j = 0; j < ST_COUNT; ++j) nw->st[j] = stt[j];
        lp.k = k;
        lp.cnt = cnt.get();
        lp.cls_pos = clspos.get();
        lp.tri_off = trioff.get();
        lp.node_db = L[k].db.get();
        lp.ocls = nw->cls.get();
        lp.opre = nw->pre.get();
        lp.pcls_out = pcls_k.get();
        lp.ztri = nw->tri.get();
        lp.nz = Tn;
        lp.geo = make_geom(Wmax, PM, PV, PVW, PT, tu);
        lp.mfma_min_q = tu.mfma_min_q;
        lp.dfs = tu.dfs ? 1u : 0u;
        for (auto& c : nw->ccount) c.alloc(ncls, s);
        lp.cm = nw->ccount[0].get();
        lp.cv = nw->ccount[1].get();
        lp.ct = nw->ccount[2].get();
        lp.cb = nw->ccount[3].get();
        lp.cs = nw->ccount[4].get();
        nw->counts_ready = true;
        for (uint32_t j = 1; j <= k; ++j) {
          lp.lv.item[j] = L[j].item.get();
          lp.lv.parent[j] = L[j].parent.get();
        }
        if (proj && tot[3]) {
          // views of the next step's projected classes: level_post writes their
          // descriptors, the projection kernels fill them before the class kernels
          if (tot[3] > 0xffffffffull) fail(BM_ERR_UNSUPPORTED, "too many projected classes");
          nw->nproj = tot[3];
          nw->proj_rows = tot[4];
          nw->proj_words = tot[5];
          nw->proj_cols = stt[NC_PJ_COLS];
          nw->pj_cand[0] = (double)stt[NC_PJ_CAND_M];
          nw->pj_work[0] = (double)stt[NC_PJ_WORK_M];
          nw->pj_cand[1] = (double)stt[NC_PJ_CAND_B];
          nw->pj_work[1] = (double)stt[NC_PJ_WORK_B];
          nw->views.alloc(nw->nproj, s);
          nw->pwork.alloc(nw->nproj, s);
          nw->vbuf.alloc(nw->proj_words, s);
          lp.pflag = pflag.get();
          lp.pslot = pslot.get();
          lp.prow_off = prow_off.get();
          lp.pword_off = pword_off.get();
          lp.nodesupp = L[k].supp.get();
          lp.vbuf = nw->vbuf.get();
          lp.views = nw->views.get();
          lp.pwork = nw->pwork.get();
        }
        launch_level_post(lp, s);
        prepare_tasks(*nw, ddb_p, Wmax, PM, PB, PV, PVW, PT, tu, tu.dfs, k + 1, s);
        tm.end();
        w = std::move(nw);
        pcls_prev = pcls_k;
        k += 1;
      }
    }

    // ---- depth-first subtrees of the small classes, then the merged levels
    uint64_t D = 0;
    for (const auto& pt : parts) D += pt.n;
    if (D > 0) {
      if (D > 0xffffffffull) fail(BM_ERR_UNSUPPORTED, "too many subtree tasks");
      st.dfs_tasks = D;
      const uint32_t Kls = (uint32_t)L.size() - 1;
      TBuf<DfsTask> tasks(D, s);
      uint64_t at = 0;
      for (const auto& pt : parts) {
        BM_HIP(hipMemcpyAsync(tasks.get() + at, pt.p, pt.n * sizeof(DfsTask), hipMemcpyDeviceToDevice,
                              s));
        at += pt.n;
      }
      const bool trace = (flags & BM_FLAG_TRACE) != 0;
      TBuf<uint32_t> order;
      TBuf<float> feats;
      // subset counting needs no queue order: the model is not consulted
      const bool ordered = sched && !tu.subsets;
      tm.begin(BM_K_SCHED);
      if (ordered || trace) {
        feats.alloc(D * MLP_IN, s);
        FeatArgs fa{};
        fa.dbs = ddb_p;
        fa.tasks = tasks.get();
        fa.ntasks = (uint32_t)D;
        for (uint32_t j = 1; j <= Kls; ++j) {
          fa.lv_supp[j] = L[j].supp.get();
          fa.lv_parent[j] = L[j].parent.get();
        }
        fa.feats = feats.get();
        launch_dfs_features(fa, s);
      }
      std::vector<uint32_t> perm;
      if (ordered) {
        TBuf<float> pred(D, s);
        TBuf<uint32_t> hist(256, s);
        TBuf<uint64_t> hoff(257, s);
        order.alloc(D, s);
        model_predict_device(sched, feats.get(), D, pred.get(), s);
        launch_order_by_key(pred.get(), (uint32_t)D, hist.get(), hoff.get(), order.get(), s);
      } else if ((flags & BM_FLAG_SHUFFLE) && !tu.subsets) {
        perm.resize(D);
        for (uint64_t i = 0; i < D; ++i) perm[i] = (uint32_t)i;
        uint64_t x = 0x243F6A8885A308D3ull ^ (opt ? opt->shuffle_seed : 0u);
        for (uint64_t i = D - 1; i > 0; --i) {  // Fisher-Yates with splitmix64 draws
          x += 0x9E3779B97F4A7C15ull;
          uint64_t z = x;
          z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
          z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
          z ^= z >> 31;
          std::swap(perm[i], perm[z % (i + 1)]);
        }
        order.alloc(D, s);
        upload(order.get(), perm, s);
      }
      tm.end();
      // short-column databases' tasks go to the one-stack-per-wave kernel, the
      // rest to the one-stack-per-workgroup kernel; a stable split keeps the
      // queue order within each
      TBuf<uint32_t> qshort, qlong, qcnt;
      if (tu.dfs_wave_words && !tu.subsets) {
        TBuf<uint32_t> qflag(D, s);
        TBuf<uint64_t> qpos(D + 1, s);
        qshort.alloc(D, s);
        qlong.alloc(D, s);
        qcnt.alloc(2, s);
        launch_dfs_short_flags(tasks.get(), ddb_p, order.get(), (uint32_t)D, tu.dfs_wave_words,
                               qflag.get(), s);
        scan32(qflag.get(), qpos.get(), D, s);
        launch_dfs_split(order.get(), (uint32_t)D, qflag.get(), qpos.get(), qshort.get(), qlong.get(),
                         qcnt.get(), s);
      }
      std::vector<TBuf<uint32_t>> ls_first(Kls + 2), ls_count(Kls + 2);
      // one status block, zeroed and read back whole: statistics (candidates and
      // frequent sets by length, words read), then the queue heads and arena
      // count ([0] workgroup-queue head, [1] arena count, [2] wave-queue head)
      // and the flags
      constexpr size_t kStatWords = 2 * (BM_MAX_LEVELS + 1) + 1;
      TBuf<unsigned long long> status(kStatWords + 2, s);
      unsigned long long* lstat = status.get();
      uint32_t* ctrl = reinterpret_cast<uint32_t*>(status.get() + kStatWords);
      uint32_t* dflags = ctrl + 3;
      TBuf<float> cost;
      if (trace) cost.alloc(D, s);
      // subset counting: a counter block per task, and word ranges per task
      // enough for about eight workgroups per CU (ranges of >= 1,024 words)
      TBuf<uint32_t> scnt;
      uint32_t splits = 1;
      if (tu.subsets) {
        scnt.alloc(D << SUBSET_Q, s);
        const uint64_t want = ceil_div((uint64_t)cu_count() * 8, D);
        splits = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, Wmax / 1024));
        if (tu.split_words) splits = (uint32_t)ceil_div(std::max<uint64_t>(1, Wmax), tu.split_words);
        splits = std::max(splits, subset_min_splits(Wmax));
      }
      // workers reserve arena space ARENA_CHUNK (256) nodes at a time
      const uint64_t workers = (uint64_t)cu_count() * (16 + 2048 / tu.dfs_threads);
      uint64_t cap = tu.arena_nodes ? (uint64_t)tu.arena_nodes
                                    : std::max<uint64_t>(1u << 16, 32 * D) + workers * 256;
      TBuf<ArenaNode> arena;
      std::vector<unsigned long long> hstat(kStatWords);
      for (int attempt = 0;; ++attempt) {
        if (cap > 0xffffffffull) fail(BM_ERR_UNSUPPORTED, "depth-first output too large");
        arena.alloc(cap, s);
        ZeroSegs z{};
        auto zero = [&](uint32_t* p, uint64_t n) {
          if (z.count == kZeroSegs) {
            launch_zero_segs(z, s);
            z = ZeroSegs{};
          }
          z.p[z.count] = p;
          z.n[z.count] = n;
          ++z.count;
        };
        for (uint32_t j = 1; j <= Kls; ++j) {
          if (!ls_first[j].p) {
            ls_first[j].alloc(L[j].n, s);
            ls_count[j].alloc(L[j].n, s);
          }
          zero(ls_count[j].get(), L[j].n);
        }
        zero(reinterpret_cast<uint32_t*>(status.get()), 2 * (kStatWords + 2));
        if (tu.subsets) zero(scnt.get(), D << SUBSET_Q);
        launch_zero_segs(z, s);
        DfsArgs da{};
        da.dbs = ddb_p;
        da.tasks = tasks.get();
        da.ntasks = (uint32_t)D;
        da.order = order.get();
        da.queue_head = ctrl;
        for (uint32_t j = 1; j <= Kls; ++j) {
          da.lv_item[j] = L[j].item.get();
          da.step_pre[j] = step_pre[j];
          da.ls_first[j] = ls_first[j].get();
          da.ls_count[j] = ls_count[j].get();
        }
        da.arena = arena.get();
        da.arena_count = ctrl + 1;
        da.arena_cap = (uint32_t)cap;
        da.flags = dflags;
        da.level_cand = lstat;
        da.level_freq = lstat + (BM_MAX_LEVELS + 1);
        da.words_read = lstat + 2 * (BM_MAX_LEVELS + 1);
        da.task_cost = trace ? cost.get() : nullptr;
        tm.begin(BM_K_DFS);
        if (tu.subsets) {
          launch_subset_count(da, scnt.get(), splits, tu.tiny_q, s);
          launch_subset_emit(da, scnt.get(), s);
        } else if (tu.dfs_wave_words) {
          DfsArgs dw = da;
          dw.order = qshort.get();
          dw.ntasks_dev = qcnt.get();
          dw.queue_head = ctrl + 2;
          launch_dfs_wave(dw, (uint32_t)std::min<uint64_t>((D + 3) / 4, (uint64_t)cu_count() * 4), s);
          da.order = qlong.get();
          da.ntasks_dev = qcnt.get() + 1;
        }
        if (!tu.subsets)
          launch_dfs(da, tu.dfs_threads,
                     (uint32_t)std::min<uint64_t>(D, (uint64_t)cu_count() * (2048 / tu.dfs_threads)),
                     s);
        tm.end();
        unsigned long long* pst = pinned_array<unsigned long long>(kStatWords + 2);
        BM_HIP(hipMemcpyAsync(pst, status.get(), (kStatWords + 2) * 8, hipMemcpyDeviceToHost, s));
        BM_HIP(hipStreamSynchronize(s));
        const uint32_t* hc = reinterpret_cast<const uint32_t*>(pst + kStatWords);
        const uint32_t hf = hc[3];
        std::copy(pst, pst + kStatWords, hstat.begin());
        st.host_syncs++;
        if (hf & DFS_TOO_LONG)
          fail(BM_ERR_UNSUPPORTED, "frequent itemsets longer than %d items", BM_MAX_LEVELS);
        if (hf & DFS_STACK) fail(BM_ERR_DEVICE, "depth-first stack exhausted");
        if (hf & DFS_OVERFLOW) {
          // the count includes the blocks that did not fit but not their
          // unexplored subtrees: grow at least fourfold per attempt
          if (attempt >= 8) fail(BM_ERR_OOM, "depth-first output keeps overflowing");
          cap = std::max<uint64_t>(4 * cap, 2 * (uint64_t)hc[1]);
          continue;
        }
        break;
      }
      double dfs_cand = 0;
      for (int len = 0; len <= BM_MAX_LEVELS; ++len) {
        st.candidates[len] += hstat[len];
        st.candidates_total += hstat[len];
        dfs_cand += (double)hstat[len];
      }
      tm.set_last(8.0 * (double)hstat[2 * (BM_MAX_LEVELS + 1)], dfs_cand * nW);
      if (trace) {
        store->trace_rows = D;
        store->trace_feats.reset(D * MLP_IN, s);
        store->trace_cost.reset(D, s);
        BM_HIP(hipMemcpyAsync(store->trace_feats.get(), feats.get(), D * MLP_IN * 4,
                              hipMemcpyDeviceToDevice, s));
        BM_HIP(hipMemcpyAsync(store->trace_cost.get(), cost.get(), D * 4, hipMemcpyDeviceToDevice, s));
      }

      // merge: final level k+1 = the children of final level k's nodes, in order,
      // taken from the level-synchronous level k+1 or from the arena
      tm.begin(BM_K_EMIT);
      std::vector<Level> FL(2);
      std::vector<TBuf<uint32_t>> skind(2), sfirst(2), scount(2);
      FL[1].n = L[1].n;
      FL[1].item.alloc(L[1].n, s);
      FL[1].parent.alloc(L[1].n, s);
      FL[1].supp.alloc(L[1].n, s);
      FL[1].db.alloc(L[1].n, s);
      skind[1].alloc(L[1].n, s);
      sfirst[1].alloc(L[1].n, s);
      scount[1].alloc(L[1].n, s);
      launch_fin_level1(L[1].n, L[1].item.get(), L[1].parent.get(), L[1].supp.get(), L[1].db.get(),
                        Kls >= 2 ? L[1].cstart.get() : nullptr, ls_first[1].get(),
                        ls_count[1].get(), FL[1].item.get(), FL[1].parent.get(), FL[1].supp.get(),
                        FL[1].db.get(), skind[1].get(), sfirst[1].get(), scount[1].get(), s);
      // every level-synchronous node and every arena node is final, so the
      // final level sizes are known without reading anything back
      for (uint32_t k = 1;; ++k) {
        const uint64_t nk = FL[k].n;
        FL[k].cstart.alloc(nk + 1, s);
        scan32(scount[k].get(), FL[k].cstart.get(), nk, s);
        const uint64_t nn = (k + 1 <= Kls ? L[k + 1].n : 0) +
                            (k + 1 <= BM_MAX_LEVELS ? (uint64_t)hstat[BM_MAX_LEVELS + 1 + k + 1] : 0);
        if (nn == 0) break;
        if (k + 1 > BM_MAX_LEVELS)
          fail(BM_ERR_UNSUPPORTED, "frequent itemsets longer than %d items", BM_MAX_LEVELS);
        FL.emplace_back();
        skind.emplace_back();
        sfirst.emplace_back();
        scount.emplace_back();
        Level& Fn = FL[k + 1];
        Fn.n = nn;
        Fn.item.alloc(nn, s);
        Fn.parent.alloc(nn, s);
        Fn.supp.alloc(nn, s);
        Fn.db.alloc(nn, s);
        skind[k + 1].alloc(nn, s);
        sfirst[k + 1].alloc(nn, s);
        scount[k + 1].alloc(nn, s);
        const bool has_ls = k + 1 <= Kls;
        launch_fin_gather(nk, FL[k].db.get(), skind[k].get(), sfirst[k].get(), scount[k].get(),
                          FL[k].cstart.get(), has_ls ? L[k + 1].item.get() : nullptr,
                          has_ls ? L[k + 1].supp.get() : nullptr, has_ls ? L[k + 1].db.get() : nullptr,
                          (k + 2 <= Kls) ? L[k + 1].cstart.get() : nullptr,
                          has_ls ? ls_first[k + 1].get() : nullptr,
                          has_ls ? ls_count[k + 1].get() : nullptr, arena.get(), Fn.item.get(),
                          Fn.parent.get(), Fn.supp.get(), Fn.db.get(), skind[k + 1].get(),
                          sfirst[k + 1].get(), scount[k + 1].get(), s);
      }
      tm.end();
      for (uint32_t k = 1; k < FL.size(); ++k) st.frequent[k] = FL[k].n;
      L.swap(FL);
    }

    // ---- canonical output (all databases as one forest, database by database)
    K = (uint32_t)L.size() - 1;
    uint64_t F = 0, TI = 0;
    for (uint32_t k = 1; k <= K; ++k) {
      F += L[k].n;
      TI += (uint64_t)k * L[k].n;
    }
    st.max_len = K;
    st.frequent_total = F;
    store->offsets.reset(F + 1, s);
    store->items.reset(TI, s);
    store->supports.reset(F, s);
    if (F == 0) {
      launch_fill_u64(store->offsets.get(), 0, 1, s);
    } else {
      tm.begin(BM_K_EMIT);
      EmitArgs ea{};
      uint64_t acc = 0;
      for (uint32_t k = 1; k <= K; ++k) {
        ea.item[k] = L[k].item.get();
        ea.parent[k] = L[k].parent.get();
        ea.cstart[k] = k < K ? L[k].cstart.get() : nullptr;
        ea.supp[k] = L[k].supp.get();
        ea.node_db[k] = L[k].db.get();
        ea.base[k] = acc;
        acc += L[k].n;
      }
      ea.base[K + 1] = acc;
      const size_t rows = (size_t)N + 1, nhb = (size_t)(K + 1) * rows;
      uint64_t* phb = pinned_array<uint64_t>(nhb + 2 * rows);
      ea.dbs = ddb_p;
      ea.first_root = dfb.get();
      ea.o_off = store->offsets.get();
      ea.o_items = store->items.get();
      ea.o_supp = store->supports.get();
      ea.bounds = mapped(phb);
      ea.slices = mapped(phb + nhb);
      ea.K = K;
      ea.N = N;
      launch_emit_all(ea, F, s);
      tm.end();
      BM_HIP(hipStreamSynchronize(s));
      st.host_syncs++;
      const uint64_t* pFs = phb + nhb;
      const uint64_t* pIs = phb + nhb + rows;
      std::copy(pFs, pFs + N + 1, Fs.begin());
      std::copy(pIs, pIs + N + 1, Is.begin());
      const std::vector<uint64_t> hb(phb, phb + nhb);
      per_level.assign(K + 1, {});
      for (uint32_t k = 1; k <= K; ++k)
        per_level[k].assign(hb.begin() + (size_t)k * (N + 1), hb.begin() + (size_t)(k + 1) * (N + 1));
    }
    BM_HIP(hipStreamSynchronize(s));
  }
  tm.collect(&st);
  st.wall_ms = ms_since(t0);
  std::vector<bm_result*> out(N, nullptr);
  for (uint32_t d = 0; d < N; ++d) {
    auto r = std::make_unique<bm_result>();
    r->device = device;
    r->store = store;
    r->set0 = Fs[d];
    r->n_sets = Fs[d + 1] - Fs[d];
    r->item0 = Is[d];
    r->n_items = Is[d + 1] - Is[d];
    r->stats = st;
    if (N > 1) {
      // per-database counts; candidates and kernel times stay batch-wide
      std::fill(std::begin(r->stats.frequent), std::end(r->stats.frequent), 0ull);
      uint32_t ml = 0;
      for (uint32_t k = 1; k <= K && !per_level.empty(); ++k) {
        const uint64_t c = per_level[k][d + 1] - per_level[k][d];
        r->stats.frequent[k] = c;
        if (c) ml = k;
      }
      r->stats.max_len = ml;
      r->stats.frequent_total = r->n_sets;
      r->stats.n_frequent_items = (uint32_t)r->stats.frequent[1];
    }
    r->max_len = r->stats.max_len;
    r->n_tx = dbs[d] ? dbs[d]->n : 0;
    out[d] = r.release();
  }
  return out;
}

void result_copy(const bm_result* r, uint64_t* offsets, uint32_t* items, uint32_t* supports,
                 hipStream_t s) {
  CallScope scope(s);
  const ResultStore& st = *r->store;
  if (offsets) {
    if (r->item0 == 0) {
      BM_HIP(hipMemcpyAsync(offsets, st.offsets.get() + r->set0, (r->n_sets + 1) * 8,
                            hipMemcpyDefault, s));
    } else if (is_device_ptr(offsets)) {
      launch_rebase(st.offsets.get() + r->set0, r->n_sets + 1, r->item0, offsets, s);
    } else {
      TBuf<uint64_t> tmp(r->n_sets + 1, s);
      launch_rebase(st.offsets.get() + r->set0, r->n_sets + 1, r->item0, tmp.get(), s);
      BM_HIP(hipMemcpyAsync(offsets, tmp.get(), (r->n_sets + 1) * 8, hipMemcpyDeviceToHost, s));
    }
  }
  if (items && r->n_items)
    BM_HIP(hipMemcpyAsync(items, st.items.get() + r->item0, r->n_items * 4, hipMemcpyDefault, s));
  if (supports && r->n_sets)
    BM_HIP(hipMemcpyAsync(supports, st.supports.get() + r->set0, r->n_sets * 4, hipMemcpyDefault, s));
  BM_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------ rules

bm_rules* rules_mine(const bm_result* r, uint32_t min_conf_ppm, uint32_t max_len, hipStream_t s) {
  if (min_conf_ppm > 1000000u) fail(BM_ERR_INVALID_ARG, "min_conf_ppm must be at most 10^6");
  if (max_len == 0) max_len = RULE_DEFAULT_LEN;
  if (max_len > RULE_MAX_LEN)
    fail(BM_ERR_UNSUPPORTED, "rules of itemsets longer than %u items are not listed", RULE_MAX_LEN);
  std::unique_ptr<bm_rules> out(new bm_rules);
  CallScope scope(s);  // after out: on failure it synchronises before out is freed
  BM_HIP(hipGetDevice(&out->device));
  const uint64_t nF = r->n_sets;
  if (nF == 0) return out.release();
  const ResultStore& st = *r->store;
  RuleArgs a{};
  a.offs = st.offsets.get() + r->set0;  // item offsets count from the store's first item
  a.items = st.items.get();
  a.supp = st.supports.get() + r->set0;
  a.nF = nF;
  a.n = r->n_tx;
  a.min_conf_ppm = min_conf_ppm;
  a.max_len = max_len;
  TBuf<uint32_t> cnt(nF, s), status(1, s);
  TBuf<uint64_t> pos(nF + 1, s);
  launch_fill_u32(status.get(), 0, 1, s);
  a.count = cnt.get();
  a.status = status.get();
  launch_rules_count(a, s);
  scan32(cnt.get(), pos.get(), nF, s);
  const uint64_t R = read_back(pos.get() + nF, s);
  if (read_back(status.get(), s))
    fail(BM_ERR_DEVICE, "a subset of a mined itemset is missing from the result");
  out->n = R;
  out->z.reset(R, s);
  out->mask.reset(R, s);
  out->sx.reset(R, s);
  out->sy.reset(R, s);
  out->sz.reset(R, s);
  out->conf.reset(R, s);
  out->lift.reset(R, s);
  if (R) {
    a.pos = pos.get();
    a.rz = out->z.get();
    a.rmask = out->mask.get();
    a.rsx = out->sx.get();
    a.rsy = out->sy.get();
    a.rsz = out->sz.get();
    a.rconf = out->conf.get();
    a.rlift = out->lift.get();
    launch_rules_emit(a, s);
  }
  BM_HIP(hipStreamSynchronize(s));
  return out.release();
}

void rules_copy(const bm_rules* rs, uint64_t* z, uint32_t* mask, uint32_t* sx, uint32_t* sy,
                uint32_t* sz, double* conf, double* lift, hipStream_t s) {
  const uint64_t R = rs->n;
  if (R == 0) return;
  if (z) BM_HIP(hipMemcpyAsync(z, rs->z.get(), R * 8, hipMemcpyDefault, s));
  if (mask) BM_HIP(hipMemcpyAsync(mask, rs->mask.get(), R * 4, hipMemcpyDefault, s));
  if (sx) BM_HIP(hipMemcpyAsync(sx, rs->sx.get(), R * 4, hipMemcpyDefault, s));
  if (sy) BM_HIP(hipMemcpyAsync(sy, rs->sy.get(), R * 4, hipMemcpyDefault, s));
  if (sz) BM_HIP(hipMemcpyAsync(sz, rs->sz.get(), R * 4, hipMemcpyDefault, s));
  if (conf) BM_HIP(hipMemcpyAsync(conf, rs->conf.get(), R * 8, hipMemcpyDefault, s));
  if (lift) BM_HIP(hipMemcpyAsync(lift, rs->lift.get(), R * 8, hipMemcpyDefault, s));
  BM_HIP(hipStreamSynchronize(s));
}

void result_trace(const bm_result* r, float* feats, float* labels, uint64_t* rows) {
  const ResultStore& st = *r->store;
  const uint64_t n = st.trace_rows;
  if (rows) *rows = n;
  if (n == 0) return;
  if (feats) BM_HIP(hipMemcpy(feats, st.trace_feats.get(), n * MLP_IN * 4, hipMemcpyDefault));
  if (labels) {
    std::vector<float> c(n);
    BM_HIP(hipMemcpy(c.data(), st.trace_cost.get(), n * 4, hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < n; ++i) labels[i] = std::log2(1.0f + c[i]);
  }
}

}  // namespace bm
