// Matrix construction, pair supports and the level-synchronous miner.
//
// bm_build (Section III, matrix construction, Eq. 1) validates the CSR on the
// device, packs it into column bitsets and counts every column (Eq. 3's
// column aggregation).  bm_mine extends frequent prefixes level by level
// (the paper's recursive mining by sequential column ANDs):
//   level 1: frequent single items (column popcounts >= minsup);
//   level 2: all pairs of frequent items -- the Gram matrix A^T A on int8 MFMA
//            (or AND+popcount when there are few items);
//   level k+1: every prefix class of level k (nodes sharing a parent) evaluates
//            its q(q-1)/2 sibling pairs, big classes as a masked Gram matrix on
//            MFMA, small ones with AND+popcount;
// and finally writes the frequent itemsets in canonical order.  One host sync
// per level reads back the next level's sizes.
#include <algorithm>
#include <chrono>
#include <memory>
#include <vector>

#include "handles.hpp"
#include "levels.hpp"

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

template <class T>
struct TBuf {  // temporary device buffer bound to the current call scope
  T* p = nullptr;
  size_t n = 0;
  TBuf() = default;
  TBuf(size_t count, hipStream_t s) { alloc(count, s); }
  void alloc(size_t count, hipStream_t s) {
    n = count;
    p = count ? static_cast<T*>(dalloc(count * sizeof(T), s)) : nullptr;
    if (p) t_scope->held.push_back(p);
  }
  T* get() const { return p; }
};

class CallScope {
 public:
  explicit CallScope(hipStream_t s) : sc_{s, {}} {
    prev_ = t_scope;
    t_scope = &sc_;
  }
  ~CallScope() {
    (void)hipStreamSynchronize(sc_.s);
    for (void* p : sc_.held) dfree(p, sc_.s);
    t_scope = prev_;
  }

 private:
  Scope sc_;
  Scope* prev_;
};

template <class T>
T read_back(const T* dev, hipStream_t s) {
  T v{};
  BM_HIP(hipMemcpyAsync(&v, dev, sizeof(T), hipMemcpyDeviceToHost, s));
  BM_HIP(hipStreamSynchronize(s));
  return v;
}

void scan_ge(const uint32_t* in, uint32_t thr, uint64_t* out, uint64_t n, hipStream_t s) {
  TBuf<uint64_t> tmp(scan_tmp_words(n), s);
  scan_ge_u32(in, thr, out, n, tmp.get(), s);
}
void scan32(const uint32_t* in, uint64_t* out, uint64_t n, hipStream_t s) {
  TBuf<uint64_t> tmp(scan_tmp_words(n), s);
  scan_u32_to_u64(in, out, n, tmp.get(), s);
}
void scan64(const uint64_t* in, uint64_t* out, uint64_t n, hipStream_t s) {
  TBuf<uint64_t> tmp(scan_tmp_words(n), s);
  scan_u64(in, out, n, tmp.get(), s);
}

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
uint64_t round_up(uint64_t a, uint64_t b) { return ceil_div(a, b) * b; }

TaskGeom make_geom(uint64_t W, uint64_t pairs_m, uint64_t pairs_v, uint64_t classes_t,
                   const Tuning& tu) {
  const uint64_t target = (uint64_t)cu_count() * 8;
  TaskGeom g{};
  const uint64_t Wm = std::max<uint64_t>(16, round_up(W, GRAM_KW));
  uint64_t sm;
  if (tu.split_words) {
    sm = round_up(tu.split_words, GRAM_KW);
  } else {
    uint64_t ns = pairs_m ? ceil_div(target, pairs_m) : 1;
    ns = std::min<uint64_t>(ns, std::max<uint64_t>(1, Wm / 256));
    sm = round_up(ceil_div(Wm, ns), GRAM_KW);
  }
  g.split_m = (uint32_t)sm;
  g.nsplit_m = (uint32_t)ceil_div(Wm, sm);
  g.wend_m = (uint32_t)Wm;
  const uint64_t Wv = std::max<uint64_t>(1, W);
  uint64_t sv;
  if (tu.split_words) {
    sv = tu.split_words;
  } else {
    uint64_t ns = pairs_v ? ceil_div(target, pairs_v) : 1;
    ns = std::min<uint64_t>(ns, std::max<uint64_t>(1, Wv / 512));
    sv = ceil_div(Wv, ns);
  }
  g.split_v = (uint32_t)sv;
  g.nsplit_v = (uint32_t)ceil_div(Wv, sv);
  g.wend_v = (uint32_t)Wv;
  uint64_t st;
  if (tu.split_words) {
    st = tu.split_words;
  } else {
    uint64_t ns = classes_t ? ceil_div(target, classes_t) : 1;
    ns = std::min<uint64_t>(ns, std::max<uint64_t>(1, Wv / 2048));
    st = round_up(ceil_div(Wv, ns), 64);
  }
  g.split_t = (uint32_t)st;
  g.nsplit_t = (uint32_t)ceil_div(Wv, st);
  g.wend_t = (uint32_t)Wv;
  return g;
}

// Device-side work of one level step.
struct StepWork {
  TBuf<ClassDesc> cls;
  TBuf<uint32_t> pre;
  TBuf<Task> tm, tv, tt;
  uint64_t ntm = 0, ntv = 0, ntt = 0;
  TBuf<uint32_t> tri;
  uint64_t T = 0;
  uint64_t st[ST_COUNT] = {};
};

void run_class_kernels(const bm_db* db, const uint32_t* f1, const uint32_t* child_item,
                       const StepWork& w, const Tuning& tu, KTimer& tm, hipStream_t s) {
  ClassArgs a{db->B.get(), db->Wp, f1, child_item, w.cls.get(), w.pre.get(), nullptr, 0, w.tri.get()};
  const uint64_t ncu = (uint64_t)cu_count();
  if (w.ntm) {
    if (w.ntm > 0xffffffffull) fail(BM_ERR_UNSUPPORTED, "too many MFMA tasks");
    a.tasks = w.tm.get();
    a.ntasks = (uint32_t)w.ntm;
    tm.begin(BM_K_GRAM_MFMA);
    launch_gram_mfma(a, (uint32_t)std::min<uint64_t>(w.ntm, ncu * 4), s);
    tm.end(8.0 * (double)db->W * (double)w.st[ST_COLS_M],
           2.0 * (double)w.st[ST_CAND_M] * (double)db->n);
  }
  if (w.ntv) {
    if (w.ntv > 0xffffffffull) fail(BM_ERR_UNSUPPORTED, "too many AND+popcount tasks");
    a.tasks = w.tv.get();
    a.ntasks = (uint32_t)w.ntv;
    tm.begin(BM_K_ANDPOP);
    launch_andpop(a, tu.andpop_chunk, (uint32_t)std::min<uint64_t>(w.ntv, ncu * 8), s);
    tm.end(8.0 * (double)db->W * (double)w.st[ST_COLS_V], (double)w.st[ST_CAND_V] * (double)db->W);
  }
  if (w.ntt) {
    if (w.ntt > 0xffffffffull) fail(BM_ERR_UNSUPPORTED, "too many AND+popcount tasks");
    a.tasks = w.tt.get();
    a.ntasks = (uint32_t)w.ntt;
    tm.begin(BM_K_ANDPOP_REG);
    launch_andpop_reg(a, (uint32_t)std::min<uint64_t>(w.ntt, ncu * 8), s);
    tm.end(8.0 * (double)db->W * (double)w.st[ST_COLS_T], (double)w.st[ST_CAND_T] * (double)db->W);
  }
}

// One class (the root, or an explicit column list) with q children.
void single_class(StepWork& w, uint32_t q, uint64_t W, const Tuning& tu, hipStream_t s) {
  ClassDesc cd{0, 0, q, 0, 0};
  w.cls.alloc(1, s);
  BM_HIP(hipMemcpyAsync(w.cls.get(), &cd, sizeof(cd), hipMemcpyHostToDevice, s));
  w.pre.alloc(1, s);
  launch_fill_u32(w.pre.get(), 0, 1, s);
  w.T = (uint64_t)q * (q - 1) / 2;
  w.tri.alloc(w.T, s);
  launch_fill_u32(w.tri.get(), 0, w.T, s);
  const int kind = class_kind(q, tu.mfma_min_q);
  const uint64_t pm = kind == 0 ? host_mfma_pairs(q) : 0;
  const uint64_t pv = kind == 1 ? host_andpop_pairs(q) : 0;
  const TaskGeom g = make_geom(W, pm, pv, kind == 2 ? 1 : 0, tu);
  if (kind == 0) {
    w.ntm = pm * g.nsplit_m;
    w.tm.alloc(w.ntm, s);
    launch_root_tasks(q, (uint32_t)pm, GRAM_TILE, g.nsplit_m, g.split_m, g.wend_m, w.tm.get(), s);
  } else if (kind == 1) {
    w.ntv = pv * g.nsplit_v;
    w.tv.alloc(w.ntv, s);
    launch_root_tasks(q, (uint32_t)pv, AP_BLOCK, g.nsplit_v, g.split_v, g.wend_v, w.tv.get(), s);
  } else {
    w.ntt = g.nsplit_t;
    w.tt.alloc(w.ntt, s);
    launch_root_tasks(q, 1, TINY_Q, g.nsplit_t, g.split_t, g.wend_t, w.tt.get(), s);
  }
  w.st[ST_CAND_M + kind] = w.T;
  w.st[ST_COLS_M + kind] = q;
  w.st[ST_CLS_M + kind] = 1;
  // hipMemcpyAsync from pageable memory may still read `cd` after returning
  BM_HIP(hipStreamSynchronize(s));
}

struct Level {
  uint64_t n = 0;
  TBuf<uint32_t> item, parent, supp;
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
  if (opt->flags & BM_FLAG_NO_MFMA) t.mfma_min_q = 0xffffffffu;
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
  uint64_t rp0 = 0, nnz = 0;
  if (rp_dev) {
    BM_HIP(hipMemcpy(&rp0, row_ptr, 8, hipMemcpyDeviceToHost));
    BM_HIP(hipMemcpy(&nnz, row_ptr + n, 8, hipMemcpyDeviceToHost));
  } else {
    rp0 = row_ptr[0];
    nnz = row_ptr[n];
  }
  if (rp0 != 0) fail(BM_ERR_CSR, "row_ptr[0] = %llu, expected 0", (unsigned long long)rp0);
  if (nnz > 0 && !col_idx) fail(BM_ERR_INVALID_ARG, "col_idx is NULL but row_ptr[n] = %llu",
                                (unsigned long long)nnz);
  const double words = (double)m * (double)db->Wp;
  if (words * 8.0 > 1.0e15) fail(BM_ERR_UNSUPPORTED, "bitset matrix too large");

  const uint64_t* d_rp = row_ptr;
  TBuf<uint64_t> rp_copy;
  if (!rp_dev) {
    rp_copy.alloc(n + 1, s);
    BM_HIP(hipMemcpyAsync(rp_copy.get(), row_ptr, (n + 1) * 8, hipMemcpyHostToDevice, s));
    d_rp = rp_copy.get();
  }
  const uint32_t* d_ci = col_idx;
  TBuf<uint32_t> ci_copy;
  if (nnz > 0 && !is_device_ptr(col_idx)) {
    ci_copy.alloc(nnz, s);
    BM_HIP(hipMemcpyAsync(ci_copy.get(), col_idx, nnz * 4, hipMemcpyHostToDevice, s));
    d_ci = ci_copy.get();
  }
  TBuf<uint32_t> err(1, s);
  launch_fill_u32(err.get(), 0, 1, s);
  db->B.reset((size_t)m * db->Wp, s);
  db->colsum.reset(m, s);
  if (m > 0) {
    launch_fill_u32(db->colsum.get(), 0, m, s);
    // row_ptr monotonicity first (flag only); the tiled pack clamps element
    // ranges, flags ids >= m and writes every word of M.
    launch_validate(d_rp, nullptr, n, 0, m, err.get(), s);
    if (!launch_pack_tiled(d_rp, d_ci, n, nnz, m, db->B.get(), db->Wp, db->colsum.get(), err.get(),
                           s)) {
      launch_validate(d_rp, d_ci, n, nnz, m, err.get(), s);
      const uint32_t e0 = read_back(err.get(), s);
      if (e0 & 1u) fail(BM_ERR_CSR, "row_ptr is not non-decreasing");
      if (e0 & 2u) fail(BM_ERR_CSR, "an item id is >= n_items (%u)", m);
      launch_fill_u64(db->B.get(), 0, (uint64_t)m * db->Wp, s);
      launch_pack(d_rp, d_ci, n, db->B.get(), db->Wp, s);
      launch_colsum(db->B.get(), db->Wp, m, db->colsum.get(), s);
    }
  } else {
    launch_validate(d_rp, d_ci, n, nnz, m, err.get(), s);
  }
  const uint32_t e = read_back(err.get(), s);
  if (e & 1u) fail(BM_ERR_CSR, "row_ptr is not non-decreasing");
  if (e & 2u) fail(BM_ERR_CSR, "an item id is >= n_items (%u)", m);
  BM_HIP(hipStreamSynchronize(s));
  return db.release();
}

// ------------------------------------------------------------------ pairs

void pair_support(const bm_db* db, const uint32_t* items, uint32_t k, uint32_t* out,
                  hipStream_t s) {
  if (k == 0) return;
  if (!out) fail(BM_ERR_INVALID_ARG, "out is NULL");
  if (!items && k != db->m) fail(BM_ERR_INVALID_ARG, "items == NULL requires k == n_items");
  CallScope scope(s);
  TBuf<uint32_t> d_items(k, s);
  if (!items) {
    std::vector<uint32_t> h(k);
    for (uint32_t i = 0; i < k; ++i) h[i] = i;
    BM_HIP(hipMemcpyAsync(d_items.get(), h.data(), (size_t)k * 4, hipMemcpyHostToDevice, s));
    BM_HIP(hipStreamSynchronize(s));
  } else if (is_device_ptr(items)) {
    BM_HIP(hipMemcpyAsync(d_items.get(), items, (size_t)k * 4, hipMemcpyDeviceToDevice, s));
    TBuf<uint32_t> err(1, s);
    launch_fill_u32(err.get(), 0, 1, s);
    launch_validate(nullptr, d_items.get(), 0, k, db->m, err.get(), s);
    if (read_back(err.get(), s)) fail(BM_ERR_INVALID_ARG, "an item id is >= n_items");
  } else {
    for (uint32_t i = 0; i < k; ++i)
      if (items[i] >= db->m) fail(BM_ERR_INVALID_ARG, "items[%u] = %u >= n_items", i, items[i]);
    BM_HIP(hipMemcpyAsync(d_items.get(), items, (size_t)k * 4, hipMemcpyHostToDevice, s));
    BM_HIP(hipStreamSynchronize(s));
  }
  const Tuning tu;
  StepWork w;
  if (k >= 2) {
    single_class(w, k, db->W, tu, s);
    KTimer tm(false, s);
    run_class_kernels(db, nullptr, d_items.get(), w, tu, tm, s);
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

// ------------------------------------------------------------------ mining

bm_result* mine(const bm_db* db, uint32_t minsup, const bm_options* opt, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  if (minsup == 0) fail(BM_ERR_INVALID_ARG, "minsup must be >= 1");
  const Tuning tu = tuning_from(opt);
  const uint32_t flags = opt ? opt->flags : 0u;
  std::unique_ptr<bm_result> res(new bm_result);
  res->device = db->device;
  bm_stats& st = res->stats;
  KTimer tm((flags & BM_FLAG_TIMING) != 0, s);
  {
    CallScope scope(s);
    const uint32_t m = db->m;
    const uint64_t n = db->n;
    std::vector<Level> L(1);
    TBuf<uint32_t> f1;
    uint64_t m1 = 0;
    if (n > 0 && m > 0 && minsup <= n) {
      TBuf<uint64_t> pos(m + 1, s);
      tm.begin(BM_K_LEVEL);
      scan_ge(db->colsum.get(), minsup, pos.get(), m, s);
      tm.end();
      m1 = read_back(pos.get() + m, s);
      st.host_syncs++;
      if (m1 > 0) {
        f1.alloc(m1, s);
        launch_f1_fill(db->colsum.get(), m, minsup, pos.get(), f1.get(), s);
        L.emplace_back();
        L[1].n = m1;
        L[1].item.alloc(m1, s);
        L[1].parent.alloc(m1, s);
        L[1].supp.alloc(m1, s);
        launch_init_level1(db->colsum.get(), f1.get(), (uint32_t)m1, L[1].item.get(),
                           L[1].parent.get(), L[1].supp.get(), s);
      }
    }
    st.n_frequent_items = (uint32_t)m1;
    if (m1 > 0) st.frequent[1] = m1;

    // ---- level steps
    if (m1 >= 2) {
      TBuf<int32_t> pcls_prev(1, s);
      launch_fill_u32(reinterpret_cast<uint32_t*>(pcls_prev.get()), 0, 1, s);
      auto w = std::make_unique<StepWork>();
      single_class(*w, (uint32_t)m1, db->W, tu, s);
      uint32_t k = 1;
      for (;;) {
        const uint64_t nk = L[k].n;
        st.candidates[k + 1] = w->T;
        st.candidates_total += w->T;
        st.classes_mfma += w->st[ST_CLS_M];
        st.classes_andpop += w->st[ST_CLS_V] + w->st[ST_CLS_T];
        run_class_kernels(db, f1.get(), L[k].item.get(), *w, tu, tm, s);

        tm.begin(BM_K_LEVEL);
        TBuf<uint64_t> S(w->T + 1, s);
        scan_ge(w->tri.get(), minsup, S.get(), w->T, s);
        TBuf<uint32_t> cnt(nk, s), iscls(nk, s), pm(nk, s), pv(nk, s), pt(nk, s);
        TBuf<uint64_t> trisz(nk, s);
        TBuf<unsigned long long> dst(ST_COUNT, s);
        launch_fill_u64(reinterpret_cast<uint64_t*>(dst.get()), 0, ST_COUNT, s);
        launch_node_counts(nk, k, L[k].parent.get(), pcls_prev.get(), w->cls.get(), S.get(),
                           tu.mfma_min_q, cnt.get(), iscls.get(), trisz.get(), pm.get(), pv.get(),
                           pt.get(), dst.get(), s);
        L[k].cstart.alloc(nk + 1, s);
        TBuf<uint64_t> clspos(nk + 1, s), trioff(nk + 1, s), pmoff(nk + 1, s), pvoff(nk + 1, s),
            ptoff(nk + 1, s);
        ScanMulti sm{};
        const void* ins[6] = {cnt.get(), iscls.get(), trisz.get(), pm.get(), pv.get(), pt.get()};
        uint64_t* outs[6] = {L[k].cstart.get(), clspos.get(), trioff.get(), pmoff.get(), pvoff.get(),
                             ptoff.get()};
        for (int j = 0; j < 6; ++j) {
          sm.in[j] = ins[j];
          sm.is64[j] = j == 2;
          sm.out[j] = outs[j];
        }
        if (!scan_multi_single(sm, 6, nk, s)) {
          for (int j = 0; j < 6; ++j) {
            if (j == 2) scan64(trisz.get(), outs[j], nk, s);
            else scan32(static_cast<const uint32_t*>(ins[j]), outs[j], nk, s);
          }
        }
        tm.end();
        uint64_t tot[6 + ST_COUNT];
        GatherU64 gsrc{};
        for (int j = 0; j < 6; ++j) gsrc.src[j] = outs[j] + nk;
        for (int j = 0; j < ST_COUNT; ++j)
          gsrc.src[6 + j] = reinterpret_cast<const uint64_t*>(dst.get()) + j;
        TBuf<uint64_t> dtot(6 + ST_COUNT, s);
        launch_gather_u64(gsrc, 6 + ST_COUNT, dtot.get(), s);
        BM_HIP(hipMemcpyAsync(tot, dtot.get(), sizeof(tot), hipMemcpyDeviceToHost, s));
        BM_HIP(hipStreamSynchronize(s));
        st.host_syncs++;
        const uint64_t n_next = tot[0], ncls = tot[1], Tn = tot[2], PM = tot[3], PV = tot[4],
                       PT = tot[5];
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
        tm.begin(BM_K_LEVEL);
        launch_fill_level(nk, L[k].parent.get(), pcls_prev.get(), w->cls.get(), L[k].item.get(),
                          w->tri.get(), S.get(), minsup, Ln.item.get(), Ln.parent.get(),
                          Ln.supp.get(), s);
        tm.end();
        st.frequent[k + 1] = n_next;
        if (ncls == 0) {
          k += 1;
          break;
        }
        auto nw = std::make_unique<StepWork>();
        nw->cls.alloc(ncls, s);
        nw->pre.alloc(ncls * k, s);
        TBuf<int32_t> pcls_k(nk, s);
        nw->T = Tn;
        nw->tri.alloc(Tn, s);
        launch_fill_u32(nw->tri.get(), 0, Tn, s);
        const TaskGeom g = make_geom(db->W, PM, PV, PT, tu);
        nw->ntm = PM * g.nsplit_m;
        nw->ntv = PV * g.nsplit_v;
        nw->ntt = PT * g.nsplit_t;
        nw->tm.alloc(nw->ntm, s);
        nw->tv.alloc(nw->ntv, s);
        nw->tt.alloc(nw->ntt, s);
        for (int j = 0; j < ST_COUNT; ++j) nw->st[j] = tot[6 + j];
        LevelPtrs lv{};
        for (uint32_t j = 1; j <= k; ++j) {
          lv.item[j] = L[j].item.get();
          lv.parent[j] = L[j].parent.get();
        }
        tm.begin(BM_K_LEVEL);
        launch_fill_classes(nk, k, cnt.get(), L[k].cstart.get(), clspos.get(), trioff.get(),
                            pmoff.get(), pvoff.get(), ptoff.get(), tu.mfma_min_q, lv, f1.get(),
                            nw->cls.get(), nw->pre.get(), pcls_k.get(), g, nw->tm.get(),
                            nw->tv.get(), nw->tt.get(), s);
        tm.end();
        w = std::move(nw);
        pcls_prev = pcls_k;
        k += 1;
      }
    }

    // ---- canonical output
    const uint32_t K = (uint32_t)L.size() - 1;
    uint64_t F = 0, TI = 0;
    for (uint32_t k = 1; k <= K; ++k) {
      F += L[k].n;
      TI += (uint64_t)k * L[k].n;
    }
    res->n_sets = F;
    res->n_items = TI;
    res->max_len = K;
    st.max_len = K;
    st.frequent_total = F;
    res->offsets.reset(F + 1, s);
    res->items.reset(TI, s);
    res->supports.reset(F, s);
    if (F == 0) {
      launch_fill_u64(res->offsets.get(), 0, 1, s);
    } else {
      tm.begin(BM_K_EMIT);
      std::vector<TBuf<uint64_t>> SZ(K + 2), ISZ(K + 2), pre(K + 1), off(K + 1);
      for (uint32_t k = K; k >= 1; --k) {
        TBuf<uint64_t> sz(L[k].n, s), isz(L[k].n, s);
        const bool last = k == K;
        launch_emit_sizes(L[k].n, k, last ? nullptr : L[k].cstart.get(),
                          last ? nullptr : SZ[k + 1].get(), last ? nullptr : ISZ[k + 1].get(),
                          sz.get(), isz.get(), s);
        SZ[k].alloc(L[k].n + 1, s);
        ISZ[k].alloc(L[k].n + 1, s);
        ScanMulti sm{};
        sm.in[0] = sz.get();
        sm.in[1] = isz.get();
        sm.is64[0] = sm.is64[1] = 1;
        sm.out[0] = SZ[k].get();
        sm.out[1] = ISZ[k].get();
        if (!scan_multi_single(sm, 2, L[k].n, s)) {
          scan64(sz.get(), SZ[k].get(), L[k].n, s);
          scan64(isz.get(), ISZ[k].get(), L[k].n, s);
        }
      }
      LevelPtrs lv{};
      for (uint32_t k = 1; k <= K; ++k) {
        lv.item[k] = L[k].item.get();
        lv.parent[k] = L[k].parent.get();
      }
      for (uint32_t k = 2; k <= K; ++k) {
        pre[k].alloc(L[k].n, s);
        off[k].alloc(L[k].n, s);
        launch_emit_pos(L[k].n, k, L[k].parent.get(), k == 2 ? SZ[1].get() : pre[k - 1].get(),
                        k == 2 ? ISZ[1].get() : off[k - 1].get(), L[k - 1].cstart.get(),
                        SZ[k].get(), ISZ[k].get(), pre[k].get(), off[k].get(), s);
      }
      for (uint32_t k = 1; k <= K; ++k) {
        launch_emit_write(L[k].n, k, k == 1 ? SZ[1].get() : pre[k].get(),
                          k == 1 ? ISZ[1].get() : off[k].get(), L[k].supp.get(), lv, f1.get(),
                          res->offsets.get(), res->items.get(), res->supports.get(), s);
      }
      launch_put_u64(res->offsets.get() + F, ISZ[1].get() + L[1].n, s);
      tm.end();
    }
    BM_HIP(hipStreamSynchronize(s));
  }
  tm.collect(&st);
  st.wall_ms = ms_since(t0);
  return res.release();
}

}  // namespace bm
