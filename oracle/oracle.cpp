// CPU oracle: frequent-itemset mining over sorted transaction-id vectors.
//
// TEST INFRASTRUCTURE ONLY: linked by nothing but the oracle's ctypes wrapper
// (tests, smoke check, benchmark CPU-baseline leg).  Shares no code with the
// HIP library.
//
// What it computes follows Section III of the paper:
//   * Eq. 1: column j of the Boolean matrix M is kept as the ascending list of
//     transaction ids containing item j (duplicate ids in a row collapse);
//   * Eq. 2 and the "AND further columns in sequence" rule: the support of
//     X + {j} is the size of tid(X) intersected with tid(X + {j'})..., here
//     computed with std::set_intersection on sorted vectors;
//   * Eq. 3: an itemset is frequent when its support reaches minsup (absolute
//     count, `>=`).
// The recursion extends a frequent prefix only by its later frequent siblings
// (anti-monotonicity), exactly like the Python set oracle.  Threads take whole
// top-level classes (all itemsets whose smallest item is a given frequent
// item) from an atomic counter; the final list is sorted explicitly.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

namespace {

struct Db {
  uint64_t n = 0;
  uint32_t m = 0;
  std::vector<std::vector<uint32_t>> tid;  // tid[j] ascending, unique
};

struct Set {
  std::vector<uint32_t> items;
  uint32_t support;
};

struct Result {
  std::vector<Set> sets;
  uint64_t candidates = 0;
  uint64_t n_items = 0;
};

struct Cand {
  uint32_t item;
  std::vector<uint32_t> tids;
};

void rec(const std::vector<uint32_t>& prefix, std::vector<Cand>& cands, uint32_t minsup,
         std::vector<Set>& out, uint64_t& ncand) {
  std::vector<uint32_t> X = prefix;
  X.push_back(0);
  for (size_t idx = 0; idx < cands.size(); ++idx) {
    X.back() = cands[idx].item;
    out.push_back(Set{X, static_cast<uint32_t>(cands[idx].tids.size())});
    std::vector<Cand> next;
    for (size_t l = idx + 1; l < cands.size(); ++l) {
      ++ncand;
      Cand c;
      c.item = cands[l].item;
      c.tids.reserve(std::min(cands[idx].tids.size(), cands[l].tids.size()));
      std::set_intersection(cands[idx].tids.begin(), cands[idx].tids.end(), cands[l].tids.begin(),
                            cands[l].tids.end(), std::back_inserter(c.tids));
      if (c.tids.size() >= minsup) next.push_back(std::move(c));
    }
    if (!next.empty()) rec(X, next, minsup, out, ncand);
  }
}

void set_err(char* err, int errlen, const char* msg) {
  if (err && errlen > 0) {
    std::snprintf(err, static_cast<size_t>(errlen), "%s", msg);
  }
}

}  // namespace

extern "C" {

void* orc_open(const uint64_t* row_ptr, const uint32_t* col_idx, uint64_t n, uint32_t m, char* err,
               int errlen) {
  if (!row_ptr) {
    set_err(err, errlen, "row_ptr is NULL");
    return nullptr;
  }
  if (row_ptr[0] != 0) {
    set_err(err, errlen, "row_ptr[0] != 0");
    return nullptr;
  }
  for (uint64_t i = 0; i < n; ++i) {
    if (row_ptr[i + 1] < row_ptr[i]) {
      set_err(err, errlen, "row_ptr not monotone");
      return nullptr;
    }
  }
  const uint64_t nnz = row_ptr[n];
  if (nnz > 0 && !col_idx) {
    set_err(err, errlen, "col_idx is NULL");
    return nullptr;
  }
  for (uint64_t e = 0; e < nnz; ++e) {
    if (col_idx[e] >= m) {
      set_err(err, errlen, "item id out of range");
      return nullptr;
    }
  }
  Db* db = new (std::nothrow) Db;
  if (!db) {
    set_err(err, errlen, "out of memory");
    return nullptr;
  }
  db->n = n;
  db->m = m;
  db->tid.assign(m, {});
  std::vector<uint64_t> cnt(m, 0);
  for (uint64_t e = 0; e < nnz; ++e) cnt[col_idx[e]]++;
  for (uint32_t j = 0; j < m; ++j) db->tid[j].reserve(cnt[j]);
  for (uint64_t i = 0; i < n; ++i) {
    for (uint64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      auto& v = db->tid[col_idx[e]];
      // rows are scanned in order, so a duplicate id in row i can only repeat the last entry
      if (v.empty() || v.back() != static_cast<uint32_t>(i)) v.push_back(static_cast<uint32_t>(i));
    }
  }
  return db;
}

void orc_close(void* h) { delete static_cast<Db*>(h); }

uint32_t orc_item_support(void* h, uint32_t j) {
  Db* db = static_cast<Db*>(h);
  return j < db->m ? static_cast<uint32_t>(db->tid[j].size()) : 0u;
}

// Frequent single items in ascending id order; returns their count, writes up to cap ids.
uint32_t orc_frequent_items(void* h, uint32_t minsup, uint32_t* out, uint32_t cap) {
  Db* db = static_cast<Db*>(h);
  uint32_t k = 0;
  for (uint32_t j = 0; j < db->m; ++j) {
    if (db->tid[j].size() >= minsup) {
      if (out && k < cap) out[k] = j;
      ++k;
    }
  }
  return k;
}

// Mine the subtrees rooted at frequent items number [top_first, top_last) of the
// ascending frequent-item list (the full result when the range covers all of them).
void* orc_mine(void* h, uint32_t minsup, int threads, uint32_t top_first, uint32_t top_last) {
  Db* db = static_cast<Db*>(h);
  if (minsup < 1) return nullptr;
  std::vector<uint32_t> f1;
  for (uint32_t j = 0; j < db->m; ++j)
    if (db->tid[j].size() >= minsup) f1.push_back(j);
  top_last = std::min<uint32_t>(top_last, static_cast<uint32_t>(f1.size()));
  Result* res = new Result;
  if (top_first >= top_last) return res;
  if (threads < 1) threads = 1;
  std::atomic<uint32_t> next{top_first};
  std::vector<std::vector<Set>> outs(threads);
  std::vector<uint64_t> ncands(threads, 0);
  auto worker = [&](int t) {
    for (;;) {
      uint32_t a = next.fetch_add(1);
      if (a >= top_last) break;
      const auto& Ta = db->tid[f1[a]];
      outs[t].push_back(Set{{f1[a]}, static_cast<uint32_t>(Ta.size())});
      std::vector<Cand> cands;
      for (uint32_t b = a + 1; b < f1.size(); ++b) {
        ++ncands[t];
        const auto& Tb = db->tid[f1[b]];
        Cand c;
        c.item = f1[b];
        c.tids.reserve(std::min(Ta.size(), Tb.size()));
        std::set_intersection(Ta.begin(), Ta.end(), Tb.begin(), Tb.end(), std::back_inserter(c.tids));
        if (c.tids.size() >= minsup) cands.push_back(std::move(c));
      }
      if (!cands.empty()) rec({f1[a]}, cands, minsup, outs[t], ncands[t]);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < threads; ++t) pool.emplace_back(worker, t);
  worker(0);
  for (auto& th : pool) th.join();
  for (int t = 0; t < threads; ++t) {
    res->candidates += ncands[t];
    for (auto& s : outs[t]) res->sets.push_back(std::move(s));
  }
  std::sort(res->sets.begin(), res->sets.end(),
            [](const Set& x, const Set& y) { return x.items < y.items; });
  for (const auto& s : res->sets) res->n_items += s.items.size();
  return res;
}

uint64_t orc_res_count(void* r) { return static_cast<Result*>(r)->sets.size(); }
uint64_t orc_res_items(void* r) { return static_cast<Result*>(r)->n_items; }
uint64_t orc_res_candidates(void* r) { return static_cast<Result*>(r)->candidates; }

void orc_res_copy(void* r, uint64_t* offsets, uint32_t* items, uint32_t* supports) {
  Result* res = static_cast<Result*>(r);
  uint64_t off = 0;
  for (size_t i = 0; i < res->sets.size(); ++i) {
    offsets[i] = off;
    for (uint32_t x : res->sets[i].items) items[off++] = x;
    supports[i] = res->sets[i].support;
  }
  offsets[res->sets.size()] = off;
}

void orc_res_free(void* r) { delete static_cast<Result*>(r); }

// Support of one itemset by successive intersection of its columns.
uint32_t orc_support(void* h, const uint32_t* items, uint32_t k) {
  Db* db = static_cast<Db*>(h);
  if (k == 0) return static_cast<uint32_t>(db->n);
  for (uint32_t i = 0; i < k; ++i)
    if (items[i] >= db->m) return 0;
  std::vector<uint32_t> cur = db->tid[items[0]];
  std::vector<uint32_t> tmp;
  for (uint32_t i = 1; i < k && !cur.empty(); ++i) {
    const auto& t = db->tid[items[i]];
    tmp.clear();
    std::set_intersection(cur.begin(), cur.end(), t.begin(), t.end(), std::back_inserter(tmp));
    cur.swap(tmp);
  }
  return static_cast<uint32_t>(cur.size());
}

// Supports of `count` itemsets given in CSR form (offsets[count+1], items).
void orc_supports(void* h, const uint64_t* offsets, const uint32_t* items, uint64_t count,
                  uint32_t* out, int threads) {
  if (threads < 1) threads = 1;
  std::atomic<uint64_t> next{0};
  auto worker = [&]() {
    for (;;) {
      uint64_t i = next.fetch_add(64);
      if (i >= count) break;
      uint64_t e = std::min<uint64_t>(count, i + 64);
      for (; i < e; ++i)
        out[i] = orc_support(h, items + offsets[i], static_cast<uint32_t>(offsets[i + 1] - offsets[i]));
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < threads; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
}

}  // extern "C"
