// extern "C" entry points of libbm (declared and documented in bm.h).
#include <cstring>

#include "handles.hpp"

namespace {

template <class F>
bm_status guarded(F&& f) {
  try {
    bm::set_last_error("");
    f();
    return BM_OK;
  } catch (const bm::Error& e) {
    bm::set_last_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    bm::set_last_error("host allocation failed");
    return BM_ERR_OOM;
  } catch (const std::exception& e) {
    bm::set_last_error(e.what());
    return BM_ERR_DEVICE;
  } catch (...) {
    bm::set_last_error("unknown failure");
    return BM_ERR_DEVICE;
  }
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

uint32_t bm_abi_version(void) { return BM_ABI_VERSION; }

const char* bm_status_string(bm_status s) {
  switch (s) {
    case BM_OK: return "ok";
    case BM_ERR_INVALID_ARG: return "invalid argument";
    case BM_ERR_CSR: return "malformed CSR transaction list";
    case BM_ERR_OOM: return "out of memory";
    case BM_ERR_DEVICE: return "device error";
    case BM_ERR_UNSUPPORTED: return "unsupported size";
  }
  return "unknown status";
}

const char* bm_last_error(void) { return bm::last_error(); }

bm_status bm_set_allocator(void* (*alloc)(size_t, void*, void*), void (*free_fn)(void*, void*, void*),
                           void* ctx) {
  return bm::set_allocator(alloc, free_fn, ctx);
}

bm_status bm_release_cached_memory(void) {
  return guarded([&] { bm::release_cached(); });
}

bm_status bm_build(const uint64_t* row_ptr, const uint32_t* col_idx, uint64_t n_tx,
                   uint32_t n_items, void* stream, bm_db** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!out) bm::fail(BM_ERR_INVALID_ARG, "out is NULL");
    *out = bm::build_db(row_ptr, col_idx, n_tx, n_items, as_stream(stream));
  });
}

bm_status bm_db_info(const bm_db* db, uint64_t* n_tx, uint32_t* n_items, uint64_t* words) {
  return guarded([&] {
    if (!db) bm::fail(BM_ERR_INVALID_ARG, "db is NULL");
    if (n_tx) *n_tx = db->n;
    if (n_items) *n_items = db->m;
    if (words) *words = db->Wp;
  });
}

bm_status bm_item_support(const bm_db* db, uint32_t* out, void* stream) {
  return guarded([&] {
    if (!db || !out) bm::fail(BM_ERR_INVALID_ARG, "db or out is NULL");
    if (db->m == 0) return;
    hipStream_t s = as_stream(stream);
    BM_HIP(hipMemcpyAsync(out, db->colsum.get(), (size_t)db->m * 4, hipMemcpyDefault, s));
    BM_HIP(hipStreamSynchronize(s));
  });
}

bm_status bm_pair_support(const bm_db* db, const uint32_t* items, uint32_t k, uint32_t* out,
                          void* stream) {
  return guarded([&] {
    if (!db) bm::fail(BM_ERR_INVALID_ARG, "db is NULL");
    bm::pair_support(db, items, k, out, as_stream(stream));
  });
}

bm_status bm_pair_support_noalloc(const bm_db* db, const uint32_t* items, uint32_t k, uint32_t* out,
                                  void* stream) {
  return guarded([&] {
    if (!db) bm::fail(BM_ERR_INVALID_ARG, "db is NULL");
    bm::pair_support_noalloc(db, items, k, out, as_stream(stream));
  });
}

bm_status bm_mine_ex(const bm_db* db, uint32_t minsup, const bm_options* opt, void* stream,
                     bm_result** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!db || !out) bm::fail(BM_ERR_INVALID_ARG, "db or out is NULL");
    auto r = bm::mine_many(&db, &minsup, 1, nullptr, opt, as_stream(stream));
    *out = r[0];
  });
}

bm_status bm_mine_blocked(const uint64_t* row_ptr, const uint32_t* col_idx, uint64_t n_tx,
                          uint32_t n_items, uint32_t minsup, uint64_t block_rows,
                          const bm_options* opt, void* stream, bm_result** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!out) bm::fail(BM_ERR_INVALID_ARG, "out is NULL");
    *out = bm::mine_blocked(row_ptr, col_idx, n_tx, n_items, minsup, block_rows, opt,
                            as_stream(stream));
  });
}

bm_status bm_mine_batch(const bm_db* const* dbs, const uint32_t* minsups, uint32_t count,
                        const bm_model* sched, const bm_options* opt, void* stream,
                        bm_result** out) {
  if (out)
    for (uint32_t i = 0; i < count; ++i) out[i] = nullptr;
  return guarded([&] {
    if (count == 0) return;
    if (!dbs || !minsups || !out) bm::fail(BM_ERR_INVALID_ARG, "dbs, minsups or out is NULL");
    auto r = bm::mine_many(dbs, minsups, count, sched, opt, as_stream(stream));
    for (uint32_t i = 0; i < count; ++i) out[i] = r[i];
  });
}

bm_status bm_build_batch(uint32_t count, const uint64_t* const* row_ptrs,
                         const uint32_t* const* col_idxs, const uint64_t* n_tx,
                         const uint32_t* n_items, void* stream, bm_db** out) {
  if (out)
    for (uint32_t i = 0; i < count; ++i) out[i] = nullptr;
  return guarded([&] {
    if (count == 0) return;
    if (!row_ptrs || !n_tx || !n_items || !out)
      bm::fail(BM_ERR_INVALID_ARG, "row_ptrs, n_tx, n_items or out is NULL");
    auto r = bm::build_many(count, row_ptrs, col_idxs, n_tx, n_items, as_stream(stream));
    for (uint32_t i = 0; i < count; ++i) out[i] = r[i];
  });
}

bm_status bm_autotune(const bm_db* const* dbs, const uint32_t* minsups, uint32_t count,
                      const bm_model* sched, const bm_options* base, uint32_t reps, void* stream,
                      bm_options* best, double* best_ms) {
  return guarded([&] {
    if (count == 0 || !dbs || !minsups || !best)
      bm::fail(BM_ERR_INVALID_ARG, "dbs, minsups or best is NULL, or count is 0");
    *best = bm::autotune(dbs, minsups, count, sched, base, reps, as_stream(stream), best_ms);
  });
}

bm_status bm_mine(const bm_db* db, uint32_t minsup, void* stream, bm_result** out) {
  return bm_mine_ex(db, minsup, nullptr, stream, out);
}

bm_status bm_result_info(const bm_result* r, uint64_t* n_sets, uint64_t* n_items_total,
                         uint32_t* max_len) {
  return guarded([&] {
    if (!r) bm::fail(BM_ERR_INVALID_ARG, "result is NULL");
    if (n_sets) *n_sets = r->n_sets;
    if (n_items_total) *n_items_total = r->n_items;
    if (max_len) *max_len = r->max_len;
  });
}

bm_status bm_result_copy(const bm_result* r, uint64_t* offsets, uint32_t* items,
                         uint32_t* supports, void* stream) {
  return guarded([&] {
    if (!r) bm::fail(BM_ERR_INVALID_ARG, "result is NULL");
    bm::result_copy(r, offsets, items, supports, as_stream(stream));
  });
}

bm_status bm_result_stats(const bm_result* r, bm_stats* out) {
  return guarded([&] {
    if (!r || !out) bm::fail(BM_ERR_INVALID_ARG, "result or out is NULL");
    std::memcpy(out, &r->stats, sizeof(bm_stats));
  });
}

bm_status bm_result_trace(const bm_result* r, float* feats, float* labels, uint64_t* rows) {
  return guarded([&] {
    if (!r) bm::fail(BM_ERR_INVALID_ARG, "result is NULL");
    bm::result_trace(r, feats, labels, rows);
  });
}

bm_status bm_rules_mine(const bm_result* r, uint32_t min_conf_ppm, uint32_t max_len, void* stream,
                        bm_rules** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!r || !out) bm::fail(BM_ERR_INVALID_ARG, "result or out is NULL");
    *out = bm::rules_mine(r, min_conf_ppm, max_len, as_stream(stream));
  });
}

bm_status bm_rules_info(const bm_rules* rs, uint64_t* n_rules) {
  return guarded([&] {
    if (!rs) bm::fail(BM_ERR_INVALID_ARG, "rules is NULL");
    if (n_rules) *n_rules = rs->n;
  });
}

bm_status bm_rules_copy(const bm_rules* rs, uint64_t* z_index, uint32_t* ante_mask, uint32_t* supp_x,
                        uint32_t* supp_y, uint32_t* supp_z, double* conf, double* lift,
                        void* stream) {
  return guarded([&] {
    if (!rs) bm::fail(BM_ERR_INVALID_ARG, "rules is NULL");
    bm::rules_copy(rs, z_index, ante_mask, supp_x, supp_y, supp_z, conf, lift, as_stream(stream));
  });
}

bm_status bm_model_create(uint32_t seed, bm_model** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!out) bm::fail(BM_ERR_INVALID_ARG, "out is NULL");
    *out = bm::model_create(seed);
  });
}

bm_status bm_model_load(const char* path, bm_model** out) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!out || !path) bm::fail(BM_ERR_INVALID_ARG, "path or out is NULL");
    *out = bm::model_load(path);
  });
}

bm_status bm_model_save(const bm_model* m, const char* path) {
  return guarded([&] {
    if (!m || !path) bm::fail(BM_ERR_INVALID_ARG, "model or path is NULL");
    bm::model_save(m, path);
  });
}

bm_status bm_model_train_ex(bm_model* m, const float* feats, const float* labels, uint64_t rows,
                            uint32_t epochs, float lr, uint32_t batch, uint32_t flags,
                            float* epoch_losses, void* stream) {
  return guarded([&] {
    if (!m || (rows && (!feats || !labels))) bm::fail(BM_ERR_INVALID_ARG, "NULL argument");
    if (!(lr > 0.f)) bm::fail(BM_ERR_INVALID_ARG, "lr must be > 0");
    if (flags & ~BM_FLAG_GRAPH) bm::fail(BM_ERR_INVALID_ARG, "only BM_FLAG_GRAPH applies to training");
    const std::vector<float> l = bm::model_train(m, feats, labels, rows, epochs, lr, batch,
                                                 (flags & BM_FLAG_GRAPH) != 0, as_stream(stream));
    if (epoch_losses)
      for (size_t i = 0; i < l.size(); ++i) epoch_losses[i] = l[i];
  });
}

bm_status bm_model_train(bm_model* m, const float* feats, const float* labels, uint64_t rows,
                         uint32_t epochs, float lr, uint32_t batch, float* final_loss, void* stream) {
  return guarded([&] {
    if (!m || (rows && (!feats || !labels))) bm::fail(BM_ERR_INVALID_ARG, "NULL argument");
    if (!(lr > 0.f)) bm::fail(BM_ERR_INVALID_ARG, "lr must be > 0");
    const std::vector<float> l =
        bm::model_train(m, feats, labels, rows, epochs, lr, batch, true, as_stream(stream));
    if (final_loss) *final_loss = l.empty() ? 0.f : l.back();
  });
}

bm_status bm_model_predict(const bm_model* m, const float* feats, uint64_t rows, float* out,
                           void* stream) {
  return guarded([&] {
    if (!m || (rows && (!feats || !out))) bm::fail(BM_ERR_INVALID_ARG, "NULL argument");
    bm::model_predict(m, feats, rows, out, as_stream(stream));
  });
}

bm_status bm_model_grad(bm_model* m, const float* feats, const float* labels, uint64_t rows,
                        float* grad, float* loss, void* stream) {
  return guarded([&] {
    if (!m || (rows && (!feats || !labels))) bm::fail(BM_ERR_INVALID_ARG, "NULL argument");
    const float l = bm::model_grad(m, feats, labels, rows, grad, as_stream(stream));
    if (loss) *loss = l;
  });
}

bm_status bm_model_params(const bm_model* m, float* master, float* weights_bf16, float* norm) {
  return guarded([&] {
    if (!m) bm::fail(BM_ERR_INVALID_ARG, "model is NULL");
    bm::model_params(m, master, weights_bf16, norm);
  });
}

bm_status bm_model_set_params(bm_model* m, const float* master, const float* norm) {
  return guarded([&] {
    if (!m) bm::fail(BM_ERR_INVALID_ARG, "model is NULL");
    bm::model_set_params(m, master, norm);
  });
}

void bm_model_free(bm_model* m) { delete m; }

void bm_db_free(bm_db* db) { delete db; }
void bm_result_free(bm_result* r) { delete r; }
void bm_rules_free(bm_rules* r) { delete r; }

}  // extern "C"
