// Handle types behind the opaque pointers of bm.h.
#pragma once

#include <memory>
#include <vector>

#include "internal.hpp"

struct bm_db {
  int device = 0;
  uint64_t n = 0;       // transactions
  uint32_t m = 0;       // items
  uint64_t W = 0;       // words holding n bits
  uint64_t Wp = 0;      // padded words per column
  bm::DBuf<uint64_t> B;         // m * Wp bitset words
  bm::DBuf<uint32_t> colsum;    // m single-item supports
};

namespace bm {
// Device arrays of one mining call, shared by the results of all its databases.
struct ResultStore {
  DBuf<uint64_t> offsets;   // all sets + 1, item offsets counted over the whole call
  DBuf<uint32_t> items;
  DBuf<uint32_t> supports;
  // with BM_FLAG_TRACE: features and realised cost of every subtree task
  DBuf<float> trace_feats;  // [rows][8]
  DBuf<float> trace_cost;   // [rows] candidates evaluated in the subtree
  uint64_t trace_rows = 0;
};
}  // namespace bm

// Scheduler cost model (8 -> 64 -> 64 -> 1 perceptron).
struct bm_model {
  int device = 0;
  bm::DBuf<float> master, m, v, grad, norm;  // FP32 master copy, Adam moments, gradient, norm
  bm::DBuf<uint16_t> wbf;                    // BF16 weights used by the kernels
  float h_norm[16] = {};                     // feature mean[8], 1/std[8]
  bool has_norm = false;
  uint64_t step = 0;
};

// One database's result: a slice [set0, set0 + n_sets) of the call's sets whose
// item ids are [item0, item0 + n_items) of the call's items.
struct bm_result {
  int device = 0;
  std::shared_ptr<bm::ResultStore> store;
  uint64_t set0 = 0, n_sets = 0;
  uint64_t item0 = 0, n_items = 0;
  uint32_t max_len = 0;
  uint64_t n_tx = 0;  // transactions of the mined database
  bm_stats stats{};
};

// Association rules of one result (bm_rules_mine), in order of Z's position
// in the result, then of the antecedent as a tuple.
struct bm_rules {
  int device = 0;
  uint64_t n = 0;
  bm::DBuf<uint64_t> z;                // position of Z = X + Y in the result
  bm::DBuf<uint32_t> mask;             // antecedent X: bit p = p-th item of Z
  bm::DBuf<uint32_t> sx, sy, sz;       // supports of X, Y and Z
  bm::DBuf<double> conf, lift;
};

namespace bm {

bool is_device_ptr(const void* p);
bm_status set_allocator(void* (*alloc)(size_t, void*, void*), void (*free_fn)(void*, void*, void*),
                        void* ctx);
void release_cached();
const char* last_error();

// Defaults of the tuning knobs (no knob changes the result).
struct Tuning {
  uint32_t mfma_min_q = 64;     // classes with this many children or more go to 128-wide MFMA tiles
  bool mfma_small = true;       // classes of 9 .. mfma_min_q - 1 children: 32-wide MFMA tiles
  uint32_t mfma_big_q = 0xffffffffu;  // ... and with this many, to the 256-wide MFMA tiles
  uint32_t andpop_chunk = 256;  // AND+popcount LDS chunk (words)
  uint32_t split_words = 0;     // 0 = automatic word split
  bool dfs = true;              // small classes: depth-first subtree kernel
  bool mfma_fp4 = true;         // MFMA kernels in the e2m1 form (else int8)
  uint32_t dfs_threads = 256;   // threads per depth-first workgroup
  uint32_t dfs_max_words = 4096;  // depth-first only when every column has <= this many words
  uint32_t dfs_wave_words = 1024;  // tasks of databases with <= this many words: one stack per wave
                                   // (0: every task on the one-stack-per-workgroup kernel)
  // Longer columns: classes of at most subset_q children (0: none) are mined
  // whole by counting every subset of their children over word ranges
  uint32_t subset_q = SUBSET_DEFAULT_Q;
  bool subsets = false;            // this call mines small subtrees by subset counting
  uint32_t tiny_q = TINY_Q;        // small-class threshold of this call
  uint32_t arena_nodes = 0;        // initial subtree-output arena (0: sized from the task count)
  uint32_t project_gain = 512;     // big deep classes counted over projected views (0: never)
};
Tuning tuning_from(const bm_options* opt);

bm_db* build_db(const uint64_t* row_ptr, const uint32_t* col_idx, uint64_t n, uint32_t m,
                hipStream_t s);
std::vector<bm_db*> build_many(uint32_t count, const uint64_t* const* row_ptrs,
                               const uint32_t* const* col_idxs, const uint64_t* ns,
                               const uint32_t* ms, hipStream_t s);
void pair_support(const bm_db* db, const uint32_t* items, uint32_t k, uint32_t* out, hipStream_t s);
// The same with every temporary in the library's static per-device scratch
// (16 MiB): no allocation; items (or NULL) and out in device memory.
constexpr uint32_t kNoAllocMaxItems = 2048;
void pair_support_noalloc(const bm_db* db, const uint32_t* items, uint32_t k, uint32_t* out,
                          hipStream_t s);
// Mine `count` databases in one level-synchronous pass; one result per database.
bm_options autotune(const bm_db* const* dbs, const uint32_t* minsups, uint32_t count,
                    const bm_model* sched, const bm_options* base, uint32_t reps, hipStream_t s,
                    double* best_ms);
// Row blocks of an out-of-core database (bm_mine_blocked): before each launch
// of the class kernels the miner loads every block in turn into the one
// device matrix the database handle points at, and the kernels add each
// block's counts into the same supports.
struct BlockSource {
  virtual ~BlockSource() = default;
  virtual uint64_t blocks() const = 0;
  virtual void load(uint64_t b, hipStream_t s) = 0;
};
std::vector<bm_result*> mine_many(const bm_db* const* dbs, const uint32_t* minsups, uint32_t count,
                                  const bm_model* sched, const bm_options* opt, hipStream_t s,
                                  BlockSource* blocks = nullptr);
// Out-of-core mining of a host CSR, block_rows transactions at a time.
bm_result* mine_blocked(const uint64_t* row_ptr, const uint32_t* col_idx, uint64_t n, uint32_t m,
                        uint32_t minsup, uint64_t block_rows, const bm_options* opt, hipStream_t s);
bm_rules* rules_mine(const bm_result* r, uint32_t min_conf_ppm, uint32_t max_len, hipStream_t s);
void rules_copy(const bm_rules* rs, uint64_t* z, uint32_t* mask, uint32_t* sx, uint32_t* sy,
                uint32_t* sz, double* conf, double* lift, hipStream_t s);
void result_trace(const bm_result* r, float* feats, float* labels, uint64_t* rows);

bm_model* model_create(uint32_t seed);
bm_model* model_load(const char* path);
void model_save(const bm_model* m, const char* path);
void model_set_norm_from(bm_model* m, const float* feats, uint64_t rows, hipStream_t s);
std::vector<float> model_train(bm_model* m, const float* feats, const float* labels, uint64_t rows,
                               uint32_t epochs, float lr, uint32_t batch, bool graph, hipStream_t s);
void model_predict(const bm_model* m, const float* feats, uint64_t rows, float* out, hipStream_t s);
void model_predict_device(const bm_model* m, const float* dfeats, uint64_t rows, float* dout,
                          hipStream_t s);
float model_grad(bm_model* m, const float* feats, const float* labels, uint64_t rows,
                 float* grad_out, hipStream_t s);
void model_params(const bm_model* m, float* master, float* rounded, float* norm);
void model_set_params(bm_model* m, const float* master, const float* norm);
void result_copy(const bm_result* r, uint64_t* offsets, uint32_t* items, uint32_t* supports,
                 hipStream_t s);

}  // namespace bm
