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
};
}  // namespace bm

// One database's result: a slice [set0, set0 + n_sets) of the call's sets whose
// item ids are [item0, item0 + n_items) of the call's items.
struct bm_result {
  int device = 0;
  std::shared_ptr<bm::ResultStore> store;
  uint64_t set0 = 0, n_sets = 0;
  uint64_t item0 = 0, n_items = 0;
  uint32_t max_len = 0;
  bm_stats stats{};
};

namespace bm {

int cu_count();
bool is_device_ptr(const void* p);
bm_status set_allocator(void* (*alloc)(size_t, void*, void*), void (*free_fn)(void*, void*, void*),
                        void* ctx);
void release_cached();
const char* last_error();

// Defaults of the tuning knobs (no knob changes the result).
struct Tuning {
  uint32_t mfma_min_q = 64;     // classes with this many children or more go to MFMA
  uint32_t andpop_chunk = 256;  // AND+popcount LDS chunk (words)
  uint32_t split_words = 0;     // 0 = automatic word split
};
Tuning tuning_from(const bm_options* opt);

bm_db* build_db(const uint64_t* row_ptr, const uint32_t* col_idx, uint64_t n, uint32_t m,
                hipStream_t s);
void pair_support(const bm_db* db, const uint32_t* items, uint32_t k, uint32_t* out, hipStream_t s);
// Mine `count` databases in one level-synchronous pass; one result per database.
std::vector<bm_result*> mine_many(const bm_db* const* dbs, const uint32_t* minsups, uint32_t count,
                                  const bm_options* opt, hipStream_t s);
void result_copy(const bm_result* r, uint64_t* offsets, uint32_t* items, uint32_t* supports,
                 hipStream_t s);

}  // namespace bm
