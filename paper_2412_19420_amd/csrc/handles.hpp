// Handle types behind the opaque pointers of bm.h.
#pragma once

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

struct bm_result {
  int device = 0;
  uint64_t n_sets = 0;
  uint64_t n_items = 0;
  uint32_t max_len = 0;
  bm::DBuf<uint64_t> offsets;   // n_sets + 1
  bm::DBuf<uint32_t> items;     // n_items
  bm::DBuf<uint32_t> supports;  // n_sets
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
bm_result* mine(const bm_db* db, uint32_t minsup, const bm_options* opt, hipStream_t s);

}  // namespace bm
