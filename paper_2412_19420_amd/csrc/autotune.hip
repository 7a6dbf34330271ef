// Autotuner of the miner's launch choices (bm_autotune).
//
// Every tuning field changes only speed, never the result, so the tuner can
// time real calls on the caller's own databases: a coordinate search over
//   * the depth-first phase (on at any column length / off),
//   * the MFMA routing thresholds (children per class, for 128- and 256-wide tiles),
//   * the word-range length of one task (automatic or fixed),
//   * the AND+popcount LDS chunk,
//   * the depth-first workgroup size and the column length below which a
//     subtree task runs one stack per wave,
// keeping each field's fastest value before moving to the next.  Each point
// is the minimum wall time of `reps` calls.
#include <algorithm>
#include <chrono>
#include <vector>

#include "handles.hpp"

namespace bm {

namespace {

double time_call(const bm_db* const* dbs, const uint32_t* minsups, uint32_t count,
                 const bm_model* sched, const bm_options& o, uint32_t reps, hipStream_t s) {
  double best = 1e300;
  for (uint32_t r = 0; r < reps; ++r) {
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<bm_result*> out = mine_many(dbs, minsups, count, sched, &o, s);
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (bm_result* p : out) delete p;
    best = std::min(best, ms);
  }
  return best;
}

}  // namespace

bm_options autotune(const bm_db* const* dbs, const uint32_t* minsups, uint32_t count,
                    const bm_model* sched, const bm_options* base, uint32_t reps, hipStream_t s,
                    double* best_ms) {
  bm_options cur{};
  if (base) cur = *base;
  // tuning runs are timed without events, in queue order, and keep no trace
  cur.flags &= ~(BM_FLAG_TIMING | BM_FLAG_TRACE | BM_FLAG_SHUFFLE);
  if (reps == 0) reps = 3;
  double best = time_call(dbs, minsups, count, sched, cur, reps, s);

  auto try_field = [&](auto set, const std::vector<uint32_t>& values) {
    bm_options keep = cur;
    for (uint32_t v : values) {
      bm_options o = keep;
      set(o, v);
      const double ms = time_call(dbs, minsups, count, sched, o, reps, s);
      if (ms < best) {
        best = ms;
        cur = o;
      }
    }
  };
  // small subtrees: level by level throughout (0), the defaults (1), the
  // depth-first kernel on short columns (2) or on every column (3)
  try_field(
      [](bm_options& o, uint32_t v) {
        o.flags &= ~(BM_FLAG_LEVELSYNC | BM_FLAG_DEPTH_FIRST);
        o.dfs_max_words = 0;
        if (v == 0) o.flags |= BM_FLAG_LEVELSYNC;
        if (v >= 2) o.flags |= BM_FLAG_DEPTH_FIRST;
        if (v == 3) o.dfs_max_words = 0xffffffffu;
      },
      {0u, 1u, 2u, 3u});
  try_field([](bm_options& o, uint32_t v) { o.mfma_min_children = v; }, {24u, 32u, 48u, 64u, 96u, 128u});
  try_field([](bm_options& o, uint32_t v) { o.mfma_big_children = v; }, {192u, 256u, 512u, 0xffffffffu});
  try_field([](bm_options& o, uint32_t v) { o.split_words = v; }, {0u, 512u, 1024u, 2048u, 4096u});
  try_field([](bm_options& o, uint32_t v) { o.andpop_chunk_words = v; }, {128u, 256u});
  // projected views of big deep classes: the default cost rule, more eager ones, or none
  try_field(
      [](bm_options& o, uint32_t v) {
        o.flags &= ~BM_FLAG_NO_PROJECT;
        if (v == 0) o.flags |= BM_FLAG_NO_PROJECT;
        o.project_gain = v;
      },
      {0u, 16u, 64u, 512u});
  if (!(cur.flags & BM_FLAG_LEVELSYNC)) {
    // long columns: small subtrees by subset counting, up to 4, 6 or 8 children, or not at all
    try_field([](bm_options& o, uint32_t v) { o.subset_max_children = v; }, {1u, 4u, 6u, 8u});
    try_field([](bm_options& o, uint32_t v) { o.dfs_threads = v; }, {256u, 512u, 1024u});
    try_field(
        [](bm_options& o, uint32_t v) {
          if (v == 0) {
            o.flags |= BM_FLAG_DFS_BLOCK_ONLY;
          } else {
            o.flags &= ~BM_FLAG_DFS_BLOCK_ONLY;
            o.dfs_wave_max_words = v;
          }
        },
        {0u, 256u, 1024u, 4096u});
  }
  if (best_ms) *best_ms = best;
  return cur;
}

}  // namespace bm
