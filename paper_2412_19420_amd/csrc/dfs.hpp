// Depth-first subtree mining of small prefix classes (k_dfs.hip): task and
// arena records, kernel arguments, launchers.
#pragma once

#include "internal.hpp"

namespace bm {

// One subtree task: a prefix class with <= TINY_Q children whose children are
// level-synchronous nodes [child0, child0 + q) of level `level`.
struct DfsTask {
  uint32_t db;
  uint32_t level;
  uint32_t child0;
  uint32_t q;
  uint32_t pre_off;  // prefix columns in the step's prefix array
  uint32_t pre_len;  // level - 1
};

// A frequent itemset found by the depth-first kernel; its own children are the
// arena block [first, first + count).
struct ArenaNode {
  uint32_t item;  // frequent-item index of the last item
  uint32_t supp;
  uint32_t first;
  uint32_t count;
};

enum : uint32_t { DFS_OVERFLOW = 1u, DFS_TOO_LONG = 2u, DFS_STACK = 4u };

struct DfsArgs {
  const DbInfo* dbs;
  const DfsTask* tasks;
  uint32_t ntasks;
  const uint32_t* ntasks_dev;  // if set, the queue length is read from device memory
  const uint32_t* order;       // queue order (nullptr: task order)
  uint32_t* queue_head;
  const uint32_t* lv_item[BM_MAX_LEVELS + 2];
  const uint32_t* step_pre[BM_MAX_LEVELS + 2];
  uint32_t* ls_first[BM_MAX_LEVELS + 2];  // per level-synchronous level: arena block of each node
  uint32_t* ls_count[BM_MAX_LEVELS + 2];
  ArenaNode* arena;
  uint32_t* arena_count;
  uint32_t arena_cap;
  uint32_t* flags;
  unsigned long long* level_cand;  // [BM_MAX_LEVELS + 1] candidates by itemset length
  unsigned long long* level_freq;  // [BM_MAX_LEVELS + 1] frequent itemsets by length
  float* task_cost;                // column words streamed in each task's subtree (or nullptr)
  unsigned long long* words_read;  // column words streamed (prefix + children), for the roofline
};

// Features of a task for the cost model (8 per task).
struct FeatArgs {
  const DbInfo* dbs;
  const DfsTask* tasks;
  uint32_t ntasks;
  const uint32_t* lv_supp[BM_MAX_LEVELS + 2];
  const uint32_t* lv_parent[BM_MAX_LEVELS + 2];
  float* feats;
};

// Child source of a node while the final levels are merged.
enum : uint32_t { SRC_NONE = 0u, SRC_LS = 1u, SRC_ARENA = 2u };

// threads: 256, 512 or 1024 per workgroup
void launch_dfs(const DfsArgs& a, uint32_t threads, uint32_t grid, hipStream_t s);
// One subtree stack per wave (four waves per workgroup): for databases with
// short columns, where a whole workgroup per class would mostly wait.
void launch_dfs_wave(const DfsArgs& a, uint32_t grid, hipStream_t s);
// Subset counting (k_subsets.hip), for tasks of at most SUBSET_Q children:
// counts[t << SUBSET_Q | mask] (zeroed by the caller) receives the support of
// task t's prefix plus the children in mask, for every mask of two or more
// children, from `splits` word ranges per task.  Then one wave per task
// writes the subtree's frequent itemsets into the arena and links them as the
// depth-first kernel does (same flags and statistics; queue fields unused).
// max_q: most children of any task (the grid holds 2^(max_q - 6) passes per
// word range when it exceeds 6).
void launch_subset_count(const DfsArgs& a, uint32_t* counts, uint32_t splits, uint32_t max_q,
                         hipStream_t s);
// Fewest word ranges per task for columns of W words (the counting kernel's
// per-thread counters are 16 bits wide).
uint32_t subset_min_splits(uint64_t W);
void launch_subset_emit(const DfsArgs& a, const uint32_t* counts, hipStream_t s);
// flags[t] = 1 if queue entry t (order[t], or t) belongs to a database with at
// most max_words words per column.
void launch_dfs_short_flags(const DfsTask* tasks, const DbInfo* dbs, const uint32_t* order,
                            uint32_t n, uint32_t max_words, uint32_t* flags, hipStream_t s);
// Stable split of the queue by flags (pos = exclusive scan of flags, n + 1):
// short[] gets the flagged entries, long_[] the others, counts[0..1] their sizes.
void launch_dfs_split(const uint32_t* order, uint32_t n, const uint32_t* flags, const uint64_t* pos,
                      uint32_t* short_, uint32_t* long_, uint32_t* counts, hipStream_t s);
void launch_dfs_features(const FeatArgs& a, hipStream_t s);
// order[0..n) = tasks sorted by descending key (bucketed, ties in arbitrary order)
void launch_order_by_key(const float* key, uint32_t n, uint32_t* hist, uint64_t* hist_off,
                         uint32_t* order, hipStream_t s);
void launch_fin_level1(uint64_t n, const uint32_t* item, const uint32_t* parent, const uint32_t* supp,
                       const uint32_t* db, const uint64_t* cstart, const uint32_t* ls_first,
                       const uint32_t* ls_count, uint32_t* fitem, uint32_t* fparent, uint32_t* fsupp,
                       uint32_t* fdb, uint32_t* skind, uint32_t* sfirst, uint32_t* scount,
                       hipStream_t s);
void launch_fin_gather(uint64_t n, const uint32_t* fdb, const uint32_t* skind, const uint32_t* sfirst,
                       const uint32_t* scount, const uint64_t* fcstart, const uint32_t* ls_item,
                       const uint32_t* ls_supp, const uint32_t* ls_db, const uint64_t* ls_cstart,
                       const uint32_t* ls_first, const uint32_t* ls_count, const ArenaNode* arena,
                       uint32_t* nitem, uint32_t* nparent, uint32_t* nsupp, uint32_t* ndb,
                       uint32_t* nkind, uint32_t* nfirst, uint32_t* ncount, hipStream_t s);

}  // namespace bm
