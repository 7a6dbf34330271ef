// Launchers of the level-step and output kernels (k_levels.hip).
#pragma once

#include "internal.hpp"

namespace bm {

// Device pointers of every level's arrays, passed by value to kernels that walk
// an itemset's ancestors (level 1 .. k).
struct LevelPtrs {
  const uint32_t* item[BM_MAX_LEVELS + 2];
  const uint32_t* parent[BM_MAX_LEVELS + 2];
};

// Everything the one-pass output kernel reads and writes.  Per level k = 1..K:
// the node arrays, the child-start array (k < K; n_k + 1 entries, the last
// one n_{k+1}) and base[k] = nodes on levels below k (base[K + 1] = F).
// first_root[d] = first level-1 node of database d (N + 1 entries).  bounds
// is (K + 1) x (N + 1), row k = first level-k node of each database; slices
// holds the first itemset (N + 1 entries) then the first item id (N + 1) of
// each database's slice.  bounds and slices may be mapped host memory.
struct EmitArgs {
  const uint32_t* item[BM_MAX_LEVELS + 2];
  const uint32_t* parent[BM_MAX_LEVELS + 2];
  const uint64_t* cstart[BM_MAX_LEVELS + 2];
  const uint32_t* supp[BM_MAX_LEVELS + 2];
  const uint32_t* node_db[BM_MAX_LEVELS + 2];
  uint64_t base[BM_MAX_LEVELS + 2];
  const DbInfo* dbs;
  const uint64_t* first_root;
  uint64_t* o_off;
  uint32_t* o_items;
  uint32_t* o_supp;
  uint64_t* bounds;
  uint64_t* slices;
  uint32_t K, N;
};

// Word-range length of one task, per kernel (MFMA splits are multiples of 16 words).
struct TaskGeom {
  uint32_t split_m, split_v, split_t, split_b, split_s;
  uint32_t big_q;     // classes with at least this many children (and MFMA-routed) use 256-wide tiles
  uint32_t small_on;  // mid-size classes use the 32-wide MFMA kernel (else LDS AND+popcount)
  uint32_t tiny_q;    // classes with at most this many children are small (registers / subtrees)
};

// Per-step totals accumulated on the device for statistics.
// Index = base + kernel type (0 = MFMA 128-wide tiles, 1 = LDS-blocked AND+popcount,
// 2 = register AND+popcount, 3 = MFMA 256-wide tiles, 4 = MFMA 32-wide tiles).
enum { ST_CAND_M = 0, ST_CAND_V, ST_CAND_T, ST_CAND_B, ST_CAND_S, ST_COLS_M, ST_COLS_V, ST_COLS_T,
       ST_COLS_B, ST_COLS_S, ST_CLS_M, ST_CLS_V, ST_CLS_T, ST_CLS_B, ST_CLS_S, ST_COUNT };
// The node-count kernel also sums the next step's task counts: 128-wide tile
// pairs, 16-wide block pairs and tiny classes (sizes for the task lists), the
// 256-wide tile pairs of big classes (NC_PAIRS_B), the 16-wide block pairs
// weighted by their databases' words (NC_PAIRS_VW: the split of the 32-wide
// kernel's word ranges),
// and for the projected classes on the 128-wide (M) and 256-wide (B) kernels
// their candidates and work (the prefix's support times the class's
// candidates), and their children.
enum { NC_PAIRS_M = ST_COUNT, NC_PAIRS_V, NC_TINY, NC_PJ_CAND_M, NC_PJ_WORK_M, NC_PJ_CAND_B,
       NC_PJ_WORK_B, NC_PJ_COLS, NC_PAIRS_B, NC_PAIRS_VW, NC_COUNT };

// Whether a class of q children whose prefix has support s_prefix (in a
// database of n transactions) is projected: its children's columns are
// re-packed over the prefix's transactions before counting.  Only classes on
// the 128- and 256-wide MFMA kernels, where the contraction reads every column
// many times, and only when the work it saves, about q^2 (n - s) MFMA
// operations, outweighs gathering the q columns (about q n / 64 word loads):
// q (n - s) >= gain * n.  gain == 0: never.
__host__ __device__ inline bool project_class(int kind, uint32_t q, uint64_t s_prefix, uint64_t n,
                                              uint32_t gain) {
  return gain && (kind == 0 || kind == 3) && s_prefix < n &&
         (double)q * (double)(n - s_prefix) >= (double)gain * (double)n;
}
// Words of a projected view over s transactions (unpadded, padded).
__host__ __device__ inline uint64_t view_words(uint64_t s) { return (s + 63) / 64; }
__host__ __device__ inline uint64_t view_padded_words(uint64_t s) {
  const uint64_t w = (view_words(s) + 63) / 64 * 64;
  return w ? w : 64;
}

void launch_f1_flags(const DbInfo* dbs, uint32_t ndb, const uint64_t* item_base, uint64_t total,
                     uint32_t* flags, hipStream_t s);
void launch_f1_fill(const uint32_t* flags, const uint64_t* pos, uint32_t ndb,
                    const uint64_t* item_base, uint64_t total, uint32_t* f1, hipStream_t s);
// Level 1 of every database; also sets each table entry's f1 slice.
void launch_init_level1(DbInfo* dbs, uint32_t ndb, const uint64_t* f1_base, uint64_t n1,
                        const uint32_t* f1, uint32_t* item, uint32_t* parent, uint32_t* supp,
                        uint32_t* ndbv, hipStream_t s);
// out[i] = arr[idx[i]], i < k; also into out2 (e.g. mapped host memory) when not NULL.
void launch_gather_idx(const uint64_t* arr, const uint64_t* idx, uint32_t k, uint64_t* out,
                       uint64_t* out2, hipStream_t s);
// Per node of level k (a wave each): frequent children (cnt: the entries of
// its row of its class's triangle tri that meet the class's threshold),
// whether it becomes a class (is_cls) and its candidate triangle size
// (tri_sz); sums the step statistics and the task-count bounds into
// st[0, NC_COUNT) (zeroed by the caller).
// With proj_on (the projection gain, 0 = off), also per node: whether its
// class will be projected (pflag),
// the length of its prefix's row list (prows: the node's support) and the
// words of its view (pwords: children x padded view words), else zeros.
// Nodes per wave of the node-count and next-level kernels for n nodes whose
// rows hold tri_total entries in all.
uint32_t node_batch(uint64_t n, uint64_t tri_total);
void launch_node_counts(uint64_t n, uint32_t nb, uint32_t k, const uint32_t* parent,
                        const int32_t* pcls,
                        const ClassDesc* cls, const DbInfo* dbs, const uint32_t* tri,
                        uint32_t mfma_min_q, uint32_t big_q, uint32_t small_on, uint32_t tiny_q,
                        uint32_t* cnt, uint32_t* is_cls, uint64_t* tri_sz, unsigned long long* st,
                        const uint32_t* supp, uint32_t proj_on, uint32_t* pflag, uint32_t* prows,
                        uint64_t* pwords, hipStream_t s);
// Arguments of the launch between two level steps (k_level_post): node i < n
// of level k writes its frequent extensions into the next level and, if it
// has at least two, its class of the next step and that class's task counts
// (skipped when ocls is NULL); the next step's support triangle ztri[0, nz)
// is zeroed.
struct LevelPost {
  uint64_t n;
  const uint32_t* parent;
  const int32_t* pcls;
  const ClassDesc* cls;
  const DbInfo* dbs;
  const uint32_t* child_item;
  const uint32_t* tri;
  uint32_t* nitem;
  uint32_t* nparent;
  uint32_t* nsupp;
  uint32_t* ndbv;
  uint32_t k;
  const uint32_t* cnt;
  const uint64_t* child_start;
  const uint64_t* cls_pos;
  const uint64_t* tri_off;
  const uint32_t* node_db;
  ClassDesc* ocls;
  uint32_t* opre;
  int32_t* pcls_out;
  uint32_t* ztri;
  uint64_t nz;
  uint32_t nb;              // nodes per wave (node_batch)
  uint32_t b_level, b_cls;  // set by the launcher
  // the next step's per-class task counts (as k_class_task_counts writes them)
  TaskGeom geo;
  uint32_t mfma_min_q, dfs;
  uint32_t *cm, *cv, *ct, *cb, *cs;
  LevelPtrs lv;
  // projected classes (views == NULL: none): the node-count kernel's flags,
  // scanned into slot numbers, row-list offsets and view-word offsets
  const uint32_t* pflag;
  const uint64_t* pslot;
  const uint64_t* prow_off;
  const uint64_t* pword_off;
  const uint32_t* nodesupp;  // supports of the level-k nodes (the prefixes)
  uint64_t* vbuf;            // the step's view words
  DbInfo* views;
  ProjWork* pwork;
};
void launch_level_post(LevelPost a, hipStream_t s);
void launch_class_task_counts(const ClassDesc* cls, uint64_t ncls, const DbInfo* dbs,
                              const DbInfo* views, uint32_t mfma_min_q, const TaskGeom& geo,
                              bool dfs, uint32_t* cm, uint32_t* cv, uint32_t* ct, uint32_t* cb,
                              uint32_t* cs, hipStream_t s);
struct DfsTask;
void launch_write_class_tasks(const ClassDesc* cls, uint64_t ncls, const DbInfo* dbs,
                              const DbInfo* views, uint32_t mfma_min_q, const TaskGeom& geo,
                              const uint64_t* om,
                              const uint64_t* ov, const uint64_t* ot, Task* tm, Task* tv, Task* tt,
                              DfsTask* dt, uint32_t level, const uint64_t* ob, Task* tb,
                              const uint64_t* os, Task* ts, hipStream_t s);
void launch_emit_all(const EmitArgs& a, uint64_t F, hipStream_t s);
// Projected views of a step's nprj classes (k_project.hip): popcounts of each
// prefix over 1,024-word chunks (cnt_tmp: nprj x view_chunks(Wmax) counts),
// then, from their exclusive scan (off_tmp, offsets counted from the first
// class's first row, so a class's own rows start at its ProjWork::row_off),
// the children's columns compressed into the (zeroed) views.
uint64_t view_chunks(uint64_t Wmax);
void launch_project_count(const ProjWork* pw, uint32_t nprj, const ClassDesc* cls,
                          const DbInfo* dbs, const uint32_t* pre_cols, uint64_t Wmax,
                          uint32_t* cnt_tmp, hipStream_t s);
void launch_project_compact(const ProjWork* pw, uint32_t nprj, const ClassDesc* cls,
                            const DbInfo* dbs, const DbInfo* views, const uint32_t* pre_cols,
                            const uint32_t* child_item, uint64_t Wmax, const uint64_t* off_tmp,
                            hipStream_t s);
// dst[i] = words[i] for i < n <= kWriteWordsMax; the words travel as a kernel
// argument (no staging copy).
constexpr uint32_t kWriteWordsMax = 64;
void launch_write_words(uint32_t* dst, const uint32_t* words, uint32_t n, hipStream_t s);
// dst[i] = i for i < n.
void launch_iota_u32(uint32_t* dst, uint32_t n, hipStream_t s);
void launch_rebase(const uint64_t* src, uint64_t n, uint64_t base, uint64_t* dst, hipStream_t s);
void launch_expand_pairs(uint32_t k, const uint32_t* items, const uint32_t* colsum,
                         const uint32_t* tri, uint32_t* out, hipStream_t s);

// Host-side helpers shared by the miner and the pair-support call.
inline uint32_t host_mfma_pairs(uint32_t q, uint32_t tile = GRAM_TILE) {
  const uint32_t nb = (q + tile - 1) / tile;
  return nb * (nb + 1) / 2;
}
// Kernel that evaluates a class of q children: 0 = MFMA (128-wide tiles),
// 1 = LDS-blocked AND+popcount, 2 = registers, 3 = MFMA (256-wide tiles),
// 4 = MFMA (32-wide tiles, one wave per block pair).
__host__ __device__ inline int class_kind(uint32_t q, uint32_t mfma_min_q, uint32_t big_q,
                                          uint32_t small_on, uint32_t tiny_q) {
  if (q >= mfma_min_q) return q >= big_q ? 3 : 0;
  if (q <= tiny_q) return 2;
  return small_on ? 4 : 1;
}
// Narrow tails: a class on the 128-wide tiles (kind 0) whose last column
// block holds at most 32 children has that block's pairs computed by the
// 32-wide kernel (when it is on): a 128-wide tile there would spend all its
// MFMAs on a few columns.  The 128-wide tasks then cover the first
// gram_tail_q(q) children, and the tail is gram_tail_pairs(q) 32-wide block
// pairs: every 32-wide row block up to and including the tail's own against
// the tail's block.
__host__ __device__ inline bool gram_tail(uint32_t q) {
  return q > GRAM_TILE && q - (q - 1) / GRAM_TILE * GRAM_TILE <= GRAM_SMALL_TILE;
}
__host__ __device__ inline uint32_t gram_tail_q(uint32_t q) { return (q - 1) / GRAM_TILE * GRAM_TILE; }
__host__ __device__ inline uint32_t gram_tail_pairs(uint32_t q) {
  return gram_tail_q(q) / GRAM_SMALL_TILE + 1;
}
// Kinds whose task word ranges are rounded to GRAM_KW (LDS-staged MFMA kernels).
__host__ __device__ inline bool is_mfma_kind(int kind) { return kind == 0 || kind == 3; }
inline uint32_t host_andpop_pairs(uint32_t q) {
  const uint32_t nb = (q + AP_BLOCK - 1) / AP_BLOCK;
  return nb * (nb + 1) / 2 - ((q % AP_BLOCK) == 1 ? 1u : 0u);
}

}  // namespace bm
