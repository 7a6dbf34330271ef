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

// How class work is cut into tasks: word-split counts and lengths per kernel.
struct TaskGeom {
  uint32_t nsplit_m, split_m, wend_m;  // MFMA: splits are multiples of 16 words
  uint32_t nsplit_v, split_v, wend_v;  // AND+popcount, LDS-blocked (mid-size classes)
  uint32_t nsplit_t, split_t, wend_t;  // AND+popcount, registers only (<= TINY_Q children)
};

// Per-step totals accumulated on the device for statistics.
// Index = base + kernel type (0 = MFMA, 1 = LDS-blocked AND+popcount, 2 = register AND+popcount).
enum { ST_CAND_M = 0, ST_CAND_V, ST_CAND_T, ST_COLS_M, ST_COLS_V, ST_COLS_T, ST_CLS_M, ST_CLS_V,
       ST_CLS_T, ST_COUNT };

void launch_f1_fill(const uint32_t* colsum, uint32_t m, uint32_t minsup, const uint64_t* pos,
                    uint32_t* f1, hipStream_t s);
void launch_init_level1(const uint32_t* colsum, const uint32_t* f1, uint32_t n1, uint32_t* item,
                        uint32_t* parent, uint32_t* supp, hipStream_t s);
void launch_node_counts(uint64_t n, uint32_t k, const uint32_t* parent, const int32_t* pcls,
                        const ClassDesc* cls, const uint64_t* S, uint32_t mfma_min_q,
                        uint32_t* cnt, uint32_t* is_cls, uint64_t* tri_sz, uint32_t* pm,
                        uint32_t* pv, uint32_t* pt, unsigned long long* st, hipStream_t s);
void launch_fill_level(uint64_t n, const uint32_t* parent, const int32_t* pcls,
                       const ClassDesc* cls, const uint32_t* child_item, const uint32_t* tri,
                       const uint64_t* S, uint32_t minsup, uint32_t* nitem, uint32_t* nparent,
                       uint32_t* nsupp, hipStream_t s);
void launch_fill_classes(uint64_t n, uint32_t k, const uint32_t* cnt, const uint64_t* child_start,
                         const uint64_t* cls_pos, const uint64_t* tri_off, const uint64_t* pm_off,
                         const uint64_t* pv_off, const uint64_t* pt_off, uint32_t mfma_min_q,
                         const LevelPtrs& lv, const uint32_t* f1, ClassDesc* ocls, uint32_t* opre,
                         int32_t* pcls_out, const TaskGeom& geo, Task* tm, Task* tv, Task* tt,
                         hipStream_t s);
void launch_root_tasks(uint32_t q, uint32_t npairs, uint32_t block, uint32_t nsplit,
                       uint32_t split_len, uint32_t wend, Task* out, hipStream_t s);
void launch_emit_sizes(uint64_t n, uint32_t k, const uint64_t* cstart, const uint64_t* SZn,
                       const uint64_t* ISZn, uint64_t* sz, uint64_t* isz, hipStream_t s);
void launch_emit_pos(uint64_t n, uint32_t k, const uint32_t* parent, const uint64_t* ppre,
                     const uint64_t* poff, const uint64_t* pcstart, const uint64_t* SZ,
                     const uint64_t* ISZ, uint64_t* pre, uint64_t* off, hipStream_t s);
void launch_emit_write(uint64_t n, uint32_t k, const uint64_t* pre, const uint64_t* off,
                       const uint32_t* supp, const LevelPtrs& lv, const uint32_t* f1,
                       uint64_t* o_off, uint32_t* o_items, uint32_t* o_supp, hipStream_t s);
void launch_put_u64(uint64_t* dst, const uint64_t* src, hipStream_t s);
void launch_expand_pairs(uint32_t k, const uint32_t* items, const uint32_t* colsum,
                         const uint32_t* tri, uint32_t* out, hipStream_t s);

// Host-side helpers shared by the miner and the pair-support call.
inline uint32_t host_mfma_pairs(uint32_t q) {
  const uint32_t nb = (q + GRAM_TILE - 1) / GRAM_TILE;
  return nb * (nb + 1) / 2;
}
// Kernel that evaluates a class of q children: 0 = MFMA, 1 = LDS-blocked, 2 = registers.
__host__ __device__ inline int class_kind(uint32_t q, uint32_t mfma_min_q) {
  if (q >= mfma_min_q) return 0;
  return q <= (uint32_t)TINY_Q ? 2 : 1;
}
inline uint32_t host_andpop_pairs(uint32_t q) {
  const uint32_t nb = (q + AP_BLOCK - 1) / AP_BLOCK;
  return nb * (nb + 1) / 2 - ((q % AP_BLOCK) == 1 ? 1u : 0u);
}

}  // namespace bm
