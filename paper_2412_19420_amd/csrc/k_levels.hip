// Frequent-itemset extraction (Eq. 3) and the recursive extension of frequent
// prefixes, level by level, plus the canonical-order output.
//
// Level k holds the frequent k-itemsets in lexicographic order as records
// (parent index in level k-1, last item, support); the children of a node are
// contiguous in level k+1.  A step turns level k into level k+1:
//   * classes: the level-k nodes grouped by parent.  A parent with q >= 2
//     frequent children forms a prefix class whose candidates are the q(q-1)/2
//     pairs of children; supports land in the step's triangle buffer, class by
//     class, row by row -- which is exactly lexicographic order of the
//     candidate itemsets;
//   * threshold + exclusive scan over the triangle give each frequent candidate
//     its index in level k+1, so the next level comes out already sorted;
//   * a node with c >= 2 frequent children becomes a class of the next step.
#include "internal.hpp"
#include "levels.hpp"

namespace bm {

namespace {

constexpr int kThreads = 256;

uint32_t grid_for(uint64_t work, uint32_t per_block, uint32_t cap = 65535) {
  uint64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

__global__ void k_f1_fill(const uint32_t* __restrict__ colsum, uint32_t m, uint32_t minsup,
                          const uint64_t* __restrict__ pos, uint32_t* __restrict__ f1) {
  for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < m;
       j += (uint64_t)gridDim.x * blockDim.x)
    if (colsum[j] >= minsup) f1[pos[j]] = (uint32_t)j;
}

__global__ void k_init_level1(const uint32_t* __restrict__ colsum, const uint32_t* __restrict__ f1,
                              uint32_t n1, uint32_t* __restrict__ item, uint32_t* __restrict__ parent,
                              uint32_t* __restrict__ supp) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n1;
       i += (uint64_t)gridDim.x * blockDim.x) {
    item[i] = (uint32_t)i;
    parent[i] = 0;
    supp[i] = colsum[f1[i]];
  }
}

__device__ inline uint32_t mfma_pairs(uint32_t q) {
  const uint32_t nb = (q + GRAM_TILE - 1) / GRAM_TILE;
  return nb * (nb + 1) / 2;
}
__device__ inline uint32_t andpop_pairs(uint32_t q) {
  const uint32_t nb = (q + AP_BLOCK - 1) / AP_BLOCK;
  // the diagonal block of a lone last child holds no pair
  return nb * (nb + 1) / 2 - ((q % AP_BLOCK) == 1 ? 1u : 0u);
}

// Per node of level k: number of frequent children, and what it contributes
// to the next step if it becomes a class.  Also accumulates per-step totals
// (candidates, columns read, classes per kernel) for the statistics.
__global__ __launch_bounds__(kThreads) void k_node_counts(
    uint64_t n, uint32_t k, const uint32_t* __restrict__ parent, const int32_t* __restrict__ pcls,
    const ClassDesc* __restrict__ cls, const uint64_t* __restrict__ S, uint32_t mfma_min_q,
    uint32_t* __restrict__ cnt, uint32_t* __restrict__ is_cls, uint64_t* __restrict__ tri_sz,
    uint32_t* __restrict__ pm, uint32_t* __restrict__ pv, uint32_t* __restrict__ pt,
    unsigned long long* __restrict__ st) {
  __shared__ unsigned long long s_st[ST_COUNT];
  if (threadIdx.x < ST_COUNT) s_st[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long loc[ST_COUNT];
#pragma unroll
  for (int j = 0; j < ST_COUNT; ++j) loc[j] = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const int32_t c = pcls[parent[i]];
    uint32_t kc = 0;
    if (c >= 0) {
      const ClassDesc cd = cls[c];
      const uint64_t li = i - cd.child0;
      if (li + 1 < cd.q) {
        const uint64_t rs = cd.tri_off + tri_index(li, li + 1, cd.q);
        const uint64_t len = cd.q - li - 1;
        kc = (uint32_t)(S[rs + len] - S[rs]);
      }
    }
    cnt[i] = kc;
    const bool cl = kc >= 2;
    const int kind = cl ? class_kind(kc, mfma_min_q) : -1;
    const uint64_t tsz = cl ? (uint64_t)kc * (kc - 1) / 2 : 0ull;
    is_cls[i] = cl ? 1u : 0u;
    tri_sz[i] = tsz;
    pm[i] = kind == 0 ? mfma_pairs(kc) : 0u;
    pv[i] = kind == 1 ? andpop_pairs(kc) : 0u;
    pt[i] = kind == 2 ? 1u : 0u;
    if (cl) {
      loc[ST_CAND_M + kind] += tsz;
      loc[ST_COLS_M + kind] += kc + k;
      loc[ST_CLS_M + kind] += 1;
    }
  }
  for (int j = 0; j < ST_COUNT; ++j)
    if (loc[j]) atomicAdd(&s_st[j], loc[j]);
  __syncthreads();
  if (threadIdx.x < ST_COUNT && s_st[threadIdx.x]) atomicAdd(&st[threadIdx.x], s_st[threadIdx.x]);
}

// Wave per node: write the node's frequent extensions into the next level.
__global__ void k_fill_level(uint64_t n, const uint32_t* __restrict__ parent,
                             const int32_t* __restrict__ pcls, const ClassDesc* __restrict__ cls,
                             const uint32_t* __restrict__ child_item, const uint32_t* __restrict__ tri,
                             const uint64_t* __restrict__ S, uint32_t minsup,
                             uint32_t* __restrict__ nitem, uint32_t* __restrict__ nparent,
                             uint32_t* __restrict__ nsupp) {
  const int lane = threadIdx.x & 63;
  const uint64_t wave0 = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t i = wave0; i < n; i += nwaves) {
    const int32_t c = pcls[parent[i]];
    if (c < 0) continue;
    const ClassDesc cd = cls[c];
    const uint64_t li = i - cd.child0;
    if (li + 1 >= cd.q) continue;
    const uint64_t rs = cd.tri_off + tri_index(li, li + 1, cd.q);
    const uint64_t len = cd.q - li - 1;
    for (uint64_t t = lane; t < len; t += 64) {
      const uint32_t v = tri[rs + t];
      if (v >= minsup) {
        const uint64_t pos = S[rs + t];
        nitem[pos] = child_item[cd.child0 + li + 1 + t];
        nparent[pos] = (uint32_t)i;
        nsupp[pos] = v;
      }
    }
  }
}

// Task records of one class: MFMA block pairs x word splits, or AND+popcount
// block pairs x word splits.  Lanes of a wave stride over the class's tasks.
__device__ void write_tasks(uint32_t ci, uint32_t q, uint32_t npairs, uint32_t block,
                            uint32_t nsplit, uint32_t split_len, uint32_t wend, Task* out,
                            int lane, int nl) {
  const uint32_t nb = (q + block - 1) / block;
  const uint64_t total = (uint64_t)npairs * nsplit;
  for (uint64_t t = lane; t < total; t += nl) {
    uint32_t tp = (uint32_t)(t / nsplit);
    const uint32_t sp = (uint32_t)(t % nsplit);
    uint32_t bi = 0;
    while (tp >= nb - bi) {
      tp -= nb - bi;
      ++bi;
    }
    Task k;
    k.cls = ci;
    k.bi = (uint16_t)bi;
    k.bl = (uint16_t)(bi + tp);
    k.w0 = sp * split_len;
    k.w1 = min(wend, (sp + 1) * split_len);
    out[t] = k;
  }
}

// Wave per node of level k: if the node has >= 2 frequent children it becomes
// a class of the next step (its prefix = the node's itemset).
__global__ void k_fill_classes(uint64_t n, uint32_t k, const uint32_t* __restrict__ cnt,
                               const uint64_t* __restrict__ child_start,
                               const uint64_t* __restrict__ cls_pos,
                               const uint64_t* __restrict__ tri_off,
                               const uint64_t* __restrict__ pm_off, const uint64_t* __restrict__ pv_off,
                               const uint64_t* __restrict__ pt_off, uint32_t mfma_min_q, LevelPtrs lv,
                               const uint32_t* __restrict__ f1, ClassDesc* __restrict__ ocls,
                               uint32_t* __restrict__ opre, int32_t* __restrict__ pcls_out,
                               TaskGeom geo, Task* __restrict__ tm, Task* __restrict__ tv,
                               Task* __restrict__ tt) {
  const int lane = threadIdx.x & 63;
  const uint64_t wave0 = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
  const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t i = wave0; i < n; i += nwaves) {
    const uint32_t q = cnt[i];
    if (q < 2) {
      if (lane == 0) pcls_out[i] = -1;
      continue;
    }
    const uint32_t ci = (uint32_t)cls_pos[i];
    if (lane == 0) {
      pcls_out[i] = (int32_t)ci;
      ClassDesc cd;
      cd.tri_off = tri_off[i];
      cd.child0 = (uint32_t)child_start[i];
      cd.q = q;
      cd.pre_off = ci * k;
      cd.pre_len = k;
      ocls[ci] = cd;
      uint64_t x = i;
      for (int lev = (int)k; lev >= 1; --lev) {
        opre[(uint64_t)ci * k + (k - lev)] = f1[lv.item[lev][x]];
        x = lv.parent[lev][x];
      }
    }
    const int kind = class_kind(q, mfma_min_q);
    if (kind == 0) {
      const uint32_t np = (uint32_t)(pm_off[i + 1] - pm_off[i]);
      write_tasks(ci, q, np, GRAM_TILE, geo.nsplit_m, geo.split_m, geo.wend_m,
                  tm + pm_off[i] * geo.nsplit_m, lane, 64);
    } else if (kind == 1) {
      const uint32_t np = (uint32_t)(pv_off[i + 1] - pv_off[i]);
      write_tasks(ci, q, np, AP_BLOCK, geo.nsplit_v, geo.split_v, geo.wend_v,
                  tv + pv_off[i] * geo.nsplit_v, lane, 64);
    } else {
      write_tasks(ci, q, 1, TINY_Q, geo.nsplit_t, geo.split_t, geo.wend_t,
                  tt + pt_off[i] * geo.nsplit_t, lane, 64);
    }
  }
}

__global__ void k_root_tasks(uint32_t q, uint32_t npairs, uint32_t block, uint32_t nsplit,
                             uint32_t split_len, uint32_t wend, Task* __restrict__ out) {
  write_tasks(0, q, npairs, block, nsplit, split_len, wend, out,
              (int)(blockIdx.x * blockDim.x + threadIdx.x), (int)(gridDim.x * blockDim.x));
}

// ---------------------------------------------------------------- output

// Subtree sizes (itemsets, item ids) of each level-k node from the next level's scans.
__global__ void k_emit_sizes(uint64_t n, uint32_t k, const uint64_t* __restrict__ cstart,
                             const uint64_t* __restrict__ SZn, const uint64_t* __restrict__ ISZn,
                             uint64_t* __restrict__ sz, uint64_t* __restrict__ isz) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t a = 1, b = k;
    if (SZn) {
      const uint64_t c0 = cstart[i], c1 = cstart[i + 1];
      a += SZn[c1] - SZn[c0];
      b += ISZn[c1] - ISZn[c0];
    }
    sz[i] = a;
    isz[i] = b;
  }
}

// Preorder rank and item offset of each level-k node (k >= 2) from its parent's.
__global__ void k_emit_pos(uint64_t n, uint32_t k, const uint32_t* __restrict__ parent,
                           const uint64_t* __restrict__ ppre, const uint64_t* __restrict__ poff,
                           const uint64_t* __restrict__ pcstart, const uint64_t* __restrict__ SZ,
                           const uint64_t* __restrict__ ISZ, uint64_t* __restrict__ pre,
                           uint64_t* __restrict__ off) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t p = parent[i];
    const uint64_t first = pcstart[p];
    pre[i] = ppre[p] + 1 + (SZ[i] - SZ[first]);
    off[i] = poff[p] + (k - 1) + (ISZ[i] - ISZ[first]);
  }
}

__global__ void k_emit_write(uint64_t n, uint32_t k, const uint64_t* __restrict__ pre,
                             const uint64_t* __restrict__ off, const uint32_t* __restrict__ supp,
                             LevelPtrs lv, const uint32_t* __restrict__ f1,
                             uint64_t* __restrict__ o_off, uint32_t* __restrict__ o_items,
                             uint32_t* __restrict__ o_supp) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t r = pre[i], o = off[i];
    o_off[r] = o;
    o_supp[r] = supp[i];
    uint64_t x = i;
    for (int lev = (int)k; lev >= 1; --lev) {
      o_items[o + lev - 1] = f1[lv.item[lev][x]];
      x = lv.parent[lev][x];
    }
  }
}

__global__ void k_put_u64(uint64_t* __restrict__ dst, const uint64_t* __restrict__ src) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

__global__ void k_expand_pairs(uint32_t k, const uint32_t* __restrict__ items,
                               const uint32_t* __restrict__ colsum, const uint32_t* __restrict__ tri,
                               uint32_t* __restrict__ out) {
  const uint64_t total = (uint64_t)k * k;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t a = e / k, b = e % k;
    uint32_t v;
    if (a == b) v = colsum[items[a]];
    else v = tri[a < b ? tri_index(a, b, k) : tri_index(b, a, k)];
    out[e] = v;
  }
}

}  // namespace

void launch_f1_fill(const uint32_t* colsum, uint32_t m, uint32_t minsup, const uint64_t* pos,
                    uint32_t* f1, hipStream_t s) {
  if (m == 0) return;
  k_f1_fill<<<grid_for(m, kThreads), kThreads, 0, s>>>(colsum, m, minsup, pos, f1);
  BM_LAUNCH_CHECK();
}

void launch_init_level1(const uint32_t* colsum, const uint32_t* f1, uint32_t n1, uint32_t* item,
                        uint32_t* parent, uint32_t* supp, hipStream_t s) {
  if (n1 == 0) return;
  k_init_level1<<<grid_for(n1, kThreads), kThreads, 0, s>>>(colsum, f1, n1, item, parent, supp);
  BM_LAUNCH_CHECK();
}

void launch_node_counts(uint64_t n, uint32_t k, const uint32_t* parent, const int32_t* pcls,
                        const ClassDesc* cls, const uint64_t* S, uint32_t mfma_min_q,
                        uint32_t* cnt, uint32_t* is_cls, uint64_t* tri_sz, uint32_t* pm,
                        uint32_t* pv, uint32_t* pt, unsigned long long* st, hipStream_t s) {
  if (n == 0) return;
  k_node_counts<<<grid_for(n, kThreads, 2048), kThreads, 0, s>>>(n, k, parent, pcls, cls, S,
                                                                  mfma_min_q, cnt, is_cls, tri_sz,
                                                                  pm, pv, pt, st);
  BM_LAUNCH_CHECK();
}

void launch_fill_level(uint64_t n, const uint32_t* parent, const int32_t* pcls,
                       const ClassDesc* cls, const uint32_t* child_item, const uint32_t* tri,
                       const uint64_t* S, uint32_t minsup, uint32_t* nitem, uint32_t* nparent,
                       uint32_t* nsupp, hipStream_t s) {
  if (n == 0) return;
  k_fill_level<<<grid_for(n * 64, kThreads), kThreads, 0, s>>>(n, parent, pcls, cls, child_item, tri,
                                                                 S, minsup, nitem, nparent, nsupp);
  BM_LAUNCH_CHECK();
}

void launch_fill_classes(uint64_t n, uint32_t k, const uint32_t* cnt, const uint64_t* child_start,
                         const uint64_t* cls_pos, const uint64_t* tri_off, const uint64_t* pm_off,
                         const uint64_t* pv_off, const uint64_t* pt_off, uint32_t mfma_min_q,
                         const LevelPtrs& lv, const uint32_t* f1, ClassDesc* ocls, uint32_t* opre,
                         int32_t* pcls_out, const TaskGeom& geo, Task* tm, Task* tv, Task* tt,
                         hipStream_t s) {
  if (n == 0) return;
  k_fill_classes<<<grid_for(n * 64, kThreads), kThreads, 0, s>>>(
      n, k, cnt, child_start, cls_pos, tri_off, pm_off, pv_off, pt_off, mfma_min_q, lv, f1, ocls,
      opre, pcls_out, geo, tm, tv, tt);
  BM_LAUNCH_CHECK();
}

void launch_root_tasks(uint32_t q, uint32_t npairs, uint32_t block, uint32_t nsplit,
                       uint32_t split_len, uint32_t wend, Task* out, hipStream_t s) {
  const uint64_t total = (uint64_t)npairs * nsplit;
  if (total == 0) return;
  k_root_tasks<<<grid_for(total, kThreads, 1024), kThreads, 0, s>>>(q, npairs, block, nsplit,
                                                                     split_len, wend, out);
  BM_LAUNCH_CHECK();
}

void launch_emit_sizes(uint64_t n, uint32_t k, const uint64_t* cstart, const uint64_t* SZn,
                       const uint64_t* ISZn, uint64_t* sz, uint64_t* isz, hipStream_t s) {
  if (n == 0) return;
  k_emit_sizes<<<grid_for(n, kThreads), kThreads, 0, s>>>(n, k, cstart, SZn, ISZn, sz, isz);
  BM_LAUNCH_CHECK();
}

void launch_emit_pos(uint64_t n, uint32_t k, const uint32_t* parent, const uint64_t* ppre,
                     const uint64_t* poff, const uint64_t* pcstart, const uint64_t* SZ,
                     const uint64_t* ISZ, uint64_t* pre, uint64_t* off, hipStream_t s) {
  if (n == 0) return;
  k_emit_pos<<<grid_for(n, kThreads), kThreads, 0, s>>>(n, k, parent, ppre, poff, pcstart, SZ, ISZ,
                                                         pre, off);
  BM_LAUNCH_CHECK();
}

void launch_emit_write(uint64_t n, uint32_t k, const uint64_t* pre, const uint64_t* off,
                       const uint32_t* supp, const LevelPtrs& lv, const uint32_t* f1,
                       uint64_t* o_off, uint32_t* o_items, uint32_t* o_supp, hipStream_t s) {
  if (n == 0) return;
  k_emit_write<<<grid_for(n, kThreads), kThreads, 0, s>>>(n, k, pre, off, supp, lv, f1, o_off,
                                                           o_items, o_supp);
  BM_LAUNCH_CHECK();
}

void launch_put_u64(uint64_t* dst, const uint64_t* src, hipStream_t s) {
  k_put_u64<<<1, 64, 0, s>>>(dst, src);
  BM_LAUNCH_CHECK();
}

void launch_expand_pairs(uint32_t k, const uint32_t* items, const uint32_t* colsum,
                         const uint32_t* tri, uint32_t* out, hipStream_t s) {
  const uint64_t total = (uint64_t)k * k;
  if (total == 0) return;
  k_expand_pairs<<<grid_for(total, kThreads), kThreads, 0, s>>>(k, items, colsum, tri, out);
  BM_LAUNCH_CHECK();
}

}  // namespace bm
