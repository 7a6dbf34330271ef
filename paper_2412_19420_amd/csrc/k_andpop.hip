// Candidate supports of small prefix classes by AND + popcount (VALU).
//
// The method's support step (Eq. 2 and the sequential-AND rule for longer
// itemsets): for a class with prefix P and children c_0..c_{q-1}, the support of
// P + {c_i, c_l} is popcount(t(P) & M[:, c_i] & M[:, c_l]) summed over 64-bit
// words.  One task covers a 16 x 16 block pair of the class's children over a
// word range:
//   * each chunk of TC words of the prefix tidset t(P) (AND of P's columns) is
//     computed once and ANDed into every staged child column, so the LDS holds
//     X_i = t(P) & M[:, c_i] for up to 32 children -- the prefix is read once
//     and reused by every sibling extension of the block;
//   * the block's candidate pairs are spread over the 256 threads: G threads
//     (a power of two) per pair, each summing popcount(X_i & X_l) over a strided
//     share of the chunk's words, accumulated across all chunks in a register;
//   * the G partial counts of a pair are reduced with wavefront shuffles (DPP /
//     swizzle), and one integer atomic add per wave puts the task's count into
//     the class triangle (exact and order-independent across word splits);
//   * the next chunk's global loads are issued before the current chunk is
//     counted (software pipelining).
#include "internal.hpp"

namespace bm {

namespace {

// Pair number p of the triangle ordered by l then i: (0,1), (0,2), (1,2), (0,3), ...
// The first n(n-1)/2 pairs are exactly the pairs of the first n children.
__device__ __forceinline__ void unrank_pair(int p, int* i, int* l) {
  int L = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)p)) * 0.5f);
  while (L * (L - 1) / 2 > p) --L;
  while ((L + 1) * L / 2 <= p) ++L;
  *l = L;
  *i = p - L * (L - 1) / 2;
}

template <int TC>
__global__ __launch_bounds__(256) void k_andpop(ClassArgs a) {
  constexpr int RG = 256 / TC;  // threads per staged word
  constexpr int RPT = 32 / RG;  // staged rows per thread
  __shared__ uint64_t X[32][TC + 1];
  __shared__ uint64_t s_col[32];
  const int tid = threadIdx.x;
  const int wi = tid % TC;
  const int rg = tid / TC;
  const int lane = tid & 63;
  const uint64_t ntasks = *a.ntasks;

  for (uint64_t t = blockIdx.x; t < ntasks; t += gridDim.x) {
    const Task task = a.tasks[t];
    const ClassDesc cd = a.cls[task.cls];
    const DbInfo db = class_view(cd, a.dbs, a.views);
    const uint32_t q = cd.q;
    const uint32_t i0 = (uint32_t)task.bi * AP_BLOCK, l0 = (uint32_t)task.bl * AP_BLOCK;
    const int NI = (int)min<uint32_t>(AP_BLOCK, q - i0);
    const int NL = (int)min<uint32_t>(AP_BLOCK, q - l0);
    const bool diag = task.bi == task.bl;
    const int NP = diag ? NI * (NI - 1) / 2 : NI * NL;
    if (NP == 0) continue;  // uniform across the workgroup

    __syncthreads();  // previous task finished with s_col / X
    if (tid < 32) {
      const int r = tid;
      uint64_t off = ~0ull;
      if (r < 16 && r < NI) {
        const uint32_t item = a.child_item[cd.child0 + i0 + r];
        off = (uint64_t)class_col(cd, db, i0 + r, item) * db.Wp;
      } else if (!diag && r >= 16 && r - 16 < NL) {
        const uint32_t item = a.child_item[cd.child0 + l0 + (r - 16)];
        off = (uint64_t)class_col(cd, db, l0 + (r - 16), item) * db.Wp;
      }
      s_col[r] = off;
    }
    __syncthreads();

    // pair owned by this thread
    int G = 256;
    while (G > 1 && G * NP > 256) G >>= 1;
    const int p = tid / G, g = tid % G;
    const bool active = p < NP;
    int ri = 0, rl = 0;
    if (active) {
      if (diag) {
        unrank_pair(p, &ri, &rl);
      } else {
        ri = p / NL;
        rl = 16 + p % NL;
      }
    }

    const uint32_t* pre = a.pre_cols + cd.pre_off;
    const uint32_t pre_len = cd.proj ? 0u : cd.pre_len;  // a view has the prefix applied
    const uint32_t w0 = task.w0, w1 = task.w1;
    const uint32_t nch = (w1 - w0 + TC - 1) / TC;

    // the first PREFIX_REG prefix columns addressed once per task; every load
    // goes through the global address space, so the LDS waits of the count
    // loop do not wait for the next chunk's loads
    const uint64_t* pc[PREFIX_REG];
#pragma unroll
    for (int j = 0; j < PREFIX_REG; ++j)
      pc[j] = (uint32_t)j < pre_len ? db.B + (uint64_t)load_global_u32(pre + j) * db.Wp : nullptr;
    uint64_t v[RPT];
    uint64_t pv[PREFIX_REG];
    uint64_t msk = 0;
    auto load_chunk = [&](uint32_t c) {
      const uint32_t w = w0 + c * TC + wi;
      const bool inb = w < w1;
      msk = inb ? ~0ull : 0ull;
      for (uint32_t j = PREFIX_REG; j < pre_len && inb; ++j)
        msk &= load_global_u64(db.B + (uint64_t)load_global_u32(pre + j) * db.Wp + w);
#pragma unroll
      for (int j = 0; j < PREFIX_REG; ++j) pv[j] = (inb && pc[j]) ? load_global_u64(pc[j] + w) : ~0ull;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const uint64_t off = s_col[rg + RG * k];
        v[k] = (inb && off != ~0ull) ? load_global_u64(db.B + off + w) : 0ull;
      }
    };

    uint32_t acc = 0;
    load_chunk(0);
    for (uint32_t c = 0; c < nch; ++c) {
      __syncthreads();  // previous chunk counted
#pragma unroll
      for (int j = 0; j < PREFIX_REG; ++j) msk &= pv[j];
#pragma unroll
      for (int k = 0; k < RPT; ++k) X[rg + RG * k][wi] = v[k] & msk;
      __syncthreads();
      if (c + 1 < nch) load_chunk(c + 1);
      const int cw = (int)min<uint32_t>(TC, w1 - (w0 + c * TC));
      if (active) {
        const uint64_t* xi = X[ri];
        const uint64_t* xl = X[rl];
        for (int w = g; w < cw; w += G) acc += (uint32_t)__popcll(xi[w] & xl[w]);
      }
    }

    // reduce the G partial counts of each pair inside the wavefront
    const int span = G < 64 ? G : 64;
    for (int off = span >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (active && (lane % span) == 0 && acc) {
      const uint32_t gi = i0 + ri;
      const uint32_t gl = (diag ? i0 : l0 - 16) + rl;
      atomicAdd(a.tri + cd.tri_off + tri_index(gi, gl, q), acc);
    }
  }
}

// Classes with at most TINY_Q children: no LDS staging.  Each thread streams
// four consecutive words of the prefix and of every child column with two
// independent 16-byte loads (task word ranges start at multiples of 64 and
// columns are padded to 64 words, so the four words stay inside the column),
// ANDs them in registers and keeps one popcount accumulator per child pair;
// the accumulators are reduced across the wavefront with shuffles and across
// the workgroup through LDS once per task.
constexpr int TQ = TINY_Q;
constexpr int TNP = TQ * (TQ - 1) / 2;

__global__ __launch_bounds__(256) void k_andpop_reg(ClassArgs a) {
  __shared__ uint32_t s_red[4][TNP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t ntasks = *a.ntasks;
  for (uint64_t t = blockIdx.x; t < ntasks; t += gridDim.x) {
    const Task task = a.tasks[t];
    const ClassDesc cd = a.cls[task.cls];
    const DbInfo db = class_view(cd, a.dbs, a.views);
    const int q = (int)cd.q;
    const uint64_t* col[TQ];
#pragma unroll
    for (int i = 0; i < TQ; ++i) {
      col[i] = db.B;
      if (i < q) {
        const uint32_t item = a.child_item[cd.child0 + i];
        col[i] = db.B + (uint64_t)class_col(cd, db, i, item) * db.Wp;
      }
    }
    const uint32_t* pre = a.pre_cols + cd.pre_off;
    const uint32_t pre_len = cd.proj ? 0u : cd.pre_len;  // a view has the prefix applied
    // the first PREFIX_REG prefix columns addressed once per task, so their
    // loads go out with the column loads (global address space throughout)
    const uint64_t* pc[PREFIX_REG];
#pragma unroll
    for (int j = 0; j < PREFIX_REG; ++j)
      pc[j] = (uint32_t)j < pre_len ? db.B + (uint64_t)load_global_u32(pre + j) * db.Wp : nullptr;
    uint32_t acc[TNP];
#pragma unroll
    for (int p = 0; p < TNP; ++p) acc[p] = 0;
    for (uint32_t w = task.w0 + 4 * tid; w < task.w1; w += 1024) {
      uint64_t m[4];
#pragma unroll
      for (int h = 0; h < 4; ++h) m[h] = (w + h < task.w1) ? ~0ull : 0ull;
      prefix_and(pc, db.B, db.Wp, pre, pre_len, w, m[0], m[1]);
      {
        const uint64_t* pc2[PREFIX_REG];
#pragma unroll
        for (int j = 0; j < PREFIX_REG; ++j) pc2[j] = pc[j] ? pc[j] + 2 : nullptr;
        prefix_and(pc2, db.B + 2, db.Wp, pre, pre_len, w, m[2], m[3]);
      }
      uint64_t xv[TQ][4];
#pragma unroll
      for (int i = 0; i < TQ; ++i) {
#pragma unroll
        for (int h = 0; h < 4; ++h) xv[i][h] = 0;
        if (i < q) {
          const uint4 v = load_global16(col[i] + w);
          const uint4 u = load_global16(col[i] + w + 2);
          xv[i][0] = ((uint64_t)v.x | ((uint64_t)v.y << 32)) & m[0];
          xv[i][1] = ((uint64_t)v.z | ((uint64_t)v.w << 32)) & m[1];
          xv[i][2] = ((uint64_t)u.x | ((uint64_t)u.y << 32)) & m[2];
          xv[i][3] = ((uint64_t)u.z | ((uint64_t)u.w << 32)) & m[3];
        }
      }
      int p = 0;
#pragma unroll
      for (int i = 0; i < TQ; ++i)
#pragma unroll
        for (int l = i + 1; l < TQ; ++l, ++p)
          if (l < q)
            acc[p] += (uint32_t)(__popcll(xv[i][0] & xv[l][0]) + __popcll(xv[i][1] & xv[l][1]) +
                                 __popcll(xv[i][2] & xv[l][2]) + __popcll(xv[i][3] & xv[l][3]));
    }
#pragma unroll
    for (int p = 0; p < TNP; ++p) {
      uint32_t v = acc[p];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) s_red[wave][p] = v;
    }
    __syncthreads();
    if (tid < TNP) {
      int i = 0, r = tid;
      while (r >= TQ - 1 - i) {
        r -= TQ - 1 - i;
        ++i;
      }
      const int l = i + 1 + r;
      const uint32_t v = s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
      if (l < q && v) atomicAdd(a.tri + cd.tri_off + tri_index(i, l, q), v);
    }
    __syncthreads();
  }
}

}  // namespace

void launch_andpop_reg(const ClassArgs& a, uint32_t grid, hipStream_t s) {
  if (grid == 0) return;
  k_andpop_reg<<<grid, 256, 0, s>>>(a);
  BM_LAUNCH_CHECK();
}

void launch_andpop(const ClassArgs& a, uint32_t chunk_words, uint32_t grid, hipStream_t s) {
  if (grid == 0) return;
  if (chunk_words == 128) {
    k_andpop<128><<<grid, 256, 0, s>>>(a);
  } else {
    k_andpop<256><<<grid, 256, 0, s>>>(a);
  }
  BM_LAUNCH_CHECK();
}

}  // namespace bm
