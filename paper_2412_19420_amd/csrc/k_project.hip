// Projected views of big prefix classes: a sparse/dense hybrid of the
// paper's Boolean matrix for the deep levels of the recursion.
//
// A class with prefix P and children c_1..c_q only ever needs the rows of M
// that hold P: the supports of its candidates are popcounts of
// t(P) & col(c_i) & col(c_l) over all n transactions, but every term outside
// t(P) is zero.  When supp(P) is small enough against n, the class is counted
// over a view instead: the children's columns with every row outside t(P)
// squeezed out, i.e. bitsets of ceil(supp(P) / 64) words over P's
// transactions in order.  The class's Gram kernel then streams supp(P) / n of
// the words it would otherwise read, with the prefix already applied.  The
// paper points at sparse representations and block computing for large data
// (Section I; Section III's closing paragraph); the view is this project's
// form of that idea on the GPU: the prefix's tidset decides which bits
// survive, the children stay dense bitsets.
//
// Per level step, for all projected classes at once (views zeroed first):
//   count   -- popcount of t(P) over 64-word chunks (a wave each), then a
//              scan: each chunk's first bit in its class's view;
//   compact -- a wave per (chunk, child group) compresses every child word
//              by its prefix word and assembles the chunk's view words in
//              LDS.  Padding words past supp(P) stay zero.
#include "internal.hpp"
#include "levels.hpp"

namespace bm {

namespace {

constexpr int kThreads = 256;
constexpr uint32_t kChunkWords = 64;    // prefix words per wave (one per lane)
constexpr uint32_t kCompactChildren = 16;  // children per compaction group
constexpr int kImages = 4;                  // children compacted per round (LDS images)
constexpr uint32_t kGroupLanes = 64;        // child groups of one chunk handled side by side

// Word w of t(P): the AND of the prefix's columns (zero past the last word).
__device__ inline uint64_t prefix_word(const DbInfo& db, const uint32_t* __restrict__ pre,
                                       uint32_t pre_len, uint64_t w) {
  if (w >= db.W) return 0;
  uint64_t t = ~0ull;
  for (uint32_t j = 0; j < pre_len; ++j) t &= db.B[(uint64_t)pre[j] * db.Wp + w];
  return t;
}

// blockIdx.y = projected class; wave w of workgroup b counts the set bits of
// the prefix over 64-word chunk 4b + w (a word per lane).
__global__ __launch_bounds__(kThreads) void k_project_count(const ProjWork* __restrict__ pw,
                                                            const ClassDesc* __restrict__ cls,
                                                            const DbInfo* __restrict__ dbs,
                                                            const uint32_t* __restrict__ pre_cols,
                                                            uint32_t nchunks,
                                                            uint32_t* __restrict__ cnt) {
  const uint32_t slot = blockIdx.y;
  const uint32_t chunk = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (chunk >= nchunks) return;  // uniform per wave
  const ClassDesc cd = cls[pw[slot].cls];
  const DbInfo db = dbs[cd.db];
  const uint32_t* pre = pre_cols + cd.pre_off;
  uint32_t c = (uint32_t)__popcll(
      prefix_word(db, pre, cd.pre_len, (uint64_t)chunk * kChunkWords + (threadIdx.x & 63)));
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0) cnt[(uint64_t)slot * nchunks + chunk] = c;
}

// Bit compress (the PEXT operation) of x by mask m: the bits of x at the set
// positions of m, packed at the low end in order.  Warren's method (Hacker's
// Delight, 2nd ed., Section 7-4): six rounds, round i moving the selected bits
// right by 2^i; the moves depend only on m, so they are computed once per
// prefix word (compress_masks) and shared by every child column.
__device__ inline void compress_masks(uint64_t m, uint64_t mv[6]) {
  uint64_t mk = ~m << 1;  // at each position: the zeros of m to its right, in parity form below
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    uint64_t mp = mk ^ (mk << 1);  // parallel prefix (XOR) of mk: odd counts move this round
    mp ^= mp << 2;
    mp ^= mp << 4;
    mp ^= mp << 8;
    mp ^= mp << 16;
    mp ^= mp << 32;
    const uint64_t v = mp & m;
    mv[i] = v;
    m = (m ^ v) | (v >> (1 << i));
    mk &= ~mp;
  }
}

__device__ inline uint64_t compress(uint64_t x, uint64_t m, const uint64_t mv[6]) {
  x &= m;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const uint64_t t = x & mv[i];
    x = (x ^ t) | (t >> (1 << i));
  }
  return x;
}

// Orders one wave's LDS writes before its own later reads (and reads before
// later writes): a wave's LDS operations are performed in issue order, and the
// fence keeps the compiler from moving them across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// blockIdx.y = projected class.  Each wave takes one 64-word chunk of the
// prefix (lane l: word 64 c + l, its prefix word, the masks of its compress
// and, by a wave scan of the popcounts plus the chunk's scanned offset, its
// first bit in the view) and strides over groups of the class's children.
// Per child, every lane compresses its word and ORs the result into the
// wave's LDS image of the chunk's view words (at most 65); the image is then
// written out -- plain stores for the words the chunk covers whole, atomic
// ORs for the two it may share with its neighbours (the views are zeroed
// first).  No workgroup barrier: each wave works alone, kImages children at
// a time.
__global__ __launch_bounds__(kThreads) void k_project_compact(
    const ProjWork* __restrict__ pw, const ClassDesc* __restrict__ cls,
    const DbInfo* __restrict__ dbs, const DbInfo* __restrict__ views,
    const uint32_t* __restrict__ pre_cols, const uint32_t* __restrict__ child_item,
    const uint64_t* __restrict__ off, uint32_t nchunks, uint32_t gx) {
  constexpr int NWV = kThreads / 64;
  __shared__ unsigned long long s_img[NWV][kImages][kChunkWords + 1];
  const uint32_t slot = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t wid = (uint64_t)blockIdx.x * NWV + wave;
  const uint32_t chunk = (uint32_t)(wid % nchunks);
  const uint32_t g0 = (uint32_t)(wid / nchunks);
  if (g0 >= gx) return;  // uniform per wave
  const ProjWork w = pw[slot];
  const ClassDesc cd = cls[w.cls];
  const uint32_t q = cd.q;
  if (g0 * kCompactChildren >= q) return;  // uniform per wave
  const DbInfo db = dbs[cd.db];
  const DbInfo v = views[slot];
  const uint32_t* pre = pre_cols + cd.pre_off;
  const uint64_t word = (uint64_t)chunk * kChunkWords + lane;
  const uint64_t t = prefix_word(db, pre, cd.pre_len, word);
  uint64_t mv[6];
  compress_masks(t, mv);
  const uint32_t k = (uint32_t)__popcll(t);
  uint32_t inc = k;
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  const uint32_t total = __shfl(inc, 63);
  if (total == 0) return;  // uniform: the prefix has no transaction in this chunk
  const uint64_t cbase = off[(uint64_t)slot * nchunks + chunk] - w.row_off;  // first view bit
  // the chunks' counts sum to the prefix's support, so the range lies in the
  // view; checked all the same so that no write can leave it
  if (cbase + total > v.n) return;  // uniform
  const uint32_t sh = (uint32_t)(cbase & 63);
  const uint32_t nwords = (sh + total + 63) >> 6;  // <= 65
  const uint32_t bit = sh + inc - k;               // this lane's first bit in the image
  const uint32_t bi = bit >> 6, bo = bit & 63;
  const bool spill = k && bo + k > 64;
  unsigned long long(*img)[kChunkWords + 1] = s_img[wave];
  for (int j = 0; j < kImages; ++j) {
    img[j][lane] = 0ull;
    if (lane == 0) img[j][kChunkWords] = 0ull;
  }
  wave_lds_sync();
  const bool in_word = word < db.W;
  for (uint32_t g = g0; g * kCompactChildren < q; g += gx) {
    const uint32_t c1 = min(q, (g + 1) * kCompactChildren);
    for (uint32_t cb = g * kCompactChildren; cb < c1; cb += kImages) {
      uint64_t x[kImages];
#pragma unroll
      for (int j = 0; j < kImages; ++j) {
        x[j] = 0ull;
        if (cb + j < c1 && in_word) {
          const uint32_t item = child_item[cd.child0 + cb + j];
          x[j] = db.B[(uint64_t)(db.f1 ? db.f1[item] : item) * db.Wp + word];
        }
      }
#pragma unroll
      for (int j = 0; j < kImages; ++j) {
        const uint64_t y = k ? compress(x[j], t, mv) : 0ull;
        if (y) {
          atomicOr(&img[j][bi], (unsigned long long)(y << bo));
          if (spill) atomicOr(&img[j][bi + 1], (unsigned long long)(y >> (64 - bo)));
        }
      }
      wave_lds_sync();  // the images are complete
#pragma unroll
      for (int j = 0; j < kImages; ++j) {
        if (cb + j >= c1) break;  // uniform
        uint64_t* dst = const_cast<uint64_t*>(v.B) + (uint64_t)(cb + j) * v.Wp + (cbase >> 6);
        for (uint32_t i = lane; i < nwords; i += 64) {
          const unsigned long long val = img[j][i];
          img[j][i] = 0ull;
          if ((i == 0 && sh != 0) || (i == nwords - 1 && ((sh + total) & 63) != 0)) {
            if (val) atomicOr(reinterpret_cast<unsigned long long*>(dst + i), val);
          } else {
            dst[i] = val;
          }
        }
      }
      wave_lds_sync();  // the images are clear for the next round
    }
  }
}

}  // namespace

uint64_t view_chunks(uint64_t Wmax) { return (Wmax + kChunkWords - 1) / kChunkWords; }

// Grids put the projected classes on blockIdx.y, at most 65,535 per launch.
constexpr uint32_t kMaxGridY = 65535;

void launch_project_count(const ProjWork* pw, uint32_t nprj, const ClassDesc* cls,
                          const DbInfo* dbs, const uint32_t* pre_cols, uint64_t Wmax,
                          uint32_t* cnt_tmp, hipStream_t s) {
  const uint64_t ch = view_chunks(Wmax);
  const uint64_t gxb = (ch + kThreads / 64 - 1) / (kThreads / 64);
  if (gxb > 0x7fffffffull) fail(BM_ERR_UNSUPPORTED, "column too long for projected views");
  for (uint32_t b = 0; b < nprj; b += kMaxGridY) {
    const dim3 grid((uint32_t)gxb, min(kMaxGridY, nprj - b));
    k_project_count<<<grid, kThreads, 0, s>>>(pw + b, cls, dbs, pre_cols, (uint32_t)ch,
                                               cnt_tmp + b * ch);
    BM_LAUNCH_CHECK();
  }
}

void launch_project_compact(const ProjWork* pw, uint32_t nprj, const ClassDesc* cls,
                            const DbInfo* dbs, const DbInfo* views, const uint32_t* pre_cols,
                            const uint32_t* child_item, uint64_t Wmax, const uint64_t* off_tmp,
                            hipStream_t s) {
  const uint64_t ch = view_chunks(Wmax);
  // waves: every (chunk, child-group lane) pair; a wave walks its lane's groups
  const uint64_t waves = ch * kGroupLanes;
  const uint64_t gxb = (waves + kThreads / 64 - 1) / (kThreads / 64);
  if (gxb > 0x7fffffffull || ch > 0xffffffffull)
    fail(BM_ERR_UNSUPPORTED, "column too long for projected views");
  for (uint32_t b = 0; b < nprj; b += kMaxGridY) {
    const dim3 grid((uint32_t)gxb, min(kMaxGridY, nprj - b));
    k_project_compact<<<grid, kThreads, 0, s>>>(pw + b, cls, dbs, views + b, pre_cols, child_item,
                                                 off_tmp + b * ch, (uint32_t)ch, kGroupLanes);
    BM_LAUNCH_CHECK();
  }
}

}  // namespace bm
