// Matrix construction (Eq. 1) and column aggregation (Eq. 3), plus the
// generic fill and prefix-sum kernels the level bookkeeping uses.
//
// Layout of M: one bitset per item column, Wp 64-bit words per column
// (column-major), transaction i at bit (i & 63) of word (i >> 6).  Column-major
// keeps every column contiguous, so the support kernels stream whole columns
// with coalesced 16-byte loads.
#include "internal.hpp"

namespace bm {

namespace {

constexpr int kThreads = 256;

__global__ void k_validate_rows(const uint64_t* __restrict__ rp, uint64_t n, uint32_t* err) {
  uint32_t bad = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    if (rp[i + 1] < rp[i]) bad |= 1u;
  }
  if (bad) atomicOr(err, bad);
}

__global__ void k_validate_cols(const uint32_t* __restrict__ ci, uint64_t nnz, uint32_t m,
                                uint32_t* err) {
  uint32_t bad = 0;
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (uint64_t)gridDim.x * blockDim.x) {
    if (ci[e] >= m) bad |= 2u;
  }
  if (bad) atomicOr(err, bad);
}

// One workgroup per 256 consecutive rows.  The rows' slice of row_ptr is kept
// in LDS; threads walk the rows' item ids with unit stride (coalesced) and find
// each id's row by binary search in LDS, then set the bit with a 64-bit atomic
// OR (idempotent, so duplicate ids collapse as M is 0/1).
__global__ __launch_bounds__(kThreads) void k_pack(const uint64_t* __restrict__ rp,
                                                   const uint32_t* __restrict__ ci, uint64_t n,
                                                   unsigned long long* __restrict__ B, uint64_t Wp) {
  __shared__ uint64_t s_rp[kThreads + 1];
  const uint64_t r0 = (uint64_t)blockIdx.x * kThreads;
  const uint32_t nr = (uint32_t)min<uint64_t>(kThreads, n - r0);
  for (uint32_t t = threadIdx.x; t <= nr; t += kThreads) s_rp[t] = rp[r0 + t];
  __syncthreads();
  const uint64_t e0 = s_rp[0], e1 = s_rp[nr];
  for (uint64_t e = e0 + threadIdx.x; e < e1; e += kThreads) {
    // largest r with s_rp[r] <= e (rows may be empty, so skip equal starts)
    uint32_t lo = 0, hi = nr;  // invariant: s_rp[lo] <= e < s_rp[hi]
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) >> 1;
      if (s_rp[mid] <= e) lo = mid; else hi = mid;
    }
    const uint64_t row = r0 + lo;
    const uint32_t j = ci[e];
    atomicOr(&B[(uint64_t)j * Wp + (row >> 6)], 1ull << (row & 63));
  }
}

// Tiled construction: one workgroup builds a 256-row block of M (4 words per
// column), one 512-column window at a time in LDS, and writes each window out
// as 32-byte column segments.  Every word of M is written exactly once (zeros
// included), so no clearing pass is needed, and each window's column popcounts
// are added to the single-item supports on the way out.
//   * the block's item ids are loaded once, coalesced and several per thread in
//     flight, into LDS as packed (column << 8 | local row) entries -- the row is
//     filled in row by row -- and then held in registers (12 per thread), so
//     every column window takes its bits from registers, not from LDS;
//   * bits are set with LDS atomic ORs (idempotent: duplicate ids collapse, as
//     M is 0/1); ids >= m are flagged;
//   * two window bitmaps (the second over the entry buffer, free once the
//     entries are in registers): window w is written out of one while window
//     w + 1 is ORed into the other, one barrier per window;
//   * row_ptr is checked on the way in (non-decreasing: flag 1); element
//     ranges are clamped to [0, nnz] and local rows are masked, so a malformed
//     row_ptr cannot send any access out of bounds.
// 256-row tiles keep a workgroup's LDS at 70 KB, so two workgroups (32 waves)
// share a CU and one's loads overlap the other's window passes: measured 15%
// faster than 512-row tiles with one workgroup per CU on the T40-style
// 1M x 2,000 build, 3% on the dense 1M x 4,096 one.
constexpr int PK_KR = 4;                  // words per column per tile
constexpr int PK_ROWS = PK_KR * 64;       // 256 rows
constexpr int PK_RBITS = 8;               // bits of a local row
constexpr int PK_CW = 512;                // columns per window
constexpr int PK_LD = PK_KR + 1;          // padded LDS row (conflict-free OR)
// Staged elements per chunk (48 KB): a tile with more runs its window passes
// once per chunk, later chunks adding to what B holds.  12,288 covers every
// 256-row tile of the dense 1M x 4,096 workload (mean 9,941 ids, at most
// 10,719), 10,240 missed 9% of them, and those tiles' second passes made the
// build 29% slower (0.363 against 0.281 ms).
constexpr int PK_ECAP = 12288;
constexpr int PK_UNROLL = 8;
// 16 waves per workgroup hide the latency of the staging loads and LDS atomics
// (measured 2.1x faster than 4 waves on the dense 1M x 4,096 workload).
constexpr int PK_T = 1024;
// Sparse databases (at most PK_SPARSE_ROW elements per row on average: a
// tile's mean fits one chunk) are packed by 512-thread workgroups with
// 6,144-element chunks: 46 KB of LDS, so three tiles share a CU instead of
// two.  Their tiles hold few ids and are bound by the latency of each tile's
// steps, which more tiles in flight hide: the batch of 256 Quest-style
// databases builds in 1.21 against 1.29 ms (1,024 threads, 8,192 elements).
constexpr int PK_ECAP_SPARSE = 6144;
constexpr int PK_T_SPARSE = 512;
constexpr int PK_SPARSE_ROW = 24;  // 24 x 256 rows = one chunk

// Workgroups are dispatched to the 8 XCDs in turn, so block b runs on XCD
// b % 8.  Giving each XCD a contiguous range of tiles lets the 32-byte
// pieces of a 128-byte line of M (neighbouring tiles) meet in one XCD's L2
// before they are written back (measured 7% faster on the dense 1M x 4,096
// build than tiles in block order).
__device__ __forceinline__ uint64_t xcd_tile(uint32_t b, uint32_t nb) {
  const uint32_t per = nb / 8, extra = nb % 8, x = b % 8, j = b / 8;
  return (uint64_t)x * per + min(x, extra) + j;
}

template <int ECAP>
struct PackSmem {
  unsigned long long X[PK_CW * PK_LD];
  uint32_t s_e[ECAP];
  uint64_t s_rp[PK_ROWS + 1];
};

// The bits of one column window [c0, c0 + cw) from a thread's entries, ORed
// into the window bitmap X.  The empty asm keeps the entries in registers and
// the per-window work recomputed from them, so values derived from all of a
// thread's entries are not held across windows.
template <int EPT>
__device__ __forceinline__ void pack_or_window(uint32_t (&xe)[EPT], unsigned long long* X,
                                               uint32_t c0, uint32_t cw) {
#pragma unroll
  for (int u = 0; u < EPT; ++u) asm volatile("" : "+v"(xe[u]));
#pragma unroll
  for (int u = 0; u < EPT; ++u) {
    const uint32_t x = xe[u];
    if (x == 0xffffffffu) continue;
    const uint32_t d = (x >> PK_RBITS) - c0;
    if (d < cw) {
      const int lr = x & (PK_ROWS - 1);
      atomicOr(X + d * PK_LD + (lr >> 6), 1ull << (lr & 63));
    }
  }
}

template <int ECAP, int T>
__device__ __forceinline__ void pack_tile(PackSmem<ECAP>& sm, const uint64_t* __restrict__ rp,
                                          const uint32_t* __restrict__ ci, uint64_t n, uint64_t nnz,
                                          uint32_t m, unsigned long long* __restrict__ B, uint64_t Wp,
                                          uint32_t* __restrict__ colsum, uint32_t* __restrict__ err,
                                          uint64_t blk) {
  static_assert(ECAP % T == 0, "whole entries per thread");
  static_assert(ECAP * sizeof(uint32_t) >= PK_CW * PK_LD * sizeof(unsigned long long),
                "the entry buffer holds a window bitmap");
  constexpr int EPT = ECAP / T;  // entries per thread
  static_assert(PK_KR == 4, "a column's words are the four lanes of a quad");
  // two window bitmaps: XA, and XB over the entry buffer once the entries are
  // in registers -- window w is written out of one while window w + 1 is
  // ORed into the other, so a window costs one barrier
  unsigned long long* XA = sm.X;
  unsigned long long* XB = reinterpret_cast<unsigned long long*>(sm.s_e);
  uint32_t* s_e = sm.s_e;
  uint64_t* s_rp = sm.s_rp;
  const int tid = threadIdx.x;
  const uint64_t r0 = blk * PK_ROWS;
  const int nr = (int)(r0 < n ? min<uint64_t>(PK_ROWS, n - r0) : 0);
  uint32_t bad = 0;
  if (nr == 0) {
    if (tid == 0) s_rp[0] = 0;
  } else {
    // the tile's rows r0 .. r0 + nr - 1 check row_ptr[r] <= row_ptr[r + 1], so
    // the tiles together check every row
    for (int t = tid; t <= nr; t += T) {
      const uint64_t v = rp[r0 + t];
      s_rp[t] = min(v, nnz);
      if (t < nr && rp[r0 + t + 1] < v) bad |= 1u;
    }
  }
  __syncthreads();
  const uint64_t e0 = s_rp[0];
  const uint64_t e1 = max(e0, s_rp[nr]);
  const uint32_t nwin = (m + PK_CW - 1) / PK_CW;
  // XA starts clear; each window's write-out clears what it read
  for (int i = tid; i < PK_CW * PK_LD; i += T) XA[i] = 0ull;
  const int wi = tid & (PK_KR - 1), cs = tid / PK_KR;  // write-out: word wi of columns cs, cs + 256, ..
  for (uint64_t ea = e0; ea < e1 || (ea == e0 && e0 == e1); ea += ECAP) {
    const uint64_t eb = min<uint64_t>(e1, ea + ECAP);
    const int ne = (int)(eb - ea);
    const bool first = ea == e0, last = eb == e1;
    __syncthreads();  // previous chunk fully consumed
    for (int base = 0; base < ne; base += T * PK_UNROLL) {
      uint32_t v[PK_UNROLL];
#pragma unroll
      for (int u = 0; u < PK_UNROLL; ++u) {
        const int k = base + u * T + tid;
        v[u] = k < ne ? ci[ea + k] : 0u;
      }
#pragma unroll
      for (int u = 0; u < PK_UNROLL; ++u) {
        const int k = base + u * T + tid;
        if (k < ne) {
          if (v[u] >= m) bad |= 2u;
          s_e[k] = v[u] < m ? (v[u] << PK_RBITS) : 0xffffffffu;
        }
      }
    }
    __syncthreads();
    for (int r = tid; r < nr; r += T) {
      const uint64_t a = max(s_rp[r], ea), b = max(a, min(s_rp[r + 1], eb));
      uint64_t e = a;
      for (; e + 4 <= b; e += 4) {  // four independent LDS round trips at a time
        const uint32_t x0 = s_e[e - ea], x1 = s_e[e - ea + 1], x2 = s_e[e - ea + 2],
                       x3 = s_e[e - ea + 3];
        s_e[e - ea] = x0 | (uint32_t)r;
        s_e[e - ea + 1] = x1 | (uint32_t)r;
        s_e[e - ea + 2] = x2 | (uint32_t)r;
        s_e[e - ea + 3] = x3 | (uint32_t)r;
      }
      for (; e < b; ++e) s_e[e - ea] |= (uint32_t)r;
    }
    __syncthreads();  // rows filled in before the entries are read
    uint32_t xe[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int k = u * T + tid;
      xe[u] = k < ne ? s_e[k] : 0xffffffffu;
    }
    __syncthreads();  // every entry is in registers: the entry buffer becomes XB
    for (int i = tid; i < PK_CW * PK_LD; i += T) XB[i] = 0ull;
    if (nwin) pack_or_window(xe, XA, 0, min<uint32_t>(PK_CW, m));
    __syncthreads();
    for (uint32_t win = 0; win < nwin; ++win) {
      unsigned long long* Xc = (win & 1) ? XB : XA;
      unsigned long long* Xn = (win & 1) ? XA : XB;
      const uint32_t c0 = win * PK_CW;
      const uint32_t cw = min<uint32_t>(PK_CW, m - c0);
      for (uint32_t c = cs; c < cw; c += T / PK_KR) {
        unsigned long long v = Xc[c * PK_LD + wi];
        Xc[c * PK_LD + wi] = 0ull;  // clear for a later window as it is written out
        unsigned long long* dst = B + (uint64_t)(c0 + c) * Wp + blk * PK_KR + wi;
        // a later chunk of the tile adds to what the earlier ones wrote (this
        // same thread wrote it)
        if (!first) v |= *dst;
        *dst = v;
        if (last) {
          // the column's four words are in the four lanes of a quad (all
          // active together): sum their popcounts with DPP quad permutes
          int pc = __popcll(v);
          pc += __builtin_amdgcn_mov_dpp(pc, 0xb1, 0xf, 0xf, false);  // quad_perm 1,0,3,2
          pc += __builtin_amdgcn_mov_dpp(pc, 0x4e, 0xf, 0xf, false);  // quad_perm 2,3,0,1
          if (wi == 0 && pc) atomicAdd(colsum + c0 + c, (uint32_t)pc);
        }
      }
      if (win + 1 < nwin) pack_or_window(xe, Xn, c0 + PK_CW, min<uint32_t>(PK_CW, m - c0 - PK_CW));
      __syncthreads();
    }
    if (e0 == e1) break;
  }
  if (bad) atomicOr(err, bad);
}

// One database: nnz = row_ptr[n] is read here, so the host needs no read-back
// before the launch.  Flags row_ptr[0] != 0 (8) and a NULL col_idx with
// nnz > 0 (4, nothing is packed).
__global__ __launch_bounds__(PK_T) __attribute__((amdgpu_waves_per_eu(8))) void k_pack_tiled(
    const uint64_t* __restrict__ rp, const uint32_t* __restrict__ ci, uint64_t n, uint32_t m,
    unsigned long long* __restrict__ B, uint64_t Wp, uint32_t* __restrict__ colsum,
    uint32_t* __restrict__ err) {
  __shared__ PackSmem<PK_ECAP> sm;
  const uint64_t nnz = rp[n];
  if (ci == nullptr && nnz > 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(err, 4u);
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && rp[0] != 0) atomicOr(err, 8u);
  pack_tile<PK_ECAP, PK_T>(sm, rp, ci, n, nnz, m, B, Wp, colsum, err, xcd_tile(blockIdx.x, gridDim.x));
}

// Batched construction, part 1 -- one workgroup per database: read nnz =
// row_ptr[n] into the job (and into hnnz, host memory the host reads to pick
// each database's pack), set err to the flags row_ptr[0] != 0 (8) and NULL
// col_idx with nnz > 0 (4), and zero the column sums.  The pack checks the rows.
__global__ __launch_bounds__(kThreads) void k_build_multi_pre(PackJob* __restrict__ jobs,
                                                              uint32_t* __restrict__ err,
                                                              uint64_t* __restrict__ hnnz) {
  PackJob& j = jobs[blockIdx.x];
  const uint64_t n = j.n;
  if (threadIdx.x == 0) {
    const uint64_t nnz = j.rp[n];
    uint32_t bad = 0;
    j.nnz = nnz;
    hnnz[blockIdx.x] = nnz;
    if (j.rp[0] != 0) bad |= 8u;
    if (nnz > 0 && j.ci == nullptr) bad |= 4u;
    err[blockIdx.x] = bad;
  }
  for (uint32_t c = threadIdx.x; c < j.m; c += kThreads) j.colsum[c] = 0u;
}

// Batched construction, part 2 -- the 256-row tiles of a list of databases in
// one grid: block b belongs to list entry e with kstart[e] <= b < kstart[e + 1],
// database kjob[e].
template <int ECAP, int T>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(8))) void k_pack_tiled_multi(const PackJob* __restrict__ jobs,
                                                           const uint32_t* __restrict__ kjob,
                                                           uint32_t nk,
                                                           const uint64_t* __restrict__ kstart,
                                                           uint32_t* __restrict__ err) {
  __shared__ PackSmem<ECAP> sm;
  const uint64_t b = xcd_tile(blockIdx.x, gridDim.x);
  uint32_t lo = 0, hi = nk;  // kstart[lo] <= b < kstart[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (kstart[mid] <= b) lo = mid; else hi = mid;
  }
  const uint32_t jd = kjob[lo];
  const PackJob j = jobs[jd];
  pack_tile<ECAP, T>(sm, j.rp, j.ci, j.n, j.nnz, j.m, reinterpret_cast<unsigned long long*>(j.B),
                     j.Wp, j.colsum, err + jd, b - kstart[lo]);
}

// Support of each single item: popcount of its column, one workgroup per column.
__global__ __launch_bounds__(kThreads) void k_colsum(const uint64_t* __restrict__ B, uint64_t Wp,
                                                     uint32_t m, uint32_t* __restrict__ out) {
  __shared__ uint32_t s_part[kThreads / 64];
  for (uint64_t j = blockIdx.x; j < m; j += gridDim.x) {
    const uint64_t* col = B + j * Wp;
    uint32_t c = 0;
    for (uint64_t w = threadIdx.x; w < Wp; w += kThreads) c += __popcll(col[w]);
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
      for (int k = 0; k < kThreads / 64; ++k) t += s_part[k];
      out[j] += t;  // one workgroup per column: adds to the (zeroed or running) sums
    }
    __syncthreads();
  }
}

template <class T>
__global__ void k_fill(T* __restrict__ p, T v, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

uint32_t grid_for(uint64_t work, uint32_t per_block = kThreads, uint32_t cap = 65536) {
  uint64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

// ---------------------------------------------------------------- prefix sums
// Three-phase exclusive scan: each workgroup scans 1024 values (4 per thread),
// the per-workgroup totals are scanned recursively, and offsets are added back.

constexpr int kScanPer = 4;
constexpr int kScanBlock = kThreads * kScanPer;

struct InU64 {
  const uint64_t* p;
  __device__ uint64_t operator()(uint64_t i) const { return p[i]; }
};
struct InU32 {
  const uint32_t* p;
  __device__ uint64_t operator()(uint64_t i) const { return p[i]; }
};

__device__ inline uint64_t block_exclusive_scan(uint64_t v, uint64_t* s_wave, uint64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t inc = v;
  for (int off = 1; off < 64; off <<= 1) {
    uint64_t y = __shfl_up(inc, off);
    if (lane >= off) inc += y;
  }
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  uint64_t base = 0, tot = 0;
  for (int k = 0; k < kThreads / 64; ++k) {
    if (k < wave) base += s_wave[k];
    tot += s_wave[k];
  }
  *total = tot;
  return base + inc - v;
}

template <class In>
__global__ __launch_bounds__(kThreads) void k_scan_local(In in, uint64_t* __restrict__ out,
                                                         uint64_t n, uint64_t* __restrict__ sums) {
  __shared__ uint64_t s_wave[kThreads / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)threadIdx.x * kScanPer;
  uint64_t v[kScanPer];
  uint64_t t = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = (base + k < n) ? in(base + k) : 0;
    t += v[k];
  }
  uint64_t total;
  uint64_t ex = block_exclusive_scan(t, s_wave, &total);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void k_scan_add(uint64_t* __restrict__ out, uint64_t n,
                                                       const uint64_t* __restrict__ offs) {
  const uint64_t add = offs[blockIdx.x];
  const uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
  for (int k = threadIdx.x; k < kScanBlock; k += kThreads) {
    if (base + k < n) out[base + k] += add;
  }
}

__global__ void k_scan_total(uint64_t* __restrict__ out, uint64_t n, const uint64_t* __restrict__ s) {
  // out[n] = scanned offset of the last block + its total
  if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = s[0];
}

template <class In>
void scan_impl(In in, uint64_t* out, uint64_t n, uint64_t* tmp, hipStream_t s) {
  if (n == 0) {
    k_fill<uint64_t><<<1, 64, 0, s>>>(out, 0ull, 1);
    BM_LAUNCH_CHECK();
    return;
  }
  const uint64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb > 0x7fffffffull) fail(BM_ERR_UNSUPPORTED, "scan of %llu elements", (unsigned long long)n);
  uint64_t* sums = tmp;           // nb + 1 entries
  uint64_t* rest = tmp + nb + 1;  // recursion scratch
  k_scan_local<<<(uint32_t)nb, kThreads, 0, s>>>(in, out, n, sums);
  BM_LAUNCH_CHECK();
  if (nb == 1) {
    // total of the single block sits in sums[0]
    k_scan_total<<<1, 64, 0, s>>>(out, n, sums);
    BM_LAUNCH_CHECK();
    return;
  }
  // scan the block totals in place into sums (exclusive, sums[nb] = grand total)
  uint64_t* soff = rest;               // nb + 1 entries
  uint64_t* rest2 = rest + nb + 1;
  scan_impl(InU64{sums}, soff, nb, rest2, s);
  k_scan_add<<<(uint32_t)nb, kThreads, 0, s>>>(out, n, soff);
  BM_LAUNCH_CHECK();
  k_scan_total<<<1, 64, 0, s>>>(out, n, soff + nb);
  BM_LAUNCH_CHECK();
}

// Single-workgroup looped scan of up to 8 arrays at once (one workgroup per
// array): for the per-node arrays of a level step, one launch replaces three
// launches per array.
constexpr int kSingleThreads = 1024;
constexpr int kSingleChunk = kSingleThreads * kScanPer;

__global__ __launch_bounds__(kSingleThreads) void k_scan_single(ScanMulti sm, uint64_t n) {
  __shared__ uint64_t s_wave[kSingleThreads / 64];
  const int a = blockIdx.x;
  const void* in = sm.in[a];
  const bool is64 = sm.is64[a] != 0;
  uint64_t* out = sm.out[a];
  if (a == 0 && sm.tot)
    for (uint32_t j = threadIdx.x; j < sm.nextra; j += kSingleThreads)
      sm.tot[gridDim.x + j] = sm.extra[j];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t base = 0;
  for (uint64_t c0 = 0; c0 < n; c0 += kSingleChunk) {
    const uint64_t i0 = c0 + (uint64_t)threadIdx.x * kScanPer;
    uint64_t v[kScanPer];
    uint64_t t = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const uint64_t i = i0 + k;
      uint64_t x = 0;
      if (i < n) {
        x = is64 ? static_cast<const uint64_t*>(in)[i] : static_cast<const uint32_t*>(in)[i];
      }
      v[k] = x;
      t += v[k];
    }
    uint64_t inc = t;
    for (int off = 1; off < 64; off <<= 1) {
      uint64_t y = __shfl_up(inc, off);
      if (lane >= off) inc += y;
    }
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    uint64_t wb = 0, tot = 0;
    for (int k = 0; k < kSingleThreads / 64; ++k) {
      if (k < wave) wb += s_wave[k];
      tot += s_wave[k];
    }
    uint64_t ex = base + wb + inc - t;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      if (i0 + k < n) out[i0 + k] = ex;
      ex += v[k];
    }
    base += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[n] = base;
    if (sm.tot) sm.tot[a] = base;
  }
}

// Element i of array a of a ScanMulti: 64-bit or 32-bit.
__device__ __forceinline__ uint64_t scan_elem(const ScanMulti& sm, int a, uint64_t i) {
  if (sm.is64[a]) return static_cast<const uint64_t*>(sm.in[a])[i];
  return static_cast<const uint32_t*>(sm.in[a])[i];
}

// Three-launch scan of up to 8 arrays of any length (grid.y = array): tiles of
// kTileScan elements are scanned locally and their totals kept (1), one
// workgroup per array scans the totals (2, k_scan_single), and each tile adds
// its offset and the totals are written (3).
constexpr int kTilePer = 8;
constexpr int kTileScan = kThreads * kTilePer;

__global__ __launch_bounds__(kThreads) void k_scan_tiles(ScanMulti sm, uint64_t n,
                                                          uint64_t* __restrict__ sums, uint32_t nb) {
  __shared__ uint64_t s_wave[kThreads / 64];
  const int a = blockIdx.y;
  const uint32_t b = blockIdx.x;
  const uint64_t i0 = (uint64_t)b * kTileScan + (uint64_t)threadIdx.x * kTilePer;
  uint64_t* out = sm.out[a];
  // a thread's 8 elements are contiguous: 16-byte accesses when the arrays
  // are 16-byte aligned and the 8 are all inside
  const bool vec = i0 + kTilePer <= n &&
                   ((reinterpret_cast<uintptr_t>(sm.in[a]) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
  uint64_t v[kTilePer];
  uint64_t t = 0;
  if (vec) {
    if (sm.is64[a]) {
      const uint4* q = reinterpret_cast<const uint4*>(static_cast<const uint64_t*>(sm.in[a]) + i0);
#pragma unroll
      for (int k = 0; k < kTilePer / 2; ++k) {
        const uint4 x = q[k];
        v[2 * k] = (uint64_t)x.x | ((uint64_t)x.y << 32);
        v[2 * k + 1] = (uint64_t)x.z | ((uint64_t)x.w << 32);
      }
    } else {
      const uint4* q = reinterpret_cast<const uint4*>(static_cast<const uint32_t*>(sm.in[a]) + i0);
#pragma unroll
      for (int k = 0; k < kTilePer / 4; ++k) {
        const uint4 x = q[k];
        v[4 * k] = x.x;
        v[4 * k + 1] = x.y;
        v[4 * k + 2] = x.z;
        v[4 * k + 3] = x.w;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < kTilePer; ++k) v[k] = i0 + k < n ? scan_elem(sm, a, i0 + k) : 0;
  }
#pragma unroll
  for (int k = 0; k < kTilePer; ++k) t += v[k];
  uint64_t total;
  uint64_t ex = block_exclusive_scan(t, s_wave, &total);
  if (vec) {
    uint4* q = reinterpret_cast<uint4*>(out + i0);
#pragma unroll
    for (int k = 0; k < kTilePer / 2; ++k) {
      const uint64_t e0 = ex, e1 = ex + v[2 * k];
      ex = e1 + v[2 * k + 1];
      q[k] = make_uint4((uint32_t)e0, (uint32_t)(e0 >> 32), (uint32_t)e1, (uint32_t)(e1 >> 32));
    }
  } else {
#pragma unroll
    for (int k = 0; k < kTilePer; ++k) {
      if (i0 + k < n) out[i0 + k] = ex;
      ex += v[k];
    }
  }
  if (threadIdx.x == 0) sums[(uint64_t)a * nb + b] = total;
}

__global__ __launch_bounds__(kThreads) void k_scan_tiles_add(ScanMulti sm, uint64_t n,
                                                              const uint64_t* __restrict__ soff,
                                                              uint32_t nb) {
  const int a = blockIdx.y;
  const uint32_t b = blockIdx.x;
  const uint64_t* so = soff + (uint64_t)a * (nb + 1);
  const uint64_t add = so[b];
  uint64_t* out = sm.out[a];
  const uint64_t base = (uint64_t)b * kTileScan;
  if (add)
    for (int k = threadIdx.x; k < kTileScan; k += kThreads)
      if (base + k < n) out[base + k] += add;
  if (b == 0 && threadIdx.x == 0) {
    out[n] = so[nb];
    if (sm.tot) sm.tot[a] = so[nb];
  }
  if (a == 0 && b == 0 && sm.tot)
    for (uint32_t j = threadIdx.x; j < sm.nextra; j += kThreads) sm.tot[gridDim.y + j] = sm.extra[j];
}

__global__ void k_gather_u64(GatherU64 g, int count, uint64_t* __restrict__ dst) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = *g.src[i];
}

}  // namespace

void launch_gather_u64(const GatherU64& g, int count, uint64_t* dst, hipStream_t s) {
  k_gather_u64<<<1, 64, 0, s>>>(g, count, dst);
  BM_LAUNCH_CHECK();
}

size_t scan_tmp_words(uint64_t n) {
  if (n == 0) return 2;
  uint64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb == 1) return 2;
  return 2 * (nb + 1) + scan_tmp_words(nb);
}

size_t scan_tiles_tmp_words(int count, uint64_t n) {
  const uint64_t nb = (n + kTileScan - 1) / kTileScan;
  return (size_t)count * (2 * nb + 1);
}

bool scan_multi_tiles(const ScanMulti& sm, int count, uint64_t n, uint64_t* tmp, hipStream_t s) {
  const uint64_t nb = (n + kTileScan - 1) / kTileScan;
  if (n == 0 || nb > kSingleMaxN || count < 1 || count > 8) return false;
  uint64_t* sums = tmp;
  uint64_t* soff = tmp + (size_t)count * nb;
  k_scan_tiles<<<dim3((uint32_t)nb, count), kThreads, 0, s>>>(sm, n, sums, (uint32_t)nb);
  BM_LAUNCH_CHECK();
  ScanMulti st{};
  for (int a = 0; a < count; ++a) {
    st.in[a] = sums + (size_t)a * nb;
    st.is64[a] = 1;
    st.out[a] = soff + (size_t)a * (nb + 1);
  }
  k_scan_single<<<count, kSingleThreads, 0, s>>>(st, nb);
  BM_LAUNCH_CHECK();
  k_scan_tiles_add<<<dim3((uint32_t)nb, count), kThreads, 0, s>>>(sm, n, soff, (uint32_t)nb);
  BM_LAUNCH_CHECK();
  return true;
}

bool scan_multi_single(const ScanMulti& sm, int count, uint64_t n, hipStream_t s) {
  if (n > kSingleMaxN || count < 1 || count > 8) return false;
  k_scan_single<<<count, kSingleThreads, 0, s>>>(sm, n);
  BM_LAUNCH_CHECK();
  return true;
}

void scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* tmp, hipStream_t s) {
  scan_impl(InU64{in}, out, n, tmp, s);
}
void scan_u32_to_u64(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* tmp, hipStream_t s) {
  scan_impl(InU32{in}, out, n, tmp, s);
}

void launch_validate(const uint64_t* rp, const uint32_t* ci, uint64_t n, uint64_t nnz, uint32_t m,
                     uint32_t* err, hipStream_t s) {
  if (n > 0) {
    k_validate_rows<<<grid_for(n, kThreads, 4096), kThreads, 0, s>>>(rp, n, err);
    BM_LAUNCH_CHECK();
  }
  if (nnz > 0) {
    k_validate_cols<<<grid_for(nnz, kThreads, 8192), kThreads, 0, s>>>(ci, nnz, m, err);
    BM_LAUNCH_CHECK();
  }
}

void launch_pack(const uint64_t* rp, const uint32_t* ci, uint64_t n, uint64_t* B, uint64_t Wp,
                 hipStream_t s) {
  if (n == 0) return;
  const uint64_t nb = (n + kThreads - 1) / kThreads;
  if (nb > 0x7fffffffull) fail(BM_ERR_UNSUPPORTED, "too many rows");
  k_pack<<<(uint32_t)nb, kThreads, 0, s>>>(rp, ci, n, reinterpret_cast<unsigned long long*>(B), Wp);
  BM_LAUNCH_CHECK();
}

bool launch_pack_tiled(const uint64_t* rp, const uint32_t* ci, uint64_t n, uint32_t m, uint64_t* B,
                       uint64_t Wp, uint32_t* colsum, uint32_t* err, hipStream_t s) {
  if (!pack_tiled_ok(m, Wp)) return false;
  dim3 grid((uint32_t)(Wp / PK_KR));
  k_pack_tiled<<<grid, PK_T, 0, s>>>(rp, ci, n, m, reinterpret_cast<unsigned long long*>(B), Wp,
                                     colsum, err);
  BM_LAUNCH_CHECK();
  return true;
}

bool pack_tiled_ok(uint32_t m, uint64_t Wp) {
  const uint64_t windows = (m + PK_CW - 1) / PK_CW;
  return m > 0 && windows <= 32 && Wp % PK_KR == 0 && ((uint64_t)m << PK_RBITS) < 0xffffffffull;
}

void launch_build_multi_pre(PackJob* jobs, uint32_t njobs, uint32_t* err, uint64_t* hnnz,
                            hipStream_t s) {
  if (njobs == 0) return;
  k_build_multi_pre<<<njobs, kThreads, 0, s>>>(jobs, err, hnnz);
  BM_LAUNCH_CHECK();
}

bool pack_sparse(uint64_t nnz, uint64_t n) { return nnz <= n * (uint64_t)PK_SPARSE_ROW; }

void launch_pack_multi(const PackJob* jobs, bool sparse, const uint32_t* kjob, uint32_t nk,
                       const uint64_t* kstart, uint64_t blocks, uint32_t* err, hipStream_t s) {
  if (nk == 0 || blocks == 0) return;
  if (blocks > 0x7fffffffull) fail(BM_ERR_UNSUPPORTED, "batch too large for one build");
  if (sparse)
    k_pack_tiled_multi<PK_ECAP_SPARSE, PK_T_SPARSE>
        <<<(uint32_t)blocks, PK_T_SPARSE, 0, s>>>(jobs, kjob, nk, kstart, err);
  else
    k_pack_tiled_multi<PK_ECAP, PK_T><<<(uint32_t)blocks, PK_T, 0, s>>>(jobs, kjob, nk, kstart, err);
  BM_LAUNCH_CHECK();
}

uint64_t pack_blocks(uint64_t Wp) { return Wp / PK_KR; }

void launch_colsum(const uint64_t* B, uint64_t Wp, uint32_t m, uint32_t* colsum, hipStream_t s) {
  if (m == 0) return;
  k_colsum<<<(uint32_t)std::min<uint64_t>(m, 1u << 20), kThreads, 0, s>>>(B, Wp, m, colsum);
  BM_LAUNCH_CHECK();
}

void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
  if (n == 0) return;
  k_fill<uint32_t><<<grid_for(n, kThreads, 16384), kThreads, 0, s>>>(p, v, n);
  BM_LAUNCH_CHECK();
}

__global__ void k_zero_segs(ZeroSegs z) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  uint64_t base = 0;
  for (int k = 0; k < z.count; ++k) {
    const uint64_t end = base + z.n[k];
    for (; i < end; i += stride) z.p[k][i - base] = 0u;
    base = end;
  }
}

void launch_zero_segs(const ZeroSegs& z, hipStream_t s) {
  if (z.count < 0 || z.count > kZeroSegs) fail(BM_ERR_DEVICE, "too many zero segments");
  uint64_t total = 0;
  ZeroSegs c{};
  for (int k = 0; k < z.count; ++k)
    if (z.p[k] && z.n[k]) {
      c.p[c.count] = z.p[k];
      c.n[c.count] = z.n[k];
      total += z.n[k];
      ++c.count;
    }
  if (total == 0) return;
  k_zero_segs<<<grid_for(total, kThreads, 16384), kThreads, 0, s>>>(c);
  BM_LAUNCH_CHECK();
}

void launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s) {
  if (n == 0) return;
  k_fill<uint64_t><<<grid_for(n, kThreads, 16384), kThreads, 0, s>>>(p, v, n);
  BM_LAUNCH_CHECK();
}

}  // namespace bm
