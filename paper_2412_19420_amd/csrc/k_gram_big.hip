// Pair supports of big prefix classes (at least mfma_big_children children)
// as masked Gram tiles on MFMA: the contraction of k_gram_mfma.hip (Eq. 2 over
// all pairs of the class's children, FP4 bit planes, exact FP32 sums) on
// 256 x 256 tiles.
//
// Kernel shape (gfx950, wave64): one workgroup of 8 waves per CU computes a
// 256 x 256 block pair over a range of words; wave (r, c), r < 4, c < 2, owns
// rows 64 r .. 64 r + 63 and columns 128 c .. 128 c + 127, a 2 x 4 grid of
// 32 x 32 accumulators (128 registers; two waves per SIMD).  Per word group a
// wave builds 6 operand rows for 8 MFMAs (the 128-tile kernel: 4 for 4), a
// stage of 16 words carries 128 MFMAs per wave between two barriers (64 in
// the 128-tile kernel), and the panels of a stage (512 rows, 64 KiB) feed 8
// waves: half the load bytes per MFMA.  Staging, swizzle and prefix masks are
// the 128-tile kernel's (gram_fp4.hpp); two stages take 128 KiB of LDS.
//
// A diagonal block pair has one panel (256 columns, loaded once and read for
// both sides).  Its waves of columns 0 .. 127 and rows 128 .. 255 lie wholly
// below the diagonal and only stage loads; every other wave computes its full
// 2 x 4 grid, and the write-out keeps the pairs above the diagonal.
#include "gram_fp4.hpp"

namespace bm {

namespace {

constexpr int BT = GRAM_TILE_BIG;       // 256 children per tile side
constexpr int BROWS = 2 * BT;           // staged rows per buffer (A panel, then B panel)
constexpr int BWAVES = 8;
constexpr int BTHREADS = 64 * BWAVES;   // 512
constexpr int BLOADS = BROWS / 8 / BWAVES;  // load instructions per wave per stage (8)

// One word group: 2 A row blocks against 4 B column blocks, four planes.
template <bool MASK>
__device__ __forceinline__ void big_group(const uint4 (&a)[2], const uint4 (&b)[4], const uint4& m,
                                          v16f (&acc)[2][4]) {
  uint32_t va[2][4], vb[4][4];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    va[i][0] = MASK ? a[i].x & m.x : a[i].x;
    va[i][1] = MASK ? a[i].y & m.y : a[i].y;
    va[i][2] = MASK ? a[i].z & m.z : a[i].z;
    va[i][3] = MASK ? a[i].w & m.w : a[i].w;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    vb[i][0] = b[i].x;
    vb[i][1] = b[i].y;
    vb[i][2] = b[i].z;
    vb[i][3] = b[i].w;
  }
#pragma unroll
  for (int pl = 0; pl < 4; ++pl) {
    v8i A[2], B[4];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j) A[i][j] = (int)fp4_plane(va[i][j], pl);
      A[i][4] = A[i][5] = A[i][6] = A[i][7] = 0;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j) B[i][j] = (int)fp4_plane(vb[i][j], pl);
      B[i][4] = B[i][5] = B[i][6] = B[i][7] = 0;
    }
    const int sc = fp4_plane_scale(pl);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = fp4_mfma(A[i], B[j], acc[i][j], sc);
  }
}

// One stage of one wave: four word groups, the next group's operands read
// from LDS before the current group's MFMAs.  ra / rb: the wave's first A and
// B rows at this lane, in chunks; mk: the stage's mask row (read with MASK).
template <bool MASK>
__device__ __forceinline__ void big_stage(const uint4* ra, const uint4* rb, const uint4* mk,
                                          int lane, v16f (&acc)[2][4]) {
  const int kh = lane >> 5, sw = lane & 7;
  uint4 a[2], b[4], m;
  auto read = [&](int g, uint4 (&xa)[2], uint4 (&xb)[4], uint4& xm) {
    const int c = 2 * g + kh;
#pragma unroll
    for (int i = 0; i < 2; ++i) xa[i] = ra[i * 32 * DCH + (c ^ sw)];
#pragma unroll
    for (int i = 0; i < 4; ++i) xb[i] = rb[i * 32 * DCH + (c ^ sw)];
    xm = MASK ? mk[c] : make_uint4(~0u, ~0u, ~0u, ~0u);
  };
  read(0, a, b, m);
#pragma unroll
  for (int g = 0; g < DKW / 4; ++g) {
    uint4 na[2], nb[4], nm;
    if (g + 1 < DKW / 4) read(g + 1, na, nb, nm);
    big_group<MASK>(a, b, m, acc);
    if (g + 1 < DKW / 4) {
      a[0] = na[0];
      a[1] = na[1];
#pragma unroll
      for (int i = 0; i < 4; ++i) b[i] = nb[i];
      m = nm;
    }
  }
}

struct BigTask {
  uint32_t col[BLOADS];  // column of this lane's row in each load instruction
  uint32_t choff;        // word offset of this lane's chunk (the same in every row)
  const uint32_t* pre;   // prefix columns
  const uint64_t* pcol;  // this thread's first prefix column (j = tid / 8) at chunk tid % 8
  uint32_t pre_len;
  uint64_t Wp;
  const uint64_t* B;
  uint32_t w0, nst;
  int nload, rb0, cb0;
  bool diag, idle;  // idle: the wave's block lies below the diagonal or past the last child
};

// The wave's load instructions for the stage at word w: r < 4 stage A-panel
// rows 32 w + 8 r .. +7 (wave w), r >= 4 the same rows of the B panel.
__device__ __forceinline__ void big_issue(const BigTask& k, uint32_t w, uint4* buf, int wave) {
  uint4* dst = buf + (size_t)(32 * wave) * DCH;
#pragma unroll
  for (int r = 0; r < BLOADS; ++r)
    if (r < k.nload)
      __builtin_amdgcn_global_load_lds(k.B + (uint64_t)k.col[r] * k.Wp + k.choff + w,
                                       dst + ((r >= 4) ? BT * DCH : 0) + 8 * (r & 3) * DCH, 16, 0,
                                       0);
}

template <bool MASK>
__device__ __forceinline__ void big_stage_step(const BigTask& k, uint32_t s, const uint4* cur,
                                               uint4* nxt, uint4* smask, int tid,
                                               v16f (&acc)[2][4]) {
  const int lane = tid & 63, wave = tid >> 6;
  const uint32_t pj0 = (uint32_t)tid >> 3, pch = (uint32_t)tid & 7;
  __syncthreads();  // stage s is in LDS (each wave waited for its loads); stage s - 1 is done
  const bool more = s + 1 < k.nst;
  const uint32_t wn = k.w0 + (s + 1) * DKW;
  const bool pre_thread = MASK && more && pj0 < k.pre_len;
  uint4 pm = make_uint4(~0u, ~0u, ~0u, ~0u);
  if (pre_thread) pm = load_global16(k.pcol + wn);
  if (more) big_issue(k, wn, nxt, wave);
  if (MASK && tid < DCH) smask[((s + 2) % 3) * DCH + tid] = make_uint4(~0u, ~0u, ~0u, ~0u);

  if (!k.idle) {
    const uint4* ra = cur + (size_t)(k.rb0 * 32 + (lane & 31)) * DCH;
    const uint4* rb = cur + (size_t)((k.diag ? 0 : BT) + k.cb0 * 32 + (lane & 31)) * DCH;
    // a wave in its MFMA section outranks the waves issuing loads
    __builtin_amdgcn_s_setprio(3);
    big_stage<MASK>(ra, rb, smask + (s % 3) * DCH, lane, acc);
    __builtin_amdgcn_s_setprio(0);
  }

  if (pre_thread)
    fp4_mask_and(pm, k.B, k.Wp, k.pre, k.pre_len, pj0, pch, wn, smask + ((s + 1) % 3) * DCH,
                 BTHREADS / 8);
}

template <bool MASK>
__device__ __forceinline__ void gram_tiles_big(const ClassArgs& a, uint4* sb0, uint4* sb1,
                                               uint4* smask) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;  // rows 64 wr .., columns 128 wc ..
  const uint64_t ntasks = *a.ntasks;
  const SkRange rg = sk_range<false>(a.tcost, ntasks);  // one workgroup per CU

  for (uint64_t t = rg.i; t < ntasks; ++t) {
    const uint64_t base = a.tcost[t];
    if (base >= rg.u1) break;
    const Task task = a.tasks[t];
    uint32_t s_lo, s_hi;
    if (!sk_stages(base, a.tcost[t + 1], rg,
                   task.bi == task.bl ? GRAM_BIG_COST_DIAG : GRAM_BIG_COST_OFF, s_lo, s_hi))
      continue;
    const ClassDesc cd = a.cls[task.cls];
    const DbInfo db = class_view(cd, a.dbs, a.views);
    const uint32_t q = cd.q;
    const uint32_t I0 = (uint32_t)task.bi * BT, L0 = (uint32_t)task.bl * BT;
    BigTask k;
    k.diag = task.bi == task.bl;
    k.rb0 = 2 * wr;  // 32-wide row blocks of the panel
    k.cb0 = 4 * wc;  // 32-wide column blocks
    k.idle = (k.diag && wc == 0 && wr >= 2) || I0 + 32u * k.rb0 >= q || L0 + 32u * k.cb0 >= q;
    k.nload = k.diag ? BLOADS / 2 : BLOADS;
    k.Wp = db.Wp;
    k.B = db.B;
    k.pre = a.pre_cols + cd.pre_off;
    k.pre_len = cd.proj ? 0u : cd.pre_len;  // a view has the prefix applied
    k.w0 = task.w0 + s_lo * DKW;
    k.nst = s_hi - s_lo;
    k.pcol = nullptr;
    if (MASK && (uint32_t)tid / 8 < k.pre_len)
      k.pcol = k.B + (uint64_t)k.pre[tid / 8] * k.Wp + 2 * (tid & 7);
    // Lane L of load instruction r fetches the chunk for slot L % 8 of panel
    // row 32 w + 8 (r % 4) + L / 8, i.e. chunk (L % 8) ^ (L / 8 % 8) of that
    // row's column.  Children beyond q load column q - 1: their rows and
    // columns of the tile are never written out.
#pragma unroll
    for (int r = 0; r < BLOADS; ++r) {
      const uint32_t idx = ((r >= 4) ? L0 : I0) + 32 * wave + 8 * (r & 3) + (lane >> 3);
      k.col[r] = idx < q ? idx : q - 1;
    }
    if (!cd.proj) {
#pragma unroll
      for (int r = 0; r < BLOADS; ++r) k.col[r] = a.child_item[cd.child0 + k.col[r]];
      if (db.f1) {
#pragma unroll
        for (int r = 0; r < BLOADS; ++r) k.col[r] = load_global_u32(db.f1 + k.col[r]);
      }
    }
    k.choff = 2 * (uint32_t)((lane & 7) ^ ((lane >> 3) & 7));

    v16f acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

    __syncthreads();  // the previous task's last stage has finished reading LDS
    if (k.nst) {
      big_issue(k, k.w0, sb0, wave);
      if (MASK && tid < DCH) {  // stage 0's mask in full; stage 1's row starts at all ones
        smask[tid] = fp4_mask_full(k.B, k.Wp, k.pre, k.pre_len, k.w0, (uint32_t)tid);
        smask[DCH + tid] = make_uint4(~0u, ~0u, ~0u, ~0u);
      }
    }
    // even stages read sb0 and load into sb1, odd stages the other way round
    for (uint32_t s = 0; s < k.nst; s += 2) {
      big_stage_step<MASK>(k, s, sb0, sb1, smask, tid, acc);
      if (s + 1 < k.nst) big_stage_step<MASK>(k, s + 1, sb1, sb0, smask, tid, acc);
    }
    if (k.idle) continue;

    // 32x32 accumulator layout: lane holds column (lane & 31); register r holds
    // row 8*(r/4) + 4*(lane/32) + (r%4).
    uint32_t* tri = a.tri + cd.tri_off;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const uint32_t gi = I0 + (k.rb0 + rb) * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const uint32_t gl = L0 + (k.cb0 + cb) * 32 + (lane & 31);
          const uint32_t v = __float2uint_rn(acc[rb][cb][r]);  // exact integer counts
          if (gi < gl && gl < q && v) atomicAdd(tri + tri_index(gi, gl, q), v);
        }
  }
}

// One workgroup per CU, two waves per SIMD (256 registers per lane).
template <bool MASK>
__global__ __launch_bounds__(BTHREADS) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_gram_mfma_big(ClassArgs a) {
  __shared__ uint4 sb0[BROWS * DCH];
  __shared__ uint4 sb1[BROWS * DCH];
  __shared__ uint4 smask[3 * DCH];
  gram_tiles_big<MASK>(a, sb0, sb1, smask);
}

}  // namespace

void launch_gram_mfma_big(const ClassArgs& a, uint32_t grid, bool masked, hipStream_t s) {
  if (grid == 0) return;
  if (masked) k_gram_mfma_big<true><<<grid, BTHREADS, 0, s>>>(a);
  else k_gram_mfma_big<false><<<grid, BTHREADS, 0, s>>>(a);
  BM_LAUNCH_CHECK();
}

}  // namespace bm
