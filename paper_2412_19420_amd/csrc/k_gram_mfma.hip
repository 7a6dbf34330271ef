// Pair supports of a prefix class as a masked Gram matrix on MFMA.
//
// For a class with prefix P (tidset t(P), the AND of P's columns) and children
// c_0..c_{q-1}, the support of P + {c_i, c_l} is
//     S = sum_rows t(P)[r] & M[r, c_i] & M[r, c_l]
// (Eq. 2, with the prefix's columns ANDed in first as the method prescribes
// for longer itemsets).  Over all pairs this is the Gram matrix
// X^T X of the 0/1 matrix X[r, i] = t(P)[r] & M[r, c_i]; for the root class
// (P empty) it is the pair-support matrix A^T A itself.  With 0/1 entries the
// products are exact, in FP4 x FP4 -> FP32 (the default form) or in
// int8 x int8 -> int32.
//
// Kernel shape (gfx950, wave64):
//   * one workgroup = 4 waves computes a 128 x 128 output tile of the class's
//     triangle over a range of words; waves own 64 x 64 sub-tiles, each a 2 x 2
//     grid of 32 x 32 MFMA accumulators;
//   * FP4 form: the bit panels of both tile sides go straight from global
//     memory into a double-buffered, XOR-swizzled LDS stage (gram_fp4.hpp),
//     and the prefix mask is ANDed into the A operands from a mask row;
//   * int8 form: the panels are staged through registers into LDS, with the
//     prefix mask ANDed into the A side on the way, the next stage's loads
//     issued before the current stage's MFMAs;
//   * bits become MFMA operands in registers right before each MFMA (FP4
//     bit planes, or for int8 the lane's 32-bit half-word v yields four dwords
//     (v >> d) & 0x01010101, one transaction bit per byte).  A and B fragments
//     use the identical bit -> (lane, element) map, so every transaction meets
//     itself in the K sum (t & a_i & b_l needs the mask once; a diagonal tile
//     reads its masked A panel for both sides);
//   * the accumulated tile is added atomically into the class's triangle
//     (integer adds: exact and independent of the order of word splits).
#include "gram_fp4.hpp"

namespace bm {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));


__device__ __forceinline__ v4i expand4(uint32_t v, int d0) {
  v4i r;
  r[0] = (int)((v >> (d0 + 0)) & 0x01010101u);
  r[1] = (int)((v >> (d0 + 1)) & 0x01010101u);
  r[2] = (int)((v >> (d0 + 2)) & 0x01010101u);
  r[3] = (int)((v >> (d0 + 3)) & 0x01010101u);
  return r;
}

// The int8 form.  NB = 32x32 accumulator blocks per wave side: NB = 2 gives
// 64x64 per wave and a 128x128 workgroup tile of 4 waves.
// KW = words per LDS stage (a divisor of GRAM_KW, so stages tile every task).
template <int NB, int KW>
__device__ __forceinline__ void gram_tiles_i8(const ClassArgs& a, uint32_t* sA, uint32_t* sB) {
  static_assert(GRAM_KW % KW == 0, "stages must tile the task word ranges");
  constexpr int T = 64 * NB;         // workgroup tile (children per side)
  constexpr int LDW = 2 * KW + 1;    // dwords per column row in LDS (odd stride: conflict-free reads)
  constexpr int SUBS = KW / 2;       // 16-byte slots per column per stage
  constexpr int CSL = 256 / SUBS;    // columns staged per pass of the workgroup
  constexpr int NS = T / CSL;        // column slots per side staged by each thread
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int sub = tid % SUBS;   // 16-byte slot of a column's stage slice
  const int cslot = tid / SUBS; // column slot 0..CSL-1
  const uint64_t ntasks = *a.ntasks;

  for (uint64_t t = blockIdx.x; t < ntasks; t += gridDim.x) {
    const Task task = a.tasks[t];
    const ClassDesc cd = a.cls[task.cls];
    const DbInfo db = class_view(cd, a.dbs, a.views);
    const uint64_t Wp = db.Wp;
    const uint32_t q = cd.q;
    const uint32_t I0 = (uint32_t)task.bi * T, L0 = (uint32_t)task.bl * T;
    const bool diag = task.bi == task.bl;
    // the wave's first A row block and first B column block (32-wide blocks
    // of the tile)
    const int rb0 = NB * wr;
    const int cb0 = NB * wc;
    const int nload = diag ? NS : 2 * NS;

    // base pointers of the columns this thread stages (nullptr = zero column)
    const uint64_t* colp[2 * NS];
#pragma unroll
    for (int p = 0; p < 2 * NS; ++p) {
      const uint32_t idx = ((p >= NS) ? L0 : I0) + cslot + CSL * (p % NS);
      colp[p] = nullptr;
      if (p < nload && idx < q) {
        const uint32_t item = a.child_item[cd.child0 + idx];
        const uint32_t col = class_col(cd, db, idx, item);
        colp[p] = db.B + (uint64_t)col * Wp + 2 * sub;
      }
    }
    const uint32_t* pre = a.pre_cols + cd.pre_off;
    const uint32_t pre_len = cd.proj ? 0u : cd.pre_len;  // a view has the prefix applied

    uint4 reg[2 * NS];
    uint64_t m0 = ~0ull, m1 = ~0ull;
    auto load_stage = [&](uint32_t w) {
      m0 = ~0ull;
      m1 = ~0ull;
      for (uint32_t j = 0; j < pre_len; ++j) {
        const uint4 x = *reinterpret_cast<const uint4*>(db.B + (uint64_t)pre[j] * Wp + w + 2 * sub);
        m0 &= (uint64_t)x.x | ((uint64_t)x.y << 32);
        m1 &= (uint64_t)x.z | ((uint64_t)x.w << 32);
      }
#pragma unroll
      for (int p = 0; p < 2 * NS; ++p) {
        if (colp[p]) reg[p] = *reinterpret_cast<const uint4*>(colp[p] + w);
        else reg[p] = make_uint4(0, 0, 0, 0);
      }
    };

    v16i acc[NB][NB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

    const uint32_t nst = (task.w1 - task.w0) / KW;
    if (nst) load_stage(task.w0);
    for (uint32_t s = 0; s < nst; ++s) {
      __syncthreads();  // previous stage (or task) finished reading LDS
#pragma unroll
      for (int p = 0; p < 2 * NS; ++p) {
        if (p < nload) {
          uint32_t* dst = ((p >= NS) ? sB : sA) + (cslot + CSL * (p % NS)) * LDW + 4 * sub;
          uint4 v = reg[p];
          if (pre_len && p < NS) {  // the prefix mask on the A side only: t & a_i & b_l
            v.x &= (uint32_t)m0;
            v.y &= (uint32_t)(m0 >> 32);
            v.z &= (uint32_t)m1;
            v.w &= (uint32_t)(m1 >> 32);
          }
          dst[0] = v.x;
          dst[1] = v.y;
          dst[2] = v.z;
          dst[3] = v.w;
        }
      }
      __syncthreads();
      if (s + 1 < nst) load_stage(task.w0 + (s + 1) * KW);

      const uint32_t* pa = sA + (rb0 * 32 + (lane & 31)) * LDW + (lane >> 5);
      const uint32_t* pb = (diag ? sA : sB) + (cb0 * 32 + (lane & 31)) * LDW + (lane >> 5);
      {
#pragma unroll
        for (int w = 0; w < KW; ++w) {
          uint32_t va[NB], vb[NB];
#pragma unroll
          for (int i = 0; i < NB; ++i) {
            va[i] = pa[i * 32 * LDW + 2 * w];
            vb[i] = pb[i * 32 * LDW + 2 * w];
          }
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            v4i A[NB], B[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
              A[i] = expand4(va[i], 4 * e);
              B[i] = expand4(vb[i], 4 * e);
            }
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
              for (int j = 0; j < NB; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[i], B[j], acc[i][j], 0, 0, 0);
          }
        }
      }
    }

    // 32x32 accumulator layout: lane holds column (lane & 31); register r holds
    // row 8*(r/4) + 4*(lane/32) + (r%4).
    uint32_t* tri = a.tri + cd.tri_off;
#pragma unroll
    for (int rb = 0; rb < NB; ++rb)
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const uint32_t gi = I0 + (rb0 + rb) * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const uint32_t gl = L0 + (cb0 + cb) * 32 + (lane & 31);
          const uint32_t v = (uint32_t)acc[rb][cb][r];
          if (gi < gl && gl < q && v) atomicAdd(tri + tri_index(gi, gl, q), v);
        }
  }
}

// FP4 form, staged directly into LDS (gram_fp4.hpp).  On a diagonal tile (A
// and B the same panel) the 10 useful 32 x 32 blocks of the 4 x 4 are shared
// out so that no wave does more than three products or builds more than
// three operand rows:
//   MODE 1 (waves on the diagonal): its two blocks against themselves,
//     (0,0), (0,1), (1,1), with B taken from A's operands;
//   MODE 2 (the two off-diagonal waves): one A block against B blocks 0, 1;
// MODE 0 is an off-diagonal tile: A blocks 0, 1 against B blocks 0, 1.
template <int MODE>
__device__ __forceinline__ void fp4_group(const uint4 (&a)[2], const uint4 (&b)[2], const uint4& m,
                                          v16f (&acc)[2][2]) {
  constexpr int NA = MODE == 2 ? 1 : 2;  // A row blocks this wave builds
  constexpr bool BSAME = MODE == 1;      // B operands are A's
  uint32_t va[2][4], vb[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    va[i][0] = a[i].x & m.x;
    va[i][1] = a[i].y & m.y;
    va[i][2] = a[i].z & m.z;
    va[i][3] = a[i].w & m.w;
    vb[i][0] = b[i].x;
    vb[i][1] = b[i].y;
    vb[i][2] = b[i].z;
    vb[i][3] = b[i].w;
  }
#pragma unroll
  for (int pl = 0; pl < 4; ++pl) {
    v8i A[2], B[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        A[i][j] = i < NA ? (int)fp4_plane(va[i][j], pl) : 0;
        B[i][j] = BSAME ? 0 : (int)fp4_plane(vb[i][j], pl);
      }
      A[i][4] = A[i][5] = A[i][6] = A[i][7] = 0;
      B[i][4] = B[i][5] = B[i][6] = B[i][7] = 0;
    }
    const int sc = fp4_plane_scale(pl);
    if constexpr (MODE == 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = fp4_mfma(A[i], B[j], acc[i][j], sc);
    } else if constexpr (MODE == 1) {
      acc[0][0] = fp4_mfma(A[0], A[0], acc[0][0], sc);
      acc[0][1] = fp4_mfma(A[0], A[1], acc[0][1], sc);
      acc[1][1] = fp4_mfma(A[1], A[1], acc[1][1], sc);
    } else {
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[0][j] = fp4_mfma(A[0], B[j], acc[0][j], sc);
    }
  }
}

// One stage of one wave: four word groups, the next group's operands read
// from LDS before the current group's MFMAs.  ra / rb: the wave's first A and
// B rows at this lane (row l % 32 of the first block), in chunks; mk: the
// stage's mask row, read only with MASK.  Launches whose classes have no
// prefix (the root classes) use a kernel without the mask reads and ANDs: 5%
// faster on the dense root, and the masked code paths in the same kernel would
// cost the unmasked ones registers.
template <int MODE, bool MASK>
__device__ __forceinline__ void fp4_stage(const uint4* ra, const uint4* rb, const uint4* mk,
                                          int lane, v16f (&acc)[2][2]) {
  constexpr int NA = MODE == 2 ? 1 : 2;
  constexpr bool BSAME = MODE == 1;
  const int kh = lane >> 5, sw = lane & 7;
  uint4 a[2], b[2], m;
  auto read = [&](int g, uint4 (&xa)[2], uint4 (&xb)[2], uint4& xm) {
    const int c = 2 * g + kh;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      xa[i] = i < NA ? ra[i * 32 * DCH + (c ^ sw)] : make_uint4(0, 0, 0, 0);
      xb[i] = BSAME ? make_uint4(0, 0, 0, 0) : rb[i * 32 * DCH + (c ^ sw)];
    }
    xm = MASK ? mk[c] : make_uint4(~0u, ~0u, ~0u, ~0u);
  };
  read(0, a, b, m);
#pragma unroll
  for (int g = 0; g < DKW / 4; ++g) {
    uint4 na[2], nb[2], nm;
    if (g + 1 < DKW / 4) read(g + 1, na, nb, nm);
    fp4_group<MODE>(a, b, m, acc);
    if (g + 1 < DKW / 4) {
      a[0] = na[0];
      a[1] = na[1];
      b[0] = nb[0];
      b[1] = nb[1];
      m = nm;
    }
  }
}

// A task's constants for the stage steps.
struct Fp4Task {
  const uint64_t* src[8];  // this lane's chunk of each load instruction, at word 0
  const uint32_t* pre;     // prefix columns
  const uint64_t* pcol;    // this thread's first prefix column (j = tid / 8) at chunk tid % 8
  uint32_t pre_len;
  uint64_t Wp;
  const uint64_t* B;
  uint32_t w0, nst;
  int mode, nload, rb0, cb0;
  bool diag;
};

// The wave's load instructions for the stage at word w: r < 4 stage A-panel
// rows 32 w + 8 r .. +7 (wave w), r >= 4 the same rows of the B panel.
__device__ __forceinline__ void fp4_issue(const Fp4Task& k, uint32_t w, uint4* buf, int wave) {
  constexpr int T = GRAM_TILE;
  uint4* dst = buf + (size_t)(32 * wave) * DCH;
#pragma unroll
  for (int r = 0; r < 8; ++r)
    if (r < k.nload)
      __builtin_amdgcn_global_load_lds(k.src[r] + w,
                                       dst + ((r >= 4) ? T * DCH : 0) + 8 * (r & 3) * DCH, 16, 0,
                                       0);
}

// Stage s of a task: wait for its loads (the barrier), start stage s + 1's
// loads into the other buffer, multiply stage s.
template <bool MASK>
__device__ __forceinline__ void fp4_stage_step(const Fp4Task& k, uint32_t s, const uint4* cur,
                                               uint4* nxt, uint4* smask, int tid,
                                               v16f (&acc)[2][2]) {
  constexpr int T = GRAM_TILE;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // LDS destinations in SGPRs
  const uint32_t pj0 = (uint32_t)tid >> 3, pch = (uint32_t)tid & 7;
  __syncthreads();  // stage s is in LDS (each wave waited for its loads); stage s - 1 is done
  const bool more = s + 1 < k.nst;
  const uint32_t wn = k.w0 + (s + 1) * DKW;
  // this thread's first prefix chunk of stage s + 1, issued before the stage
  // loads so that waiting for it does not wait for them
  const bool pre_thread = MASK && more && pj0 < k.pre_len;
  uint4 pm = make_uint4(~0u, ~0u, ~0u, ~0u);
  if (pre_thread) pm = load_global16(k.pcol + wn);
  if (more) fp4_issue(k, wn, nxt, wave);
  if (MASK && tid < DCH) smask[((s + 2) % 3) * DCH + tid] = make_uint4(~0u, ~0u, ~0u, ~0u);

  const uint4* ra = cur + (size_t)(k.rb0 * 32 + (lane & 31)) * DCH;
  const uint4* rb = cur + (size_t)((k.diag ? 0 : T) + k.cb0 * 32 + (lane & 31)) * DCH;
  const uint4* mk = smask + (s % 3) * DCH;
  // a wave in its MFMA section outranks the other workgroup's waves that are
  // issuing loads
  __builtin_amdgcn_s_setprio(3);
  if (k.mode == 0) fp4_stage<0, MASK>(ra, rb, mk, lane, acc);
  else if (k.mode == 1) fp4_stage<1, MASK>(ra, rb, mk, lane, acc);
  else fp4_stage<2, MASK>(ra, rb, mk, lane, acc);
  __builtin_amdgcn_s_setprio(0);

  if (pre_thread)
    fp4_mask_and(pm, k.B, k.Wp, k.pre, k.pre_len, pj0, pch, wn, smask + ((s + 1) % 3) * DCH, 32);
}

template <bool MASK>
__device__ __forceinline__ void gram_tiles_fp4(const ClassArgs& a, uint4* sb0, uint4* sb1,
                                               uint4* smask) {
  constexpr int T = GRAM_TILE;  // 128 children per tile side
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const uint64_t ntasks = *a.ntasks;
  const SkRange rg = sk_range<true>(a.tcost, ntasks);  // two workgroups per CU

  for (uint64_t t = rg.i; t < ntasks; ++t) {
    const uint64_t base = a.tcost[t];
    if (base >= rg.u1) break;
    const Task task = a.tasks[t];
    uint32_t s_lo, s_hi;
    if (!sk_stages(base, a.tcost[t + 1], rg,
                   task.bi == task.bl ? GRAM_COST_DIAG : GRAM_COST_OFF, s_lo, s_hi))
      continue;
    const ClassDesc cd = a.cls[task.cls];
    const DbInfo db = class_view(cd, a.dbs, a.views);
    const uint32_t q = cd.q;
    const uint32_t I0 = (uint32_t)task.bi * T, L0 = (uint32_t)task.bl * T;
    Fp4Task k;
    k.diag = task.bi == task.bl;
    // the wave's first A row block and first B column block (32-wide blocks
    // of the tile)
    k.mode = k.diag ? (wr == wc ? 1 : 2) : 0;
    k.rb0 = k.mode == 2 ? wr : 2 * wr;
    k.cb0 = k.mode == 2 ? 2 : 2 * wc;
    k.nload = k.diag ? 4 : 8;
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
    // row 32 w + 8 (r % 4) + L / 8.  Children beyond q load column q - 1:
    // their rows and columns of the tile are never written out.  (class_col
    // for the eight children, with the loads of each step issued together.)
    uint32_t col[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint32_t idx = ((r >= 4) ? L0 : I0) + 32 * wave + 8 * (r & 3) + (lane >> 3);
      col[r] = idx < q ? idx : q - 1;
    }
    if (!cd.proj) {
#pragma unroll
      for (int r = 0; r < 8; ++r) col[r] = a.child_item[cd.child0 + col[r]];
      if (db.f1) {
#pragma unroll
        for (int r = 0; r < 8; ++r) col[r] = load_global_u32(db.f1 + col[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint32_t row = 32 * wave + 8 * (r & 3) + (lane >> 3);
      const uint32_t chunk = (uint32_t)((lane & 7) ^ (row & 7));
      k.src[r] = db.B + (uint64_t)col[r] * k.Wp + 2 * chunk;
    }

    v16f acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0;

    __syncthreads();  // the previous task's last stage has finished reading LDS
    if (k.nst) {
      fp4_issue(k, k.w0, sb0, wave);
      if (MASK && tid < DCH) {  // stage 0's mask in full; stage 1's row starts at all ones
        smask[tid] = fp4_mask_full(k.B, k.Wp, k.pre, k.pre_len, k.w0, (uint32_t)tid);
        smask[DCH + tid] = make_uint4(~0u, ~0u, ~0u, ~0u);
      }
    }
    // even stages read sb0 and load into sb1, odd stages the other way round
    for (uint32_t s = 0; s < k.nst; s += 2) {
      fp4_stage_step<MASK>(k, s, sb0, sb1, smask, tid, acc);
      if (s + 1 < k.nst) fp4_stage_step<MASK>(k, s + 1, sb1, sb0, smask, tid, acc);
    }

    // 32x32 accumulator layout: lane holds column (lane & 31); register r holds
    // row 8*(r/4) + 4*(lane/32) + (r%4).
    uint32_t* tri = a.tri + cd.tri_off;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const uint32_t gi = I0 + (k.rb0 + rb) * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const uint32_t gl = L0 + (k.cb0 + cb) * 32 + (lane & 31);
          const uint32_t v = __float2uint_rn(acc[rb][cb][r]);  // exact integer counts
          if (gi < gl && gl < q && v) atomicAdd(tri + tri_index(gi, gl, q), v);
        }
  }
}

// Two workgroups per CU (two waves per SIMD; each workgroup holds 64 KiB of
// LDS stages): the register budget is capped at 256 so the three stage
// variants do not push the kernel to one wave.
template <bool F4, bool MASK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_gram_mfma(ClassArgs a) {
  if constexpr (F4) {
    // two stages of both panels (2 x 32 KiB) and three mask rows
    __shared__ uint4 sb0[2 * GRAM_TILE * DCH];
    __shared__ uint4 sb1[2 * GRAM_TILE * DCH];
    __shared__ uint4 smask[3 * DCH];
    gram_tiles_fp4<MASK>(a, sb0, sb1, smask);
  } else {
    constexpr int KW = 16;
    __shared__ uint32_t sA[GRAM_TILE * (2 * KW + 1)];
    __shared__ uint32_t sB[GRAM_TILE * (2 * KW + 1)];
    gram_tiles_i8<2, KW>(a, sA, sB);
  }
}

}  // namespace

void launch_gram_mfma(const ClassArgs& a, uint32_t grid, bool fp4, bool masked, hipStream_t s) {
  if (grid == 0) return;
  if (fp4 && masked) k_gram_mfma<true, true><<<grid, 256, 0, s>>>(a);
  else if (fp4) k_gram_mfma<true, false><<<grid, 256, 0, s>>>(a);
  else k_gram_mfma<false, true><<<grid, 256, 0, s>>>(a);
  BM_LAUNCH_CHECK();
}


}  // namespace bm
