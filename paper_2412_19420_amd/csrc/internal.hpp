// Internal declarations of libbm: device data layout, task records, launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "bm.h"

namespace bm {

// ------------------------------------------------------------------ errors

struct Error {
  bm_status status;
  std::string msg;
};

[[noreturn]] void fail(bm_status st, const char* fmt, ...);
void set_last_error(const std::string& s);

#define BM_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      ::bm::fail(BM_ERR_DEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),       \
                 __FILE__, __LINE__);                                                         \
  } while (0)

#define BM_LAUNCH_CHECK() BM_HIP(hipGetLastError())

// ------------------------------------------------------------------ memory

void* dalloc(size_t bytes, hipStream_t s);  // throws Error{BM_ERR_OOM}
void dfree(void* p, hipStream_t s) noexcept;

// Owning device buffer, returned to the pool on destruction.
template <class T>
class DBuf {
 public:
  DBuf() = default;
  DBuf(size_t n, hipStream_t s) : s_(s) { reset(n, s); }
  ~DBuf() { release(); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p_(o.p_), n_(o.n_), s_(o.s_) { o.p_ = nullptr; o.n_ = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p_ = o.p_; n_ = o.n_; s_ = o.s_;
      o.p_ = nullptr; o.n_ = 0;
    }
    return *this;
  }
  void reset(size_t n, hipStream_t s) {
    release();
    s_ = s;
    n_ = n;
    p_ = n ? static_cast<T*>(dalloc(n * sizeof(T), s)) : nullptr;
  }
  void release() {
    if (p_) dfree(p_, s_);
    p_ = nullptr;
    n_ = 0;
  }
  T* get() const { return p_; }
  size_t size() const { return n_; }
  size_t bytes() const { return n_ * sizeof(T); }

 private:
  T* p_ = nullptr;
  size_t n_ = 0;
  hipStream_t s_ = nullptr;
};

// ------------------------------------------------------------------ layout

// Words per bitset column: ceil(n/64) rounded up to a multiple of 64 words, so
// every 16-word MFMA stage and 64-word split boundary stays inside the column;
// padding bits are zero.
inline uint64_t padded_words(uint64_t n_tx) {
  uint64_t w = (n_tx + 63) / 64;
  uint64_t wp = (w + 63) / 64 * 64;
  return wp ? wp : 64;
}

// One prefix class of a level step: a frequent prefix P and its q frequent
// one-item extensions ("children").  The class's candidates are the q(q-1)/2
// pairs of children (i < l); candidate (i, l) is P + child_i + child_l.
struct ClassDesc {
  uint64_t tri_off;   // offset of this class's q(q-1)/2 supports in the step's buffer
  uint32_t child0;    // index of the first child in the child-item array
  uint32_t q;         // number of children
  uint32_t pre_off;   // offset of P's columns in the prefix-column array
  uint32_t pre_len;   // |P| (0 for the root class of single items)
  uint32_t db;        // database the class belongs to
  uint32_t proj;      // 0, or 1 + index of the class's projected column block (see ProjWork)
};

// One database of a (batched) mining call, as the kernels see it.
struct DbInfo {
  const uint64_t* B;       // bitset matrix, column-major, Wp words per column
  uint64_t Wp;             // padded words per column
  uint64_t W;              // words holding n bits
  uint64_t n;              // transactions
  const uint32_t* f1;      // frequent-item index -> column id (nullptr: identity)
  const uint32_t* colsum;  // single-item supports
  uint32_t minsup;
  uint32_t m;
};

// The database view a class kernel reads: the class's database, or, for a
// projected class, its children's columns re-packed over the transactions that
// hold the prefix (views[cd.proj - 1]: B = those columns in child order, n = the
// prefix's support, W/Wp its words; the prefix is already applied).
// Loads through the global address space.  A pointer read from memory (a
// column base in a DbInfo, a task's prefix list) is generic, and a load
// through it compiles to a flat load, which also counts against the LDS
// counter: every LDS wait of a kernel that stages through LDS would then
// wait for its global loads in flight too.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 load_global16(const void* p) {
  const u32x4 v = *(const __attribute__((address_space(1))) u32x4*)p;
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint64_t load_global_u64(const uint64_t* p) {
  return *(const __attribute__((address_space(1))) uint64_t*)p;
}
__device__ __forceinline__ uint32_t load_global_u32(const uint32_t* p) {
  return *(const __attribute__((address_space(1))) uint32_t*)p;
}

// The AND of a class's prefix columns at words w, w + 1 (m0, m1 ANDed in
// place; 16-byte loads at an even word).  The first PREFIX_REG columns come
// from bases set up once per class (pc[j], nullptr beyond the prefix), so
// their loads need no index load first and go out together with the other
// loads of the step; further columns (prefixes longer than PREFIX_REG) are
// read through the prefix list.
constexpr int PREFIX_REG = 4;
__device__ __forceinline__ void prefix_and(const uint64_t* const (&pc)[PREFIX_REG],
                                           const uint64_t* B, uint64_t Wp, const uint32_t* pre,
                                           uint32_t pre_len, uint32_t w, uint64_t& m0,
                                           uint64_t& m1) {
  uint4 x[PREFIX_REG];
#pragma unroll
  for (int j = 0; j < PREFIX_REG; ++j)
    x[j] = pc[j] ? load_global16(pc[j] + w) : make_uint4(~0u, ~0u, ~0u, ~0u);
  for (uint32_t j = PREFIX_REG; j < pre_len; ++j) {
    const uint4 y = load_global16(B + (uint64_t)pre[j] * Wp + w);
    m0 &= (uint64_t)y.x | ((uint64_t)y.y << 32);
    m1 &= (uint64_t)y.z | ((uint64_t)y.w << 32);
  }
#pragma unroll
  for (int j = 0; j < PREFIX_REG; ++j) {
    m0 &= (uint64_t)x[j].x | ((uint64_t)x[j].y << 32);
    m1 &= (uint64_t)x[j].z | ((uint64_t)x[j].w << 32);
  }
}

__host__ __device__ inline DbInfo class_view(const ClassDesc& cd, const DbInfo* dbs,
                                             const DbInfo* views) {
  return cd.proj ? views[cd.proj - 1] : dbs[cd.db];
}
// Column of child idx (item = its frequent-item index) in a class's view.
__host__ __device__ inline uint32_t class_col(const ClassDesc& cd, const DbInfo& v, uint32_t idx,
                                              uint32_t item) {
  return cd.proj ? idx : (v.f1 ? v.f1[item] : item);
}

// One projected class of a level step.  row_off: the supports of the step's
// earlier projected prefixes summed, i.e. where this class's transactions
// start when all the step's prefixes' transactions are counted in class order.
struct ProjWork {
  uint64_t row_off;
  uint32_t cls;  // class index in the step
  uint32_t pad;
};

// One unit of kernel work: a block pair (bi <= bl) of a class's q x q triangle
// over a word range.  Block size is the kernel's (128 for MFMA, 16 for AND+popcount).
struct Task {
  uint32_t cls;
  uint16_t bi, bl;
  uint32_t w0, w1;
};

// Upper-triangle index of pair (i, l), i < l, in a q x q triangle.
__host__ __device__ inline uint64_t tri_index(uint64_t i, uint64_t l, uint64_t q) {
  return i * (2 * q - i - 1) / 2 + (l - i - 1);
}

constexpr int GRAM_TILE = 128;  // MFMA kernel output tile (children per block)
constexpr int GRAM_TILE_BIG = 256;  // big-class MFMA kernel output tile
constexpr int GRAM_KW = 16;     // MFMA kernel words per LDS stage
constexpr int AP_BLOCK = 16;    // AND+popcount kernel children per block
constexpr int GRAM_SMALL_TILE = 32;  // mid-size-class MFMA kernel children per block
constexpr int GRAM_SMALL_KW = 32;    // its task word ranges are multiples of this
constexpr int TINY_Q = 8;       // classes up to this many children use the register kernel
constexpr int SUBSET_Q = 8;     // largest class mined whole by subset counting (2^8 counters)
constexpr int SUBSET_LAT = 6;   // children walked in registers per subset-counting pass
// Default limit: classes of 7-8 children need 2-4 passes, which measured
// slower than evaluating them level by level (dense 1M x 4,096: 1.79 against
// 1.64 ms per mine call; T40-style: 4.77 against 4.45 ms).
constexpr int SUBSET_DEFAULT_Q = 6;

// Arguments shared by the class kernels.  They loop over the task list from
// the launched workgroups (persistent, grid-stride); the task count is read
// from device memory so the host need not know it.
struct ClassArgs {
  const DbInfo* dbs;
  const uint32_t* child_item; // item of each child (indexed by class child0 + i)
  const ClassDesc* cls;
  const uint32_t* pre_cols;   // prefix column ids
  const DbInfo* views;        // projected classes' views (ClassDesc::proj)
  const Task* tasks;
  const uint64_t* ntasks;     // device-side task count
  uint32_t* tri;              // per-class triangles of supports (accumulated atomically)
  // FP4 Gram kernels: exclusive prefix sums of the tasks' costs (ntasks + 1
  // entries; launch_task_costs then a scan), for the balanced split of the
  // launch's stages over its workgroups
  const uint64_t* tcost = nullptr;
};

// ------------------------------------------------------------------ launchers

// Device timing of launches (hipEvents on the call's stream).
class KTimer {
 public:
  // Times the launch kinds whose bit is set in `kinds` (none: off).
  KTimer(uint32_t kinds, hipStream_t s);
  ~KTimer();
  void begin(int kind);
  void end(double bytes = 0, double ops = 0);
  // Work counts of the last recorded launch, when they are known only afterwards.
  void set_last(double bytes, double ops);
  // Adds accumulated times to stats (synchronises on the recorded events).
  void collect(bm_stats* st);
  bool on() const { return on_; }

 private:
  struct Rec {
    int kind;
    hipEvent_t a, b;
    double bytes, ops;
  };
  bool on_;
  uint32_t kinds_;
  bool skip_ = false;
  hipStream_t s_;
  int dev_ = 0;
  std::vector<Rec> recs_;
  int cur_kind_ = -1;
  hipEvent_t cur_a_ = nullptr;
};

// build
void launch_validate(const uint64_t* rp, const uint32_t* ci, uint64_t n, uint64_t nnz, uint32_t m,
                     uint32_t* err, hipStream_t s);
void launch_pack(const uint64_t* rp, const uint32_t* ci, uint64_t n, uint64_t* B, uint64_t Wp,
                 hipStream_t s);
// Adds each column's popcount to colsum[j] (zero it first for plain sums).
void launch_colsum(const uint64_t* B, uint64_t Wp, uint32_t m, uint32_t* colsum, hipStream_t s);
// Tiled build of M and its column sums in one pass, with the CSR checks
// (colsum and err must be zeroed; err gets the flags of launch_build_multi;
// nnz is read on the device); returns false when the shape needs the atomic
// path (m > 16384).
bool launch_pack_tiled(const uint64_t* rp, const uint32_t* ci, uint64_t n, uint32_t m, uint64_t* B,
                       uint64_t Wp, uint32_t* colsum, uint32_t* err, hipStream_t s);
// One database of a batched matrix construction (nnz is filled on the device).
struct PackJob {
  const uint64_t* rp;
  const uint32_t* ci;
  uint64_t n;
  uint32_t m;
  uint32_t pad;
  uint64_t* B;
  uint64_t Wp;
  uint32_t* colsum;
  uint64_t nnz;
};
// Whether the tiled construction handles m items (else the atomic one is used).
bool pack_tiled_ok(uint32_t m, uint64_t Wp);
uint64_t pack_blocks(uint64_t Wp);
// Compute units of the current device (cached per device).
int cu_count();

// Batched build, step 1: one workgroup per database reads nnz into the job
// and into hnnz (host memory), sets err[j] to the flags row_ptr[0] != 0 (8)
// and NULL col_idx with nnz > 0 (4), and zeroes the column sums.
void launch_build_multi_pre(PackJob* jobs, uint32_t njobs, uint32_t* err, uint64_t* hnnz,
                            hipStream_t s);
// Whether a database of nnz elements over n rows takes the sparse pack (small
// LDS chunks, two workgroups per CU).
bool pack_sparse(uint64_t nnz, uint64_t n);
// Step 2, per kind: the tiles of databases kjob[0..nk) (tile offsets kstart,
// nk + 1 entries; `blocks` tiles in all) packed in one grid; err[j] gets the
// row flags (1 decreasing row_ptr, 2 item id >= m).
void launch_pack_multi(const PackJob* jobs, bool sparse, const uint32_t* kjob, uint32_t nk,
                       const uint64_t* kstart, uint64_t blocks, uint32_t* err, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
void launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s);
// Zero up to kZeroSegs arrays of 32-bit words in one launch (segments with
// p == nullptr or n == 0 are skipped).
constexpr int kZeroSegs = 16;
struct ZeroSegs {
  uint32_t* p[kZeroSegs];
  uint64_t n[kZeroSegs];
  int count;
};
void launch_zero_segs(const ZeroSegs& z, hipStream_t s);

// scans: out[0..n] exclusive, out[n] = total.  tmp sized by scan_tmp_words(n).
size_t scan_tmp_words(uint64_t n);
void scan_u64(const uint64_t* in, uint64_t* out, uint64_t n, uint64_t* tmp, hipStream_t s);
void scan_u32_to_u64(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* tmp, hipStream_t s);
// Up to 8 arrays of the same length n <= kSingleMaxN scanned by one launch
// (false when n is too large: use the per-array scans).
struct ScanMulti {
  const void* in[8];
  uint32_t is64[8];
  uint64_t* out[8];
  uint64_t* tot;        // if set: tot[j] = total of array j, then tot[count + e] = extra[e]
  const uint64_t* extra;
  uint32_t nextra;
};
constexpr uint64_t kSingleMaxN = 1ull << 18;
// dst[i] = *src[i] for i < count (count <= 32); dst may be mapped host memory.
struct GatherU64 {
  const uint64_t* src[32];
};
void launch_gather_u64(const GatherU64& g, int count, uint64_t* dst, hipStream_t s);
bool scan_multi_single(const ScanMulti& sm, int count, uint64_t n, hipStream_t s);
// The same (tot and extra included) for long arrays in three launches;
// tmp holds scan_tiles_tmp_words(count, n) words.  False if n is 0 or too long.
size_t scan_tiles_tmp_words(int count, uint64_t n);
bool scan_multi_tiles(const ScanMulti& sm, int count, uint64_t n, uint64_t* tmp, hipStream_t s);

// class kernels
// fp4: the scaled e2m1 MFMA form (64 transactions per instruction, exact FP32
// integer sums for counts up to 2^24); else int8 x int8 -> int32.
// masked: some class of the launch has a prefix (FP4 form: without, a lighter
// kernel that never reads a mask; every class must then have none)
void launch_gram_mfma(const ClassArgs& a, uint32_t grid, bool fp4, bool masked, hipStream_t s);
// Same contraction with 256 x 256 tiles (tasks index 256-wide blocks).
void launch_gram_mfma_big(const ClassArgs& a, uint32_t grid, bool masked, hipStream_t s);  // FP4 only
// Cost of each FP4 Gram task: its stages (GRAM_KW words each) times w_diag on
// a diagonal block pair, else w_off; 0 for t in [*ntasks, ub).
void launch_task_costs(const Task* tasks, const uint64_t* ntasks, uint64_t ub, uint32_t w_off,
                       uint32_t w_diag, uint32_t* cost, hipStream_t s);
// Per-stage costs of the two FP4 Gram kernels, off and on the diagonal: the
// most MFMAs any one wave issues per word group (128-wide tiles 16 / 12;
// 256-wide tiles 32 / 32, their diagonal waves computing whole grids).
constexpr uint32_t GRAM_COST_OFF = 4, GRAM_COST_DIAG = 3;
constexpr uint32_t GRAM_BIG_COST_OFF = 1, GRAM_BIG_COST_DIAG = 1;
// Mid-size classes: one wave per 32 x 32 block pair (tasks index 32-wide blocks).
void launch_gram_small(const ClassArgs& a, uint32_t grid, bool fp4, hipStream_t s);
// Longest word range one MFMA task may cover in the fp4 form (2^24 transactions).
constexpr uint32_t GRAM_FP4_MAX_WORDS = 1u << 18;
void launch_andpop(const ClassArgs& a, uint32_t chunk_words, uint32_t grid, hipStream_t s);
void launch_andpop_reg(const ClassArgs& a, uint32_t grid, hipStream_t s);

}  // namespace bm
