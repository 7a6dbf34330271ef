/* bm.h -- Boolean-matrix frequent-itemset mining on MI355X (gfx950).
 *
 * C ABI of libbm.so.  The operations follow the method of "A Matrix Logic
 * Approach to Efficient Frequent Itemset Discovery in Large Data Sets"
 * (arXiv 2412.19420), Section III:
 *   - matrix construction (Eq. 1): the transaction list becomes the n x m
 *     Boolean matrix M, M[i,j] = 1 iff item j is in transaction i;
 *   - support calculation (Eq. 2): the joint support of items a and b is the
 *     number of rows where columns a and b are both 1; longer itemsets AND
 *     further columns one after another;
 *   - frequent-itemset extraction (Eq. 3): an itemset is frequent when its
 *     support passes the threshold.  This library takes the threshold as an
 *     absolute count `minsup` and reports X iff S(X) >= minsup; the paper's
 *     strict S(X) > theta is minsup = floor(theta) + 1.
 *
 * Conventions shared by every call
 *   Status     every call returns a bm_status; no C++ exception crosses the ABI.
 *              On failure `*out` (where present) is set to NULL, nothing leaks,
 *              and bm_last_error() holds a thread-local description.
 *   Pointers   "host or device" arguments may point to host memory or to device
 *              memory of the current HIP device; the library tells them apart
 *              with hipPointerGetAttributes.  Inputs are borrowed: the caller
 *              may free or reuse them as soon as the call returns.
 *   Streams    `stream` is a hipStream_t (NULL = the default stream).  All work
 *              of a call is issued on it and the call returns only once that
 *              work has completed.
 *   Ownership  handles (bm_db, bm_result, bm_model) belong to the library until
 *              the matching *_free call; *_free(NULL) is a no-op.
 *   Threads    distinct handles may be used from different host threads; one
 *              handle must not be used by two calls at once.
 *   Limits     n_tx < 2^31 (supports are counted in int32, exact); item ids are
 *              uint32 and must be < n_items.  Larger n_tx gives BM_ERR_UNSUPPORTED.
 *   Devices    a handle lives on the HIP device that was current when it was
 *              created; later calls on it must be made with that device current.
 */
#ifndef BM_H_
#define BM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BM_ABI_VERSION 2u
#define BM_MAX_LEVELS 64

typedef struct bm_db bm_db;
typedef struct bm_result bm_result;
typedef struct bm_model bm_model;
typedef struct bm_rules bm_rules;

typedef enum {
  BM_OK = 0,
  BM_ERR_INVALID_ARG = 1, /* NULL where a pointer is required, minsup == 0, bad option */
  BM_ERR_CSR = 2,         /* row_ptr[0] != 0, row_ptr not monotone, or an item id >= n_items */
  BM_ERR_OOM = 3,         /* a device or host allocation failed */
  BM_ERR_DEVICE = 4,      /* a HIP runtime call or kernel failed */
  BM_ERR_UNSUPPORTED = 5  /* size beyond the documented limits */
} bm_status;

/* Kernel classes timed in bm_stats (index into the per-kernel arrays). */
enum {
  BM_K_BUILD = 0,     /* CSR validation + packing of column bitsets */
  BM_K_COLSUM = 1,    /* column popcount: single-item supports */
  BM_K_GRAM_MFMA = 2, /* MFMA (masked) Gram matrix of a class, 128 x 128 tiles: pair supports
                       * (scaled FP4 operands by default, int8 with BM_FLAG_INT8_MFMA) */
  BM_K_ANDPOP = 3,    /* AND + popcount of a prefix class's columns, LDS-blocked (VALU) */
  BM_K_ANDPOP_REG = 4,/* AND + popcount of a small prefix class held in registers (VALU) */
  BM_K_LEVEL = 5,     /* candidate/level bookkeeping: thresholds, scans, compaction */
  BM_K_EMIT = 6,      /* canonical-order output (and the merge of depth-first output) */
  BM_K_DFS = 7,       /* persistent depth-first subtree kernel (small classes) */
  BM_K_SCHED = 8,     /* cost-model features, prediction and task ordering */
  BM_K_GRAM_MFMA_BIG = 9, /* as BM_K_GRAM_MFMA with 256 x 256 tiles (classes of at least
                           * mfma_big_children children; FP4 form only) */
  BM_K_GRAM_SMALL = 10,   /* MFMA Gram of mid-size classes, one wave per 32 x 32 block pair */
  BM_K_PROJECT = 11,      /* projected views of big deep classes: prefix row lists and the
                           * children's columns gathered over them */
  BM_K_COUNT = 12
};

/* Statistics of one mining call.  Kernel times are filled only when the call
 * ran with BM_FLAG_TIMING (hipEvents recorded around every launch on the call's
 * stream); `ops` counts algorithmic work: 2 n per candidate pair (one AND and
 * one add per transaction) for the Gram kernels, AND+popcount word operations
 * for the AND+popcount kernels; `bytes` counts
 * algorithmic bytes (see the library's design notes for each kernel). */
typedef struct {
  uint32_t max_len;                            /* longest frequent itemset */
  uint32_t n_frequent_items;                   /* frequent single items (m') */
  uint64_t candidates[BM_MAX_LEVELS + 1];      /* [k]: supports evaluated for length-k sets */
  uint64_t frequent[BM_MAX_LEVELS + 1];        /* [k]: frequent length-k sets */
  uint64_t candidates_total;                   /* sum over k >= 2 of candidates[k] */
  uint64_t frequent_total;
  uint64_t classes_mfma, classes_andpop;       /* prefix classes sent to MFMA / to AND+popcount */
  double kernel_ms[BM_K_COUNT];
  uint64_t kernel_launches[BM_K_COUNT];
  double kernel_bytes[BM_K_COUNT];
  double kernel_ops[BM_K_COUNT];
  double wall_ms;                              /* host wall time of the call */
  uint32_t host_syncs;                         /* device->host synchronisations */
  uint64_t dfs_tasks;                          /* subtree tasks run by the depth-first kernel */
  uint32_t mfma_form;                          /* 1: Gram kernels ran in FP4 (e2m1) form, 0: int8 */
} bm_stats;

/* Tuning and behaviour switches for bm_mine_ex / bm_mine_batch.  Zero fields
 * take the library default (or the autotuned value, see bm_autotune).  No option
 * changes the mined result. */
#define BM_FLAG_TIMING 1u      /* record per-kernel hipEvent times into bm_stats */
#define BM_FLAG_NO_MFMA 2u     /* send every class to the AND+popcount kernels (no MFMA) */
#define BM_FLAG_ALL_MFMA 4u    /* send every class with >= 2 children to the MFMA kernel */
#define BM_FLAG_GRAPH 8u       /* bm_model_train_ex: replay each training epoch as a hipGraph */
#define BM_FLAG_TRACE 16u      /* keep per-class features and subtree costs (bm_result_trace) */
#define BM_FLAG_SHUFFLE 32u    /* random subtree-task order (order-invariance tests) */
#define BM_FLAG_LEVELSYNC 64u  /* evaluate small classes level by level too (no depth-first kernel
                                * and no subset counting) */
#define BM_FLAG_FP4_MFMA 128u  /* Gram kernels on the block-scaled FP4 (e2m1) MFMA form (the
                                * default): each transaction bit sits in one e2m1 element of a
                                * bit plane, coded 0.5, 1 or 2 by plane, and the planes' E8M0
                                * scales (2, 1, 1/2, 1) make every product of two set bits
                                * exactly 1.0; FP32 sums are exact while a task's counts stay
                                * below 2^24, which the word-range cap of 2^18 words per task
                                * guarantees */
#define BM_FLAG_INT8_MFMA 256u /* Gram kernels on int8 x int8 -> int32 MFMA (overrides FP4) */
#define BM_FLAG_DFS_BLOCK_ONLY 512u /* every subtree task on the one-stack-per-workgroup kernel */
#define BM_FLAG_TIMING_MAIN 1024u   /* with BM_FLAG_TIMING: events only around the support-counting
                                     * kernels (Gram, AND+popcount, depth-first), not around the
                                     * level bookkeeping, output and scheduling launches */
#define BM_FLAG_NO_PROJECT 4096u    /* count every class over all n transactions: no projected views
                                     * (by default a big class of a deep level whose prefix holds
                                     * few of the transactions is counted over a view: its
                                     * children's columns gathered over the prefix's
                                     * transactions; see project_gain) */
#define BM_FLAG_DEPTH_FIRST 2048u   /* databases with short columns (<= dfs_max_words words): mine
                                     * small subtrees with the depth-first kernel from a work queue.
                                     * Off by default (level by level measured faster there); also
                                     * on when bm_mine_batch gets a cost model to order that queue,
                                     * or with BM_FLAG_TRACE (whose rows are its tasks) */

typedef struct {
  uint32_t flags;
  uint32_t mfma_min_children; /* classes with at least this many children use 128-wide MFMA tiles,
                               * smaller ones (over 8 children) 32-wide MFMA tiles (default 64) */
  uint32_t andpop_chunk_words;/* AND+popcount LDS chunk: 128 or 256 words */
  uint32_t split_words;       /* word-range length of one task (multiple of 64; 0 = automatic) */
  uint32_t shuffle_seed;      /* with BM_FLAG_SHUFFLE */
  uint32_t dfs_threads;       /* threads per workgroup of the depth-first kernel: 256, 512 or 1024 */
  uint32_t dfs_max_words;     /* columns of at most this many 64-bit words are short: the
                               * depth-first phase may run (see BM_FLAG_DEPTH_FIRST); longer ones
                               * take subset counting (0 = default 4,096; 0xffffffff = always
                               * short) */
  uint32_t mfma_big_children; /* MFMA classes with at least this many children use 256-wide
                               * tiles, FP4 form only (0 = default: never) */
  uint32_t dfs_wave_max_words;/* subtree tasks of databases with at most this many words per
                               * column run one stack per wave, the others one per workgroup
                               * (0 = default 1024; see BM_FLAG_DFS_BLOCK_ONLY) */
  uint32_t subset_max_children;/* when columns are too long for the depth-first phase, classes of
                               * at most this many children (2..8) are mined whole: every subset
                               * of their children is counted in one pass over word ranges, and
                               * the rest of such a subtree needs no further level step
                               * (0 = default 6; 1 = never, level by level instead) */
  uint32_t dfs_arena_nodes;   /* initial capacity, in nodes, of the output arena that the subtree
                               * kernels write (0 = automatic).  When it overflows the subtree
                               * phase runs again with at least four times the room; a small value
                               * exercises that path and never changes the result */
  uint32_t project_gain;       /* a class on the 128/256-wide MFMA kernels with q children whose
                               * prefix has support s is counted over a projected view when
                               * q (n - s) >= project_gain * n: the MFMA work it saves,
                               * q^2 (n - s), then outweighs gathering q columns (0 = default
                               * 512; see BM_FLAG_NO_PROJECT) */
} bm_options;

uint32_t bm_abi_version(void);
/* Static English text for a status code. */
const char* bm_status_string(bm_status s);
/* Thread-local description of the last failure on this thread ("" if none). */
const char* bm_last_error(void);

/* Route the library's device allocations through caller callbacks (for example
 * a framework's caching allocator).  alloc(size, stream, ctx) returns device
 * memory or NULL (reported as BM_ERR_OOM); free(ptr, stream, ctx) releases it.
 * Passing alloc == NULL and free == NULL restores the built-in caching pool.
 * Must not be called while any handle is alive. */
bm_status bm_set_allocator(void* (*alloc)(size_t size, void* stream, void* ctx),
                           void (*free_fn)(void* ptr, void* stream, void* ctx), void* ctx);
/* Return every cached block of the built-in pool to the HIP runtime. */
bm_status bm_release_cached_memory(void);

/* Matrix construction (Section III, Eq. 1).
 * row_ptr  host or device, uint64[n_tx + 1]; row_ptr[0] == 0, non-decreasing.
 * col_idx  host or device, uint32[row_ptr[n_tx]]; item ids of transaction i are
 *          col_idx[row_ptr[i] .. row_ptr[i+1]); order within a row is free and
 *          duplicate ids collapse (M is 0/1).  May be NULL when row_ptr[n_tx] == 0.
 * On success *out holds M as one bitset per item column on the device: 64-bit
 * words, transaction i at bit (i & 63) of word (i >> 6), padding bits zero,
 * plus every column's popcount (the single-item supports, Eq. 3).
 * Errors: BM_ERR_INVALID_ARG (out or row_ptr NULL), BM_ERR_CSR, BM_ERR_UNSUPPORTED
 * (n_tx >= 2^31), BM_ERR_OOM, BM_ERR_DEVICE.  n_tx == 0 or n_items == 0 is valid. */
bm_status bm_build(const uint64_t* row_ptr, const uint32_t* col_idx, uint64_t n_tx,
                   uint32_t n_items, void* stream, bm_db** out);

/* Batched bm_build: `count` databases (host arrays of per-database row_ptr
 * and col_idx pointers, each host or device, and of sizes; col_idxs may be
 * NULL when every database is empty) are validated and packed by three kernel
 * launches for the whole batch and two synchronisations, instead of one call
 * each.  out[i] equals what bm_build would return for database i.  All or
 * nothing: on failure every out[i] is NULL and bm_last_error names the first
 * failing database. */
bm_status bm_build_batch(uint32_t count, const uint64_t* const* row_ptrs,
                         const uint32_t* const* col_idxs, const uint64_t* n_tx,
                         const uint32_t* n_items, void* stream, bm_db** out);
bm_status bm_db_info(const bm_db* db, uint64_t* n_tx, uint32_t* n_items, uint64_t* words_per_column);

/* Single-item supports S({j}) = popcount of column j (Eq. 3's column aggregation).
 * out: host or device uint32[n_items]. */
bm_status bm_item_support(const bm_db* db, uint32_t* out, void* stream);

/* Pair supports (Eq. 2) of the k items `items` (host or device uint32[k], ids <
 * n_items, repeats allowed; NULL means all n_items items in id order, k must then
 * equal n_items).  out: host or device uint32[k*k], row-major and symmetric,
 * out[a*k+b] = S({items[a], items[b]}), diagonal = single-item supports.
 * Computed as the Gram matrix A^T A of the selected columns with the mining
 * path's class kernels: MFMA in the FP4 (e2m1) form with FP32 sums, exact
 * because every task's counts stay below 2^24 (small k: AND+popcount).  k == 0
 * is a no-op. */
bm_status bm_pair_support(const bm_db* db, const uint32_t* items, uint32_t k, uint32_t* out,
                          void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): bm_pair_support
 * with every temporary buffer (item list, task lists, the support triangle)
 * carved from a static 16 MiB scratch array that the library holds on each GPU
 * it runs on until the process ends; the call makes no hipMalloc, hipFree or
 * other allocating call.  items (or NULL, meaning all n_items items) and out
 * (uint32[k*k], as bm_pair_support) must be device memory (else
 * BM_ERR_INVALID_ARG).  k <= 2048 (BM_ERR_UNSUPPORTED beyond, or if the
 * database's shape would need more scratch than the array holds).  Results are
 * those of bm_pair_support.  All calls on one GPU share its scratch array, which
 * keeps the last call's contents: calls that overlap on one GPU (from several
 * threads or streams) race and must be serialised by the caller. */
bm_status bm_pair_support_noalloc(const bm_db* db, const uint32_t* items, uint32_t k, uint32_t* out,
                                  void* stream);

/* Frequent-itemset mining (Section III, Eqs. 1-3 and the recursive extension of
 * frequent prefixes by further column ANDs).  Reports every non-empty itemset X
 * with S(X) >= minsup.  minsup == 0 gives BM_ERR_INVALID_ARG; minsup > n_tx or an
 * empty database gives an empty result.  The result is in canonical order:
 * each itemset is an ascending tuple of the caller's item ids and the list is
 * sorted lexicographically, a proper prefix before its extensions. */
bm_status bm_mine(const bm_db* db, uint32_t minsup, void* stream, bm_result** out);
/* As bm_mine with options (NULL = defaults). */
bm_status bm_mine_ex(const bm_db* db, uint32_t minsup, const bm_options* opt, void* stream,
                     bm_result** out);

/* Out-of-core mining (the paper's block storage and block computing of large
 * matrices: Section I, the closing paragraph of Section III, Section V): the
 * transactions stay in host memory and the device holds only one block of
 * block_rows transactions at a time, as column bitsets.  A first pass over the
 * blocks sums the single-item supports; then every level step loads the
 * blocks one after another and adds each block's candidate counts into the
 * same supports, so every support is exact (a sum of integer counts over the
 * blocks) and no recount pass is needed.  Small classes are mined level by
 * level.  Device memory: the block matrix (n_items x ceil(block_rows/64)
 * words, padded) plus the level arrays, independent of n_tx; every level re-reads
 * the whole CSR over the host link.  row_ptr (uint64[n_tx + 1]) and col_idx
 * (uint32[row_ptr[n_tx]]) must be host memory (else BM_ERR_INVALID_ARG); their
 * checks and limits are bm_build's, plus block_rows >= 1 and minsup >= 1.  The
 * result equals bm_mine on the whole database. */
bm_status bm_mine_blocked(const uint64_t* row_ptr, const uint32_t* col_idx, uint64_t n_tx,
                          uint32_t n_items, uint32_t minsup, uint64_t block_rows,
                          const bm_options* opt, void* stream, bm_result** out);

/* Batched mining: `count` independent databases (each with its own minsup) are
 * mined together -- every level step covers the prefix classes of all of them,
 * so the whole batch needs one device->host synchronisation per itemset length
 * instead of one per length per database.  dbs: host array of count handles
 * (NULL entries give empty results); minsups: host uint32[count]; out: host
 * array of count result pointers, each filled exactly as bm_mine would fill
 * it for that database alone (bit-identical output).  sched: a trained cost
 * model or NULL; it only orders work and never changes a result.  On failure
 * every out[i] is NULL. */
bm_status bm_mine_batch(const bm_db* const* dbs, const uint32_t* minsups, uint32_t count,
                        const bm_model* sched, const bm_options* opt, void* stream,
                        bm_result** out);

/* Autotuner (batching design, word tiles and block shapes): times real calls of
 * bm_mine_batch on these databases over a coordinate search of the tuning
 * fields of bm_options -- small subtrees level by level / defaults /
 * depth-first on short columns / depth-first everywhere, mfma_min_children,
 * mfma_big_children, split_words, andpop_chunk_words, project_gain (or no
 * projected views), subset_max_children, dfs_threads, dfs_wave_max_words --
 * and writes
 * the fastest combination to *best (base's other flags kept; NULL base =
 * defaults).  Each point is the minimum of `reps` calls (0 = 3); *best_ms
 * (optional) receives its wall time.  No tuning field changes the mined
 * result, so *best can be passed to bm_mine_ex / bm_mine_batch as is. */
bm_status bm_autotune(const bm_db* const* dbs, const uint32_t* minsups, uint32_t count,
                      const bm_model* sched, const bm_options* base, uint32_t reps, void* stream,
                      bm_options* best, double* best_ms);

/* Result access.  n_sets frequent itemsets holding n_items_total item ids. */
bm_status bm_result_info(const bm_result* r, uint64_t* n_sets, uint64_t* n_items_total,
                         uint32_t* max_len);
/* Copy the result (any pointer may be NULL to skip that array):
 *   offsets  host or device uint64[n_sets + 1]; itemset s is items[offsets[s] .. offsets[s+1])
 *   items    host or device uint32[n_items_total]
 *   supports host or device uint32[n_sets] */
bm_status bm_result_copy(const bm_result* r, uint64_t* offsets, uint32_t* items,
                         uint32_t* supports, void* stream);
bm_status bm_result_stats(const bm_result* r, bm_stats* out);

/* Trace of a call made with BM_FLAG_TRACE (shared by all results of a batch):
 * one row per subtree task handed to the depth-first kernel -- 8 features of
 * the task's prefix class (itemset length of its children, log2 support of the
 * prefix, log2(1 + children), mean log2 child support, max and mean child /
 * prefix support ratio, log2 minsup, log2 words per column) and the label
 * log2(1 + 64-bit column words the depth-first kernel streams for the task's
 * whole subtree: prefix and child columns of every class it evaluates), which
 * is deterministic and proportional to the task's run time.  feats: host float[rows*8] or NULL; labels: host float[rows]
 * or NULL; *rows receives the row count (0 without a trace). */
bm_status bm_result_trace(const bm_result* r, float* feats, float* labels, uint64_t* rows);

/* Scheduler cost model: an 8 -> 64 -> 64 -> 1 perceptron with ReLU, BF16
 * weights and FP32 accumulation, predicting the trace label (log2 of the
 * subtree's streamed column words) of a subtree task from its 8 features.  Passed to bm_mine_batch it only
 * orders the depth-first work queue (longest predicted first); results are
 * identical with and without it.  Training runs on the device (forward,
 * backward and Adam kernels on an FP32 master copy); inputs are standardised
 * with statistics of the first training set.  Arrays are host or device. */
bm_status bm_model_create(uint32_t seed, bm_model** out);  /* He-uniform init from `seed` */
bm_status bm_model_load(const char* path, bm_model** out);
bm_status bm_model_save(const bm_model* m, const char* path);
/* Minibatch Adam (batch rows per step, 0 = 256) over `epochs` passes, rows in
 * order; *final_loss (may be NULL) receives the last epoch's mean over batches
 * of the batch mean squared error.  Epochs after capture are replayed as one
 * hipGraph each (bm_model_train_ex with BM_FLAG_GRAPH).  Training is
 * deterministic: gradients are summed per workgroup and then in a fixed order. */
bm_status bm_model_train(bm_model* m, const float* feats, const float* labels, uint64_t rows,
                         uint32_t epochs, float lr, uint32_t batch, float* final_loss,
                         void* stream);
/* As bm_model_train; flags: 0 (every launch issued from the host) or
 * BM_FLAG_GRAPH (one epoch captured as a hipGraph and replayed `epochs`
 * times; identical results).  epoch_losses: NULL or host float[epochs]. */
bm_status bm_model_train_ex(bm_model* m, const float* feats, const float* labels, uint64_t rows,
                            uint32_t epochs, float lr, uint32_t batch, uint32_t flags,
                            float* epoch_losses, void* stream);
bm_status bm_model_predict(const bm_model* m, const float* feats, uint64_t rows, float* out,
                           void* stream);
/* Gradient of the mean squared error over `rows` (float[4801]) and the loss,
 * without updating the model (for checking the backward kernel). */
bm_status bm_model_grad(bm_model* m, const float* feats, const float* labels, uint64_t rows,
                        float* grad, float* loss, void* stream);
/* Parameters: FP32 master copy, the BF16 weights the kernels use (as floats),
 * and the 16 normalisation values (mean[8], 1/std[8]); any pointer may be NULL. */
bm_status bm_model_params(const bm_model* m, float* master, float* weights_bf16, float* norm);
bm_status bm_model_set_params(bm_model* m, const float* master, const float* norm);

/* Association rules (the paper's use of frequent itemsets: abstract and
 * Section I; support, confidence and lift are its indicators, Section IV-A).
 * From every itemset Z of a mining result with 2 <= |Z| <= max_len and every
 * split Z = X + Y into non-empty disjoint X (antecedent) and Y (consequent):
 *   conf(X => Y) = supp(Z) / supp(X),
 *   lift(X => Y) = supp(Z) * n / (supp(X) * supp(Y)),  n = transactions,
 * keeping the rule iff supp(Z) * 10^6 >= min_conf_ppm * supp(X) (exact integer
 * test; min_conf_ppm <= 10^6, 0 keeps all 2^|Z| - 2 rules of each Z).  Both
 * supports are looked up in the result itself (every subset of a frequent
 * set is frequent) by a device join of the canonical list with itself.
 * max_len: 0 = 20; at most 24 (BM_ERR_UNSUPPORTED beyond), itemsets longer
 * than max_len give no rules.  conf and lift are IEEE double quotients of the
 * integers (exact operands while supp(Z) * n < 2^53).  Rules are ordered by
 * Z's position in the result, then by X as an ascending tuple
 * (lexicographically, a prefix first).  The result may be freed afterwards. */
bm_status bm_rules_mine(const bm_result* r, uint32_t min_conf_ppm, uint32_t max_len, void* stream,
                        bm_rules** out);
bm_status bm_rules_info(const bm_rules* rs, uint64_t* n_rules);
/* Copy the rules (host or device arrays of n_rules entries; any may be NULL):
 *   z_index   uint64: position of Z in the result's itemset list
 *   ante_mask uint32: X as a mask over Z's items, bit p = p-th (ascending) item
 *   supp_x, supp_y, supp_z uint32; conf, lift double */
bm_status bm_rules_copy(const bm_rules* rs, uint64_t* z_index, uint32_t* ante_mask, uint32_t* supp_x,
                        uint32_t* supp_y, uint32_t* supp_z, double* conf, double* lift,
                        void* stream);

void bm_db_free(bm_db* db);
void bm_result_free(bm_result* r);
void bm_rules_free(bm_rules* rs);
void bm_model_free(bm_model* m);

#ifdef __cplusplus
}
#endif

#endif /* BM_H_ */
