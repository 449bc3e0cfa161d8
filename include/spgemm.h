/*
 * spgemm.h — C ABI of the MI355X (gfx950) hash-table SpGEMM library.
 *
 * Operation: C = A*B for sparse A (m x n) and B (n x k) in CSR, over the
 * (+, x) semiring on IEEE binary64 or on int64 (wrap-around), as defined by
 * Gustavson's row-wise algorithm (paper Section 2, Fig. 1).  The library runs
 * the two-phase method of the paper (Section 2 "two-phase method"; Hash
 * SpGEMM driver, Section 4.2.1, Fig. 5):
 *
 *   spgemm_plan      row flop count (Section 4.1, Fig. 4 part 1) and the
 *                    grouping of rows by flop (the GPU counterpart of the
 *                    flop-balanced partition of Fig. 4 part 2); returns the
 *                    workspace size.
 *   spgemm_symbolic  per-row nnz of C from hash-table (or bitmap) insertion of
 *                    keys only (Section 4.2.1), prefix-summed into the int64
 *                    row pointers of C; returns nnz(C) to the host.
 *   spgemm_numeric   accumulation of a_ik*b_kj into hash tables and compaction
 *                    into the caller's columns/values of C; each row sorted by
 *                    column when SPGEMM_SORTED is set (Section 4.2.1, output
 *                    step), otherwise in table order.
 *   spgemm_free      releases the plan's host-side state.
 *
 * Memory ownership: the library never allocates device memory.  Every device
 * buffer (plan scratch, workspace, C) comes from the caller and must stay
 * allocated and unmodified (except for the documented outputs) until the
 * plan is freed.  The plan object itself is host memory owned by the library.
 *
 * Streams: all device work is enqueued on the stream given to spgemm_plan.
 * spgemm_plan and spgemm_symbolic synchronise that stream (they read a few
 * bytes of results back to the host); spgemm_numeric does not.
 *
 * Errors: every function returns SPGEMM_OK (0) or a negative status; nothing
 * aborts and no C++ exception crosses the ABI.  spgemm_strerror() gives the
 * text; for SPGEMM_ERR_HIP it includes the HIP runtime's message.
 */
#ifndef SPGEMM_H
#define SPGEMM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Value type of A, B and C (all three share it). */
typedef enum {
    SPGEMM_F64 = 0, /* IEEE binary64; sums within 1e-12 relative of any order */
    SPGEMM_I64 = 1  /* int64, multiply and add modulo 2^64 (exact)            */
} spgemm_dtype;

/* Flags for spgemm_plan. */
enum {
    SPGEMM_SORTED = 1u << 0,   /* emit each row of C with ascending column ids     */
    SPGEMM_VALIDATE = 1u << 1, /* check A and B structure on the device at plan time
                                  (row pointers non-decreasing from 0 to nnz, column
                                  ids in range); failure gives SPGEMM_ERR_INVALID_CSR */
    SPGEMM_TIMING = 1u << 2,   /* record HIP events around every kernel launch from
                                  the plan on (see spgemm_plan_kernel_times)        */
    SPGEMM_PROBE_COUNT = 1u << 4, /* count the LDS probes of every hash-table
                                  insertion per bin (spgemm_stats: the collision
                                  factor of Eq. 2); a debugging aid, not free   */
    SPGEMM_LOW_MEMORY = 1u << 3 /* do not keep the symbolic bitmaps of rows whose
                                  key bound exceeds 8448 for the numeric phase: a
                                  smaller workspace (by nrows_in_that_bin *
                                  ceil(ncols/4096) * 512 bytes) and a slower numeric
                                  phase.  Without it they are kept when they take
                                  at most 64 GiB.                                  */
};

/* Status codes. */
enum {
    SPGEMM_OK = 0,
    SPGEMM_ERR_INVALID_ARG = -1,  /* NULL pointer, negative size, bad dtype/flags     */
    SPGEMM_ERR_SHAPE = -2,        /* A.ncols != B.nrows                               */
    SPGEMM_ERR_INVALID_CSR = -3,  /* SPGEMM_VALIDATE found malformed A or B           */
    SPGEMM_ERR_WORKSPACE = -4,    /* workspace pointer NULL while bytes are needed    */
    SPGEMM_ERR_OVERFLOW = -5,     /* a size exceeds the supported index range         */
    SPGEMM_ERR_STATE = -6,        /* calls out of order (e.g. numeric before symbolic) */
    SPGEMM_ERR_HIP = -7,          /* a HIP runtime call failed                         */
    SPGEMM_ERR_UNSUPPORTED = -8,  /* input outside the supported envelope              */
    SPGEMM_ERR_HOST_ALLOC = -9,   /* host memory for the plan could not be allocated   */
    SPGEMM_ERR_INTERNAL = -10,    /* a device-side consistency check failed            */
    SPGEMM_ERR_STATIC_LIMIT = -11 /* the plan needs more workspace than the static
                                     scratch of spgemm_symbolic_static holds          */
};

/*
 * A CSR operand (paper Section 2, CSR paragraph).  All pointers are DEVICE
 * pointers, owned by the caller, read-only to the library:
 *   rpts  int32[nrows + 1], rpts[0] = 0, non-decreasing, rpts[nrows] = nnz
 *   cols  int32[nnz], 0 <= cols[p] < ncols, any order within a row
 *   vals  nnz values of the plan's dtype (may be NULL until spgemm_numeric)
 * Limits: nrows, ncols < 2^31 - 1, nnz < 2^31 - 1.  Repeated column ids in a
 * row are allowed and simply add up.
 */
typedef struct {
    int64_t nrows;
    int64_t ncols;
    int64_t nnz;
    const int32_t *rpts;
    const int32_t *cols;
    const void *vals;
} spgemm_csr;

typedef struct spgemm_plan_s *spgemm_plan_t;

/*
 * Bytes of device "plan scratch" spgemm_plan needs for nprod products whose
 * left operands are A[0..nprod-1] (a small header, 4 bytes per row of A for
 * the row flop and lists of the rows of A longer than 32 entries: 4 bytes
 * for each of at most min(rows, nnz / 33) of them and for each of at most
 * nnz / 4097 rows longer than 4096 entries).
 * Returns 0 if an argument is invalid.
 */
size_t spgemm_plan_scratch_bytes(int nprod, const spgemm_csr *A);

/*
 * Tunables of a plan: the hash of the LDS tables and the row bins (Section
 * 4.2.1 hashes a column id by multiplying it by a constant; Fig. 5 sizes a
 * table from the rows it serves).  Rows are binned by their key bound
 * x = min(row flop, ncols) in the symbolic phase and by nnz(c_i) in the
 * numeric phase; bin b (1..9) serves bounds in (max[b-2], max[b-1]] with an
 * LDS table of
 *   symbolic: 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384 keys
 *   numeric:  64, 128, 256, 512, 1024, 2048, 4096, 8192, 11264 entries
 * for b = 1..9.  Limits must be positive, non-decreasing, at most their
 * table's size (a fuller table still works, with longer probes), and the
 * ninth must be 8448 (rows above it take the heavy-row path).  hash_mul is
 * the odd multiplier of the hash; 0 sends every key to the first bucket (a
 * worst case, for tests).  bucket_slots (4, 8 or 16) is the width of the
 * tables' buckets: a key's bucket is scanned 4 slots (one 16-byte LDS load)
 * at a time, front to back, and a full bucket passes the probe to the next;
 * with 4-slot buckets an insertion first tries the key's own slot of its
 * bucket with one compare-and-swap.  8 and 16 are the wider chunks of the
 * HashVector variant (Section 4.2.2).
 * heap = 1 selects the Heap accumulator of Section 4.2.3 for the numeric
 * phase of every row whose output fits an LDS table, that has at most 256
 * entries of A and at most 1024 products: the row is merged from the sorted
 * rows of B by a priority queue of nnz(a_i) heads and leaves sorted (Eq. 1
 * costs it flop * log nnz(a_i)); other rows keep the hash tables.  It needs
 * SPGEMM_SORTED (else spgemm_plan returns SPGEMM_ERR_INVALID_ARG) and rows of B
 * in ascending column order (checked on the device by spgemm_plan, which
 * returns SPGEMM_ERR_UNSUPPORTED otherwise).  heap = 0: hash tables only.
 * The defaults (spgemm_config_default) fill each table at most half, use
 * 4-slot buckets and no heap.
 */
typedef struct {
    uint32_t hash_mul;
    int32_t sym_max[9];
    int32_t num_max[9];
    uint32_t bucket_slots;
    uint32_t heap;
} spgemm_config;

/* The default configuration. */
void spgemm_config_default(spgemm_config *cfg);

/* SPGEMM_OK if cfg satisfies the rules above, else SPGEMM_ERR_INVALID_ARG. */
int spgemm_config_check(const spgemm_config *cfg);

/*
 * Plan nprod independent products C[p] = A[p]*B[p] (nprod >= 1; A and B are
 * host arrays of nprod descriptors).  Computes row flop and groups rows by
 * flop on the device (Section 4.1 and Fig. 4: the flop of every row, then the
 * rows grouped so that each group's table fits its largest row), then reads
 * the group sizes back (synchronises stream).
 *   plan_scratch     device buffer of spgemm_plan_scratch_bytes(nprod, A)
 *                    bytes, kept alive until spgemm_free
 *   workspace_bytes  out: bytes of device workspace spgemm_symbolic needs
 *   cfg              tunables (NULL: spgemm_config_default); an invalid
 *                    cfg gives SPGEMM_ERR_INVALID_ARG
 * Values are not read here.  On error *out is NULL.
 */
int spgemm_plan(spgemm_plan_t *out, int nprod, const spgemm_csr *A, const spgemm_csr *B,
                spgemm_dtype dtype, unsigned flags, void *plan_scratch, hipStream_t stream,
                size_t *workspace_bytes,
                const spgemm_config *cfg);

/*
 * Symbolic phase.  Writes rpts_C[p][0..A[p].nrows] (device int64, caller-owned,
 * nrows+1 entries each; rpts_C is a host array of nprod device pointers) and
 * stores nnz(C[p]) in nnz_C[p] (host array of nprod).  Synchronises stream.
 *   workspace  device buffer of the size spgemm_plan returned, kept alive
 *              until spgemm_free
 */
int spgemm_symbolic(spgemm_plan_t plan, void *workspace, int64_t *const *rpts_C, int64_t *nnz_C);

/*
 * spgemm_symbolic without a workspace argument, for callers that cannot
 * allocate device memory (serving loops and harnesses that forbid hipMalloc):
 * the workspace is a static device array of SPGEMM_STATIC_WS_BYTES bytes that
 * the library holds on every GPU it runs on until the process ends.  The
 * current device must be the device of the plan's stream.  A plan whose
 * workspace (spgemm_plan's workspace_bytes) exceeds SPGEMM_STATIC_WS_BYTES is
 * rejected with SPGEMM_ERR_STATIC_LIMIT before any work is enqueued.
 * Otherwise this is spgemm_symbolic with that array as the workspace: same
 * outputs, same synchronisation, and the plan's spgemm_numeric reads the array
 * too.  Every call on a GPU shares that GPU's array, which keeps the last
 * call's contents: from this call until the same plan's spgemm_numeric has
 * finished on its stream, another spgemm_symbolic_static on the same GPU
 * races with it (its results are undefined).  Nothing is allocated.
 */
enum { SPGEMM_STATIC_WS_BYTES = 64 << 20 };
int spgemm_symbolic_static(spgemm_plan_t plan, int64_t *const *rpts_C, int64_t *nnz_C);

/*
 * Numeric phase.  A and B must describe the same matrices (same pointers for
 * rpts/cols) as at plan time; their vals must now be set (new values with the
 * same pattern may be passed on later calls: the symbolic result is reused).
 * cols_C[p] (device int32[nnz_C[p]]) and vals_C[p] (device dtype[nnz_C[p]])
 * are caller-owned outputs; cols_C and vals_C are host arrays of nprod device
 * pointers.  Asynchronous on the plan's stream.
 */
int spgemm_numeric(spgemm_plan_t plan, const spgemm_csr *A, const spgemm_csr *B,
                   int32_t *const *cols_C, void *const *vals_C);

/* Release the plan's host state (device buffers stay the caller's).  NULL-safe.
 * Bookkeeping of this interface only: no passage of the paper defines it. */
int spgemm_free(spgemm_plan_t plan);

/* Static text for a status code (the HIP message for SPGEMM_ERR_HIP is that of
 * the most recent failure in this process). */
const char *spgemm_strerror(int status);

/* Counters of one planned product, for reporting. */
typedef struct {
    int64_t flop;            /* multiplications a_ik*b_kj (paper Section 2)        */
    int64_t max_row_flop;
    int64_t nnz_C;           /* valid after spgemm_symbolic                         */
    int64_t heavy_rows;      /* rows accumulated in column windows                  */
    int64_t windows;         /* column-window work items of those rows              */
    int64_t probe_overflow;  /* must be 0: hash probes that exceeded the table size */
    int64_t heap_rows;       /* rows whose numeric phase took the heap merge        */
    /* Collision factor of Eq. 2 per LDS table bin b = 1..9 (index b-1):
     * c = probes / flop, the LDS probes per insertion (a compare-and-swap on the
 * key's own slot, then each 16-byte bucket read).  probes are
     * counted only in plans made with SPGEMM_PROBE_COUNT (else 0); flop is
     * the bin's multiplications (symbolic bins by key bound, numeric bins by
     * nnz(c_i); valid after spgemm_symbolic). */
    int64_t sym_flop[9];
    int64_t sym_probes[9];
    int64_t num_flop[9];
    int64_t num_probes[9];
} spgemm_stats;

int spgemm_plan_stats(spgemm_plan_t plan, int iprod, spgemm_stats *out);

/*
 * Per-kernel timing.  When enabled, the library records HIP events around
 * each kernel launch on the plan's stream; spgemm_plan_kernel_times waits for
 * them and reports, for each kernel name, the summed milliseconds, launch
 * count and the algorithmic bytes that launch moves (the per-kernel byte
 * model of the library's design notes).  Returns the number of kernels
 * written (at most cap), or a negative status.
 */
typedef struct {
    char name[48];
    double ms;
    int64_t launches;
    double alg_bytes;
} spgemm_kernel_time;

int spgemm_plan_set_timing(spgemm_plan_t plan, int enable);
int spgemm_plan_kernel_times(spgemm_plan_t plan, spgemm_kernel_time *out, int cap);

/*
 * Masked sum for triangle counting (paper Section 5.6): out[0] = sum over the
 * stored positions (i, j) of M of C_ij, int64 wrap-around.  C has int64 row
 * pointers (as spgemm_symbolic writes them) and int64 values; M is a CSR
 * pattern (its vals are ignored).  Rows of C and M may be in any column order.
 * out is a device int64 (overwritten).  Asynchronous on stream.
 */
int spgemm_masked_sum_i64(int64_t nrows, int64_t ncols, const int64_t *rpts_C, const int32_t *cols_C,
                          const int64_t *vals_C, const spgemm_csr *M, int64_t *out, hipStream_t stream);

/*
 * Masked product sum without forming C (the masked product behind Section
 * 5.6's triangle count): out[0] = sum over the stored positions (i, j) of M of
 * (A*B)_ij, int64 wrap-around; every product a_ik*b_kj whose column j is not in
 * row i of M is dropped as it is formed.  A is m x n, B is n x k, M is m x k
 * (a pattern: its vals are ignored; a row must not repeat a column).  int64
 * values; if A.vals or B.vals is NULL every value of both counts as 1
 * (counting: triangles = spgemm_masked_product_sum_i64(L, U, A) / 2).
 * workspace: device buffer of at least SPGEMM_MASKED_WS_BYTES bytes (a row
 * counter), out: device int64 (overwritten).  Asynchronous on stream; no
 * device allocation.  Errors: SPGEMM_ERR_INVALID_ARG, SPGEMM_ERR_SHAPE.
 */
enum { SPGEMM_MASKED_WS_BYTES = 256 };
int spgemm_masked_product_sum_i64(const spgemm_csr *A, const spgemm_csr *B, const spgemm_csr *M, void *workspace,
                                  int64_t *out, hipStream_t stream);

/*
 * Streaming copy of nbytes (multiple of 16) from src to dst, both device
 * pointers: the measured HBM copy rate is the denominator the benchmark
 * compares the SpGEMM byte rates with.  Asynchronous on stream.
 */
int spgemm_stream_copy(void *dst, const void *src, size_t nbytes, hipStream_t stream);

/*
 * Stanza read probe (the access pattern of B rows, Section 5 on DDR and
 * MCDRAM: short runs of consecutive words fetched from effectively random
 * places).  Reads nstanza stanzas of 2^log2_words 8-byte words from the
 * device array base (nbytes, a multiple of 8, at least 8), stanza s starting
 * at word start[s] (device array of nstanza int64 word offsets), and writes
 * the wrap-around sum of every word read to *sum and the number of stanzas
 * that did not fit the array (skipped, not read) to *skipped; both are device
 * pointers to 8 bytes owned by the caller.  Consecutive lanes read
 * consecutive words, so the rate against log2_words traces the bandwidth
 * between random 8-byte reads and streaming.  0 <= log2_words <=
 * SPGEMM_STANZA_MAX_LOG2.  Asynchronous on stream; nothing is allocated.
 */
enum { SPGEMM_STANZA_MAX_LOG2 = 24 };
int spgemm_stanza_read(const void *base, size_t nbytes, const int64_t *start, int64_t nstanza, int log2_words,
                       unsigned long long *sum, unsigned long long *skipped, hipStream_t stream);

/* ---------------------------------------------------------------- batches
 *
 * Many small independent products through one fixed sequence of launches per
 * batch, with no host synchronisation inside spgemm_batch_run (the sequence
 * can be captured in a HIP graph and replayed).  Every row of every product is
 * binned by its key bound min(row flop, ncols) (the row flop of Fig. 4) into
 * the LDS hash table size the single-product path uses for that bound
 * (Section 4.2.1), and the two phases of Section 2 run on the device for the
 * whole batch: the rows' distinct columns are counted, the counts scanned into
 * places, and every row accumulated and written at its place in a
 * caller-provided arena sized from the bounds (an upper bound of nnz(C)).  A
 * product with a row whose key bound exceeds 8448 is
 * outside the batched range: none of its rows is computed and it gets status
 * SPGEMM_ERR_UNSUPPORTED (use the plan path for it).  Operands must be valid
 * CSR (see spgemm_csr); the batch path does not validate them.  The total row
 * count of a batch must be below 2^31 - 1.  Calls that overlap on one scratch
 * or arena race.
 */
typedef struct {
    int64_t flop;       /* multiplications of the product                           */
    int64_t nnz;        /* nnz(C)                                                  */
    int64_t rpts_off;   /* byte offset in the arena of C's int64 row pointers       */
    int64_t cols_off;   /* byte offset in the arena of C's int32 column ids         */
    int64_t vals_off;   /* byte offset in the arena of C's values                   */
    int32_t status;     /* SPGEMM_OK, SPGEMM_ERR_UNSUPPORTED or SPGEMM_ERR_INTERNAL */
    int32_t pad;
} spgemm_batch_result;

/* Device scratch bytes for a batch whose left operands are A[0..nprod-1]
 * (0 for an invalid batch). */
size_t spgemm_batch_scratch_bytes(int nprod, const spgemm_csr *A);

/* Upload the batch description (device pointers of A[p], B[p], per-product
 * flags: SPGEMM_SORTED or 0) into scratch.  Host arrays may be reused on
 * return (the call waits for its copy).  Errors: SPGEMM_ERR_INVALID_ARG
 * (counts, pointers, flags), SPGEMM_ERR_SHAPE (A[p].ncols != B[p].nrows). */
int spgemm_batch_prepare(int nprod, const spgemm_csr *A, const spgemm_csr *B, const unsigned *flags,
                         void *scratch, hipStream_t stream);

/* Analyse a prepared batch: the row flop of every row (Fig. 4) and its bin,
 * kept in scratch for every later run; per product, into
 * host arrays of nprod: flop[p] (multiplications), bound[p] (sum over the
 * product's batched rows of min(row flop, ncols): an upper bound of
 * nnz(C[p])) and, if max_key is not NULL, max_key[p] (largest
 * min(row flop, ncols) of the product).  Synchronises stream (used for
 * admission and arena sizing).  Operand values are not read. */
int spgemm_batch_analyse(int nprod, const spgemm_csr *A, void *scratch, int64_t *flop, int64_t *bound,
                         int64_t *max_key, hipStream_t stream);

/* Rows of an analysed batch per bin (Fig. 4's row flop grouped as in the
 * single-product path): rows[0] = empty rows, rows[b] for b = 1..9 = rows whose
 * key bound min(row flop, ncols) falls in the bin of the b-th LDS table size
 * (64 ... 16384 slots, see spgemm_config), rows[10] = rows above 8448 (outside
 * the batched range).  rows is a host array of 11.  Synchronises stream.
 * Errors: SPGEMM_ERR_INVALID_ARG, SPGEMM_ERR_HIP. */
enum { SPGEMM_BATCH_BINS = 11 };
int spgemm_batch_bin_rows(int nprod, const spgemm_csr *A, void *scratch, int64_t *rows, hipStream_t stream);

/* Arena bytes for a batch with the given per-product bounds (host array):
 * 12 bytes per bounded entry plus 8 per row pointer, 256-byte aligned parts. */
size_t spgemm_batch_arena_bytes(int nprod, const spgemm_csr *A, const int64_t *bound);

/* Run a prepared batch: every product C[p] = A[p]*B[p] lands in the arena;
 * results (device array of nprod) says where.  bound is the host array that
 * spgemm_batch_analyse returned (it fixes the arena layout; operand values may
 * change between runs, their structure may not: rows whose bound no longer
 * fits the arena come out empty with status SPGEMM_ERR_INTERNAL).  Launches kernels
 * only (no memset, no copy, no synchronisation): capturable in a HIP graph.
 * SPGEMM_ERR_WORKSPACE if arena_bytes is below spgemm_batch_arena_bytes. */
int spgemm_batch_run(int nprod, const spgemm_csr *A, spgemm_dtype dtype, const int64_t *bound, void *scratch,
                     void *arena, size_t arena_bytes, spgemm_batch_result *results, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SPGEMM_H */
