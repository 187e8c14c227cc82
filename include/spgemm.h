/*
 * spgemm.h -- C ABI of the MI355X (gfx950) two-phase sparse matrix-matrix
 * multiply C = A * B on CSR (Deveci, Trott, Rajamanickam, "Multi-threaded
 * Sparse Matrix-Matrix Multiplication for Many-Core and GPU Architectures").
 *
 * The product is computed in the paper's two phases (Algorithms section,
 * Algorithm 2):
 *   1. spgemm_symbolic: compress B into column-set bit words (Compression
 *      subsection), find the size of every row of C by a union of those words
 *      (core kernel, Algorithm 3, symbolic branch), exclusive-scan the sizes
 *      into C.row_ptr and return nnz(C) so the caller can allocate C.
 *   2. spgemm_numeric: Gustavson row-by-row multiply-accumulate (Background
 *      section, Algorithm 1; Algorithm 3, numeric branch) writing C.col_idx
 *      (strictly increasing per row) and C.values.
 * The symbolic result is kept in the handle, so spgemm_numeric can be called
 * again with new values on the same structure (the reuse case the paper argues
 * for in its Background section and measures as "Reuse" in Experiments).
 *
 * Conventions (every entry point):
 *  - Pointers inside spg_csr / spg_csr_out are DEVICE pointers (memory the
 *    caller allocated on the GPU the handle was created on) unless the
 *    parameter says "host".
 *  - Every call returns an spg_status; nothing is thrown across the ABI.
 *    Arguments are validated before any launch.  HIP runtime failures map to
 *    SPG_ERR_HIP; spg_last_error(h) gives the text of the last failure.
 *  - All device work is enqueued on the handle's stream, in stream order.
 *    Inputs are borrowed: they must stay valid until the stream has reached
 *    the call.  spgemm_symbolic blocks the host twice (to read global flop
 *    counts and nnz(C)); spgemm_numeric never blocks the host.
 *  - The handle owns all scratch memory (compressed B, row bins, per-row
 *    windows, spill arenas); the caller owns A, B and C.
 *  - A handle is not thread-safe: use one handle per host thread / stream.
 *  - Indices: col_idx is always int32.  row_ptr is int32 or int64
 *    (spg_itype).  Input rows may hold columns in any order but no duplicate
 *    column within a row.  Stored zeros are structure.
 */
#ifndef SPGEMM_MI355X_H
#define SPGEMM_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPG_OK = 0,
    SPG_ERR_INVALID_ARG = 1,        /* NULL pointer, negative size, bad enum, bad CSR */
    SPG_ERR_DIM_MISMATCH = 2,       /* A.ncols != B.nrows, or C's shape is not m x k */
    SPG_ERR_INDEX_OVERFLOW = 3,     /* nnz(C) does not fit the requested row_ptr type */
    SPG_ERR_OUT_OF_MEMORY = 4,      /* device allocation failed, or a scratch limit */
    SPG_ERR_NOT_READY = 5,          /* numeric called before a successful symbolic */
    SPG_ERR_STRUCTURE_MISMATCH = 6, /* numeric inputs differ from the symbolic ones */
    SPG_ERR_HIP = 7,                /* HIP runtime error (text in spg_last_error) */
    SPG_ERR_UNSUPPORTED = 8,        /* valid input the library does not handle */
    SPG_ERR_INTERNAL = 9
} spg_status;

typedef enum { SPG_F64 = 0, SPG_F32 = 1 } spg_dtype;
typedef enum { SPG_I32 = 0, SPG_I64 = 1 } spg_itype;

/* Accumulator selection for every row of C (Accumulators subsection). */
typedef enum {
    SPG_ACC_AUTO = 0,   /* per-row choice by the library's selector */
    SPG_ACC_DENSE = 1,  /* bit-window dense accumulator where it fits, else hash */
    SPG_ACC_HASH = 2,   /* linear-probing hash (LDS level 1, HBM level 2) */
    SPG_ACC_HASH_L2 = 3, /* two-level hash for every non-empty row (tests the spill path) */
    SPG_ACC_LL = 4       /* the paper's kkmem choice: linked-list hashmap (Begins / Nexts /
                            Ids / Values) per row, a group of lanes per row walking its B
                            rows in turn (Thread-Sequential); rows of up to 1024 entries come
                            out UNSORTED (slot order); longer rows use the two-level hash,
                            sorted.  Position maps (spgemm_numeric_values) and
                            spgemm_backward need sorted rows and are not available. */
} spg_accumulator;

/* Floating-point forms of the numeric phase for FP32 values. */
typedef enum {
    SPG_FP32_PLAIN = 0,       /* FP32 products, FP32 accumulation */
    SPG_FP32_COMPENSATED = 1, /* FP32 with a compensated (TwoSum / TwoProduct) pair per entry */
    SPG_FP32_WIDE = 2         /* FP32 inputs and outputs, FP64 accumulation */
} spg_fp32_mode;

/* Read-only CSR operand.  values may be NULL for the symbolic phase. */
typedef struct {
    int64_t nrows, ncols, nnz;
    spg_itype rp_type;
    const void *row_ptr;      /* nrows+1 entries of rp_type, row_ptr[0] == 0 */
    const int32_t *col_idx;   /* nnz entries in [0, ncols) */
    const void *values;       /* nnz entries of dtype */
    spg_dtype dtype;
} spg_csr;

/* Output CSR: row_ptr holds the symbolic result (read), col_idx and values
 * are written by the numeric phase; nnz must equal the symbolic nnz(C). */
typedef struct {
    int64_t nrows, ncols, nnz;
    spg_itype rp_type;
    const void *row_ptr;
    int32_t *col_idx;
    void *values;
    spg_dtype dtype;
} spg_csr_out;

typedef struct {
    /* Compression of B for the symbolic phase (Compression subsection):
     * -1 = compress only if it removes more than (1 - cf_threshold) of the
     * flops, 0 = never, 1 = always. */
    int32_t compression;
    double cf_threshold;          /* 0.85: the paper's "more than 15%" rule */
    int32_t accumulator;          /* spg_accumulator */
    int32_t fp32_mode;            /* spg_fp32_mode, FP32 values only */
    int64_t fp64_heavy_row_flops; /* FP32: rows with at least this many flops
                                     accumulate in FP64 (0 = never) */
    int32_t l1_hash_slots;        /* cap on LDS hash slots for the two-level
                                     hash (0 = sized by LDS); small values force
                                     level-2 spills */
    int32_t autotune;             /* 1 = time candidate kernels on sampled rows
                                     during symbolic and keep the fastest */
    int32_t fp32_terms_max;       /* FP32 values: rows of A with more entries than
                                     this accumulate in FP64, since each entry of C
                                     then sums more products than FP32 (plain or
                                     compensated) can add within 1e-5 of the sum of
                                     |products|.  -1 = derived from fp32_mode (167
                                     plain, 52730 compensated, none with FP64
                                     accumulation), 0 = never, n > 0 = n.  Fixed at
                                     the symbolic phase. */
    int32_t verify_structure;     /* 1 = the symbolic phase records a 64-bit digest
                                     of A's and B's row_ptr and col_idx, and every
                                     spgemm_numeric, spgemm_numeric_rows and
                                     spgemm_backward on the plan recomputes it on the
                                     device first (one pass over both structures);
                                     a difference is reported by spg_check_errors as
                                     STRUCTURE_MISMATCH.  0 = pointers and sizes are
                                     the only check.  Not applied to batch plans. */
    int32_t sorted_output;        /* 1 (default) = columns strictly increasing per row;
                                     0 = rows may come out unsorted: the autotuner
                                     (autotune = 1) also times the LL hashmap */
} spg_options;

typedef struct {
    int64_t flops;                  /* f_m: number of multiplications */
    int64_t flops_compressed;       /* symbolic inserts after compression */
    int64_t max_row_flops;          /* maxrf */
    int64_t max_row_flops_compressed;
    int64_t nnz_c;                  /* nnz(C) */
    int64_t max_row_nnz;            /* maxrs */
    int64_t nnz_b_compressed;       /* (column-set index, column-set) pairs of compressed
                                       B (0 when the symbolic phase did not compress B) */
    int32_t compressed;             /* 1 if the symbolic phase used compressed B */
    int32_t n_kinds;                /* kinds in use: 0 empty, 1 bit window (wavefront),
                                       2 hash (wavefront), 3 bit window (workgroup),
                                       4 two-level hash, 5 word hash (numeric),
                                       6 short rows (a team of lanes per row),
                                       7 stored structure (numeric on the (word, bits)
                                       pairs the symbolic phase kept) */
    int64_t rows_symbolic[8];       /* rows per symbolic kernel kind */
    int64_t rows_numeric[8];        /* rows per numeric kernel kind */
    int32_t l2_spill_rows;          /* rows that used the level-2 (HBM) hash */
    int32_t tuned_policy;           /* autotune: 0 selector, 1 bit window first, 2 hash first,
                                       4 LL hashmap (unsorted rows) */
    int32_t tuned_lanes;            /* autotune: lanes per B row in the numeric phase (0 = not tuned) */
    int32_t fp64_rows;              /* rows kept in the FP64-accumulated kind lists
                                       (fp64_heavy_row_flops, fp32_terms_max) */
    int32_t reserved[4];
} spg_stats;

typedef struct spg_handle_s *spg_handle;

/* Fill *opt with the defaults (compression -1, cf_threshold 0.85, AUTO,
 * FP32_PLAIN, no flop threshold for FP64 rows, FP64 rows by the derived term
 * limit, LDS-sized hash, no autotune). */
void spg_default_options(spg_options *opt);

/* Create a handle on the current HIP device.  hip_stream is a hipStream_t
 * (NULL = the legacy default stream).  opt may be NULL (defaults); it is
 * copied.  Errors: INVALID_ARG (h NULL or bad option), HIP. */
spg_status spg_create(spg_handle *h, void *hip_stream, const spg_options *opt);

/* Release the handle and all scratch it owns (synchronises its stream). */
spg_status spg_destroy(spg_handle h);

/* Change the stream later calls enqueue on. */
spg_status spg_set_stream(spg_handle h, void *hip_stream);

/* Replace the options.  Takes effect at the next spgemm_symbolic. */
spg_status spg_set_options(spg_handle h, const spg_options *opt);

/* Symbolic phase (Algorithm 2, compress + symbolic lines; Algorithm 3).
 * A: m x n, B: n x k (values are not read).  C_row_ptr: device array of m+1
 * entries of c_rp_type, caller-allocated, written with the exclusive scan of
 * the row sizes of C.  *nnz_c (host) receives nnz(C).  The handle keeps the
 * plan for spgemm_numeric.  Errors: INVALID_ARG, DIM_MISMATCH,
 * INDEX_OVERFLOW (nnz(C) > INT32_MAX with SPG_I32), OUT_OF_MEMORY,
 * UNSUPPORTED, HIP. */
spg_status spgemm_symbolic(spg_handle h, const spg_csr *A, const spg_csr *B,
                           void *C_row_ptr, spg_itype c_rp_type, int64_t *nnz_c);

/* Numeric phase (Algorithm 2, numeric line; Algorithm 3; Algorithm 1).
 * A and B must have the structure (dims, nnz, row_ptr and col_idx pointers)
 * given to the last spgemm_symbolic on this handle; values may change.
 * C->row_ptr must be the array the symbolic phase wrote; C->col_idx (nnz_c
 * int32) and C->values (nnz_c of C->dtype) are written.  A, B and C must share
 * one dtype.  Columns come out strictly increasing per row.  Never blocks the
 * host.  Errors: INVALID_ARG, NOT_READY, STRUCTURE_MISMATCH, UNSUPPORTED,
 * OUT_OF_MEMORY, HIP. */
spg_status spgemm_numeric(spg_handle h, const spg_csr *A, const spg_csr *B, spg_csr_out *C);

/* Numeric phase on a known structure (the Reuse case: symbolic once, numeric
 * repeated with new values).  Same arguments and errors as spgemm_numeric,
 * but C->col_idx must already hold the columns an earlier spgemm_numeric on
 * this plan wrote (the same array contents; the pointer may differ): only
 * C->values is written.  The first call on a plan takes, from those columns,
 * a position map -- the rank in its row of C of every multiplication of the
 * rows in wavefront and team kinds (16 bits each) -- which blocks the host
 * once and allocates 2 bytes per such multiplication; later calls add every
 * product at its rank with no hashing or sorting.  Rows of the stored-
 * structure kind skip their column writes; heavy rows run their full kernels
 * (their columns are rewritten unchanged).  If the map cannot be allocated
 * the call runs the full numeric phase.  A C whose columns were changed since
 * is reported by spg_check_errors (STRUCTURE_MISMATCH) at the first call. */
spg_status spgemm_numeric_values(spg_handle h, const spg_csr *A, const spg_csr *B, spg_csr_out *C);

/* spgemm_numeric for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same numeric phase, arguments, results and errors as spgemm_numeric,
 * but it calls no hipMalloc / hipFree or other allocating routine.  Scratch
 * the heavy-row kernels need (value windows, level-2 hash tables, per-entry
 * cursors) comes from a static 64 MiB device array, one per GPU, that the
 * library holds from its first spg_create on that GPU until the process
 * ends; launches of heavy-row kinds are narrowed to fit it, and a plan whose
 * heavy rows need more than 64 MiB even for 8 workgroups returns
 * OUT_OF_MEMORY (nothing is written then).  The plan itself was allocated by
 * spgemm_symbolic.  The autotuner does not run here: an untuned plan keeps
 * the selector's kinds.  Every call on one GPU shares that array, so calls
 * that overlap in time on one GPU (several streams or host threads) race:
 * serialise them.  The current device must be the handle's device. */
spg_status spgemm_numeric_noalloc(spg_handle h, const spg_csr *A, const spg_csr *B, spg_csr_out *C);

/* Batched symbolic phase of `count` independent products C_i = A_i * B_i
 * (host arrays A[count], B[count] of device operands; C_row_ptr[count] of
 * device arrays of A_i.nrows+1 entries of c_rp_type; nnz_c[count] on the
 * host).  The batch runs as one block-diagonal product: one persistent launch
 * per row kind serves the rows of every product, in a work list binned by
 * flops.  The handle's plan then belongs to the batch (spgemm_numeric on it
 * returns STRUCTURE_MISMATCH).  Errors as spgemm_symbolic. */
spg_status spgemm_batch_symbolic(spg_handle h, int32_t count, const spg_csr *A, const spg_csr *B,
                                 void *const *C_row_ptr, spg_itype c_rp_type, int64_t *nnz_c);

/* Batched numeric phase on the plan of the last spgemm_batch_symbolic (same
 * operands' structure, new values allowed; C[i].nnz = nnz_c[i]).  When the
 * values of all A_i (and of all B_i, and the columns and values of all C_i)
 * lie back to back in one allocation, in batch order, nothing is copied and
 * the call never blocks the host (so it can be captured in a HIP graph);
 * otherwise the values are gathered / scattered through handle-owned staging
 * buffers and the call synchronises the stream to upload the pointer tables.
 * Errors as spgemm_numeric. */
spg_status spgemm_batch_numeric(spg_handle h, int32_t count, const spg_csr *A, const spg_csr *B,
                                spg_csr_out *C);

/* spgemm_batch_numeric on a known structure (see spgemm_numeric_values): the
 * C_i must lie back to back in one allocation (the zero-copy layout) and hold
 * the columns an earlier spgemm_batch_numeric wrote; only values are written.
 * With any other layout the call runs spgemm_batch_numeric. */
spg_status spgemm_batch_numeric_values(spg_handle h, int32_t count, const spg_csr *A, const spg_csr *B,
                                       spg_csr_out *C);

/* Per-product choices of a batch plan (host arrays of `count`): the
 * accumulator policy (spg_accumulator; SPG_ACC_AUTO = the selector) and the
 * lanes per B row the numeric phase uses for C_i.  With autotune = 1 the
 * first spgemm_batch_numeric groups the products by the average row size of
 * C_i (at most 16, 128, 1024 entries, more) and times the candidates per
 * group on sampled rows, so products of different shapes can get different
 * choices; each group then has its own row lists and LDS sizing.  Without
 * tuning every product reports the plan's one choice.  Errors: INVALID_ARG,
 * NOT_READY (no batch plan). */
spg_status spg_batch_choices(spg_handle h, int32_t count, int32_t *policy, int32_t *lanes);

/* Backward of C = A * B restricted to the stored entries (differentiation
 * of the numeric phase: each multiplication A(i,k)*B(k,j) of Algorithm 1
 * contributes G(i,j)*B(k,j) to dA(i,k) and A(i,k)*G(i,j) to dB(k,j)):
 *   dA = (G * B^T) on pattern(A),   dB = (A^T * G) on pattern(B).
 * A and B: the operands of the last spgemm_symbolic (same structure, current
 * values).  G: m x k with C's structure -- row_ptr and col_idx of the C the
 * numeric phase wrote (sorted columns), values = dL/dC.  dA_values (nnz(A))
 * and dB_values (nnz(B)) are device arrays of the common dtype, overwritten;
 * either may be NULL to skip it.  Never blocks the host.  Errors: INVALID_ARG,
 * NOT_READY, STRUCTURE_MISMATCH, HIP (a G column missing from C's row is
 * reported by spg_check_errors as STRUCTURE_MISMATCH). */
spg_status spgemm_backward(spg_handle h, const spg_csr *A, const spg_csr *B, const spg_csr *G,
                           void *dA_values, void *dB_values);

/* Masked product (graph analytics on the product's structure, Background
 * section; triangle counting, Compression subsection): for every stored
 * entry (i, j) of the mask M (m x k, values not read),
 *     out[e] = sum over k with A(i,k) and B(k,j) stored of A(i,k) * B(k,j)
 * (0 where no such k exists), or with structural = 1 the NUMBER of such k
 * (values of A and B not read, may be NULL): e.g. with A = B = M = L, the
 * strictly lower triangle of a graph's adjacency, out sums to the graph's
 * triangle count.  out: device array of M.nnz entries of A's dtype, in M's
 * entry order (M's rows may be unsorted, without duplicate columns).  FP32
 * inputs are accumulated in FP64 and rounded once.  No symbolic phase is
 * needed and the handle's plan is left as it was.  Blocks the host (twice:
 * to size the launches and to report malformed input).  Errors:
 * INVALID_ARG (malformed CSR, bad dtype), DIM_MISMATCH, OUT_OF_MEMORY, HIP. */
spg_status spgemm_masked(spg_handle h, const spg_csr *A, const spg_csr *B, const spg_csr *M, void *out,
                         int structural);

/* Synchronise the handle's stream and report errors the device found since
 * the last check: STRUCTURE_MISMATCH if a numeric call met a row whose size
 * differs from the plan (the caller changed A or B's structure in place; that
 * row was left unwritten), OUT_OF_MEMORY if a level-2 table did not fit its
 * arena slice.  Clears the device flags.  spgemm_numeric itself never blocks,
 * so this is how a caller confirms a numeric result. */
spg_status spg_check_errors(spg_handle h);

/* Numeric phase for the rows [row_begin, row_end) of C only (a row panel:
 * for products whose C does not fit device memory at once, the caller
 * computes C in panels into reused buffers).  Same plan and operands as
 * spgemm_numeric; the panel's entries (C.row_ptr[row_end] - C.row_ptr[row_begin]
 * of them, C.row_ptr from the symbolic phase) are written to C_col_idx[0..)
 * and C_values[0..) (device arrays, dtype of A and B).  Never blocks the host.
 * Errors as spgemm_numeric, INVALID_ARG for a bad row range. */
spg_status spgemm_numeric_rows(spg_handle h, const spg_csr *A, const spg_csr *B, int64_t row_begin,
                               int64_t row_end, int32_t *C_col_idx, void *C_values);

/* Statistics of the last symbolic phase (host struct). */
spg_status spg_get_stats(spg_handle h, spg_stats *out);

/* Static text for a status code. */
const char *spg_status_string(spg_status s);

/* Text of the last error on this handle ("" if none).  Valid until the next
 * call on the handle. */
const char *spg_last_error(spg_handle h);

/* Library version string. */
const char *spg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPGEMM_MI355X_H */
