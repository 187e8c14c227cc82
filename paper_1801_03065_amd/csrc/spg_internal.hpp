// Internal declarations of the gfx950 SpGEMM library: argument blocks of the
// kernels, 64-lane wavefront primitives and the host-side launch wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>

namespace spg {

constexpr int WAVE = 64;  // CDNA wavefront width
constexpr int XCDS = 8;   // accelerator complex dies on the MI355X
constexpr int WG_BIG = 256;
// Lanes of the bit-window workgroup kernels (one heavy row per workgroup):
// their window (up to 128 KB of LDS) leaves room for one workgroup per CU, so
// the workgroup is large to keep enough loads in flight.
constexpr int DG_WG = 1024;

// Per row of B: number of entries, number of distinct column-set words
// (col >> 5) after compression, lowest and highest word touched.
struct BRow {
    int32_t len, lenc, wmin, wmax;
};

// Kernel kinds a row of C can be assigned to (one persistent launch each).
enum Kind : int {
    K_EMPTY = 0,  // no multiplications: row size 0
    K_DW = 1,     // bit-window dense accumulator, one wavefront per row
    K_HW = 2,     // LDS linear-probing hash, one wavefront per row
    K_DG = 3,     // bit-window dense accumulator, one 256-lane workgroup per row, values in HBM
    K_HL = 4,     // two-level hash: LDS level 1 + HBM level 2, one workgroup per row
    K_WH = 5,     // word hash + ordered summary, one wavefront per row (numeric)
    K_SR = 6,     // short rows: a team of T <= 64 lanes per row, several rows per wavefront
    K_PL = 7,     // numeric on the symbolic phase's stored row structure, one wavefront per row
    NK = 8
};

// Global counters written by the analysis kernels (zeroed per symbolic call).
struct DevStats {
    unsigned long long fm, fmc, maxrf, maxrfc, nnzbc;
    unsigned long long fmb, fmcb;  // flops (raw / compressed) of rows beyond the short-row limit
    unsigned long long maxnnza;    // longest row of A
    unsigned long long nnzc;
    int bad_input;    // malformed CSR (row_ptr not monotone / not ending at nnz, column out of range)
    int unsorted;     // B rows whose columns are not sorted
    int bad_window;   // unsorted B rows too wide for the LDS window
    int mismatch;     // numeric: row size differs from the plan
    int overflow;     // level-2 arena exhausted
    int comp;         // the analysis chose compressed B (Compression subsection rule)
    unsigned long long sdigest;  // structure fingerprint of the symbolic phase's operands
    long long kcount_sym[NK];
    long long kcount_num[NK];
    long long kcount_heavy[NK];
    int kmax_sym[NK][3];   // per kind: max window words, max bound, max touched words
    int kmax_num[NK][3];   // per kind: max window words, max row size, max touched words
    int kmax_heavy[NK][3]; // numeric, rows at or above the FP64 flop threshold
};

// Limits of the kernel kinds (entries, not bytes).
constexpr int DW_NW_MAX = 2048;   // window words of the wavefront dense kernel (65536 columns)
constexpr int DW_R_MAX = 1024;    // row size of the wavefront dense kernel
constexpr int HW_KEYS_MAX = 1024; // distinct keys of the wavefront hash (table 2x)
constexpr int DG_NW_MAX = 32768;  // window words of the workgroup dense kernel (2^20 columns)
constexpr int WH_NW_MAX = 32768;  // window words of the word-hash kernel (summary of 1024 words)
constexpr int WH_R_MAX = 1024;    // row size of the word-hash kernel
constexpr int WH_T_MAX = 512;     // touched words of the word-hash kernel (table 2x)
constexpr int SR_F_MAX = 64;      // multiplications of a short row (one per lane of its team)
constexpr int PL_CAP = 64;        // stored (word, bits) pairs per row (one per lane)
constexpr int PL_NW_MAX = 8192;   // window words of the stored-structure kernel (byte map in LDS)
constexpr int PL_R_MAX = 2048;    // row size of the stored-structure kernel
constexpr int SG_NW = 4096;       // column-set words of one heavy-row segment (aligned groups)
constexpr int SG_CAP = 4096;      // entries of one heavy-row segment (LDS values)
constexpr int SG_CUT = SG_CAP - 32;  // a segment starts at the word holding each multiple of this

// ------------------------------------------------------------ argument blocks
struct RowSet {
    const int32_t *rows;   // permutation of row ids, grouped by kind
    const int64_t *koff;   // koff[kind] .. koff[kind+1] is this kind's slice
    const int64_t *range;  // when set: range[2*kind] .. range[2*kind+1] instead (row panels)
    int kind;
    int32_t *queue;        // XCDS dynamic-schedule counters (zeroed before launch)
};

__device__ __forceinline__ void rs_bounds(const RowSet &rs, int64_t &lo, int64_t &hi) {
    if (rs.range) {
        lo = rs.range[2 * rs.kind];
        hi = rs.range[2 * rs.kind + 1];
    } else {
        lo = rs.koff[rs.kind];
        hi = rs.koff[rs.kind + 1];
    }
}

struct SymArgs {
    const int64_t *arp;
    const int32_t *aci;
    const int64_t *brp;    // raw B structure
    const int32_t *bci;
    const int64_t *bcrp;   // compressed B (nullptr when not compressed)
    const uint2 *bcw;      // compressed B: (column-set word, bits) per entry
    const int2 *rwin;      // per row: lowest / highest column-set word
    int32_t *row_nnz;
    int32_t *row_words;    // touched column-set words per row (exact, or a bound)
    RowSet rs;
    int nw_max;            // LDS window words for this launch
    int ts;                // hash table slots (power of two) for hash kinds
    int lg_gs;             // log2 lanes per B row (Thread-Parallel group)
    int l1_slots;          // two-level hash: level-1 slots
    uint32_t *l2_keys;     // two-level hash arena (keys / masks), per workgroup
    uint32_t *l2_vals;
    int64_t l2_cap;        // slots per workgroup in the arena
    const int64_t *plan_off;  // bit-window rows: where the row's (word, bits) pairs go
    const int32_t *plan_len;  // room for pairs per row (0: none stored)
    uint2 *plan;              // nullptr: no pairs stored
    int b32;                  // nnz(B) < 2^30: B entries addressed with 32-bit byte offsets
    int64_t nnzb;             // nnz(B): gathers clamp their offsets to its last entry
    DevStats *st;
};

template <typename VT>
struct NumArgs {
    const int64_t *arp;
    const int32_t *aci;
    const VT *aval;
    const int64_t *brp;
    const int32_t *bci;
    const VT *bval;
    const int64_t *bcrp;
    const uint2 *bcw;      // compressed B: (column-set word, bits) per entry
    const int2 *rwin;
    const int64_t *coff;   // C row offsets (plan copy, int64)
    int32_t *cci;          // written at coff[i] - coff[cbase_row] (0 when cbase_row < 0)
    VT *cval;
    int64_t cbase_row;
    RowSet rs;
    RowSet rs2;               // K_DG (segmented, FP64): a second row set taken first in the same launch (rows unset: none)
    int nw_max;
    int r_max;
    int ts;
    int lg_gs_or;          // lanes per compressed B row in the structure pass
    int lg_gs;             // lanes per B row in the product pass
    int l1_slots;
    void *arena;           // HBM scratch: dense values (K_DG) or level-2 tables (K_HL)
    int64_t arena_cap;     // entries per workgroup
    const int64_t *plan_off;  // K_PL: the row's stored (word, bits) pairs
    const uint2 *plan;
    const int32_t *row_words; // K_PL: number of pairs of the row
    const int32_t *plan_len;  // K_DG (segmented): room in plan per row
    const uint8_t *sym_kind;  // K_DG (segmented): rows of symbolic kind K_DG with room hold a segment list
    int32_t *sg_cur;          // K_DG (segmented): per workgroup, sg_cap A entries x 3 int32 (cursor, run end, B row end)
    int sg_cap;               //   (nullptr / 0: runs found by two searches per segment)
    int b32;               // nnz(B) * 8 < 2^32: B entries addressed with 32-bit offsets
    int64_t nnzb;          // nnz(B): gathers clamp their offsets to its last entry
    const int64_t *map_off;   // reuse: per row, where its products' ranks start in map
    uint16_t *map;            // reuse: rank in C's row per multiplication
    int values_only;          // K_PL: C's columns are already in place, write values only
    DevStats *st;
};

template <typename VT>
struct BwdArgs {
    int64_t m, nnza, nnzb;
    const int64_t *arp;
    const int32_t *aci;
    const VT *aval;
    const int64_t *brp;
    const int32_t *bci;
    const VT *bval;
    const int64_t *coff;   // C row offsets (plan)
    const int32_t *gci;    // C's sorted columns (pattern of G)
    const VT *gval;        // dL/dC on pattern(C)
    VT *dA;                // nnz(A) or nullptr
    VT *dB;                // nnz(B) or nullptr
    int lg_gs;
    DevStats *st;
};

// One matrix of a batch: where its structure / values live and where they go
// in the concatenated (block-diagonal) product.
struct BatchDesc {
    const void *rp;        // row_ptr (input), or C_i.row_ptr (output)
    const int32_t *ci;
    const void *vals;      // values (gather source / scatter target)
    int64_t nrows, ncols, nnz;
    int64_t row_off;       // first row in the concatenation
    int64_t nnz_off;       // first entry in the concatenation
    int32_t col_add;       // added to column indices (A: B's row offset)
    int32_t rp64;
    int32_t cls;           // product class of the batch autotuner (A descriptors)
    int32_t pad;
};

// ------------------------------------------------------------ device helpers
__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}
__device__ __forceinline__ long long wave_sum64(long long v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d));
    return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d));
    return v;
}
// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        int t = __shfl_up(v, d);
        if (l >= d) v += t;
    }
    return v;
}
// Inclusive prefix sum over the 64 lanes with DPP lane moves (row shifts
// inside each 16-lane row, then row broadcasts of lane 15 and lane 31): no
// address registers, unlike a shuffle through ds_bpermute.
__device__ __forceinline__ int wave_scan_dpp(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
    return v;
}
__device__ __forceinline__ long long wave_incl_scan64(long long v) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        long long t = __shfl_up(v, d);
        if (l >= d) v += t;
    }
    return v;
}
// Inclusive prefix sum inside teams of 2^LG lanes with DPP lane moves (row
// shifts inside each 16-lane row, masked at team edges below 16 lanes; row
// broadcasts of lane 15 / lane 31 for teams of 32 / 64): no shuffle address
// arithmetic.
template <int LG>
__device__ __forceinline__ int team_scan(int v, int q) {
    if (LG >= 1) { const int t = __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false); v += (LG >= 4 || q >= 1) ? t : 0; }
    if (LG >= 2) { const int t = __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false); v += (LG >= 4 || q >= 2) ? t : 0; }
    if (LG >= 3) { const int t = __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false); v += (LG >= 4 || q >= 4) ? t : 0; }
    if (LG >= 4) v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);
    if (LG >= 5) v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
    if (LG >= 6) v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
    return v;
}
// Set bits of word w below bit b (b in [0, 31]): one bit-field extract of the
// low b bits (width 0 gives 0) and a popcount.
__device__ __forceinline__ int bits_below(uint32_t w, int b) {
    return __popc(__builtin_amdgcn_ubfe(w, 0u, (uint32_t)b));
}
// Number of set bits of a 64-bit lane mask below this lane.
__device__ __forceinline__ int mbcnt(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}
__device__ __forceinline__ int read_first(int v) { return __builtin_amdgcn_readfirstlane(v); }
// A wavefront-uniform 64-bit value moved to scalar registers.
__device__ __forceinline__ int64_t uni64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Load base[idx] with a 32-bit byte offset (idx * sizeof(T) < 2^32): the
// compiler then addresses with the base in SGPRs plus one 32-bit VGPR offset
// (one shift per gathered element instead of 64-bit address arithmetic).
template <typename T>
__device__ __forceinline__ T ld32(const T *base, uint32_t idx) {
    return *(const T *)((const char *)base + (uint32_t)(idx * (uint32_t)sizeof(T)));
}

// LDS hand-off between the lanes of a one-wavefront workgroup: wait for this
// wavefront's outstanding LDS operations only (lgkmcnt(0); vector-memory loads
// stay in flight) and keep the compiler from moving memory operations across.
// A workgroup barrier would also wait for every outstanding global load,
// including loads prefetched for the next row.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt = max, expcnt = max, lgkmcnt = 0
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Static, XCD-aware slice of [lo, hi) for this workgroup: the grid is a
// multiple of 8 and workgroup b runs on die b % 8, so each die walks one
// contiguous eighth of the rows (its L2 then holds that eighth's B rows),
// and the workgroups of one die interleave row by row inside it.
struct Slice {
    int64_t idx, end, step;
};
__device__ __forceinline__ Slice xcd_slice(int64_t lo, int64_t hi, int per_wg = 1, int sub = 0) {
    const int G = gridDim.x, b = blockIdx.x;
    const int x = b % XCDS, slot = b / XCDS, S = G / XCDS;
    const int64_t n = hi - lo;
    Slice s;
    const int64_t beg = lo + n * x / XCDS;
    s.end = lo + n * (x + 1) / XCDS;
    s.idx = beg + (int64_t)slot * per_wg + sub;
    s.step = (int64_t)S * per_wg;
    return s;
}

// Dynamic XCD-aware queue: a workgroup first drains its own die's eighth,
// then the other dies' eighths.  Returns -1 when everything is taken.
__device__ __forceinline__ int64_t xcd_grab(int32_t *queue, int64_t lo, int64_t hi, int &x) {
    const int64_t n = hi - lo;
    for (int k = 0; k < XCDS; ++k) {
        const int64_t beg = lo + n * x / XCDS, end = lo + n * (x + 1) / XCDS;
        if (beg < end) {
            const int64_t t = beg + atomicAdd(&queue[x], 1);
            if (t < end) return t;
        }
        x = (x + 1) % XCDS;
    }
    return -1;
}

// ------------------------------------------------------------ host launchers
struct LaunchCfg {
    hipStream_t stream;
    int grid;  // persistent workgroups (multiple of 8); 0 = all resident workgroups
    int cus;   // compute units of the device
};

// Per row of B: length, distinct column-set words, word window, sortedness
// (uflag, and the list of unsorted rows); columns out of [0, ncols) raise the
// malformed-input flag.
hipError_t launch_brow(int64_t n, int64_t nnz, int64_t ncols, const int64_t *brp, const int32_t *bci, BRow *out,
                       int32_t *unsorted_list, uint8_t *uflag, DevStats *st, hipStream_t s);
hipError_t launch_brow_unsorted(const int32_t *list, const int *count, const int64_t *brp, const int32_t *bci,
                                BRow *out, DevStats *st, hipStream_t s);
// The compression kernels and the scan take `enable` (device flag, nullable):
// they do nothing when it reads 0.
hipError_t launch_compress_sorted_flags(int64_t n, int64_t nnz, const int64_t *brp, const int32_t *bci, const BRow *bi,
                                        const uint8_t *unsorted, const int64_t *bcrp, uint2 *bcw,
                                        const int *enable, hipStream_t s);
hipError_t launch_compress_unsorted(const int32_t *list, const int *count, const int64_t *brp,
                                    const int32_t *bci, const BRow *bi, const int64_t *bcrp, uint2 *bcw,
                                    const int *enable, hipStream_t s);
// Per-block partials of the rowinfo reduction (folded by a one-workgroup
// kernel): RED_ELEMS int64 of device scratch.
constexpr int RED_ELEMS = 16384;
// Row flops, windows, A column checks; the totals are folded into st, where
// the compression decision is taken (comp_opt -1 rule / 0 / 1).
hipError_t launch_rowinfo(int64_t m, int64_t n, const int64_t *arp, const int32_t *aci, const BRow *bi,
                          int64_t *rflops, int64_t *rflopsc, int2 *rwin, DevStats *st, long long *part, int comp_opt,
                          int selector, double cf_threshold, hipStream_t s);
// Row pointers of A and B (int32 or int64) copied to int64, clamped to
// [0, nnz], with a monotonicity / end check into *bad: one launch for both.
hipError_t launch_copy_rp(int64_t n1a, const void *srca, int is64a, int64_t nnza, int64_t *dsta, int64_t n1b,
                          const void *srcb, int is64b, int64_t nnzb, int64_t *dstb, int *bad, hipStream_t s);

// Exclusive scan: out[0..n] (n+1 entries) of in[0..n), int64 result.
// tmp must hold scan_tmp_elems(n) int64.
int64_t scan_tmp_elems(int64_t n);
// in[i * stride] (e.g. one field of an array of structs)
hipError_t launch_scan_i32s(int64_t n, const int32_t *in, int stride, int64_t *out, int64_t *tmp, const int *enable,
                            hipStream_t s);
hipError_t launch_scan_i32(int64_t n, const int32_t *in, int64_t *out, int64_t *tmp, hipStream_t s);
hipError_t launch_store_rp(int64_t n1, const int64_t *src, void *dst, int is64, hipStream_t s);

// Classification parameters shared by host and device.
struct ClassParams {
    int phase;          // 0 symbolic, 1 numeric
    int accumulator;    // spg_accumulator
    int compressed;
    int dw_nw_max, dw_r_max, hw_keys_max, dg_nw_max, wh_nw_max, wh_r_max, wh_t_max;
    int sample_stride;  // numeric: only rows i with i % stride == 0 get a kind (others: empty)
    // numeric, FP64-accumulated rows: a row is "heavy" when its flops reach
    // heavy_flops (> 0) or its A row has more than heavy_alen (> 0) entries
    // (each entry of C then sums more than heavy_alen products); with split
    // set only the rows on the side named by `heavy` get a kind (others: empty)
    long long heavy_flops, heavy_alen;
    const int64_t *arp;  // A's row offsets (int64), read when heavy_alen > 0
    int split;
    int heavy;          // numeric: counts / maxima go to the heavy-row set
    int sr_f_max;       // selector: rows with at most this many multiplications are short rows (0: off)
    int plan_cap;       // stored row structure: pairs per row (0: off)
    int32_t *plan_len;  // symbolic: room for pairs per row (written); numeric: read
    const uint8_t *sym_kind;  // numeric: kind of each row in the symbolic phase
    const int *comp_flag;     // symbolic: when set, compression as decided on the device (else `compressed`)
    int32_t *words_out;       // symbolic: zeroed for every row (touched words, filled by the structure kernels)
    const int *unsorted;      // when set: segments only if it reads 0 (rows of B with unsorted columns)
    const uint8_t *row_cls;  // numeric, batch classes: only rows with row_cls[i] == cls get a kind
    int cls;
    int sg;             // heavy rows in segments (B's rows sorted): symbolic K_DG rows that may
                        // need several segments get room for a list; numeric K_DG rows must
                        // have one or fit a single segment
};
// Classification of every row into a kind, with per-kind counts and maxima
// per classify workgroup (tmp, part_tmp_elems(m)); launch_partition then folds
// them into st (counts, maxima) and koff (offsets per kind) and writes the
// rows grouped by kind.  (koff is only filled here when there are no rows.)
hipError_t launch_classify(int64_t m, const int64_t *rflops, const int64_t *rflopsc, const int2 *rwin,
                           const int32_t *row_nnz, const int32_t *row_words, ClassParams p, uint8_t *kind,
                           int32_t *row_nnz_out, DevStats *st, int64_t *tmp, int64_t *koff, hipStream_t s);
int64_t part_tmp_elems(int64_t m);
hipError_t launch_partition(int64_t m, const uint8_t *kind, int32_t *perm, const int64_t *tmp, int64_t *koff,
                            int phase, int heavy, DevStats *st, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_kind_ranges(const int32_t *perm, const int64_t *koff, int64_t rb, int64_t re, int64_t *range,
                              hipStream_t s);

// Core kernels.
hipError_t launch_sym_dw(const SymArgs &a, const LaunchCfg &c);
hipError_t launch_sym_hw(const SymArgs &a, const LaunchCfg &c);
hipError_t launch_sym_dg(const SymArgs &a, const LaunchCfg &c);
hipError_t launch_sym_hl(const SymArgs &a, const LaunchCfg &c);
// Short rows: teams of 2^lg_t lanes; rows = number of rows in the kind (grid sizing).
hipError_t launch_sym_sr(const SymArgs &a, int lg_t, const LaunchCfg &c, int64_t rows);

// acc: 0 native, 1 compensated pair (FP32), 2 FP64 accumulation (FP32)
template <typename VT>
hipError_t launch_num_dw(const NumArgs<VT> &a, int acc, const LaunchCfg &c);
template <typename VT>
hipError_t launch_num_hw(const NumArgs<VT> &a, int acc, const LaunchCfg &c);
template <typename VT>
hipError_t launch_num_dg(const NumArgs<VT> &a, int acc, const LaunchCfg &c);
template <typename VT>
hipError_t launch_num_hl(const NumArgs<VT> &a, int acc, const LaunchCfg &c);
// Heavy rows in column segments (sorted B): the segment lists are in a.plan.
template <typename VT>
hipError_t launch_num_sg(const NumArgs<VT> &a, int acc, int acc2, const LaunchCfg &c);  // acc2: rows of a.rs2
int sg_resident_grid(int acc, int acc2, bool dbl, int cus);
template <typename VT>
hipError_t launch_num_wh(const NumArgs<VT> &a, int acc, const LaunchCfg &c);
template <typename VT>
hipError_t launch_num_pl(const NumArgs<VT> &a, int acc, const LaunchCfg &c);
size_t lds_num_pl(int nw_max, int r_max, int acc_bytes);
template <typename VT>
hipError_t launch_num_sr(const NumArgs<VT> &a, int acc, int lg_t, const LaunchCfg &c, int64_t rows);
size_t lds_num_wh(int ts, int nw_max, int r_max, int acc_bytes);
template <typename VT>
hipError_t launch_backward(const BwdArgs<VT> &a, const LaunchCfg &c);
// Reuse on a known structure: position maps of a kind's rows from C's sorted
// columns (teams of 2^lgt lanes, 2^lgs lanes per B row), and the values of
// those rows on their maps (LDS rows of a.r_max entries per team).
hipError_t launch_posmap(const NumArgs<double> &a, const int32_t *cci, int lgt, int lgs, const LaunchCfg &c,
                         int64_t rows);
template <typename VT>
hipError_t launch_num_map(const NumArgs<VT> &a, int acc, int lgt, int lgs, const LaunchCfg &c, int64_t rows);
size_t lds_num_map(int r_max, int lgt, int acc_bytes);
// LL hashmap, Thread-Sequential groups of 2^lgg lanes per row, unsorted rows:
// a.ts buckets (power of two), a.r_max slots (>= the largest row of the kind).
template <typename VT>
hipError_t launch_num_ll(const NumArgs<VT> &a, int acc, int lgg, const LaunchCfg &c, int64_t rows);
size_t lds_num_ll(int hb, int cap, int lgg, int acc_bytes);
// Masked product: C = (A * B) on M's pattern, or path counts (structural).
template <typename VT>
struct MaskArgs {
    const int64_t *arp;
    const int32_t *aci;
    const VT *aval;        // nullptr in structural mode
    const int64_t *brp;
    const int32_t *bci;
    const VT *bval;
    const int64_t *mrp;
    const int32_t *mci;
    VT *out;               // nnz(M), M's entry order
    const int32_t *rows;   // rows of this launch
    int64_t nrows;
    int64_t n, k;          // A's columns < n, B's and M's < k
    int lg_gs;             // lanes per B row
    int structural;
    void *arena;           // workgroup rows: 12 B per slot per workgroup
    int64_t arena_cap;     // slots per workgroup (power of two >= 2 x longest mask row)
    int *bad;              // bit 0: a column out of range, bit 1: arena too small
};
constexpr int MW_MAX = 512;  // mask row length of the wavefront kind
hipError_t launch_mask_class(int64_t m, const int64_t *arp, const int64_t *mrp, int mw_max, int32_t *rows1,
                             int32_t *rows2, int *cnt, hipStream_t s);
template <typename VT>
hipError_t launch_mask_w(const MaskArgs<VT> &a, int lg, int mmax, const LaunchCfg &c);
template <typename VT>
hipError_t launch_mask_g(const MaskArgs<VT> &a, const LaunchCfg &c);
size_t lds_mask_w(int lg, int mmax);

// Kinds whose rows get position maps: every row fits 1024 entries (16-bit ranks).
__host__ __device__ inline bool map_kind(int k) { return k == K_SR || k == K_WH || k == K_HW || k == K_DW; }
// out[i] = multiplications of row i if it gets a map, else 0 (kind_heavy nullable).
hipError_t launch_map_rows(int64_t m, const uint8_t *kind, const uint8_t *kind_heavy, const int64_t *rflops,
                           int32_t *out, hipStream_t s);

// Operand structure of one product (caller's arrays) for the fingerprint.
struct StructRef {
    const void *arp, *brp;
    const int32_t *aci, *bci;
    int64_t m, n, nnza, nnzb;
    int arp64, brp64;
};
// Digest of A's and B's row pointers and columns: check = 0 stores it in
// *ref, check = 1 compares and counts a mismatch (device-side, no host sync).
// part: at least 1024 uint64 of scratch.
hipError_t launch_struct_digest(const StructRef &s, unsigned long long *part, unsigned long long *ref, int check,
                                int *mismatch, hipStream_t st);

hipError_t launch_batch_struct(const BatchDesc *d, int count, int64_t max_work, int64_t *dst_rp, int32_t *dst_ci,
                               int *bad, hipStream_t s);
hipError_t launch_batch_gather(const BatchDesc *d, int count, int64_t max_nnz, void *dst, int bytes,
                               hipStream_t s);
hipError_t launch_batch_scatter(const BatchDesc *d, int count, int64_t max_nnz, const void *src, int bytes,
                                hipStream_t s);
hipError_t launch_batch_rp_out(const BatchDesc *d, int count, int64_t max_rows, const int64_t *coff,
                               hipStream_t s);
hipError_t launch_batch_bounds(const BatchDesc *d, int count, const int64_t *coff, int64_t *out, hipStream_t s);
// row_cls[row_off_i + r] = d[i].cls for the rows of every product
hipError_t launch_batch_row_class(const BatchDesc *d, int count, int64_t max_rows, uint8_t *row_cls, hipStream_t s);
// kind[i] = kind_cls[row_cls[i] * m + i]: the classes' kinds merged into one array
hipError_t launch_kind_merge(int64_t m, const uint8_t *row_cls, const uint8_t *kind_cls, uint8_t *kind, hipStream_t s);

// LDS bytes of the core kernels for given limits.
size_t lds_sym_dw(int nw_max);
size_t lds_sym_hw(int ts);
size_t lds_sym_dg(int nw_max);
size_t lds_sym_hl(int l1_slots);
size_t lds_num_dw(int nw_max, int r_max, int acc_bytes, int val_bytes);
size_t lds_num_hw(int ts, int acc_bytes);
size_t lds_num_dg(int nw_max);
size_t lds_num_hl(int l1_slots, int acc_bytes);

int dg_resident_grid(int acc, bool dbl, size_t lds, int cus);
int hl_resident_grid(int acc, bool dbl, size_t lds, int cus);

}  // namespace spg
