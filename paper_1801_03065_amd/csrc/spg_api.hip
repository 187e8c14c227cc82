// Host side of the C ABI: the handle, the symbolic plan kept for reuse, and
// the orchestration of the two phases (Algorithm 2):
//   symbolic: row_ptr copies -> B row statistics -> per-row flops / windows
//             and, on the device, the compression decision (compress B if it
//             removes more than 15% of the flops) -> compressed B -> rows
//             classified by kernel kind -> [host reads the statistics and
//             per-kind sizes] -> room for stored structure -> one persistent
//             launch per kind -> scan -> numeric classification -> [host
//             reads nnz(C)]
//   numeric:  one persistent launch per kind, no host synchronisation.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "spg_accum.hpp"
#include "spg_internal.hpp"
#include "spgemm.h"

using namespace spg;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    template <typename T>
    T *as() const { return (T *)p; }
};

struct Fingerprint {
    int64_t m = -1, n = -1, k = -1, nnza = -1, nnzb = -1;
    const void *arp = nullptr, *brp = nullptr;
    const int32_t *aci = nullptr, *bci = nullptr;
    int arpt = 0, brpt = 0;
};

}  // namespace

// Scratch of spgemm_numeric_noalloc: a file-scope device array, one instance
// per GPU the library runs on, held until the process ends.  In host code
// `scratch` names a host-side stand-in; its device address comes from
// hipGetSymbolAddress, taken once per device at spg_create with that device
// current, and only that address is passed to kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
namespace {
constexpr int SCR_MAX_DEV = 64;
std::mutex g_scr_mu;
void *g_scr_ptr[SCR_MAX_DEV] = {};

hipError_t scratch_address(int dev, void **out) {
    *out = nullptr;
    if (dev < 0 || dev >= SCR_MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scr_mu);
    if (!g_scr_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scr_ptr[dev] = p;
    }
    *out = g_scr_ptr[dev];
    return hipSuccess;
}
}  // namespace

struct spg_handle_s {
    hipStream_t stream = nullptr;
    spg_options opt{};
    int device = 0, cus = 0;
    size_t lds_max = 65536;
    int dg_nw_max = DG_NW_MAX;
    std::string err;

    // plan
    bool ready = false;
    Fingerprint fp;
    int64_t nnzc = 0;
    bool compressed = false;
    double avg_len = 1, avg_len_c = 1;  // B entries (raw / compressed) read per A entry
    DevStats *hst = nullptr;            // pinned host copy of the device counters
    int64_t *hkoff = nullptr;           // pinned: [0] nnz(C), [1] stored-structure pairs
    bool planned = false;               // the symbolic phase stored row structure (K_PL rows)
    bool sg_mode = false;               // heavy rows run in segments (B's rows sorted)
    bool segmented = false;             // the symbolic phase wrote segment lists into plan
    spg_stats stats{};

    DevBuf arp64, brp64, binfo, ulist, uflag, bcrp, bcw, rflops, rflopsc, rwin, row_nnz, coff, kind_sym,
        kind_num, perm_sym, perm_num, koff_sym, koff_num, tmp, dstats, red, queue, plan_len, plan_off, plan, arena, l2k, l2v, blens, row_words;
    size_t arena_bytes_zeroed = 0;
    const int32_t *aci_used = nullptr, *bci_used = nullptr;  // column arrays the kernels read
    ClassParams cparams{};                                   // classification of the last symbolic phase
    int lg_num = 4;                                          // log2 lanes per B row, numeric phase
    bool tuned = false;
    DevBuf kind_tmp, perm_tmp, koff_tmp, krange, kind_heavy, perm_heavy, koff_heavy, krange_heavy, sgcur;
    bool heavy_split = false;  // the plan keeps FP64-accumulated rows in their own kind lists
    bool verify = false;       // numeric / backward check the operands' structure fingerprint
    DevBuf mflops, map_off, map;  // reuse: per-row mapped multiplications, map offsets, ranks
    DevBuf mk_arp, mk_brp, mk_mrp, mk_rows, mk_cnt, mk_arena;  // masked product
    bool maps_built = false;      // position maps taken for this plan (maps_ok: they exist)
    long long kc_nomap[NK] = {};  // scratch: kind counts with the mapped kinds removed
    bool maps_ok = false;
    void *scr = nullptr;       // this device's static scratch array (device address)
    bool noalloc = false;      // the current call carves its scratch from scr instead of hipMalloc
    bool values_only = false;  // the current call writes C's values only (structure known)
    int lg_map_cur = 2;        // lanes per B row (log2) of the position-map kernels in the current launch set
    int num_policy = 0;        // accumulator policy of the numeric classification (SPG_ACC_*)
    // batch plans: products fall into classes by the average row size of C_i,
    // and the autotuner picks (policy, lanes per B row) per class; each class
    // then has its own classification, row lists and LDS sizing
    int ncls = 0;              // 0: one launch set for the whole plan
    bool cls_tuned = false;
    int cls_rows[4] = {}, cls_lg[4] = {}, cls_pol[4] = {};
    double cls_avg_b[4] = {};  // average B row length of the class's products
    long long cls_kc[4][NK] = {};
    int cls_km[4][NK][3] = {};
    DevBuf row_cls, kind_cls, perm_cls, koff_cls;
    StructRef sref{};          // the symbolic phase's operand structure (caller's arrays)

    struct Batch {
        int count = 0;
        std::vector<BatchDesc> a, b, c;    // host copies (c: row_ptr outputs of C_i)
        std::vector<int64_t> c_off, c_nnz; // C_i's entries in the concatenation
        int64_t rows = 0, nnza = 0, nnzb = 0, max_rows = 0, max_nnza = 0, max_nnzb = 0, max_nnzc = 0;
        DevBuf aci, bci, desc, astage, bstage, cci, cval;
    } batch;
};

namespace {

spg_status fail(spg_handle h, spg_status s, const std::string &msg) {
    if (h) h->err = msg;
    return s;
}

spg_status hip_fail(spg_handle h, hipError_t e, const char *where) {
    return fail(h, SPG_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr)                                         \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return hip_fail(h, _e, #expr); \
    } while (0)

hipError_t ensure(DevBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.p && b.cap >= bytes) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        if (e != hipSuccess) return e;
    }
    b.p = nullptr;
    b.cap = 0;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        return e;
    }
    b.cap = bytes;
    return hipSuccess;
}

void release(DevBuf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

// Team size of the short-row kernel: the smallest power of two >= the largest
// multiplication count among its rows, at least 8 lanes.
static int sr_lg(int max_flops) {
    int lg = 3;
    while ((1 << lg) < max_flops && lg < 6) ++lg;
    return lg;
}

int lg_group(double avg) {
    // lanes per B row: the average length rounded up to a power of two, 4..64
    int lg = 2;
    while (lg < 6 && (double)(1 << lg) < avg) ++lg;
    return lg;
}

// lanes per B row of the position-map kernels: the average B row length
// rounded up to a power of two, 1..64 (products on maps carry no structure
// work, so a B row of one entry gets one lane)
static int lg_map(double avg) {
    int lg = 0;
    while (lg < 6 && (double)(1 << lg) < avg) ++lg;
    return lg;
}

int pow2_at_least(int64_t v, int lo) {
    int64_t p = lo;
    while (p < v) p <<= 1;
    return (int)p;
}

spg_status check_csr(spg_handle h, const spg_csr *M, const char *name, bool need_values) {
    if (!M) return fail(h, SPG_ERR_INVALID_ARG, std::string(name) + " is NULL");
    if (M->nrows < 0 || M->ncols < 0 || M->nnz < 0)
        return fail(h, SPG_ERR_INVALID_ARG, std::string(name) + ": negative size");
    if (M->ncols > INT32_MAX || M->nrows > INT32_MAX - 1)
        return fail(h, SPG_ERR_UNSUPPORTED, std::string(name) + ": more than 2^31-1 rows or columns");
    if (M->rp_type != SPG_I32 && M->rp_type != SPG_I64)
        return fail(h, SPG_ERR_INVALID_ARG, std::string(name) + ": bad rp_type");
    if (M->rp_type == SPG_I32 && M->nnz > INT32_MAX)
        return fail(h, SPG_ERR_INDEX_OVERFLOW, std::string(name) + ": nnz exceeds int32 row_ptr");
    if (!M->row_ptr) return fail(h, SPG_ERR_INVALID_ARG, std::string(name) + ": row_ptr is NULL");
    if (M->nnz > 0 && !M->col_idx) return fail(h, SPG_ERR_INVALID_ARG, std::string(name) + ": col_idx is NULL");
    if (need_values) {
        if (M->dtype != SPG_F64 && M->dtype != SPG_F32)
            return fail(h, SPG_ERR_INVALID_ARG, std::string(name) + ": bad dtype");
        if (M->nnz > 0 && !M->values) return fail(h, SPG_ERR_INVALID_ARG, std::string(name) + ": values is NULL");
    }
    return SPG_OK;
}

// Device counters -> pinned host copy (blocks the host).
spg_status pull_stats(spg_handle h) {
    HIPCHK(hipMemcpyAsync(h->hst, h->dstats.p, sizeof(DevStats), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return SPG_OK;
}

}  // namespace

extern "C" {

const char *spg_version(void) { return "spgemm-mi355x 0.1 (gfx950)"; }

const char *spg_status_string(spg_status s) {
    switch (s) {
        case SPG_OK: return "ok";
        case SPG_ERR_INVALID_ARG: return "invalid argument";
        case SPG_ERR_DIM_MISMATCH: return "dimension mismatch";
        case SPG_ERR_INDEX_OVERFLOW: return "index overflow";
        case SPG_ERR_OUT_OF_MEMORY: return "out of memory";
        case SPG_ERR_NOT_READY: return "numeric phase before symbolic phase";
        case SPG_ERR_STRUCTURE_MISMATCH: return "structure differs from the symbolic phase";
        case SPG_ERR_HIP: return "HIP runtime error";
        case SPG_ERR_UNSUPPORTED: return "unsupported input";
        case SPG_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char *spg_last_error(spg_handle h) { return h ? h->err.c_str() : "null handle"; }

void spg_default_options(spg_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->compression = -1;
    o->cf_threshold = 0.85;
    o->accumulator = SPG_ACC_AUTO;
    o->fp32_mode = SPG_FP32_PLAIN;
    o->fp64_heavy_row_flops = 0;
    o->l1_hash_slots = 0;
    o->autotune = 0;
    o->fp32_terms_max = -1;
    o->verify_structure = 0;
    o->sorted_output = 1;
}

// FP32 values: the most products one entry of C may sum in FP32 (plain or
// compensated) and still meet |c - exact| <= 1e-5 * sum_k |a_ik * b_kj|.
// Recursive summation of n rounded FP32 products in any order is within
// gamma_n = n*u / (1 - n*u) of that sum (u = 2^-24); gamma_n <= 1e-5 gives
// n <= 167.  The compensated pair (Dot2) is within u*|c| + gamma_n^2 * sum,
// so gamma_n^2 <= 1e-5 - u gives n <= 52730.  An entry of row i sums at most
// nnz(A(i,:)) products, so rows of A longer than the limit accumulate in FP64.
// FP32 with FP64 accumulation needs no limit.
static long long fp32_terms_limit(const spg_options &o) {
    if (o.fp32_terms_max >= 0) return o.fp32_terms_max;
    const double u = 1.0 / 16777216.0, tol = 1e-5;
    double g;
    if (o.fp32_mode == SPG_FP32_PLAIN)
        g = tol;
    else if (o.fp32_mode == SPG_FP32_COMPENSATED)
        g = std::sqrt(tol - u);
    else
        return 0;
    // largest n with n*u / (1 - n*u) <= g
    return (long long)std::floor(g / (u * (1.0 + g)));
}

static spg_status check_options(spg_handle h, const spg_options *o) {
    if (o->compression < -1 || o->compression > 1) return fail(h, SPG_ERR_INVALID_ARG, "compression must be -1, 0 or 1");
    if (!(o->cf_threshold > 0.0 && o->cf_threshold <= 1.0)) return fail(h, SPG_ERR_INVALID_ARG, "cf_threshold in (0, 1]");
    if (o->accumulator < 0 || o->accumulator > 4) return fail(h, SPG_ERR_INVALID_ARG, "bad accumulator");
    if (o->sorted_output < 0 || o->sorted_output > 1) return fail(h, SPG_ERR_INVALID_ARG, "sorted_output must be 0 or 1");
    if (o->fp32_mode < 0 || o->fp32_mode > 2) return fail(h, SPG_ERR_INVALID_ARG, "bad fp32_mode");
    if (o->verify_structure < 0 || o->verify_structure > 1)
        return fail(h, SPG_ERR_INVALID_ARG, "verify_structure must be 0 or 1");
    if (o->fp32_terms_max < -1) return fail(h, SPG_ERR_INVALID_ARG, "fp32_terms_max must be -1, 0 or positive");
    if (o->l1_hash_slots < 0 || (o->l1_hash_slots & (o->l1_hash_slots - 1)) != 0 ||
        (o->l1_hash_slots != 0 && o->l1_hash_slots < 8))
        return fail(h, SPG_ERR_INVALID_ARG, "l1_hash_slots must be 0 or a power of two >= 8");
    return SPG_OK;
}

spg_status spg_create(spg_handle *out, void *stream, const spg_options *opt) {
    if (!out) return SPG_ERR_INVALID_ARG;
    *out = nullptr;
    spg_handle h = new (std::nothrow) spg_handle_s();
    if (!h) return SPG_ERR_OUT_OF_MEMORY;
    spg_default_options(&h->opt);
    if (opt) {
        spg_status s = check_options(h, opt);
        if (s != SPG_OK) {
            delete h;
            return s;
        }
        h->opt = *opt;
    }
    h->stream = (hipStream_t)stream;
    hipError_t e = hipGetDevice(&h->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&h->cus, hipDeviceAttributeMultiprocessorCount, h->device);
    int lds = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device);
    if (e == hipSuccess) e = hipHostMalloc((void **)&h->hst, sizeof(DevStats), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&h->hkoff, sizeof(int64_t) * (2 * (NK + 1) + 2), hipHostMallocDefault);
    if (e == hipSuccess) e = ensure(h->dstats, sizeof(DevStats));
    if (e == hipSuccess) e = ensure(h->red, sizeof(long long) * RED_ELEMS);
    if (e == hipSuccess) e = ensure(h->queue, sizeof(int32_t) * XCDS * NK);
    if (e == hipSuccess) e = scratch_address(h->device, &h->scr);
    if (e != hipSuccess) {
        spg_destroy(h);
        return SPG_ERR_HIP;
    }
    h->lds_max = (size_t)lds;
    // window words the workgroup dense kernel can hold next to its staging area
    // LDS bytes = 4*nw (bits) + nw/8 (summary) + staging + alignment slack
    const size_t over = 8 * DG_WG * 3 + 8 * (DG_WG / WAVE + 2) + 128;
    int64_t words = h->lds_max > over ? (int64_t)((h->lds_max - over) * 8 / 33) : 0;
    words = (words / 32) * 32;
    h->dg_nw_max = (int)std::min<int64_t>(DG_NW_MAX, std::max<int64_t>(words, 32));
    *out = h;
    return SPG_OK;
}

spg_status spg_destroy(spg_handle h) {
    if (!h) return SPG_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(h->stream);
    DevBuf *bufs[] = {&h->arp64, &h->brp64, &h->binfo, &h->ulist, &h->uflag, &h->bcrp, &h->bcw,
                      &h->rflops, &h->rflopsc, &h->rwin, &h->row_nnz, &h->coff, &h->kind_sym, &h->kind_num,
                      &h->perm_sym, &h->perm_num, &h->koff_sym, &h->koff_num, &h->tmp, &h->dstats, &h->red, &h->queue, &h->plan_len, &h->plan_off, &h->plan,
                      &h->arena, &h->l2k, &h->l2v, &h->blens, &h->row_words, &h->kind_tmp, &h->perm_tmp, &h->koff_tmp, &h->krange, &h->kind_heavy, &h->perm_heavy, &h->koff_heavy, &h->krange_heavy, &h->sgcur, &h->mflops, &h->map_off, &h->map,
                      &h->mk_arp, &h->mk_brp, &h->mk_mrp, &h->mk_rows, &h->mk_cnt, &h->mk_arena,
                      &h->row_cls, &h->kind_cls, &h->perm_cls, &h->koff_cls};
    for (DevBuf *b : bufs) release(*b);
    if (h->hst) (void)hipHostFree(h->hst);
    if (h->hkoff) (void)hipHostFree(h->hkoff);
    delete h;
    return SPG_OK;
}

spg_status spg_set_stream(spg_handle h, void *stream) {
    if (!h) return SPG_ERR_INVALID_ARG;
    h->stream = (hipStream_t)stream;
    return SPG_OK;
}

spg_status spg_set_options(spg_handle h, const spg_options *opt) {
    if (!h || !opt) return SPG_ERR_INVALID_ARG;
    spg_status s = check_options(h, opt);
    if (s != SPG_OK) return s;
    h->opt = *opt;
    return SPG_OK;
}

spg_status spg_get_stats(spg_handle h, spg_stats *out) {
    if (!h || !out) return SPG_ERR_INVALID_ARG;
    if (!h->ready) return fail(h, SPG_ERR_NOT_READY, "no symbolic phase yet");
    *out = h->stats;
    return SPG_OK;
}

spg_status spg_check_errors(spg_handle h) {
    if (!h) return SPG_ERR_INVALID_ARG;
    spg_status s = pull_stats(h);
    if (s != SPG_OK) return s;
    const int mism = h->hst->mismatch, ovf = h->hst->overflow;
    if (mism || ovf) {
        HIPCHK(hipMemsetAsync((char *)h->dstats.p + offsetof(DevStats, mismatch), 0, 2 * sizeof(int), h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    if (mism) return fail(h, SPG_ERR_STRUCTURE_MISMATCH, std::to_string(mism) + " rows differ from the plan");
    if (ovf) return fail(h, SPG_ERR_OUT_OF_MEMORY, std::to_string(ovf) + " rows overflowed the level-2 arena");
    return SPG_OK;
}

// ------------------------------------------------------------------ symbolic
// Plan buffers for an m x n times n x k product (grow-only).
static spg_status plan_buffers(spg_handle h, int64_t m, int64_t n, int64_t nnzb) {
    HIPCHK(ensure(h->arp64, 8 * (m + 1)));
    HIPCHK(ensure(h->brp64, 8 * (n + 1)));
    HIPCHK(ensure(h->binfo, sizeof(BRow) * std::max<int64_t>(n, 1)));
    HIPCHK(ensure(h->ulist, 4 * std::max<int64_t>(n, 1)));
    HIPCHK(ensure(h->uflag, 4 * ((std::max<int64_t>(n, 1) + 3) / 4)));
    HIPCHK(ensure(h->bcrp, 8 * (n + 1)));
    HIPCHK(ensure(h->rflops, 8 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->rflopsc, 8 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->rwin, 8 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->row_nnz, 4 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->row_words, 4 * (m + 2)));  // one padding element (8-byte reads of the last row)
    HIPCHK(ensure(h->coff, 8 * (m + 1)));
    HIPCHK(ensure(h->kind_sym, std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->kind_num, std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->perm_sym, 4 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->perm_num, 4 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->koff_sym, 8 * (NK + 1)));
    HIPCHK(ensure(h->koff_num, 8 * (NK + 1)));
    const int64_t tmp_elems = std::max({scan_tmp_elems(m), scan_tmp_elems(n), part_tmp_elems(m)});
    HIPCHK(ensure(h->tmp, 8 * tmp_elems));

    return SPG_OK;
}

// Rows per numeric kind: the main lists plus, when the plan keeps FP64-
// accumulated rows apart, their lists (whose rows the main classification
// counted as empty).  main: per-kind counts of the main lists (nullptr: the
// device statistics' numeric counts).
static void rows_numeric_stats(spg_stats &o, const DevStats &hs, bool split, const long long *main) {
    if (!main) main = hs.kcount_num;
    long long heavy = 0;
    for (int kk = 0; kk < NK; ++kk) {
        o.rows_numeric[kk] = main[kk];
        if (split && kk != K_EMPTY) {
            o.rows_numeric[kk] += hs.kcount_heavy[kk];
            heavy += hs.kcount_heavy[kk];
        }
    }
    o.rows_numeric[K_EMPTY] -= heavy;
}

// The symbolic phase on validated, device-resident structure: h->arp64 (m+1),
// h->brp64 (n+1) as int64, A's columns aci (row indices of B) and B's columns
// bci.  Leaves the plan in the handle and C's int64 row offsets in h->coff.
static spg_status symbolic_core(spg_handle h, int64_t m, int64_t n, int64_t k, int64_t nnza, int64_t nnzb,
                                const int32_t *aci, const int32_t *bci, int64_t *nnzc_out) {
    spg_status s;
    hipStream_t st = h->stream;
    DevStats *dst = h->dstats.as<DevStats>();
    const int64_t *arp = h->arp64.as<int64_t>(), *brp = h->brp64.as<int64_t>();
    BRow *bi = h->binfo.as<BRow>();
    // Everything up to the first host sync runs on unchecked input: row
    // pointers are clamped copies, columns out of range only raise the flag
    // (k_brow, k_rowinfo) and are never used as indices before the sync.
    HIPCHK(launch_brow(n, nnzb, k, brp, bci, bi, h->ulist.as<int32_t>(), h->uflag.as<uint8_t>(), dst, st));
    HIPCHK(launch_brow_unsorted(h->ulist.as<int32_t>(), &dst->unsorted, brp, bci, bi, dst, st));
    const bool sel = h->opt.accumulator == SPG_ACC_AUTO;
    HIPCHK(launch_rowinfo(m, n, arp, aci, bi, h->rflops.as<int64_t>(), h->rflopsc.as<int64_t>(),
                          h->rwin.as<int2>(), dst, h->red.as<long long>(), h->opt.compression, sel ? 1 : 0,
                          h->opt.cf_threshold, st));
    // compressed B (Compression subsection): lengths -> offsets -> (word, bits)
    // pairs, built when the analysis decided so (dst->comp, on the device)
    const int *cflag = &dst->comp;
    if (h->opt.compression != 0) {
        HIPCHK(ensure(h->bcw, 8 * std::max<int64_t>(nnzb, 1)));
        static_assert(sizeof(BRow) == 4 * sizeof(int32_t), "BRow is four int32");
        HIPCHK(launch_scan_i32s(n, &bi->lenc, 4, h->bcrp.as<int64_t>(), h->tmp.as<int64_t>(), cflag, st));
        HIPCHK(launch_compress_sorted_flags(n, nnzb, brp, bci, bi, h->uflag.as<uint8_t>(), h->bcrp.as<int64_t>(),
                                            h->bcw.as<uint2>(), cflag, st));
        HIPCHK(launch_compress_unsorted(h->ulist.as<int32_t>(), &dst->unsorted, brp, bci, bi,
                                        h->bcrp.as<int64_t>(), h->bcw.as<uint2>(), cflag,
                                        st));
    }

    ClassParams cp{};
    cp.phase = 0;
    cp.accumulator = h->opt.accumulator;
    cp.compressed = 0;
    cp.comp_flag = h->opt.compression != 0 ? cflag : nullptr;
    cp.unsorted = &dst->unsorted;
    cp.dw_nw_max = DW_NW_MAX;
    cp.dw_r_max = DW_R_MAX;
    cp.hw_keys_max = HW_KEYS_MAX;
    cp.dg_nw_max = h->dg_nw_max;
    cp.wh_nw_max = WH_NW_MAX;
    cp.wh_r_max = WH_R_MAX;
    cp.wh_t_max = WH_T_MAX;
    cp.sample_stride = 1;
    cp.sr_f_max = SR_F_MAX;
    // stored row structure: bit-window rows keep their (word, bits) pairs for
    // the numeric phase (selector only); heavy rows keep their segment lists
    // (selector and dense policy, B's rows sorted: checked on the device)
    const bool want_pairs = sel;
    const bool want_segs_opt = sel || h->opt.accumulator == SPG_ACC_DENSE;
    const bool want_plan = want_pairs || want_segs_opt;
    if (want_plan) {
        HIPCHK(ensure(h->plan_len, 4 * (m + 2)));  // one padding element (8-byte reads of the last row)
        HIPCHK(ensure(h->plan_off, 8 * (m + 1)));
        cp.plan_cap = want_pairs ? PL_CAP : 0;
        cp.plan_len = h->plan_len.as<int32_t>();
        cp.sg = want_segs_opt ? 1 : 0;
    }
    cp.words_out = h->row_words.as<int32_t>();
    HIPCHK(launch_classify(m, h->rflops.as<int64_t>(), h->rflopsc.as<int64_t>(), h->rwin.as<int2>(), nullptr,
                           nullptr, cp, h->kind_sym.as<uint8_t>(), h->row_nnz.as<int32_t>(), dst, h->tmp.as<int64_t>(),
                           h->koff_sym.as<int64_t>(), st));
    HIPCHK(launch_partition(m, h->kind_sym.as<uint8_t>(), h->perm_sym.as<int32_t>(), h->tmp.as<int64_t>(),
                            h->koff_sym.as<int64_t>(), cp.phase, cp.heavy, dst, st));
    // host sync 1: input checks, flop counts, compression, per-kind sizes
    if ((s = pull_stats(h)) != SPG_OK) return s;
    const DevStats hs2 = *h->hst;
    const DevStats &hs1 = hs2;
    if (hs1.bad_input) return fail(h, SPG_ERR_INVALID_ARG, "malformed CSR: row_ptr or col_idx out of range");
    // (an unsorted row of B wider than the LDS bitmap of its word count makes
    // the analysis skip compression: the structure kernels read raw B)
    const bool comp = h->opt.compression != 0 && hs1.comp != 0;
    const double fm = (double)hs1.fm, fmc = (double)hs1.fmc;
    h->avg_len = nnza ? std::max(1.0, fm / (double)nnza) : 1.0;
    h->avg_len_c = nnza ? std::max(1.0, (comp ? fmc : fm) / (double)nnza) : 1.0;
    const bool want_segs = want_segs_opt && hs1.unsorted == 0;

    h->planned = false;
    h->segmented = false;
    const bool pairs_used = want_pairs && hs2.kcount_sym[K_DW] > 0;
    const bool segs_used = want_segs && hs2.kcount_sym[K_DG] > 0;
    // room for stored structure: the scan of the rows' room gives each row's
    // offset.  Bit-window rows hold at most PL_CAP pairs each, so while no
    // segment room is in the scan (no heavy rows with lists) and that bound
    // is modest, the plan is sized by it without waiting for the total;
    // otherwise the exact total is fetched (one more host sync).
    int64_t plan_room = 0;
    if (pairs_used || segs_used) {
        HIPCHK(launch_scan_i32(m, h->plan_len.as<int32_t>(), h->plan_off.as<int64_t>(), h->tmp.as<int64_t>(), st));
        const int64_t bound = (int64_t)PL_CAP * hs2.kcount_sym[K_DW];
        const bool seg_room = want_segs_opt && hs2.kcount_sym[K_DG] > 0;
        if (!seg_room && bound <= (int64_t(1) << 27)) {
            plan_room = bound;
        } else {
            HIPCHK(hipMemcpyAsync(h->hkoff + 1, h->plan_off.as<int64_t>() + m, sizeof(int64_t),
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            plan_room = h->hkoff[1];
        }
    }
    bool plan_ok = false;
    if ((pairs_used || segs_used) && plan_room > 0) {
        // without room for the pairs the numeric phase rebuilds the structure
        // itself; without room for the segment lists heavy rows use the
        // window-wide kernel
        plan_ok = ensure(h->plan, 8 * (size_t)plan_room) == hipSuccess;
        (void)hipGetLastError();
    }
    h->planned = plan_ok && pairs_used;
    h->segmented = plan_ok && segs_used;
    // segments need a list wherever a row may exceed one (rows with a bound
    // of room in plan_len): with lists missing, all heavy rows take the
    // window-wide kernel
    h->sg_mode = want_segs && (plan_ok || !segs_used || plan_room == 0);

    SymArgs sa{};
    sa.arp = arp;
    sa.aci = aci;
    sa.brp = brp;
    sa.bci = bci;
    if (comp) {
        sa.bcrp = h->bcrp.as<int64_t>();
        sa.bcw = h->bcw.as<uint2>();
    }
    sa.rwin = h->rwin.as<int2>();
    sa.row_nnz = h->row_nnz.as<int32_t>();
    sa.row_words = h->row_words.as<int32_t>();
    sa.rs.rows = h->perm_sym.as<int32_t>();
    sa.rs.koff = h->koff_sym.as<int64_t>();
    sa.st = dst;
    sa.lg_gs = lg_group(h->avg_len_c);
    sa.b32 = nnzb < (int64_t(1) << 29);  // 8-byte compressed records: 32-bit byte offsets
    sa.nnzb = nnzb;
    if (h->planned || h->segmented) {
        sa.plan_off = h->plan_off.as<int64_t>();
        sa.plan_len = h->plan_len.as<int32_t>();
        sa.plan = h->plan.as<uint2>();
    }
    LaunchCfg lc{st, 0, h->cus};
    auto grid_cap = [&](int64_t rows) { return (int)std::min<int64_t>(2048 * 8, ((rows + 7) / 8) * 8); };

    if (hs2.kcount_sym[K_SR] > 0) {
        sa.rs.kind = K_SR;
        lc.grid = 0;
        HIPCHK(launch_sym_sr(sa, sr_lg(hs2.kmax_sym[K_SR][1]), lc, hs2.kcount_sym[K_SR]));
    }
    if (hs2.kcount_sym[K_DW] > 0) {
        sa.rs.kind = K_DW;
        sa.nw_max = ((hs2.kmax_sym[K_DW][0] + 31) / 32) * 32;
        lc.grid = 0;
        HIPCHK(launch_sym_dw(sa, lc));
    }
    if (hs2.kcount_sym[K_HW] > 0) {
        sa.rs.kind = K_HW;
        sa.ts = pow2_at_least(2 * (int64_t)hs2.kmax_sym[K_HW][1], 64);
        lc.grid = 0;
        HIPCHK(launch_sym_hw(sa, lc));
    }
    if (hs2.kcount_sym[K_DG] > 0) {
        sa.rs.kind = K_DG;
        sa.rs.queue = h->queue.as<int32_t>() + XCDS * K_DG;
        sa.nw_max = ((hs2.kmax_sym[K_DG][0] + 31) / 32) * 32;
        HIPCHK(launch_fill_i32(sa.rs.queue, XCDS, 0, st));
        lc.grid = grid_cap(hs2.kcount_sym[K_DG]);
        lc.grid = std::min(lc.grid, 8 * h->cus);
        HIPCHK(launch_sym_dg(sa, lc));
    }
    if (hs2.kcount_sym[K_HL] > 0) {
        sa.rs.kind = K_HL;
        sa.rs.queue = h->queue.as<int32_t>() + XCDS * K_HL;
        int l1 = h->opt.l1_hash_slots ? h->opt.l1_hash_slots : 4096;
        sa.l1_slots = l1;
        const int64_t cap2 = pow2_at_least(2 * (int64_t)std::max(1, hs2.kmax_sym[K_HL][1]), 64);
        int grid = (int)std::min<int64_t>(grid_cap(hs2.kcount_sym[K_HL]), 2 * h->cus);
        sa.l2_cap = cap2;
        HIPCHK(ensure(h->l2k, (size_t)4 * cap2 * grid));
        HIPCHK(ensure(h->l2v, (size_t)4 * cap2 * grid));
        sa.l2_keys = h->l2k.as<uint32_t>();
        sa.l2_vals = h->l2v.as<uint32_t>();
        HIPCHK(launch_fill_i32(sa.rs.queue, XCDS, 0, st));
        lc.grid = grid;
        HIPCHK(launch_sym_hl(sa, lc));
    }

    // scan -> C row offsets (int64 plan copy), then the numeric classification
    HIPCHK(launch_scan_i32(m, h->row_nnz.as<int32_t>(), h->coff.as<int64_t>(), h->tmp.as<int64_t>(), st));
    cp.phase = 1;
    cp.words_out = nullptr;
    cp.plan_cap = h->planned ? PL_CAP : 0;
    cp.sym_kind = h->kind_sym.as<uint8_t>();
    cp.sg = h->sg_mode ? 1 : 0;
    const long long thr = h->opt.fp64_heavy_row_flops;
    const long long tmax = fp32_terms_limit(h->opt);
    // (no separate lists unless some row of A is longer than the term limit)
    const bool split = thr > 0 || (tmax > 0 && (long long)hs1.maxnnza > tmax);
    cp.heavy_flops = thr > 0 ? thr : 0;
    cp.heavy_alen = tmax > 0 ? tmax : 0;
    cp.arp = arp;
    cp.split = split ? 1 : 0;
    cp.heavy = 0;
    HIPCHK(launch_classify(m, h->rflops.as<int64_t>(), h->rflopsc.as<int64_t>(), h->rwin.as<int2>(),
                           h->row_nnz.as<int32_t>(), h->row_words.as<int32_t>(), cp, h->kind_num.as<uint8_t>(),
                           nullptr, dst, h->tmp.as<int64_t>(), h->koff_num.as<int64_t>(), st));
    HIPCHK(launch_partition(m, h->kind_num.as<uint8_t>(), h->perm_num.as<int32_t>(), h->tmp.as<int64_t>(),
                            h->koff_num.as<int64_t>(), cp.phase, cp.heavy, dst, st));
    h->heavy_split = false;
    if (split) {  // FP64-accumulated rows: their own kind lists (FP64 accumulation in FP32 mode)
        HIPCHK(ensure(h->kind_heavy, std::max<int64_t>(m, 1)));
        HIPCHK(ensure(h->perm_heavy, 4 * std::max<int64_t>(m, 1)));
        HIPCHK(ensure(h->koff_heavy, 8 * (NK + 1)));
        ClassParams ch = cp;
        ch.heavy = 1;
        HIPCHK(launch_classify(m, h->rflops.as<int64_t>(), h->rflopsc.as<int64_t>(), h->rwin.as<int2>(),
                               h->row_nnz.as<int32_t>(), h->row_words.as<int32_t>(), ch,
                               h->kind_heavy.as<uint8_t>(), nullptr, dst, h->tmp.as<int64_t>(),
                               h->koff_heavy.as<int64_t>(), st));
        HIPCHK(launch_partition(m, h->kind_heavy.as<uint8_t>(), h->perm_heavy.as<int32_t>(), h->tmp.as<int64_t>(),
                                h->koff_heavy.as<int64_t>(), ch.phase, ch.heavy, dst, st));
    }
    HIPCHK(hipMemcpyAsync(h->hkoff, h->coff.as<int64_t>() + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    h->hkoff[2] = 0;
    if (comp)  // pairs of compressed B: the end of its row offsets
        HIPCHK(hipMemcpyAsync(h->hkoff + 2, h->bcrp.as<int64_t>() + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    if ((s = pull_stats(h)) != SPG_OK) return s;  // host sync 2: nnz(C), numeric kinds
    const DevStats hs3 = *h->hst;
    if (hs3.overflow) return fail(h, SPG_ERR_OUT_OF_MEMORY, "level-2 hash arena too small in the symbolic phase");
    const int64_t nnzc = h->hkoff[0];
    h->compressed = comp;
    *h->hst = hs3;
    spg_stats &o = h->stats;
    std::memset(&o, 0, sizeof(o));
    o.flops = (int64_t)hs1.fm;
    o.flops_compressed = (int64_t)hs1.fmc;
    o.max_row_flops = (int64_t)hs1.maxrf;
    o.max_row_flops_compressed = (int64_t)hs1.maxrfc;
    o.nnz_c = nnzc;
    o.compressed = comp ? 1 : 0;
    o.nnz_b_compressed = comp ? h->hkoff[2] : 0;
    o.n_kinds = NK;
    int64_t maxrs = 0;
    for (int kk = 0; kk < NK; ++kk) {
        o.rows_symbolic[kk] = hs3.kcount_sym[kk];
        if (kk != K_EMPTY) maxrs = std::max<int64_t>(maxrs, hs3.kmax_num[kk][1]);
        if (kk != K_EMPTY && split) maxrs = std::max<int64_t>(maxrs, hs3.kmax_heavy[kk][1]);
    }
    rows_numeric_stats(h->stats, hs3, split, nullptr);
    o.max_row_nnz = maxrs;
    o.l2_spill_rows = (int32_t)o.rows_numeric[K_HL];
    o.fp64_rows = 0;
    if (split)
        for (int kk = 1; kk < NK; ++kk) o.fp64_rows += hs3.kcount_heavy[kk];
    h->aci_used = aci;
    h->bci_used = bci;
    h->cparams = cp;
    h->heavy_split = split;
    h->lg_num = lg_group(h->avg_len);
    h->tuned = false;
    h->maps_built = h->maps_ok = false;
    h->num_policy = h->opt.accumulator;
    *nnzc_out = nnzc;
    return SPG_OK;
}

spg_status spgemm_symbolic(spg_handle h, const spg_csr *A, const spg_csr *B, void *C_row_ptr,
                           spg_itype c_rpt, int64_t *nnz_c) {
    if (!h) return SPG_ERR_INVALID_ARG;
    h->err.clear();
    spg_status s;
    if ((s = check_csr(h, A, "A", false)) != SPG_OK) return s;
    if ((s = check_csr(h, B, "B", false)) != SPG_OK) return s;
    if (!C_row_ptr || !nnz_c) return fail(h, SPG_ERR_INVALID_ARG, "C_row_ptr / nnz_c is NULL");
    if (c_rpt != SPG_I32 && c_rpt != SPG_I64) return fail(h, SPG_ERR_INVALID_ARG, "bad C rp_type");
    if (A->ncols != B->nrows) return fail(h, SPG_ERR_DIM_MISMATCH, "A.ncols != B.nrows");
    h->ready = false;
    h->batch.count = 0;
    h->ncls = 0;
    const int64_t m = A->nrows, n = B->nrows, k = B->ncols;
    hipStream_t st = h->stream;
    if ((s = plan_buffers(h, m, n, B->nnz)) != SPG_OK) return s;
    DevStats *dst = h->dstats.as<DevStats>();
    HIPCHK(launch_fill_i32((int32_t *)dst, (int64_t)(sizeof(DevStats) / 4), 0, st));
    int *bad = &dst->bad_input;
    // Row pointers are copied clamped to [0, nnz] and out-of-range columns of A
    // are skipped by the analysis, so the kernels that run before the first
    // host sync stay in bounds on malformed input; that sync rejects it before
    // any structure kernel indexes B by A's columns.
    HIPCHK(launch_copy_rp(m + 1, A->row_ptr, A->rp_type == SPG_I64, A->nnz, h->arp64.as<int64_t>(), n + 1,
                          B->row_ptr, B->rp_type == SPG_I64, B->nnz, h->brp64.as<int64_t>(), bad, st));
    int64_t nnzc = 0;
    if ((s = symbolic_core(h, m, n, k, A->nnz, B->nnz, A->col_idx, B->col_idx, &nnzc)) != SPG_OK) return s;
    if (c_rpt == SPG_I32 && nnzc > INT32_MAX)
        return fail(h, SPG_ERR_INDEX_OVERFLOW, "nnz(C) exceeds an int32 row_ptr; ask for SPG_I64");
    HIPCHK(launch_store_rp(m + 1, h->coff.as<int64_t>(), C_row_ptr, c_rpt == SPG_I64, st));
    Fingerprint &fp = h->fp;
    fp.m = m; fp.n = n; fp.k = k; fp.nnza = A->nnz; fp.nnzb = B->nnz;
    fp.arp = A->row_ptr; fp.brp = B->row_ptr; fp.aci = A->col_idx; fp.bci = B->col_idx;
    fp.arpt = A->rp_type; fp.brpt = B->rp_type;
    h->nnzc = nnzc;
    h->sref = StructRef{A->row_ptr, B->row_ptr, A->col_idx, B->col_idx, m, n, A->nnz, B->nnz,
                        A->rp_type == SPG_I64, B->rp_type == SPG_I64};
    h->verify = h->opt.verify_structure != 0;
    if (h->verify)
        HIPCHK(launch_struct_digest(h->sref, (unsigned long long *)h->red.p, &dst->sdigest, 0, &dst->mismatch, st));
    *nnz_c = nnzc;
    h->ready = true;
    return SPG_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ numeric
// With verify_structure: the operands' structure digest against the symbolic
// phase's, on the device; a difference is counted as a mismatch that
// spg_check_errors reports (no host sync here).
static spg_status verify_struct(spg_handle h) {
    if (!h->verify || h->batch.count) return SPG_OK;
    DevStats *dst = h->dstats.as<DevStats>();
    HIPCHK(launch_struct_digest(h->sref, (unsigned long long *)h->red.p, &dst->sdigest, 1, &dst->mismatch,
                                h->stream));
    return SPG_OK;
}

static int fp32_acc(spg_handle h) {
    return h->opt.fp32_mode == SPG_FP32_COMPENSATED ? ACC_COMP
           : h->opt.fp32_mode == SPG_FP32_WIDE      ? ACC_WIDE
                                                    : ACC_NATIVE;
}

// Device scratch for one launch of the numeric phase: a handle-owned buffer
// grown with hipMalloc, or, in an allocation-free call, the front of this
// device's static scratch array (the launches of a call are stream-ordered,
// so each starts at the array's beginning).  per_wg: bytes per workgroup;
// *grid is lowered (to a multiple of 8) until the scratch fits.  Returns
// false when not even 8 workgroups fit.
static bool scratch_grid(spg_handle h, size_t per_wg, int *grid) {
    if (!h->noalloc) return true;
    const size_t fit = per_wg ? NOALLOC_SCRATCH_BYTES / per_wg : (size_t)*grid;
    int g = (int)std::min<size_t>((size_t)*grid, fit);
    g = (g / XCDS) * XCDS;
    if (g < XCDS) return false;
    *grid = g;
    return true;
}

// The numeric phase on the plan: A's values aval, B's values bval (entry order
// of the structure the symbolic phase saw), C's columns / values written at the
// plan's row offsets.
// One persistent launch per non-empty kind, sized by the kind's maxima.
// dg: DG_OWN launches this set's segmented rows; DG_MERGE also takes the
// rows of na.rs2 (rs2_count of them, accumulated with acc2) in the same
// launch; DG_SKIP leaves them to such a launch.
enum { DG_OWN = 0, DG_MERGE = 1, DG_SKIP = 2 };
template <typename VT>
static spg_status launch_kinds(spg_handle h, NumArgs<VT> na, const long long *kcount, const int (*kmax)[3],
                               int acc, bool vo = false, int pol = -1, int dg = DG_OWN, int64_t rs2_count = 0,
                               int acc2 = -1) {
    if (pol < 0) pol = h->num_policy;
    hipStream_t st = h->stream;
    const size_t sbytes = (sizeof(VT) == 8 || acc != ACC_NATIVE) ? 8 : 4;
    LaunchCfg lc{st, 0, h->cus};
    auto grid_cap = [&](int64_t rows) { return (int)std::min<int64_t>(2048 * 8, ((rows + 7) / 8) * 8); };

    na.values_only = vo ? 1 : 0;
    if (kcount[K_PL] > 0) {
        na.rs.kind = K_PL;
        na.nw_max = ((kmax[K_PL][0] + 31) / 32) * 32;
        na.r_max = std::max(kmax[K_PL][1], 1);
        HIPCHK(launch_num_pl<VT>(na, acc, lc));
    }
    if (vo && h->maps_ok) {  // structure known: every mapped kind on its position maps
        for (int K : {K_SR, K_DW, K_WH, K_HW}) {
            if (kcount[K] <= 0) continue;
            na.rs.kind = K;
            na.r_max = std::max(kmax[K][1], 1);
            const int lgt = K == K_SR ? sr_lg(kmax[K_SR][1]) : 6;
            HIPCHK(launch_num_map<VT>(na, acc, lgt, h->lg_map_cur, lc, kcount[K]));
        }
        for (int kk = 0; kk < NK; ++kk) h->kc_nomap[kk] = map_kind(kk) ? 0 : kcount[kk];
        kcount = h->kc_nomap;  // the remaining kinds below
    }
    if (kcount[K_SR] > 0) {
        na.rs.kind = K_SR;
        HIPCHK(launch_num_sr<VT>(na, acc, sr_lg(kmax[K_SR][1]), lc, kcount[K_SR]));
    }
    if (kcount[K_DW] > 0) {
        na.rs.kind = K_DW;
        na.nw_max = ((kmax[K_DW][0] + 31) / 32) * 32;
        na.r_max = std::max(kmax[K_DW][1], 1);
        HIPCHK(launch_num_dw<VT>(na, acc, lc));
    }
    if (kcount[K_WH] > 0) {
        na.rs.kind = K_WH;
        na.nw_max = ((kmax[K_WH][0] + 31) / 32) * 32;
        na.r_max = std::max(kmax[K_WH][1], 1);
        na.ts = pow2_at_least(2 * (int64_t)std::max(kmax[K_WH][2], 1), 16);
        HIPCHK(launch_num_wh<VT>(na, acc, lc));
    }
    if (kcount[K_HW] > 0 && pol == SPG_ACC_LL) {  // LL hashmap, rows unsorted
        na.rs.kind = K_HW;
        na.r_max = std::max(kmax[K_HW][1], 1);
        na.ts = pow2_at_least(na.r_max, 16);
        HIPCHK(launch_num_ll<VT>(na, acc, na.lg_gs, lc, kcount[K_HW]));
    } else if (kcount[K_HW] > 0) {
        na.rs.kind = K_HW;
        na.ts = pow2_at_least(2 * (int64_t)kmax[K_HW][1], 64);
        HIPCHK(launch_num_hw<VT>(na, acc, lc));
    }
    if ((kcount[K_DG] > 0 || (dg == DG_MERGE && rs2_count > 0)) && h->sg_mode && dg != DG_SKIP) {
        na.rs.kind = K_DG;
        na.rs.queue = h->queue.as<int32_t>() + XCDS * K_DG;
        HIPCHK(launch_fill_i32(na.rs.queue, XCDS, 0, st));
        int64_t dg_rows = kcount[K_DG];
        const int acc_b = (dg == DG_MERGE && rs2_count > 0 && acc2 >= 0) ? acc2 : acc;
        if (dg == DG_MERGE && rs2_count > 0) {
            na.rs2.kind = K_DG;
            na.rs2.queue = h->queue.as<int32_t>() + XCDS * K_EMPTY;  // the empty kind has no queue of its own
            HIPCHK(launch_fill_i32(na.rs2.queue, XCDS, 0, st));
            dg_rows += rs2_count;
        } else {
            na.rs2 = RowSet{};
        }
        lc.grid = std::min(grid_cap(dg_rows), sg_resident_grid(acc, acc_b, sizeof(VT) == 8, h->cus));
        // rows with more than one chunk of A entries keep per-entry cursors
        // (32-bit positions in B) in HBM scratch; without it (or with
        // nnz(B) >= 2^31) they search each run from the B row's start
        na.sg_cur = nullptr;
        na.sg_cap = 0;
        const int64_t mxa = (int64_t)h->hst->maxnnza;
        if (mxa > WG_BIG && h->fp.nnzb < (int64_t(1) << 31)) {
            const int cap = (int)std::min<int64_t>(mxa, 65536);
            const size_t bytes = (size_t)lc.grid * 3 * cap * sizeof(int32_t);
            if (h->noalloc) {
                if (bytes <= NOALLOC_SCRATCH_BYTES) {  // else runs are searched without cursors
                    na.sg_cur = (int32_t *)h->scr;
                    na.sg_cap = cap;
                }
            } else if (ensure(h->sgcur, bytes) == hipSuccess) {
                na.sg_cur = h->sgcur.as<int32_t>();
                na.sg_cap = cap;
            }
            (void)hipGetLastError();
        }
        HIPCHK(launch_num_sg<VT>(na, acc, acc_b, lc));
        lc.grid = 0;
    } else if (kcount[K_DG] > 0 && dg != DG_SKIP) {
        na.rs.kind = K_DG;
        na.rs.queue = h->queue.as<int32_t>() + XCDS * K_DG;
        na.nw_max = ((kmax[K_DG][0] + 31) / 32) * 32;
        int grid = std::min(grid_cap(kcount[K_DG]),
                            dg_resident_grid(acc, sizeof(VT) == 8, lds_num_dg(na.nw_max), h->cus));
        na.arena_cap = (int64_t)na.nw_max * 32;
        if (!scratch_grid(h, (size_t)na.arena_cap * sbytes, &grid))
            return fail(h, SPG_ERR_OUT_OF_MEMORY, "heavy-row value windows exceed the static scratch");
        const size_t bytes = (size_t)na.arena_cap * grid * sbytes;
        if (h->noalloc) {  // the window must start at zero; the kernel leaves it zero
            HIPCHK(launch_fill_i32((int32_t *)h->scr, (int64_t)(bytes / 4), 0, st));
            na.arena = h->scr;
        } else {
            if (h->arena.cap < bytes || h->arena_bytes_zeroed < bytes) {
                HIPCHK(ensure(h->arena, bytes));
                HIPCHK(hipMemsetAsync(h->arena.p, 0, h->arena.cap, st));
                h->arena_bytes_zeroed = h->arena.cap;
            }
            na.arena = h->arena.p;
        }
        HIPCHK(launch_fill_i32(na.rs.queue, XCDS, 0, st));
        lc.grid = grid;
        HIPCHK(launch_num_dg<VT>(na, acc, lc));
        lc.grid = 0;
    }
    if (kcount[K_HL] > 0) {
        na.rs.kind = K_HL;
        na.rs.queue = h->queue.as<int32_t>() + XCDS * K_HL;
        na.l1_slots = h->opt.l1_hash_slots ? h->opt.l1_hash_slots : (sbytes == 8 ? 4096 : 8192);
        int grid = std::min(grid_cap(kcount[K_HL]),
                            hl_resident_grid(acc, sizeof(VT) == 8, lds_num_hl(na.l1_slots, (int)sbytes), h->cus));
        na.arena_cap = pow2_at_least(2 * (int64_t)std::max(1, kmax[K_HL][1]), 64);
        if (!scratch_grid(h, (size_t)na.arena_cap * (8 + 2 * sbytes), &grid))
            return fail(h, SPG_ERR_OUT_OF_MEMORY, "level-2 hash tables exceed the static scratch");
        const size_t bytes = (size_t)na.arena_cap * grid * (8 + 2 * sbytes);
        if (h->noalloc) {
            na.arena = h->scr;
        } else {
            if (h->l2k.cap < bytes) HIPCHK(ensure(h->l2k, bytes));
            na.arena = h->l2k.p;
        }
        HIPCHK(launch_fill_i32(na.rs.queue, XCDS, 0, st));
        lc.grid = grid;
        HIPCHK(launch_num_hl<VT>(na, acc, lc));
        lc.grid = 0;
    }
    return SPG_OK;
}


// Measured selection (replaces a fixed heuristic): on a strided sample of the
// rows, time each accumulator policy (selector / bit window first / column
// hash first) with lane groups of 2^(base-1), 2^base, 2^(base+1) lanes per B
// row, keep the fastest, and classify every row with it.  Runs once per plan,
// at the first numeric call (values and C are available then); blocks the host.
template <typename VT>
static spg_status autotune(spg_handle h, NumArgs<VT> na, int acc) {
    hipStream_t st = h->stream;
    const int64_t m = h->fp.m;
    DevStats *dst = h->dstats.as<DevStats>();
    HIPCHK(ensure(h->kind_tmp, std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->perm_tmp, 4 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->koff_tmp, 8 * (NK + 1)));
    const int stride = (int)std::max<int64_t>(1, std::min<int64_t>(16, m / 16384));
    ClassParams cp = h->cparams;
    cp.phase = 1;
    cp.sample_stride = stride;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best = 3.4e38f;
    int best_pol = cp.accumulator, best_lg = h->lg_num;
    const int base = lg_group(h->avg_len);
    spg_status s = SPG_OK;
    const size_t koff_bytes = offsetof(DevStats, kcount_num);
    // candidates: selector, bit window first, column hash first, and with
    // unsorted rows allowed the LL hashmap (its classification is the hash
    // policy's; the hash-wave rows then run the LL kernel)
    const int npol = h->opt.sorted_output ? 3 : 4;
    for (int ci = 0; ci < npol && s == SPG_OK; ++ci) {
        const int pol = ci < 3 ? ci : SPG_ACC_LL;
        cp.accumulator = pol;
        h->num_policy = pol;
        HIPCHK(hipMemsetAsync((char *)dst + koff_bytes, 0, sizeof(long long) * NK, st));
        HIPCHK(hipMemsetAsync(&dst->kmax_num[0][0], 0, sizeof(dst->kmax_num), st));
        HIPCHK(launch_classify(m, h->rflops.as<int64_t>(), h->rflopsc.as<int64_t>(), h->rwin.as<int2>(),
                               h->row_nnz.as<int32_t>(), h->row_words.as<int32_t>(), cp, h->kind_tmp.as<uint8_t>(),
                               nullptr, dst, h->tmp.as<int64_t>(), h->koff_tmp.as<int64_t>(), st));
        HIPCHK(launch_partition(m, h->kind_tmp.as<uint8_t>(), h->perm_tmp.as<int32_t>(), h->tmp.as<int64_t>(),
                                h->koff_tmp.as<int64_t>(), cp.phase, cp.heavy, dst, st));
        if ((s = pull_stats(h)) != SPG_OK) break;
        const DevStats hs = *h->hst;
        na.rs.rows = h->perm_tmp.as<int32_t>();
        na.rs.koff = h->koff_tmp.as<int64_t>();
        for (int lg = std::max(2, base - 1); lg <= std::min(6, base + 1); ++lg) {
            na.lg_gs = lg;
            float ms = 0;
            HIPCHK(hipEventRecord(e0, st));
            if ((s = launch_kinds<VT>(h, na, hs.kcount_num, hs.kmax_num, acc)) != SPG_OK) break;  // warm-up
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            // a policy whose warm-up run is far behind the best so far is not
            // timed further (the column-hash policy on rows meant for the bit
            // window can be an order of magnitude slower)
            if (ms > 4.0f * best) break;
            HIPCHK(hipEventRecord(e0, st));
            if ((s = launch_kinds<VT>(h, na, hs.kcount_num, hs.kmax_num, acc)) != SPG_OK) break;
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                best_pol = pol;
                best_lg = lg;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != SPG_OK) {
        h->num_policy = h->opt.accumulator;
        return s;
    }
    // final classification of every row with the winner
    cp.accumulator = best_pol;
    h->num_policy = best_pol;
    cp.sample_stride = 1;
    HIPCHK(hipMemsetAsync((char *)dst + koff_bytes, 0, sizeof(long long) * NK, st));
    HIPCHK(hipMemsetAsync(&dst->kmax_num[0][0], 0, sizeof(dst->kmax_num), st));
    HIPCHK(launch_classify(m, h->rflops.as<int64_t>(), h->rflopsc.as<int64_t>(), h->rwin.as<int2>(),
                           h->row_nnz.as<int32_t>(), h->row_words.as<int32_t>(), cp, h->kind_num.as<uint8_t>(),
                           nullptr, dst, h->tmp.as<int64_t>(), h->koff_num.as<int64_t>(), st));
    HIPCHK(launch_partition(m, h->kind_num.as<uint8_t>(), h->perm_num.as<int32_t>(), h->tmp.as<int64_t>(),
                            h->koff_num.as<int64_t>(), cp.phase, cp.heavy, dst, st));
    if ((s = pull_stats(h)) != SPG_OK) return s;
    h->lg_num = best_lg;
    h->tuned = true;
    h->stats.tuned_policy = best_pol;
    h->stats.tuned_lanes = 1 << best_lg;
    rows_numeric_stats(h->stats, *h->hst, h->heavy_split, nullptr);
    return SPG_OK;
}

// Batch plans with product classes: the same measured selection per class.
// For class c the candidates are timed on a strided sample of the class's
// rows (other rows classified empty), lanes per B row centred on the class's
// average B row length; the winner classifies the class's rows into their own
// row lists (kinds, counts and maxima per class, so LDS is sized by the
// class's largest rows, not the batch's).  Blocks the host; once per plan.
template <typename VT>
static spg_status autotune_classes(spg_handle h, NumArgs<VT> na, int acc) {
    hipStream_t st = h->stream;
    const int64_t m = h->fp.m;
    DevStats *dst = h->dstats.as<DevStats>();
    HIPCHK(ensure(h->kind_tmp, std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->perm_tmp, 4 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->koff_tmp, 8 * (NK + 1)));
    HIPCHK(ensure(h->kind_cls, 4 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->perm_cls, 16 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->koff_cls, 8 * 4 * (NK + 1)));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const size_t koff_bytes = offsetof(DevStats, kcount_num);
    spg_status s = SPG_OK;
    const int npol = h->opt.sorted_output ? 3 : 4;
    for (int c = 0; c < 4 && s == SPG_OK; ++c) {
        for (int k = 0; k < NK; ++k) {
            h->cls_kc[c][k] = 0;
            h->cls_km[c][k][0] = h->cls_km[c][k][1] = h->cls_km[c][k][2] = 0;
        }
        h->cls_pol[c] = h->cparams.accumulator;
        h->cls_lg[c] = lg_group(h->cls_avg_b[c]);
        if (h->cls_rows[c] == 0) continue;
        ClassParams cp = h->cparams;
        cp.phase = 1;
        cp.row_cls = h->row_cls.as<uint8_t>();
        cp.cls = c;
        cp.sample_stride = (int)std::max<int64_t>(1, std::min<int64_t>(16, h->cls_rows[c] / 16384));
        float best = 3.4e38f;
        int best_pol = cp.accumulator, best_lg = h->cls_lg[c];
        const int base = lg_group(h->cls_avg_b[c]);
        for (int ci = 0; ci < npol && s == SPG_OK; ++ci) {
            const int pol = ci < 3 ? ci : SPG_ACC_LL;
            cp.accumulator = pol;
            HIPCHK(hipMemsetAsync((char *)dst + koff_bytes, 0, sizeof(long long) * NK, st));
            HIPCHK(hipMemsetAsync(&dst->kmax_num[0][0], 0, sizeof(dst->kmax_num), st));
            HIPCHK(launch_classify(m, h->rflops.as<int64_t>(), h->rflopsc.as<int64_t>(), h->rwin.as<int2>(),
                                   h->row_nnz.as<int32_t>(), h->row_words.as<int32_t>(), cp,
                                   h->kind_tmp.as<uint8_t>(), nullptr, dst, h->tmp.as<int64_t>(),
                                   h->koff_tmp.as<int64_t>(), st));
            HIPCHK(launch_partition(m, h->kind_tmp.as<uint8_t>(), h->perm_tmp.as<int32_t>(), h->tmp.as<int64_t>(),
                                    h->koff_tmp.as<int64_t>(), cp.phase, cp.heavy, dst, st));
            if ((s = pull_stats(h)) != SPG_OK) break;
            const DevStats hs = *h->hst;
            na.rs.rows = h->perm_tmp.as<int32_t>();
            na.rs.koff = h->koff_tmp.as<int64_t>();
            for (int lg = std::max(2, base - 1); lg <= std::min(6, base + 1); ++lg) {
                na.lg_gs = lg;
                float ms = 0;
                HIPCHK(hipEventRecord(e0, st));
                if ((s = launch_kinds<VT>(h, na, hs.kcount_num, hs.kmax_num, acc, false, pol)) != SPG_OK) break;
                HIPCHK(hipEventRecord(e1, st));
                HIPCHK(hipEventSynchronize(e1));
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                if (ms > 4.0f * best) break;
                HIPCHK(hipEventRecord(e0, st));
                if ((s = launch_kinds<VT>(h, na, hs.kcount_num, hs.kmax_num, acc, false, pol)) != SPG_OK) break;
                HIPCHK(hipEventRecord(e1, st));
                HIPCHK(hipEventSynchronize(e1));
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    best_pol = pol;
                    best_lg = lg;
                }
            }
        }
        if (s != SPG_OK) break;
        // the class's rows with its winner, into its own lists
        cp.accumulator = best_pol;
        cp.sample_stride = 1;
        uint8_t *kc = h->kind_cls.as<uint8_t>() + (size_t)c * m;
        int32_t *pc = h->perm_cls.as<int32_t>() + (size_t)c * m;
        int64_t *oc = h->koff_cls.as<int64_t>() + (size_t)c * (NK + 1);
        HIPCHK(hipMemsetAsync((char *)dst + koff_bytes, 0, sizeof(long long) * NK, st));
        HIPCHK(hipMemsetAsync(&dst->kmax_num[0][0], 0, sizeof(dst->kmax_num), st));
        HIPCHK(launch_classify(m, h->rflops.as<int64_t>(), h->rflopsc.as<int64_t>(), h->rwin.as<int2>(),
                               h->row_nnz.as<int32_t>(), h->row_words.as<int32_t>(), cp, kc, nullptr, dst,
                               h->tmp.as<int64_t>(), oc, st));
        HIPCHK(launch_partition(m, kc, pc, h->tmp.as<int64_t>(), oc, cp.phase, cp.heavy, dst, st));
        if ((s = pull_stats(h)) != SPG_OK) break;
        for (int k = 0; k < NK; ++k) {
            h->cls_kc[c][k] = h->hst->kcount_num[k];
            for (int f = 0; f < 3; ++f) h->cls_km[c][k][f] = h->hst->kmax_num[k][f];
        }
        h->cls_pol[c] = best_pol;
        h->cls_lg[c] = best_lg;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != SPG_OK) return s;
    // every row's kind in one array (position maps read it)
    HIPCHK(launch_kind_merge(m, h->row_cls.as<uint8_t>(), h->kind_cls.as<uint8_t>(), h->kind_num.as<uint8_t>(), st));
    h->cls_tuned = true;
    h->tuned = true;
    int major = 0;
    for (int c = 1; c < 4; ++c)
        if (h->cls_rows[c] > h->cls_rows[major]) major = c;
    h->stats.tuned_policy = h->cls_pol[major];
    h->stats.tuned_lanes = 1 << h->cls_lg[major];
    long long tot[NK] = {};
    for (int kk = 0; kk < NK; ++kk)
        for (int c = 0; c < 4; ++c) tot[kk] += h->cls_kc[c][kk];
    // every classified class's list counts the other classes' rows as empty
    int used = 0;
    for (int c = 0; c < 4; ++c) used += h->cls_rows[c] > 0;
    tot[K_EMPTY] -= (long long)(used - 1) * h->fp.m;
    rows_numeric_stats(h->stats, *h->hst, h->heavy_split, tot);
    return SPG_OK;
}

template <typename VT>
static spg_status numeric_impl(spg_handle h, const VT *aval, const VT *bval, int32_t *cci, VT *cval, int acc,
                               int64_t row_begin = -1, int64_t row_end = -1, bool vo = false) {
    hipStream_t st = h->stream;
    DevStats &hs = *h->hst;
    NumArgs<VT> na{};
    na.arp = h->arp64.as<int64_t>();
    na.aci = h->aci_used;
    na.aval = aval;
    na.brp = h->brp64.as<int64_t>();
    na.bci = h->bci_used;
    na.bval = bval;
    if (h->compressed) {
        na.bcrp = h->bcrp.as<int64_t>();
        na.bcw = h->bcw.as<uint2>();
    }
    na.rwin = h->rwin.as<int2>();
    na.coff = h->coff.as<int64_t>();
    na.b32 = h->fp.nnzb < (int64_t(1) << 29);
    na.nnzb = h->fp.nnzb;
    if (h->planned || h->segmented) {
        na.plan_off = h->plan_off.as<int64_t>();
        na.plan = h->plan.as<uint2>();
        na.row_words = h->row_words.as<int32_t>();
    }
    if (h->segmented) {
        na.plan_len = h->plan_len.as<int32_t>();
        na.sym_kind = h->kind_sym.as<uint8_t>();
    }
    na.cci = cci;
    na.cval = cval;
    na.rs.rows = h->perm_num.as<int32_t>();
    na.rs.koff = h->koff_num.as<int64_t>();
    na.st = h->dstats.as<DevStats>();
    na.lg_gs_or = lg_group(h->avg_len_c);
    na.lg_gs = h->lg_num;
    na.cbase_row = -1;
    if (row_begin >= 0) {  // one panel of rows: per-kind slices, output relative to the panel
        HIPCHK(ensure(h->krange, 16 * NK));
        HIPCHK(launch_kind_ranges(h->perm_num.as<int32_t>(), h->koff_num.as<int64_t>(), row_begin, row_end,
                                  h->krange.as<int64_t>(), h->stream));
        na.rs.rows = h->perm_num.as<int32_t>();
        na.rs.koff = h->koff_num.as<int64_t>();
        na.rs.range = h->krange.as<int64_t>();
        na.cbase_row = row_begin;
        spg_status s = launch_kinds<VT>(h, na, hs.kcount_num, hs.kmax_num, acc);
        if (s != SPG_OK || !h->heavy_split) return s;
        HIPCHK(ensure(h->krange_heavy, 16 * NK));
        HIPCHK(launch_kind_ranges(h->perm_heavy.as<int32_t>(), h->koff_heavy.as<int64_t>(), row_begin, row_end,
                                  h->krange_heavy.as<int64_t>(), h->stream));
        na.rs.rows = h->perm_heavy.as<int32_t>();
        na.rs.koff = h->koff_heavy.as<int64_t>();
        na.rs.range = h->krange_heavy.as<int64_t>();
        return launch_kinds<VT>(h, na, hs.kcount_heavy, hs.kmax_heavy, sizeof(VT) == 4 ? ACC_WIDE : acc);
    }
    if (h->opt.autotune && !h->tuned && !h->noalloc && !vo) {
        spg_status s = h->ncls ? autotune_classes<VT>(h, na, acc) : autotune<VT>(h, na, acc);
        if (s != SPG_OK) return s;
        na.lg_gs = h->lg_num;
    }
    if (vo && h->maps_ok) {
        na.map_off = h->map_off.as<int64_t>();
        na.map = h->map.as<uint16_t>();
    }
    spg_status s = SPG_OK;
    // the heaviest rows' segments (FP64 accumulation for FP32 values) go
    // through the other segmented rows' launch, taken first, so that the two
    // kinds of work overlap
    const bool merge_dg = h->heavy_split && h->sg_mode && hs.kcount_heavy[K_DG] > 0 && !(h->ncls && h->cls_tuned);
    const int acc_heavy = sizeof(VT) == 4 ? ACC_WIDE : acc;
    if (h->ncls && h->cls_tuned) {  // one launch set per product class
        for (int c = 0; c < 4 && s == SPG_OK; ++c) {
            if (h->cls_rows[c] == 0) continue;
            na.rs.rows = h->perm_cls.as<int32_t>() + (size_t)c * h->fp.m;
            na.rs.koff = h->koff_cls.as<int64_t>() + (size_t)c * (NK + 1);
            na.lg_gs = h->cls_lg[c];
            h->lg_map_cur = lg_map(h->cls_avg_b[c]);
            s = launch_kinds<VT>(h, na, h->cls_kc[c], h->cls_km[c], acc, vo, h->cls_pol[c]);
        }
        na.lg_gs = h->lg_num;
    } else {
        na.rs.rows = h->perm_num.as<int32_t>();
        na.rs.koff = h->koff_num.as<int64_t>();
        h->lg_map_cur = lg_map(h->avg_len);
        if (merge_dg) {
            na.rs2.rows = h->perm_heavy.as<int32_t>();
            na.rs2.koff = h->koff_heavy.as<int64_t>();
            na.rs2.range = nullptr;
        }
        s = launch_kinds<VT>(h, na, hs.kcount_num, hs.kmax_num, acc, vo, -1, merge_dg ? DG_MERGE : DG_OWN,
                             merge_dg ? hs.kcount_heavy[K_DG] : 0, acc_heavy);
        na.rs2 = RowSet{};
    }
    if (s != SPG_OK || !h->heavy_split) return s;
    // heaviest rows: FP64 accumulation for FP32 values (FP64 values: the same kernels)
    na.rs.rows = h->perm_heavy.as<int32_t>();
    na.rs.koff = h->koff_heavy.as<int64_t>();
    h->lg_map_cur = lg_map(h->avg_len);
    return launch_kinds<VT>(h, na, hs.kcount_heavy, hs.kmax_heavy, acc_heavy, vo, -1, merge_dg ? DG_SKIP : DG_OWN);
}
static spg_status numeric_check(spg_handle h, const spg_csr *A, const spg_csr *B, spg_csr_out *C) {
    if (!h->ready) return fail(h, SPG_ERR_NOT_READY, "spgemm_numeric before a successful spgemm_symbolic");
    spg_status s;
    if ((s = check_csr(h, A, "A", true)) != SPG_OK) return s;
    if ((s = check_csr(h, B, "B", true)) != SPG_OK) return s;
    if (!C) return fail(h, SPG_ERR_INVALID_ARG, "C is NULL");
    const Fingerprint &f = h->fp;
    if (A->nrows != f.m || A->ncols != f.n || B->ncols != f.k || A->nnz != f.nnza || B->nnz != f.nnzb ||
        A->row_ptr != f.arp || B->row_ptr != f.brp || A->col_idx != f.aci || B->col_idx != f.bci ||
        (int)A->rp_type != f.arpt || (int)B->rp_type != f.brpt)
        return fail(h, SPG_ERR_STRUCTURE_MISMATCH, "A or B differs from the operands of the symbolic phase");
    if (C->nrows != f.m || C->ncols != f.k) return fail(h, SPG_ERR_DIM_MISMATCH, "C must be A.nrows x B.ncols");
    if (C->nnz != h->nnzc) return fail(h, SPG_ERR_STRUCTURE_MISMATCH, "C.nnz differs from the symbolic nnz(C)");
    if (h->nnzc > 0 && (!C->col_idx || !C->values)) return fail(h, SPG_ERR_INVALID_ARG, "C arrays are NULL");
    if (A->dtype != B->dtype || A->dtype != C->dtype)
        return fail(h, SPG_ERR_INVALID_ARG, "A, B and C must share one dtype");
    if (h->batch.count) return fail(h, SPG_ERR_STRUCTURE_MISMATCH, "the plan is a batch: use spgemm_batch_numeric");
    return SPG_OK;
}

static spg_status numeric_entry(spg_handle h, const spg_csr *A, const spg_csr *B, spg_csr_out *C) {
    spg_status s;
    if ((s = numeric_check(h, A, B, C)) != SPG_OK) return s;
    if ((s = verify_struct(h)) != SPG_OK) return s;
    if (h->nnzc == 0) return SPG_OK;
    const bool vo = h->values_only;
    if (A->dtype == SPG_F64)
        return numeric_impl<double>(h, (const double *)A->values, (const double *)B->values, C->col_idx,
                                    (double *)C->values, ACC_NATIVE, -1, -1, vo);
    return numeric_impl<float>(h, (const float *)A->values, (const float *)B->values, C->col_idx,
                               (float *)C->values, fp32_acc(h), -1, -1, vo);
}

extern "C" spg_status spgemm_numeric(spg_handle h, const spg_csr *A, const spg_csr *B, spg_csr_out *C) {
    if (!h) return SPG_ERR_INVALID_ARG;
    h->err.clear();
    h->noalloc = false;
    return numeric_entry(h, A, B, C);
}

extern "C" spg_status spgemm_numeric_noalloc(spg_handle h, const spg_csr *A, const spg_csr *B, spg_csr_out *C) {
    if (!h) return SPG_ERR_INVALID_ARG;
    h->err.clear();
    if (!h->scr) return fail(h, SPG_ERR_INTERNAL, "no static scratch address for this device");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != h->device)
        return fail(h, SPG_ERR_INVALID_ARG, "the current device is not the handle's device");
    h->noalloc = true;
    spg_status s = numeric_entry(h, A, B, C);
    h->noalloc = false;
    return s;
}

// ------------------------------------------------------------------ reuse maps
// Position maps of the plan (Reuse case): for the rows of the wavefront and
// team kinds, the rank in C's row of every multiplication, from C's sorted
// columns cci (written by an earlier numeric call on this plan).  Sizes come
// from a scan of the mapped rows' multiplications (one host sync); if the
// maps cannot be allocated, reuse calls run the full numeric kernels.
static spg_status build_maps(spg_handle h, const int32_t *cci) {
    hipStream_t st = h->stream;
    const int64_t m = h->fp.m;
    h->maps_built = true;
    h->maps_ok = false;
    if (h->num_policy == SPG_ACC_LL) return SPG_OK;  // ranks need sorted rows: the full kernels run
    if (h->ncls && h->cls_tuned)
        for (int c = 0; c < 4; ++c)
            if (h->cls_rows[c] && h->cls_pol[c] == SPG_ACC_LL) return SPG_OK;
    HIPCHK(ensure(h->mflops, 4 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->map_off, 8 * (m + 1)));
    HIPCHK(launch_map_rows(m, h->kind_num.as<uint8_t>(), h->heavy_split ? h->kind_heavy.as<uint8_t>() : nullptr,
                           h->rflops.as<int64_t>(), h->mflops.as<int32_t>(), st));
    HIPCHK(launch_scan_i32(m, h->mflops.as<int32_t>(), h->map_off.as<int64_t>(), h->tmp.as<int64_t>(), st));
    HIPCHK(hipMemcpyAsync(h->hkoff + 3, h->map_off.as<int64_t>() + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int64_t total = h->hkoff[3];
    if (total == 0) return SPG_OK;
    if (ensure(h->map, 2 * (size_t)total) != hipSuccess) {
        (void)hipGetLastError();
        return SPG_OK;
    }
    const DevStats &hs = *h->hst;
    NumArgs<double> na{};
    na.arp = h->arp64.as<int64_t>();
    na.aci = h->aci_used;
    na.brp = h->brp64.as<int64_t>();
    na.bci = h->bci_used;
    na.coff = h->coff.as<int64_t>();
    na.map_off = h->map_off.as<int64_t>();
    na.map = h->map.as<uint16_t>();
    na.st = h->dstats.as<DevStats>();
    LaunchCfg lc{st, 0, h->cus};
    auto kinds = [&](const int32_t *perm, const int64_t *koff, const long long *kcount, const int (*kmax)[3],
                     double avg_b) {
        na.rs.rows = perm;
        na.rs.koff = koff;
        for (int K : {K_SR, K_DW, K_WH, K_HW}) {
            if (kcount[K] <= 0) continue;
            na.rs.kind = K;
            const int lgt = K == K_SR ? sr_lg(kmax[K_SR][1]) : 6;
            hipError_t e = launch_posmap(na, cci, lgt, lg_map(avg_b), lc, kcount[K]);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    if (h->ncls && h->cls_tuned) {
        for (int c = 0; c < 4; ++c) {
            if (h->cls_rows[c] == 0) continue;
            HIPCHK(kinds(h->perm_cls.as<int32_t>() + (size_t)c * m, h->koff_cls.as<int64_t>() + (size_t)c * (NK + 1),
                         h->cls_kc[c], h->cls_km[c], h->cls_avg_b[c]));
        }
    } else {
        HIPCHK(kinds(h->perm_num.as<int32_t>(), h->koff_num.as<int64_t>(), hs.kcount_num, hs.kmax_num, h->avg_len));
    }
    if (h->heavy_split)
        HIPCHK(kinds(h->perm_heavy.as<int32_t>(), h->koff_heavy.as<int64_t>(), hs.kcount_heavy, hs.kmax_heavy,
                     h->avg_len));
    h->maps_ok = true;
    return SPG_OK;
}

extern "C" spg_status spgemm_numeric_values(spg_handle h, const spg_csr *A, const spg_csr *B, spg_csr_out *C) {
    if (!h) return SPG_ERR_INVALID_ARG;
    h->err.clear();
    h->noalloc = false;
    if (!h->ready) return fail(h, SPG_ERR_NOT_READY, "spgemm_numeric_values before a successful spgemm_symbolic");
    if (h->batch.count) return fail(h, SPG_ERR_STRUCTURE_MISMATCH, "the plan is a batch: use spgemm_batch_numeric_values");
    spg_status s = numeric_check(h, A, B, C);
    if (s != SPG_OK) return s;
    if (!h->maps_built && h->nnzc > 0 && (s = build_maps(h, C->col_idx)) != SPG_OK) return s;
    h->values_only = true;
    s = numeric_entry(h, A, B, C);
    h->values_only = false;
    return s;
}

extern "C" spg_status spg_batch_choices(spg_handle h, int32_t count, int32_t *policy, int32_t *lanes) {
    if (!h || !policy || !lanes) return SPG_ERR_INVALID_ARG;
    h->err.clear();
    if (!h->ready || h->batch.count == 0) return fail(h, SPG_ERR_NOT_READY, "no batch plan");
    if (count != h->batch.count) return fail(h, SPG_ERR_INVALID_ARG, "count differs from the batch");
    for (int i = 0; i < count; ++i) {
        const int c = h->batch.a[i].cls;
        const bool per_cls = h->ncls && h->cls_tuned;
        policy[i] = per_cls ? h->cls_pol[c] : h->num_policy;
        lanes[i] = 1 << (per_cls ? h->cls_lg[c] : h->lg_num);
    }
    return SPG_OK;
}

// ------------------------------------------------------------------ masked
template <typename VT>
static spg_status masked_impl(spg_handle h, const spg_csr *A, const spg_csr *B, const spg_csr *M, VT *out,
                              int structural) {
    hipStream_t st = h->stream;
    const int64_t m = A->nrows, n = B->nrows, k = B->ncols;
    HIPCHK(ensure(h->mk_arp, 8 * (m + 1)));
    HIPCHK(ensure(h->mk_brp, 8 * (n + 1)));
    HIPCHK(ensure(h->mk_mrp, 8 * (m + 1)));
    HIPCHK(ensure(h->mk_rows, 8 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->mk_cnt, 8 * sizeof(int)));
    int *cnt = h->mk_cnt.as<int>();  // [0..1] rows per kind, [2..3] longest mask row per kind, [4] bad input
    int32_t *rows1 = h->mk_rows.as<int32_t>(), *rows2 = rows1 + m;
    HIPCHK(launch_fill_i32(cnt, 8, 0, st));
    HIPCHK(launch_copy_rp(m + 1, A->row_ptr, A->rp_type == SPG_I64, A->nnz, h->mk_arp.as<int64_t>(), n + 1,
                          B->row_ptr, B->rp_type == SPG_I64, B->nnz, h->mk_brp.as<int64_t>(), cnt + 4, st));
    HIPCHK(launch_copy_rp(m + 1, M->row_ptr, M->rp_type == SPG_I64, M->nnz, h->mk_mrp.as<int64_t>(), 0, nullptr, 0,
                          0, nullptr, cnt + 4, st));
    if (M->nnz > 0) HIPCHK(launch_fill_i32((int32_t *)out, M->nnz * (int64_t)(sizeof(VT) / 4), 0, st));
    HIPCHK(launch_mask_class(m, h->mk_arp.as<int64_t>(), h->mk_mrp.as<int64_t>(), MW_MAX, rows1, rows2, cnt, st));
    int *hc = (int *)(h->hkoff + 8);
    HIPCHK(hipMemcpyAsync(hc, cnt, 5 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hc[4]) return fail(h, SPG_ERR_INVALID_ARG, "malformed CSR: row_ptr out of range or not monotone");
    MaskArgs<VT> a{};
    a.arp = h->mk_arp.as<int64_t>();
    a.aci = A->col_idx;
    a.aval = structural ? nullptr : (const VT *)A->values;
    a.brp = h->mk_brp.as<int64_t>();
    a.bci = B->col_idx;
    a.bval = structural ? nullptr : (const VT *)B->values;
    a.mrp = h->mk_mrp.as<int64_t>();
    a.mci = M->col_idx;
    a.out = out;
    a.n = n;
    a.k = k;
    a.lg_gs = lg_group(n ? std::max(1.0, (double)B->nnz / (double)n) : 1.0);
    a.structural = structural;
    a.bad = cnt + 4;
    LaunchCfg lc{st, 0, h->cus};
    if (hc[0] > 0) {
        a.rows = rows1;
        a.nrows = hc[0];
        int lg = 4;
        while ((1 << lg) < 2 * hc[2]) ++lg;
        HIPCHK(launch_mask_w<VT>(a, lg, hc[2], lc));
    }
    if (hc[1] > 0) {
        a.rows = rows2;
        a.nrows = hc[1];
        a.arena_cap = pow2_at_least(2 * (int64_t)hc[3], 64);
        int grid = (int)std::min<int64_t>(((hc[1] + 7) / 8) * 8, 2 * (int64_t)h->cus);
        HIPCHK(ensure(h->mk_arena, (size_t)12 * a.arena_cap * grid));
        a.arena = h->mk_arena.p;
        lc.grid = grid;
        HIPCHK(launch_mask_g<VT>(a, lc));
    }
    HIPCHK(hipMemcpyAsync(hc + 4, cnt + 4, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hc[4] & 1) return fail(h, SPG_ERR_INVALID_ARG, "malformed CSR: a column index out of range");
    if (hc[4]) return fail(h, SPG_ERR_INTERNAL, "masked product: arena too small");
    return SPG_OK;
}

extern "C" spg_status spgemm_masked(spg_handle h, const spg_csr *A, const spg_csr *B, const spg_csr *M, void *out,
                                    int structural) {
    if (!h) return SPG_ERR_INVALID_ARG;
    h->err.clear();
    spg_status s;
    const bool vals = structural == 0;
    if (structural != 0 && structural != 1) return fail(h, SPG_ERR_INVALID_ARG, "structural must be 0 or 1");
    if ((s = check_csr(h, A, "A", vals)) != SPG_OK) return s;
    if ((s = check_csr(h, B, "B", vals)) != SPG_OK) return s;
    if ((s = check_csr(h, M, "M", false)) != SPG_OK) return s;
    if (A->ncols != B->nrows) return fail(h, SPG_ERR_DIM_MISMATCH, "A.ncols != B.nrows");
    if (M->nrows != A->nrows || M->ncols != B->ncols) return fail(h, SPG_ERR_DIM_MISMATCH, "M must be A.nrows x B.ncols");
    if (A->dtype != SPG_F64 && A->dtype != SPG_F32) return fail(h, SPG_ERR_INVALID_ARG, "bad dtype");
    if (vals && B->dtype != A->dtype) return fail(h, SPG_ERR_INVALID_ARG, "A and B must share one dtype");
    if (M->nnz > 0 && !out) return fail(h, SPG_ERR_INVALID_ARG, "out is NULL");
    if (M->nnz == 0) return SPG_OK;
    if (A->dtype == SPG_F64) return masked_impl<double>(h, A, B, M, (double *)out, structural);
    return masked_impl<float>(h, A, B, M, (float *)out, structural);
}

// ------------------------------------------------------------------ backward
template <typename VT>
static spg_status backward_impl(spg_handle h, const spg_csr *A, const spg_csr *B, const spg_csr *G, void *dA,
                                void *dB) {
    BwdArgs<VT> ba{};
    ba.m = h->fp.m;
    ba.nnza = A->nnz;
    ba.nnzb = B->nnz;
    ba.arp = h->arp64.as<int64_t>();
    ba.aci = A->col_idx;
    ba.aval = (const VT *)A->values;
    ba.brp = h->brp64.as<int64_t>();
    ba.bci = B->col_idx;
    ba.bval = (const VT *)B->values;
    ba.coff = h->coff.as<int64_t>();
    ba.gci = G->col_idx;
    ba.gval = (const VT *)G->values;
    ba.dA = (VT *)dA;
    ba.dB = (VT *)dB;
    ba.lg_gs = lg_group(h->avg_len);
    ba.st = h->dstats.as<DevStats>();
    LaunchCfg lc{h->stream, 0, h->cus};
    HIPCHK(launch_backward<VT>(ba, lc));
    return SPG_OK;
}

extern "C" spg_status spgemm_backward(spg_handle h, const spg_csr *A, const spg_csr *B, const spg_csr *G,
                                      void *dA, void *dB) {
    if (!h) return SPG_ERR_INVALID_ARG;
    h->err.clear();
    if (!h->ready) return fail(h, SPG_ERR_NOT_READY, "spgemm_backward before a successful spgemm_symbolic");
    if (h->batch.count) return fail(h, SPG_ERR_UNSUPPORTED, "backward of a batch plan");
    spg_status s;
    if ((s = check_csr(h, A, "A", true)) != SPG_OK) return s;
    if ((s = check_csr(h, B, "B", true)) != SPG_OK) return s;
    if ((s = check_csr(h, G, "G", true)) != SPG_OK) return s;
    if (h->num_policy == SPG_ACC_LL)
        return fail(h, SPG_ERR_UNSUPPORTED, "backward needs C's columns sorted; the plan's numeric phase leaves "
                                            "rows unsorted (SPG_ACC_LL)");
    const Fingerprint &f = h->fp;
    if (A->nrows != f.m || A->ncols != f.n || B->ncols != f.k || A->nnz != f.nnza || B->nnz != f.nnzb ||
        A->row_ptr != f.arp || B->row_ptr != f.brp || A->col_idx != f.aci || B->col_idx != f.bci ||
        (int)A->rp_type != f.arpt || (int)B->rp_type != f.brpt)
        return fail(h, SPG_ERR_STRUCTURE_MISMATCH, "A or B differs from the operands of the symbolic phase");
    if (G->nrows != f.m || G->ncols != f.k || G->nnz != h->nnzc)
        return fail(h, SPG_ERR_STRUCTURE_MISMATCH, "G must have the structure of C");
    if (A->dtype != B->dtype || A->dtype != G->dtype)
        return fail(h, SPG_ERR_INVALID_ARG, "A, B and G must share one dtype");
    if ((s = verify_struct(h)) != SPG_OK) return s;
    if (A->dtype == SPG_F64) return backward_impl<double>(h, A, B, G, dA, dB);
    return backward_impl<float>(h, A, B, G, dA, dB);
}

// ------------------------------------------------------------------ batch
static spg_status upload_desc(spg_handle h, const std::vector<BatchDesc> &d, BatchDesc **out) {
    HIPCHK(ensure(h->batch.desc, sizeof(BatchDesc) * d.size() * 4 + 16));
    // four regions: A, B, C row pointers, scratch for gather/scatter descriptors
    *out = h->batch.desc.as<BatchDesc>();
    HIPCHK(hipMemcpyAsync(*out, d.data(), sizeof(BatchDesc) * d.size(), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return SPG_OK;
}

extern "C" spg_status spgemm_batch_symbolic(spg_handle h, int32_t count, const spg_csr *A, const spg_csr *B,
                                            void *const *C_row_ptr, spg_itype c_rpt, int64_t *nnz_c) {
    if (!h) return SPG_ERR_INVALID_ARG;
    h->err.clear();
    if (count <= 0 || !A || !B || !C_row_ptr || !nnz_c) return fail(h, SPG_ERR_INVALID_ARG, "bad batch arguments");
    if (c_rpt != SPG_I32 && c_rpt != SPG_I64) return fail(h, SPG_ERR_INVALID_ARG, "bad C rp_type");
    spg_status s;
    auto &bt = h->batch;
    h->ready = false;
    bt.count = 0;
    bt.a.assign(count, BatchDesc{});
    bt.b.assign(count, BatchDesc{});
    bt.c.assign(count, BatchDesc{});
    int64_t R = 0, N = 0, NA = 0, NB = 0, K = 0;
    bt.max_rows = bt.max_nnza = bt.max_nnzb = 0;
    for (int i = 0; i < count; ++i) {
        if ((s = check_csr(h, &A[i], "A[i]", false)) != SPG_OK) return s;
        if ((s = check_csr(h, &B[i], "B[i]", false)) != SPG_OK) return s;
        if (A[i].ncols != B[i].nrows) return fail(h, SPG_ERR_DIM_MISMATCH, "A[i].ncols != B[i].nrows");
        if (!C_row_ptr[i]) return fail(h, SPG_ERR_INVALID_ARG, "C_row_ptr[i] is NULL");
        BatchDesc &a = bt.a[i], &b = bt.b[i], &c = bt.c[i];
        a.rp = A[i].row_ptr; a.ci = A[i].col_idx; a.nrows = A[i].nrows; a.ncols = A[i].ncols; a.nnz = A[i].nnz;
        a.row_off = R; a.nnz_off = NA; a.col_add = (int32_t)N; a.rp64 = A[i].rp_type == SPG_I64;
        b.rp = B[i].row_ptr; b.ci = B[i].col_idx; b.nrows = B[i].nrows; b.ncols = B[i].ncols; b.nnz = B[i].nnz;
        b.row_off = N; b.nnz_off = NB; b.col_add = 0; b.rp64 = B[i].rp_type == SPG_I64;
        c.rp = C_row_ptr[i]; c.nrows = A[i].nrows; c.ncols = B[i].ncols; c.row_off = R; c.rp64 = c_rpt == SPG_I64;
        R += A[i].nrows;
        N += B[i].nrows;
        NA += A[i].nnz;
        NB += B[i].nnz;
        K = std::max<int64_t>(K, B[i].ncols);
        bt.max_rows = std::max<int64_t>(bt.max_rows, std::max(A[i].nrows, B[i].nrows));
        bt.max_nnza = std::max<int64_t>(bt.max_nnza, A[i].nnz);
        bt.max_nnzb = std::max<int64_t>(bt.max_nnzb, B[i].nnz);
        if (N > INT32_MAX || R > INT32_MAX - 1)
            return fail(h, SPG_ERR_UNSUPPORTED, "a batch with more than 2^31-1 rows of A or B");
    }
    bt.rows = R;
    bt.nnza = NA;
    bt.nnzb = NB;
    hipStream_t st = h->stream;
    if ((s = plan_buffers(h, R, N, NB)) != SPG_OK) return s;
    HIPCHK(ensure(bt.aci, 4 * std::max<int64_t>(NA, 1)));
    HIPCHK(ensure(bt.bci, 4 * std::max<int64_t>(NB, 1)));
    DevStats *dst = h->dstats.as<DevStats>();
    HIPCHK(hipMemsetAsync(dst, 0, sizeof(DevStats), st));
    BatchDesc *dev = nullptr;
    if ((s = upload_desc(h, bt.a, &dev)) != SPG_OK) return s;
    HIPCHK(launch_batch_struct(dev, count, std::max(bt.max_rows + 1, bt.max_nnza), h->arp64.as<int64_t>(),
                               bt.aci.as<int32_t>(), &dst->bad_input, st));
    // B: the same kernel, column bound = k_i, no offset
    if ((s = upload_desc(h, bt.b, &dev)) != SPG_OK) return s;
    HIPCHK(launch_batch_struct(dev, count, std::max(bt.max_rows + 1, bt.max_nnzb), h->brp64.as<int64_t>(),
                               bt.bci.as<int32_t>(), &dst->bad_input, st));
    if ((s = pull_stats(h)) != SPG_OK) return s;
    if (h->hst->bad_input) return fail(h, SPG_ERR_INVALID_ARG, "malformed CSR in the batch");
    HIPCHK(hipMemsetAsync(dst, 0, sizeof(DevStats), st));
    int64_t nnzc = 0;
    if ((s = symbolic_core(h, R, N, K, NA, NB, bt.aci.as<int32_t>(), bt.bci.as<int32_t>(), &nnzc)) != SPG_OK)
        return s;
    // per-product entries of C, then each C_i.row_ptr
    if ((s = upload_desc(h, bt.c, &dev)) != SPG_OK) return s;
    HIPCHK(ensure(h->blens, 16 * (size_t)count));
    HIPCHK(launch_batch_bounds(dev, count, h->coff.as<int64_t>(), h->blens.as<int64_t>(), st));
    std::vector<int64_t> bnd(2 * (size_t)count);
    HIPCHK(hipMemcpyAsync(bnd.data(), h->blens.p, 16 * (size_t)count, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bt.c_off.assign(count, 0);
    bt.c_nnz.assign(count, 0);
    bt.max_nnzc = 0;
    for (int i = 0; i < count; ++i) {
        bt.c_off[i] = bnd[2 * i];
        bt.c_nnz[i] = bnd[2 * i + 1] - bnd[2 * i];
        bt.c[i].nnz = bt.c_nnz[i];
        bt.c[i].nnz_off = bt.c_off[i];
        bt.max_nnzc = std::max(bt.max_nnzc, bt.c_nnz[i]);
        if (c_rpt == SPG_I32 && bt.c_nnz[i] > INT32_MAX)
            return fail(h, SPG_ERR_INDEX_OVERFLOW, "nnz(C_i) exceeds an int32 row_ptr; ask for SPG_I64");
        nnz_c[i] = bt.c_nnz[i];
    }
    HIPCHK(launch_batch_rp_out(dev, count, bt.max_rows, h->coff.as<int64_t>(), st));
    // product classes by the average row size of C_i (<= 16, 128, 1024, more)
    h->ncls = 0;
    h->cls_tuned = false;
    {
        int64_t rows_c[4] = {}, nb_c[4] = {}, nbr_c[4] = {};
        for (int i = 0; i < count; ++i) {
            const double avg = (double)bt.c_nnz[i] / (double)std::max<int64_t>(1, bt.a[i].nrows);
            const int c = avg <= 16 ? 0 : avg <= 128 ? 1 : avg <= 1024 ? 2 : 3;
            bt.a[i].cls = c;
            rows_c[c] += bt.a[i].nrows;
            nb_c[c] += bt.b[i].nnz;
            nbr_c[c] += bt.b[i].nrows;
        }
        int used = 0;
        for (int c = 0; c < 4; ++c) {
            h->cls_rows[c] = (int)std::min<int64_t>(rows_c[c], INT32_MAX);
            h->cls_avg_b[c] = nbr_c[c] ? std::max(1.0, (double)nb_c[c] / (double)nbr_c[c]) : 1.0;
            used += rows_c[c] > 0;
        }
        if (used > 1) {
            HIPCHK(ensure(h->row_cls, std::max<int64_t>(R, 1)));
            if ((s = upload_desc(h, bt.a, &dev)) != SPG_OK) return s;
            HIPCHK(launch_batch_row_class(dev, count, bt.max_rows, h->row_cls.as<uint8_t>(), st));
            h->ncls = 4;
        }
    }
    h->nnzc = nnzc;
    Fingerprint &fp = h->fp;
    fp = Fingerprint{};
    fp.m = R; fp.n = N; fp.k = K; fp.nnza = NA; fp.nnzb = NB;
    bt.count = count;
    h->ready = true;
    return SPG_OK;
}

template <typename VT>
static spg_status batch_numeric_impl(spg_handle h, int32_t count, const spg_csr *A, const spg_csr *B,
                                     spg_csr_out *C, int acc, bool vo) {
    auto &bt = h->batch;
    hipStream_t st = h->stream;
    const size_t vb = sizeof(VT);
    // values of A / B: zero-copy when the batch is laid out back to back,
    // otherwise gathered into a staging buffer
    bool a_contig = true, b_contig = true, c_contig = true;
    for (int i = 0; i < count; ++i) {
        a_contig &= A[i].nnz == 0 || (const char *)A[i].values == (const char *)A[0].values + vb * bt.a[i].nnz_off;
        b_contig &= B[i].nnz == 0 || (const char *)B[i].values == (const char *)B[0].values + vb * bt.b[i].nnz_off;
        c_contig &= C[i].nnz == 0 || (C[i].col_idx == C[0].col_idx + bt.c_off[i] &&
                                      (const char *)C[i].values == (const char *)C[0].values + vb * bt.c_off[i]);
    }
    const VT *aval = (const VT *)A[0].values, *bval = (const VT *)B[0].values;
    int32_t *cci = C[0].col_idx;
    VT *cval = (VT *)C[0].values;
    spg_status s;
    BatchDesc *dev = nullptr;
    if (!a_contig) {
        std::vector<BatchDesc> d = bt.a;
        for (int i = 0; i < count; ++i) d[i].vals = A[i].values;
        HIPCHK(ensure(bt.astage, vb * std::max<int64_t>(bt.nnza, 1)));
        if ((s = upload_desc(h, d, &dev)) != SPG_OK) return s;
        HIPCHK(launch_batch_gather(dev, count, bt.max_nnza, bt.astage.p, (int)vb, st));
        aval = bt.astage.as<VT>();
    }
    if (!b_contig) {
        std::vector<BatchDesc> d = bt.b;
        for (int i = 0; i < count; ++i) d[i].vals = B[i].values;
        HIPCHK(ensure(bt.bstage, vb * std::max<int64_t>(bt.nnzb, 1)));
        if ((s = upload_desc(h, d, &dev)) != SPG_OK) return s;
        HIPCHK(launch_batch_gather(dev, count, bt.max_nnzb, bt.bstage.p, (int)vb, st));
        bval = bt.bstage.as<VT>();
    }
    if (!c_contig) {
        HIPCHK(ensure(bt.cci, 4 * std::max<int64_t>(h->nnzc, 1)));
        HIPCHK(ensure(bt.cval, vb * std::max<int64_t>(h->nnzc, 1)));
        cci = bt.cci.as<int32_t>();
        cval = bt.cval.as<VT>();
    }
    // structure known (values only): position maps from the back-to-back C
    // columns an earlier call wrote; outputs gathered through staging take the
    // full kernels
    vo = vo && c_contig;
    if (vo && !h->maps_built && h->nnzc > 0 && (s = build_maps(h, cci)) != SPG_OK) return s;
    if (h->nnzc > 0) {
        if ((s = numeric_impl<VT>(h, aval, bval, cci, cval, acc, -1, -1, vo)) != SPG_OK) return s;
    }
    if (!c_contig) {
        std::vector<BatchDesc> d = bt.c;
        for (int i = 0; i < count; ++i) d[i].vals = C[i].col_idx;
        if ((s = upload_desc(h, d, &dev)) != SPG_OK) return s;
        HIPCHK(launch_batch_scatter(dev, count, bt.max_nnzc, cci, 4, st));
        for (int i = 0; i < count; ++i) d[i].vals = C[i].values;
        HIPCHK(hipStreamSynchronize(st));
        if ((s = upload_desc(h, d, &dev)) != SPG_OK) return s;
        HIPCHK(launch_batch_scatter(dev, count, bt.max_nnzc, cval, (int)vb, st));
    }
    return SPG_OK;
}

static spg_status batch_entry(spg_handle h, int32_t count, const spg_csr *A, const spg_csr *B, spg_csr_out *C,
                              bool vo) {
    auto &bt = h->batch;
    if (!h->ready || bt.count == 0) return fail(h, SPG_ERR_NOT_READY, "spgemm_batch_numeric before spgemm_batch_symbolic");
    if (count != bt.count || !A || !B || !C) return fail(h, SPG_ERR_STRUCTURE_MISMATCH, "batch size differs from the plan");
    spg_status s;
    const int dt = A[0].dtype;
    for (int i = 0; i < count; ++i) {
        if ((s = check_csr(h, &A[i], "A[i]", true)) != SPG_OK) return s;
        if ((s = check_csr(h, &B[i], "B[i]", true)) != SPG_OK) return s;
        const BatchDesc &a = bt.a[i], &b = bt.b[i];
        if (A[i].row_ptr != a.rp || A[i].col_idx != a.ci || A[i].nnz != a.nnz || A[i].nrows != a.nrows ||
            B[i].row_ptr != b.rp || B[i].col_idx != b.ci || B[i].nnz != b.nnz || B[i].nrows != b.nrows ||
            B[i].ncols != b.ncols)
            return fail(h, SPG_ERR_STRUCTURE_MISMATCH, "A[i] or B[i] differs from the symbolic batch");
        if (C[i].nrows != a.nrows || C[i].ncols != b.ncols || C[i].nnz != bt.c_nnz[i])
            return fail(h, SPG_ERR_STRUCTURE_MISMATCH, "C[i] shape or nnz differs from the symbolic batch");
        if (C[i].nnz > 0 && (!C[i].col_idx || !C[i].values)) return fail(h, SPG_ERR_INVALID_ARG, "C[i] arrays are NULL");
        if ((int)A[i].dtype != dt || (int)B[i].dtype != dt || (int)C[i].dtype != dt)
            return fail(h, SPG_ERR_INVALID_ARG, "one dtype for the whole batch");
    }
    if (dt == SPG_F64) return batch_numeric_impl<double>(h, count, A, B, C, ACC_NATIVE, vo);
    return batch_numeric_impl<float>(h, count, A, B, C, fp32_acc(h), vo);
}

extern "C" spg_status spgemm_batch_numeric(spg_handle h, int32_t count, const spg_csr *A, const spg_csr *B,
                                           spg_csr_out *C) {
    if (!h) return SPG_ERR_INVALID_ARG;
    h->err.clear();
    h->noalloc = false;
    return batch_entry(h, count, A, B, C, false);
}

extern "C" spg_status spgemm_batch_numeric_values(spg_handle h, int32_t count, const spg_csr *A,
                                                  const spg_csr *B, spg_csr_out *C) {
    if (!h) return SPG_ERR_INVALID_ARG;
    h->err.clear();
    h->noalloc = false;
    return batch_entry(h, count, A, B, C, true);
}

extern "C" spg_status spgemm_numeric_rows(spg_handle h, const spg_csr *A, const spg_csr *B, int64_t row_begin,
                                          int64_t row_end, int32_t *C_col_idx, void *C_values) {
    if (!h) return SPG_ERR_INVALID_ARG;
    h->err.clear();
    if (!h->ready) return fail(h, SPG_ERR_NOT_READY, "spgemm_numeric_rows before a successful spgemm_symbolic");
    if (h->batch.count) return fail(h, SPG_ERR_STRUCTURE_MISMATCH, "the plan is a batch");
    spg_status s;
    if ((s = check_csr(h, A, "A", true)) != SPG_OK) return s;
    if ((s = check_csr(h, B, "B", true)) != SPG_OK) return s;
    const Fingerprint &f = h->fp;
    if (A->nrows != f.m || A->ncols != f.n || B->ncols != f.k || A->nnz != f.nnza || B->nnz != f.nnzb ||
        A->row_ptr != f.arp || B->row_ptr != f.brp || A->col_idx != f.aci || B->col_idx != f.bci ||
        (int)A->rp_type != f.arpt || (int)B->rp_type != f.brpt)
        return fail(h, SPG_ERR_STRUCTURE_MISMATCH, "A or B differs from the operands of the symbolic phase");
    if (row_begin < 0 || row_end < row_begin || row_end > f.m)
        return fail(h, SPG_ERR_INVALID_ARG, "need 0 <= row_begin <= row_end <= A.nrows");
    if (A->dtype != B->dtype) return fail(h, SPG_ERR_INVALID_ARG, "A and B must share one dtype");
    if (row_begin == row_end || h->nnzc == 0) return SPG_OK;
    if (!C_col_idx || !C_values) return fail(h, SPG_ERR_INVALID_ARG, "panel arrays are NULL");
    if ((s = verify_struct(h)) != SPG_OK) return s;
    if (A->dtype == SPG_F64)
        return numeric_impl<double>(h, (const double *)A->values, (const double *)B->values, C_col_idx,
                                    (double *)C_values, ACC_NATIVE, row_begin, row_end);
    return numeric_impl<float>(h, (const float *)A->values, (const float *)B->values, C_col_idx,
                               (float *)C_values, fp32_acc(h), row_begin, row_end);
}
