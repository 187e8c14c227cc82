// Host side of the C ABI: the handle, the symbolic plan kept for reuse, and
// the orchestration of the two phases (Algorithm 2):
//   symbolic: row_ptr copies -> B row statistics -> per-row flops / windows
//             -> [host reads f_m, compressed f_m] -> compression of B if it
//             removes more than 15% of the flops -> rows classified by kernel
//             kind -> [host reads per-kind sizes] -> one persistent launch per
//             kind -> scan -> numeric classification -> [host reads nnz(C)]
//   numeric:  one persistent launch per kind, no host synchronisation.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>

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
    int64_t *hkoff = nullptr;           // pinned: koff_sym[NK+1], koff_num[NK+1], nnzc
    spg_stats stats{};

    DevBuf arp64, brp64, binfo, ulist, uflag, bcrp, bcsi, bcs, rflops, rflopsc, rwin, row_nnz, coff, kind_sym,
        kind_num, perm_sym, perm_num, koff_sym, koff_num, tmp, dstats, queue, arena, l2k, l2v, blens;
    size_t arena_bytes_zeroed = 0;
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

int lg_group(double avg) {
    // lanes per B row: the average length rounded up to a power of two, 4..64
    int lg = 2;
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
}

static spg_status check_options(spg_handle h, const spg_options *o) {
    if (o->compression < -1 || o->compression > 1) return fail(h, SPG_ERR_INVALID_ARG, "compression must be -1, 0 or 1");
    if (!(o->cf_threshold > 0.0 && o->cf_threshold <= 1.0)) return fail(h, SPG_ERR_INVALID_ARG, "cf_threshold in (0, 1]");
    if (o->accumulator < 0 || o->accumulator > 3) return fail(h, SPG_ERR_INVALID_ARG, "bad accumulator");
    if (o->fp32_mode < 0 || o->fp32_mode > 2) return fail(h, SPG_ERR_INVALID_ARG, "bad fp32_mode");
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
    if (e == hipSuccess) e = ensure(h->queue, sizeof(int32_t) * XCDS * NK);
    if (e != hipSuccess) {
        spg_destroy(h);
        return SPG_ERR_HIP;
    }
    h->lds_max = (size_t)lds;
    // window words the workgroup dense kernel can hold next to its staging area
    // LDS bytes = 4*nw (bits) + nw/8 (summary) + staging + alignment slack
    const size_t over = 8 * WG_BIG * 3 + 8 * (WG_BIG / WAVE + 2) + 128;
    int64_t words = h->lds_max > over ? (int64_t)((h->lds_max - over) * 8 / 33) : 0;
    words = (words / 32) * 32;
    h->dg_nw_max = (int)std::min<int64_t>(DG_NW_MAX, std::max<int64_t>(words, 32));
    *out = h;
    return SPG_OK;
}

spg_status spg_destroy(spg_handle h) {
    if (!h) return SPG_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(h->stream);
    DevBuf *bufs[] = {&h->arp64, &h->brp64, &h->binfo, &h->ulist, &h->uflag, &h->bcrp, &h->bcsi, &h->bcs,
                      &h->rflops, &h->rflopsc, &h->rwin, &h->row_nnz, &h->coff, &h->kind_sym, &h->kind_num,
                      &h->perm_sym, &h->perm_num, &h->koff_sym, &h->koff_num, &h->tmp, &h->dstats, &h->queue,
                      &h->arena, &h->l2k, &h->l2v, &h->blens};
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
    const int64_t m = A->nrows, n = B->nrows, k = B->ncols;
    hipStream_t st = h->stream;
    Fingerprint fp;
    fp.m = m; fp.n = n; fp.k = k; fp.nnza = A->nnz; fp.nnzb = B->nnz;
    fp.arp = A->row_ptr; fp.brp = B->row_ptr; fp.aci = A->col_idx; fp.bci = B->col_idx;
    fp.arpt = A->rp_type; fp.brpt = B->rp_type;

    HIPCHK(ensure(h->arp64, 8 * (m + 1)));
    HIPCHK(ensure(h->brp64, 8 * (n + 1)));
    HIPCHK(ensure(h->binfo, sizeof(BRow) * std::max<int64_t>(n, 1)));
    HIPCHK(ensure(h->ulist, 4 * std::max<int64_t>(n, 1)));
    HIPCHK(ensure(h->uflag, std::max<int64_t>(n, 1)));
    HIPCHK(ensure(h->bcrp, 8 * (n + 1)));
    HIPCHK(ensure(h->rflops, 8 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->rflopsc, 8 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->rwin, 8 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->row_nnz, 4 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->coff, 8 * (m + 1)));
    HIPCHK(ensure(h->kind_sym, std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->kind_num, std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->perm_sym, 4 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->perm_num, 4 * std::max<int64_t>(m, 1)));
    HIPCHK(ensure(h->koff_sym, 8 * (NK + 1)));
    HIPCHK(ensure(h->koff_num, 8 * (NK + 1)));
    const int64_t tmp_elems = std::max({scan_tmp_elems(m), scan_tmp_elems(n), part_tmp_elems(m)});
    HIPCHK(ensure(h->tmp, 8 * tmp_elems));

    DevStats *dst = h->dstats.as<DevStats>();
    HIPCHK(hipMemsetAsync(dst, 0, sizeof(DevStats), st));
    int *bad = &dst->bad_input;
    HIPCHK(launch_copy_rp(m + 1, A->row_ptr, A->rp_type == SPG_I64, A->nnz, h->arp64.as<int64_t>(), bad, st));
    HIPCHK(launch_copy_rp(n + 1, B->row_ptr, B->rp_type == SPG_I64, B->nnz, h->brp64.as<int64_t>(), bad, st));
    HIPCHK(launch_check_cols(A->nnz, A->col_idx, n, bad, st));
    HIPCHK(launch_check_cols(B->nnz, B->col_idx, k, bad, st));
    // The structure kernels below index B by A's columns: they run only on
    // validated input, so a malformed operand is rejected before any of them.
    if ((s = pull_stats(h)) != SPG_OK) return s;
    if (h->hst->bad_input) return fail(h, SPG_ERR_INVALID_ARG, "malformed CSR: row_ptr or col_idx out of range");

    const int64_t *arp = h->arp64.as<int64_t>(), *brp = h->brp64.as<int64_t>();
    BRow *bi = h->binfo.as<BRow>();
    HIPCHK(launch_brow(n, brp, B->col_idx, bi, h->ulist.as<int32_t>(), dst, st));
    HIPCHK(launch_brow_unsorted(h->ulist.as<int32_t>(), &dst->unsorted, brp, B->col_idx, bi, dst, st));
    HIPCHK(launch_rowinfo(m, arp, A->col_idx, bi, h->rflops.as<int64_t>(), h->rflopsc.as<int64_t>(),
                          h->rwin.as<int2>(), dst, st));
    if ((s = pull_stats(h)) != SPG_OK) return s;  // host sync 1: flop counts
    const DevStats hs1 = *h->hst;
    if (hs1.bad_window)
        return fail(h, SPG_ERR_UNSUPPORTED, "a row of B with unsorted columns spans more than 2^19 columns");

    const double fm = (double)hs1.fm, fmc = (double)hs1.fmc;
    bool comp = false;
    if (h->opt.compression == 1) comp = true;
    else if (h->opt.compression == -1) comp = hs1.fm > 0 && fmc < h->opt.cf_threshold * fm;
    h->avg_len = A->nnz ? std::max(1.0, fm / (double)A->nnz) : 1.0;
    h->avg_len_c = A->nnz ? std::max(1.0, (comp ? fmc : fm) / (double)A->nnz) : 1.0;

    if (comp) {
        // compressed B (Compression subsection): lengths -> offsets -> (word, bits) pairs
        HIPCHK(ensure(h->blens, 8 * std::max<int64_t>(n, 1)));
        HIPCHK(launch_brow_lens(n, bi, 1, h->blens.as<int64_t>(), st));
        HIPCHK(launch_scan_i64(n, h->blens.as<int64_t>(), h->bcrp.as<int64_t>(), h->tmp.as<int64_t>(), st));
        HIPCHK(ensure(h->bcsi, 4 * std::max<int64_t>(B->nnz, 1)));
        HIPCHK(ensure(h->bcs, 4 * std::max<int64_t>(B->nnz, 1)));
        HIPCHK(hipMemsetAsync(h->bcs.p, 0, 4 * std::max<int64_t>(B->nnz, 1), st));
        HIPCHK(hipMemsetAsync(h->uflag.p, 0, std::max<int64_t>(n, 1), st));
        HIPCHK(launch_mark_unsorted(h->ulist.as<int32_t>(), &dst->unsorted, h->uflag.as<uint8_t>(), st));
        HIPCHK(launch_compress_sorted_flags(n, brp, B->col_idx, bi, h->uflag.as<uint8_t>(), h->bcrp.as<int64_t>(),
                                            h->bcsi.as<int32_t>(), h->bcs.as<uint32_t>(), st));
        HIPCHK(launch_compress_unsorted(h->ulist.as<int32_t>(), &dst->unsorted, brp, B->col_idx, bi,
                                        h->bcrp.as<int64_t>(), h->bcsi.as<int32_t>(), h->bcs.as<uint32_t>(), st));
    }

    ClassParams cp{};
    cp.phase = 0;
    cp.accumulator = h->opt.accumulator;
    cp.compressed = comp ? 1 : 0;
    cp.dw_nw_max = DW_NW_MAX;
    cp.dw_r_max = DW_R_MAX;
    cp.hw_keys_max = HW_KEYS_MAX;
    cp.dg_nw_max = h->dg_nw_max;
    HIPCHK(launch_classify(m, h->rflops.as<int64_t>(), h->rflopsc.as<int64_t>(), h->rwin.as<int2>(), nullptr, cp,
                           h->kind_sym.as<uint8_t>(), h->row_nnz.as<int32_t>(), dst, st));
    HIPCHK(launch_partition(m, h->kind_sym.as<uint8_t>(), h->perm_sym.as<int32_t>(), h->koff_sym.as<int64_t>(),
                            h->tmp.as<int64_t>(), st));
    if ((s = pull_stats(h)) != SPG_OK) return s;  // host sync 2: per-kind sizes
    const DevStats hs2 = *h->hst;

    SymArgs sa{};
    sa.arp = arp;
    sa.aci = A->col_idx;
    sa.brp = brp;
    sa.bci = B->col_idx;
    if (comp) {
        sa.bcrp = h->bcrp.as<int64_t>();
        sa.bcsi = h->bcsi.as<int32_t>();
        sa.bcs = h->bcs.as<uint32_t>();
    }
    sa.rwin = h->rwin.as<int2>();
    sa.row_nnz = h->row_nnz.as<int32_t>();
    sa.rs.rows = h->perm_sym.as<int32_t>();
    sa.rs.koff = h->koff_sym.as<int64_t>();
    sa.st = dst;
    sa.lg_gs = lg_group(h->avg_len_c);
    LaunchCfg lc{st, 0, h->cus};
    auto grid_cap = [&](int64_t rows) { return (int)std::min<int64_t>(2048 * 8, ((rows + 7) / 8) * 8); };

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
    HIPCHK(launch_classify(m, h->rflops.as<int64_t>(), h->rflopsc.as<int64_t>(), h->rwin.as<int2>(),
                           h->row_nnz.as<int32_t>(), cp, h->kind_num.as<uint8_t>(), nullptr, dst, st));
    HIPCHK(launch_partition(m, h->kind_num.as<uint8_t>(), h->perm_num.as<int32_t>(), h->koff_num.as<int64_t>(),
                            h->tmp.as<int64_t>(), st));
    HIPCHK(hipMemcpyAsync(h->hkoff, h->coff.as<int64_t>() + m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    if ((s = pull_stats(h)) != SPG_OK) return s;  // host sync 3: nnz(C), numeric kinds
    const DevStats hs3 = *h->hst;
    if (hs3.overflow) return fail(h, SPG_ERR_OUT_OF_MEMORY, "level-2 hash arena too small in the symbolic phase");
    const int64_t nnzc = h->hkoff[0];
    if (c_rpt == SPG_I32 && nnzc > INT32_MAX)
        return fail(h, SPG_ERR_INDEX_OVERFLOW, "nnz(C) exceeds an int32 row_ptr; ask for SPG_I64");
    HIPCHK(launch_store_rp(m + 1, h->coff.as<int64_t>(), C_row_ptr, c_rpt == SPG_I64, st));

    h->fp = fp;
    h->nnzc = nnzc;
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
    o.n_kinds = NK;
    int64_t maxrs = 0;
    for (int kk = 0; kk < NK; ++kk) {
        o.rows_symbolic[kk] = hs3.kcount_sym[kk];
        o.rows_numeric[kk] = hs3.kcount_num[kk];
        if (kk != K_EMPTY) maxrs = std::max<int64_t>(maxrs, hs3.kmax_num[kk][1]);
    }
    o.max_row_nnz = maxrs;
    o.l2_spill_rows = (int32_t)hs3.kcount_num[K_HL];
    *nnz_c = nnzc;
    h->ready = true;
    return SPG_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ numeric
template <typename VT>
static spg_status numeric_impl(spg_handle h, const spg_csr *A, const spg_csr *B, spg_csr_out *C, int acc) {
    hipStream_t st = h->stream;
    const DevStats &hs = *h->hst;
    NumArgs<VT> na{};
    na.arp = h->arp64.as<int64_t>();
    na.aci = A->col_idx;
    na.aval = (const VT *)A->values;
    na.brp = h->brp64.as<int64_t>();
    na.bci = B->col_idx;
    na.bval = (const VT *)B->values;
    if (h->compressed) {
        na.bcrp = h->bcrp.as<int64_t>();
        na.bcsi = h->bcsi.as<int32_t>();
        na.bcs = h->bcs.as<uint32_t>();
    }
    na.rwin = h->rwin.as<int2>();
    na.coff = h->coff.as<int64_t>();
    na.cci = C->col_idx;
    na.cval = (VT *)C->values;
    na.rs.rows = h->perm_num.as<int32_t>();
    na.rs.koff = h->koff_num.as<int64_t>();
    na.st = h->dstats.as<DevStats>();
    na.lg_gs_or = lg_group(h->avg_len_c);
    na.lg_gs = lg_group(h->avg_len);
    const size_t sbytes = (sizeof(VT) == 8 || acc != ACC_NATIVE) ? 8 : 4;
    LaunchCfg lc{st, 0, h->cus};
    auto grid_cap = [&](int64_t rows) { return (int)std::min<int64_t>(2048 * 8, ((rows + 7) / 8) * 8); };

    if (hs.kcount_num[K_DW] > 0) {
        na.rs.kind = K_DW;
        na.nw_max = ((hs.kmax_num[K_DW][0] + 31) / 32) * 32;
        na.r_max = std::max(hs.kmax_num[K_DW][1], 1);
        HIPCHK(launch_num_dw<VT>(na, acc, lc));
    }
    if (hs.kcount_num[K_HW] > 0) {
        na.rs.kind = K_HW;
        na.ts = pow2_at_least(2 * (int64_t)hs.kmax_num[K_HW][1], 64);
        HIPCHK(launch_num_hw<VT>(na, acc, lc));
    }
    if (hs.kcount_num[K_DG] > 0) {
        na.rs.kind = K_DG;
        na.rs.queue = h->queue.as<int32_t>() + XCDS * K_DG;
        na.nw_max = ((hs.kmax_num[K_DG][0] + 31) / 32) * 32;
        const int grid = std::min(grid_cap(hs.kcount_num[K_DG]),
                                  dg_resident_grid(acc, sizeof(VT) == 8, lds_num_dg(na.nw_max), h->cus));
        na.arena_cap = (int64_t)na.nw_max * 32;
        const size_t bytes = (size_t)na.arena_cap * grid * sbytes;
        if (h->arena.cap < bytes || h->arena_bytes_zeroed < bytes) {
            HIPCHK(ensure(h->arena, bytes));
            HIPCHK(hipMemsetAsync(h->arena.p, 0, h->arena.cap, st));
            h->arena_bytes_zeroed = h->arena.cap;
        }
        na.arena = h->arena.p;
        HIPCHK(launch_fill_i32(na.rs.queue, XCDS, 0, st));
        lc.grid = grid;
        HIPCHK(launch_num_dg<VT>(na, acc, lc));
        lc.grid = 0;
    }
    if (hs.kcount_num[K_HL] > 0) {
        na.rs.kind = K_HL;
        na.rs.queue = h->queue.as<int32_t>() + XCDS * K_HL;
        na.l1_slots = h->opt.l1_hash_slots ? h->opt.l1_hash_slots : (sbytes == 8 ? 4096 : 8192);
        const int grid = std::min(grid_cap(hs.kcount_num[K_HL]),
                                  hl_resident_grid(acc, sizeof(VT) == 8, lds_num_hl(na.l1_slots, (int)sbytes), h->cus));
        na.arena_cap = pow2_at_least(2 * (int64_t)std::max(1, hs.kmax_num[K_HL][1]), 64);
        const size_t bytes = (size_t)na.arena_cap * grid * (8 + 2 * sbytes);
        if (h->l2k.cap < bytes) HIPCHK(ensure(h->l2k, bytes));
        na.arena = h->l2k.p;
        HIPCHK(launch_fill_i32(na.rs.queue, XCDS, 0, st));
        lc.grid = grid;
        HIPCHK(launch_num_hl<VT>(na, acc, lc));
        lc.grid = 0;
    }
    return SPG_OK;
}

extern "C" spg_status spgemm_numeric(spg_handle h, const spg_csr *A, const spg_csr *B, spg_csr_out *C) {
    if (!h) return SPG_ERR_INVALID_ARG;
    h->err.clear();
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
    if (h->nnzc == 0) return SPG_OK;
    if (A->dtype == SPG_F64) return numeric_impl<double>(h, A, B, C, ACC_NATIVE);
    const int acc = h->opt.fp32_mode == SPG_FP32_COMPENSATED ? ACC_COMP
                    : h->opt.fp32_mode == SPG_FP32_WIDE      ? ACC_WIDE
                                                             : ACC_NATIVE;
    return numeric_impl<float>(h, A, B, C, acc);
}


