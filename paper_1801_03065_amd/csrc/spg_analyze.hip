// Analysis kernels of the symbolic phase: B row statistics and compression
// of B into column-set words (Compression subsection), per-row flop counts
// and column windows of C (memory-pool sizing by max row flops, Accumulators
// subsection), row classification into kernel kinds, stable partition of the
// rows by kind, and the exclusive scans that turn row sizes into C.row_ptr
// (Algorithm 2).
#include "spg_internal.hpp"

namespace spg {

namespace {

constexpr int BLK = 256;
constexpr int CL_GRID = 512;  // classify workgroups (rows per lane grow beyond)

__device__ __forceinline__ unsigned long long ull(long long v) { return (unsigned long long)v; }

// ------------------------------------------------------------------ row ptrs
// One row-pointer array (int32 or int64) of n1 entries.
struct RpCopy {
    const void *src;
    int is64;
    int64_t n1, nnz;
    int64_t *dst;
};
__device__ __forceinline__ int64_t rp_at(const RpCopy &c, int64_t i) {
    return c.is64 ? ((const int64_t *)c.src)[i] : (int64_t)((const int32_t *)c.src)[i];
}
// Both operands' row pointers in one launch: entries [0, a.n1) are A's, the
// rest B's.
__global__ __launch_bounds__(BLK) void k_copy_rp(RpCopy a, RpCopy b, int *bad) {
    const int64_t tot = a.n1 + b.n1;
    for (int64_t t = (int64_t)blockIdx.x * BLK + threadIdx.x; t < tot; t += (int64_t)gridDim.x * BLK) {
        const bool isa = t < a.n1;
        const RpCopy &c = isa ? a : b;
        const int64_t i = isa ? t : t - a.n1;
        const int64_t v = rp_at(c, i);
        if ((i == 0 && v != 0) || (i > 0 && v < rp_at(c, i - 1)) || (i == c.n1 - 1 && v != c.nnz))
            atomicOr(bad, 1);
        // the copy is clamped to [0, nnz]: every row range read through it is
        // empty or inside the arrays, so the analysis kernels that run before
        // the host sees the flag cannot read out of bounds
        c.dst[i] = min(max(v, (int64_t)0), c.nnz);
    }
}

// ------------------------------------------------------------------ 16-lane groups
// A group of 16 lanes is one DPP row: lane moves inside it need no shuffle
// address arithmetic.
__device__ __forceinline__ int row_prev(int v, int fill) {  // value of lane q-1 (fill at q = 0)
    return __builtin_amdgcn_update_dpp(fill, v, 0x111, 0xF, 0xF, false);
}
__device__ __forceinline__ int row_next(int v, int fill) {  // value of lane q+1 (fill at q = 15)
    return __builtin_amdgcn_update_dpp(fill, v, 0x101, 0xF, 0xF, false);
}
__device__ __forceinline__ int row_last(int v) {  // lane 15 of the row, to every lane of it
    return __builtin_amdgcn_ds_swizzle(v, 0x10 | (0x0F << 5));
}
template <int N>
__device__ __forceinline__ int row_ror(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x120 + N, 0xF, 0xF, false);
}
__device__ __forceinline__ int row_sum(int v) {
    v += row_ror<8>(v);
    v += row_ror<4>(v);
    v += row_ror<2>(v);
    return v + row_ror<1>(v);
}
__device__ __forceinline__ int row_min(int v) {
    v = min(v, row_ror<8>(v));
    v = min(v, row_ror<4>(v));
    v = min(v, row_ror<2>(v));
    return min(v, row_ror<1>(v));
}
__device__ __forceinline__ int row_max(int v) {
    v = max(v, row_ror<8>(v));
    v = max(v, row_ror<4>(v));
    v = max(v, row_ror<2>(v));
    return max(v, row_ror<1>(v));
}

// ------------------------------------------------------------------ B rows
// One group of 16 lanes per row of B.  For rows whose columns are strictly
// increasing, the number of distinct words col >> 5 is the number of word
// changes along the row; other rows are queued for the LDS-bitmap kernel.
// Columns outside [0, ncols) set the malformed-input flag.
constexpr int BR_GS = 16;

__global__ __launch_bounds__(BLK) void k_brow(int64_t n, int64_t ncols, const int64_t *brp, const int32_t *bci,
                                               BRow *out, int32_t *ulist, uint8_t *uflag, DevStats *st) {
    const int q = threadIdx.x & (BR_GS - 1);
    const int64_t g0 = ((int64_t)blockIdx.x * BLK + threadIdx.x) / BR_GS;
    const int64_t ng = (int64_t)gridDim.x * BLK / BR_GS;
    int badcol = 0;
    for (int64_t r = g0; r < n; r += ng) {
        const int64_t b = brp[r], e = brp[r + 1];
        int cmin = INT_MAX, cmax = -1, heads = 0, unsorted = 0, prev_last = -1;
        for (int64_t c0 = b; c0 < e; c0 += BR_GS) {
            const int64_t idx = c0 + q;
            const bool v = idx < e;
            const int col = v ? bci[idx] : INT_MAX;
            const int prevc = row_prev(col, prev_last);
            if (v) {
                cmin = min(cmin, col);
                cmax = max(cmax, col);
                unsorted |= (prevc >= col);
                heads += ((col >> 5) != (prevc >> 5));
                badcol |= (col < 0) | ((int64_t)col >= ncols);
            }
            prev_last = row_last(col);
        }
        cmin = row_min(cmin);
        cmax = row_max(cmax);
        heads = row_sum(heads);
        unsorted = row_max(unsorted);
        if (q == 0) {
            BRow o;
            o.len = (int32_t)(e - b);
            o.lenc = heads;
            o.wmin = (e > b) ? (cmin >> 5) : INT_MAX;
            o.wmax = (e > b) ? (cmax >> 5) : -1;
            out[r] = o;
            uflag[r] = unsorted ? 1 : 0;
            if (unsorted) ulist[atomicAdd(&st->unsorted, 1)] = (int32_t)r;
        }
    }
    if (__ballot(badcol) && lane_id() == 0) atomicOr(&st->bad_input, 1);
}

// The same per row of B for short rows (average length <= BR_SHORT): one
// lane per row walks its columns.
constexpr int BR_SHORT = 8;

__global__ __launch_bounds__(BLK) void k_brow_short(int64_t n, int64_t ncols, const int64_t *brp, const int32_t *bci,
                                                     BRow *out, int32_t *ulist, uint8_t *uflag, DevStats *st) {
    int badcol = 0;
    for (int64_t r = (int64_t)blockIdx.x * BLK + threadIdx.x; r < n; r += (int64_t)gridDim.x * BLK) {
        const int64_t b = brp[r], e = brp[r + 1];
        int cmin = INT_MAX, cmax = -1, heads = 0, unsorted = 0, prev = -1;
        for (int64_t k = b; k < e; ++k) {
            const int col = bci[k];
            cmin = min(cmin, col);
            cmax = max(cmax, col);
            unsorted |= (prev >= col);
            heads += ((col >> 5) != (prev >> 5));
            badcol |= (col < 0) | ((int64_t)col >= ncols);
            prev = col;
        }
        BRow o;
        o.len = (int32_t)(e - b);
        o.lenc = heads;
        o.wmin = (e > b) ? (cmin >> 5) : INT_MAX;
        o.wmax = (e > b) ? (cmax >> 5) : -1;
        out[r] = o;
        uflag[r] = unsorted ? 1 : 0;
        if (unsorted) ulist[atomicAdd(&st->unsorted, 1)] = (int32_t)r;
    }
    if (__ballot(badcol) && lane_id() == 0) atomicOr(&st->bad_input, 1);
}

// One wavefront per listed row: OR every column bit into an LDS bitmap over
// the row's word window; distinct words = nonzero bitmap words.  mode 0
// writes the count, mode 1 writes the (word, bits) pairs in word order.
constexpr int UB_WORDS = 16384;

__global__ __launch_bounds__(WAVE) void k_brow_unsorted(const int32_t *list, const int *count_p, const int64_t *brp,
                                                         const int32_t *bci, BRow *bi, const int64_t *bcrp,
                                                         uint2 *bcw, int mode, DevStats *st,
                                                         const int *enable) {
    __shared__ uint32_t bits[UB_WORDS];
    const int l = lane_id();
    if (enable && !*enable) return;
    const int count = *count_p;
    if ((int)blockIdx.x >= count) return;
    for (int w = l; w < UB_WORDS; w += WAVE) bits[w] = 0;
    wave_lds_sync();
    for (int t = blockIdx.x; t < count; t += gridDim.x) {
        const int64_t r = list[t];
        const int64_t b = brp[r], e = brp[r + 1];
        const BRow br = bi[r];
        const int64_t nw = (int64_t)br.wmax - br.wmin + 1;
        if (e == b) continue;
        if (nw > UB_WORDS) {
            if (l == 0 && st) atomicAdd(&st->bad_window, 1);
            continue;
        }
        for (int64_t idx = b + l; idx < e; idx += WAVE) {
            const int col = bci[idx];
            atomicOr(&bits[(col >> 5) - br.wmin], 1u << (col & 31));
        }
        wave_lds_sync();
        int run = 0;
        const int64_t out0 = mode ? bcrp[r] : 0;
        for (int w0 = 0; w0 < nw; w0 += WAVE) {
            const int w = w0 + l;
            const uint32_t m = (w < nw) ? bits[w] : 0u;
            const unsigned long long bal = __ballot(m != 0u);
            if (mode && m) {
                const int64_t pos = out0 + run + mbcnt(bal);
                bcw[pos] = make_uint2((uint32_t)(br.wmin + w), m);
            }
            if (w < nw) bits[w] = 0;
            run += __popcll(bal);
        }
        if (mode == 0 && l == 0) bi[r].lenc = run;
        wave_lds_sync();
    }
}

// Compressed B for rows with sorted columns: a 16-lane group per row; the
// last lane of each word run writes its (word, bits) record with one 8-byte
// store.  A run that crosses into the next 16-column chunk carries its partial
// bits there.
__global__ __launch_bounds__(BLK) void k_compress_sorted(int64_t n, const int64_t *brp, const int32_t *bci,
                                                          const BRow *bi, const uint8_t *unsorted,
                                                          const int64_t *bcrp, uint2 *bcw, const int *enable) {
    if (enable && !*enable) return;
    const int q = threadIdx.x & (BR_GS - 1);
    const int64_t g0 = ((int64_t)blockIdx.x * BLK + threadIdx.x) / BR_GS;
    const int64_t ng = (int64_t)gridDim.x * BLK / BR_GS;
    for (int64_t r = g0; r < n; r += ng) {
        if (unsorted[r]) continue;
        const int64_t b = brp[r], e = brp[r + 1];
        const int64_t o0 = bcrp[r];
        int heads_before = 0, prev_last = -1;
        uint32_t carry = 0;
        for (int64_t c0 = b; c0 < e; c0 += BR_GS) {
            const int64_t idx = c0 + q;
            const bool v = idx < e;
            const int col = v ? bci[idx] : INT_MAX;
            const int prevc = row_prev(col, prev_last);
            const int nextc = row_next(col, (q == BR_GS - 1 && idx + 1 < e) ? bci[idx + 1] : INT_MAX);
            const int head = v && ((col >> 5) != (prevc >> 5));
            // inclusive count of heads in this chunk = run id (0 = run from previous chunk)
            int seg = head;
            seg += __builtin_amdgcn_update_dpp(0, seg, 0x111, 0xF, 0xF, false);
            seg += __builtin_amdgcn_update_dpp(0, seg, 0x112, 0xF, 0xF, false);
            seg += __builtin_amdgcn_update_dpp(0, seg, 0x114, 0xF, 0xF, false);
            seg += __builtin_amdgcn_update_dpp(0, seg, 0x118, 0xF, 0xF, false);
            uint32_t acc = v ? (1u << (col & 31)) : 0u;
            if (seg == 0) acc |= carry;
            // OR-scan inside runs: a lane takes the bits of lane q-d when it is in the same run
#define SR_OR_STEP(CTRL)                                                                      \
    {                                                                                         \
        const uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)acc, CTRL, 0xF, 0xF, false); \
        const int ts = __builtin_amdgcn_update_dpp(-1, seg, CTRL, 0xF, 0xF, false);        \
        if (ts == seg) acc |= t;                                                              \
    }
            SR_OR_STEP(0x111)
            SR_OR_STEP(0x112)
            SR_OR_STEP(0x114)
            SR_OR_STEP(0x118)
#undef SR_OR_STEP
            // the run ends here when the next column is in another word (or there is none)
            const bool tail = v && (idx + 1 >= e || (nextc >> 5) != (col >> 5));
            const int64_t pos = o0 + heads_before + seg - 1;
            if (tail) bcw[pos] = make_uint2((uint32_t)(col >> 5), acc);  // one record per word run
            const bool open = v && !tail && q == BR_GS - 1;  // run continues into the next chunk
            carry = (uint32_t)row_last(open ? (int)acc : 0);
            heads_before += row_last(seg);
            prev_last = row_last(col);
        }
    }
}

// The same for B with short rows: one lane per row walks its columns and
// writes each word run where it ends.
__global__ __launch_bounds__(BLK) void k_compress_short(int64_t n, const int64_t *brp, const int32_t *bci,
                                                         const uint8_t *unsorted, const int64_t *bcrp, uint2 *bcw,
                                                         const int *enable) {
    if (enable && !*enable) return;
    for (int64_t r = (int64_t)blockIdx.x * BLK + threadIdx.x; r < n; r += (int64_t)gridDim.x * BLK) {
        if (unsorted[r]) continue;
        const int64_t b = brp[r], e = brp[r + 1];
        int64_t pos = bcrp[r];
        int curw = INT_MIN;
        uint32_t bits = 0;
        for (int64_t k = b; k < e; ++k) {
            const int col = bci[k];
            const int w = col >> 5;
            if (w != curw) {
                if (curw != INT_MIN) bcw[pos++] = make_uint2((uint32_t)curw, bits);
                curw = w;
                bits = 0;
            }
            bits |= 1u << (col & 31);
        }
        if (curw != INT_MIN) bcw[pos] = make_uint2((uint32_t)curw, bits);
    }
}

// ------------------------------------------------------------------ A rows
// 16 lanes per row of A: f_m(i) = sum |B(j,:)|, the same over compressed B,
// and the word window [min wmin, max wmax] of the B rows it reads.
__device__ __forceinline__ long long wave_max64(long long v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = max(v, (long long)__shfl_xor(v, d));
    return v;
}

constexpr int RI_GS = 8;
// DPP lane moves inside groups of 8 lanes (quad permutes, half-row mirror)
template <int CTRL>
__device__ __forceinline__ int ri_x32(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ long long ri_x(long long v) {
    const int lo = ri_x32<CTRL>((int)(uint32_t)v), hi = ri_x32<CTRL>((int)((uint64_t)v >> 32));
    return (long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
constexpr int RI_U = 4;  // A entries per lane in flight
constexpr int RI_GRID = 2048;
constexpr int RI_F = 7;  // rowinfo partial fields: fm, fmc, max, max compressed, fm and fmc of long rows,
                         // longest row of A
__host__ __device__ constexpr bool ri_is_max(int f) { return f == 2 || f == 3 || f == 6; }
static_assert(RI_F * RI_GRID <= RED_ELEMS && 4 * NK * CL_GRID <= RED_ELEMS, "analysis partials exceed scratch");

// Compression rule of the Compression subsection, taken on the device from
// the folded flop counts: compress when it removes more than (1 - thr) of the
// flops of the rows that read B's structure word by word (all rows, or those
// beyond the short-row limit when the selector is on).
struct CompRule {
    int opt;     // -1 by the rule, 0 never, 1 always
    int sel;     // selector active: short rows read raw B
    double thr;  // 0.85
};

__global__ __launch_bounds__(BLK) void k_rowinfo(int64_t m, int64_t n, const int64_t *arp, const int32_t *aci,
                                                  const BRow *bi, int64_t *rflops, int64_t *rflopsc,
                                                  int2 *rwin, long long *part, DevStats *st) {
    const int q = threadIdx.x & (RI_GS - 1);
    const int64_t g0 = ((int64_t)blockIdx.x * BLK + threadIdx.x) / RI_GS;
    const int64_t ng = (int64_t)gridDim.x * BLK / RI_GS;
    long long s_fm = 0, s_fmc = 0, s_mx = 0, s_mxc = 0, s_fmb = 0, s_fmcb = 0, s_mxa = 0;
    int badcol = 0;
    for (int64_t i = g0; i < m; i += ng) {
        const int64_t b = arp[i], e = arp[i + 1];
        long long f = 0, fc = 0;
        int wlo = INT_MAX, whi = -1;
        for (int64_t base = b; base < e; base += RI_GS * RI_U) {
            int j[RI_U];
#pragma unroll
            for (int u = 0; u < RI_U; ++u) {
                const int64_t idx = base + q + u * RI_GS;
                j[u] = idx < e ? aci[idx] : -1;
                if (idx < e && (uint64_t)(int64_t)j[u] >= (uint64_t)n) badcol = 1;
                if ((uint64_t)(int64_t)j[u] >= (uint64_t)n) j[u] = -1;  // out of range (flagged): skipped
            }
            BRow br[RI_U];
#pragma unroll
            for (int u = 0; u < RI_U; ++u) br[u] = bi[j[u] >= 0 ? j[u] : 0];
#pragma unroll
            for (int u = 0; u < RI_U; ++u) {
                if (j[u] >= 0) {
                    f += br[u].len;
                    fc += br[u].lenc;
                    wlo = min(wlo, br[u].wmin);
                    whi = max(whi, br[u].wmax);
                }
            }
        }
        // reductions over the 8-lane group: DPP quad permutes (lane ^ 1,
        // lane ^ 2), then the half-row mirror (lane i <-> 7 - i) joins the two
        // quads
        f += ri_x<0xB1>(f);
        fc += ri_x<0xB1>(fc);
        wlo = min(wlo, ri_x32<0xB1>(wlo));
        whi = max(whi, ri_x32<0xB1>(whi));
        f += ri_x<0x4E>(f);
        fc += ri_x<0x4E>(fc);
        wlo = min(wlo, ri_x32<0x4E>(wlo));
        whi = max(whi, ri_x32<0x4E>(whi));
        f += ri_x<0x141>(f);
        fc += ri_x<0x141>(fc);
        wlo = min(wlo, ri_x32<0x141>(wlo));
        whi = max(whi, ri_x32<0x141>(whi));
        if (q == 0) {
            rflops[i] = f;
            rflopsc[i] = fc;
            rwin[i] = make_int2(wlo, whi);
            s_fm += f;
            s_fmc += fc;
            s_mx = max(s_mx, f);
            s_mxc = max(s_mxc, fc);
            s_mxa = max(s_mxa, (long long)(e - b));
            if (f > SR_F_MAX) {  // rows that read B's structure word by word
                s_fmb += f;
                s_fmcb += fc;
            }
        }
    }
    // per-block partials; k_rowinfo_fin folds them (same-address global
    // atomics from every block would serialise)
    __shared__ long long red[RI_F][BLK / WAVE];
    s_fm = wave_sum64(s_fm);
    s_fmc = wave_sum64(s_fmc);
    s_fmb = wave_sum64(s_fmb);
    s_fmcb = wave_sum64(s_fmcb);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        s_mx = max(s_mx, (long long)__shfl_xor(s_mx, d));
        s_mxc = max(s_mxc, (long long)__shfl_xor(s_mxc, d));
        s_mxa = max(s_mxa, (long long)__shfl_xor(s_mxa, d));
    }
    const int wv = threadIdx.x / WAVE;
    if (lane_id() == 0) {
        red[0][wv] = s_fm;
        red[1][wv] = s_fmc;
        red[2][wv] = s_mx;
        red[3][wv] = s_mxc;
        red[4][wv] = s_fmb;
        red[5][wv] = s_fmcb;
        red[6][wv] = s_mxa;
    }
    __syncthreads();
    if (threadIdx.x < RI_F) {
        const int f = threadIdx.x;
        long long v = 0;
        for (int u = 0; u < BLK / WAVE; ++u) v = ri_is_max(f) ? max(v, red[f][u]) : v + red[f][u];
        part[RI_F * (int64_t)blockIdx.x + f] = v;
    }
    if (__ballot(badcol) && lane_id() == 0) atomicOr(&st->bad_input, 1);
}

// One workgroup: fold the rowinfo partials of nb blocks into the statistics
// and take the compression decision.
__global__ __launch_bounds__(BLK) void k_rowinfo_fin(int nb, const long long *part, DevStats *st, CompRule rule) {
    long long v[RI_F];
#pragma unroll
    for (int f = 0; f < RI_F; ++f) v[f] = 0;
    for (int k = threadIdx.x; k < nb; k += BLK)
#pragma unroll
        for (int f = 0; f < RI_F; ++f) {
            const long long x = part[RI_F * (int64_t)k + f];
            v[f] = ri_is_max(f) ? max(v[f], x) : v[f] + x;
        }
    __shared__ long long red[RI_F][BLK / WAVE];
    const int wv = threadIdx.x / WAVE;
#pragma unroll
    for (int f = 0; f < RI_F; ++f) {
        const long long r = ri_is_max(f) ? wave_max64(v[f]) : wave_sum64(v[f]);
        if (lane_id() == 0) red[f][wv] = r;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long a[RI_F];
        for (int f = 0; f < RI_F; ++f) {
            a[f] = 0;
            for (int u = 0; u < BLK / WAVE; ++u) a[f] = ri_is_max(f) ? max(a[f], red[f][u]) : a[f] + red[f][u];
        }
        st->fm = ull(a[0]);
        st->fmc = ull(a[1]);
        st->maxrf = ull(a[2]);
        st->maxrfc = ull(a[3]);
        st->fmb = ull(a[4]);
        st->fmcb = ull(a[5]);
        st->maxnnza = ull(a[6]);
        int comp = rule.opt == 1;
        if (rule.opt == -1) {
            const double f0 = (double)(rule.sel ? a[4] : a[0]), f1 = (double)(rule.sel ? a[5] : a[1]);
            comp = f0 > 0 && f1 < rule.thr * f0;
        }
        // an unsorted row of B too wide for the word-count bitmap has no
        // compressed form: the structure kernels then read raw B
        if (st->bad_window) comp = 0;
        st->comp = comp;
    }
}

// ------------------------------------------------------------------ classify
// One row per lane, CB rows per workgroup (contiguous, so the per-workgroup
// kind counts are the counts of the stable partition).  Each workgroup writes
// per kind: max window words, max bound, max touched words and its row count
// (int32 x 4), and the row counts again compactly (int32 per kind); the
// partition kernel folds them into the phase's statistics and the partition's
// offsets (kinds in order, workgroups in row order within a kind).
constexpr int CB = 1024;

__global__ __launch_bounds__(CB) void k_classify(int64_t m, const int64_t *rflops, const int64_t *rflopsc,
                                                  const int2 *rwin, const int32_t *row_nnz,
                                                  const int32_t *row_words, ClassParams p, uint8_t *kind,
                                                  int32_t *row_nnz_out, int32_t *blk) {
    __shared__ int smax[NK][3];
    __shared__ int scnt[NK];
    const int t = threadIdx.x, l = lane_id();
    if (t < NK) {
        smax[t][0] = 0;
        smax[t][1] = 0;
        smax[t][2] = 0;
        scnt[t] = 0;
    }
    // device-side switches: compression decided by the analysis, segments
    // only when every row of B is sorted
    const bool compressed = p.comp_flag ? (*p.comp_flag != 0) : (p.compressed != 0);
    const bool sg = p.sg && (p.unsorted == nullptr || *p.unsorted == 0);
    __syncthreads();
    {
        const int64_t i = (int64_t)blockIdx.x * CB + t;
        const bool valid = i < m;
        const bool sampled = p.sample_stride <= 1 || (i % p.sample_stride) == 0;
        long long f = (valid && sampled) ? rflops[i] : 0;
        if (p.phase == 1 && p.row_cls && valid && p.row_cls[i] != p.cls) f = 0;
        if (p.phase == 1 && p.split && f > 0) {
            const bool hv = (p.heavy_flops > 0 && f >= p.heavy_flops) ||
                            (p.heavy_alen > 0 && p.arp[i + 1] - p.arp[i] > p.heavy_alen);
            if (hv != (p.heavy != 0)) f = 0;
        }
        const int2 w = valid ? rwin[i] : make_int2(0, -1);
        int k = valid ? K_EMPTY : -1, a = 0, bnd = 0, tw = 0;
        if (f > 0) {
            const long long nw = (long long)w.y - w.x + 1;
            long long bound, words;
            if (p.phase == 0) {
                bound = compressed ? min((long long)rflopsc[i], nw) : min(f, 32 * nw);
                words = min(bound, nw);
            } else {
                bound = row_nnz[i];
                words = row_words[i];
            }
            const bool dw_fit = nw <= p.dw_nw_max && (p.phase == 0 || bound <= p.dw_r_max);
            const bool wh_fit = p.phase == 1 && nw <= p.wh_nw_max && bound <= p.wh_r_max && words <= p.wh_t_max;
            const bool hw_fit = bound <= p.hw_keys_max;
            const bool dg_fit = nw <= p.dg_nw_max;
            switch (p.accumulator) {
                case 1:  // bit-window dense wherever it fits
                    k = dw_fit ? K_DW : (dg_fit ? K_DG : (hw_fit ? K_HW : K_HL));
                    break;
                case 2:  // hash
                case 4:  // LL hashmap (numeric: hash-wave rows run the LL kernel)
                    k = hw_fit ? K_HW : K_HL;
                    break;
                case 3:  // two-level hash everywhere
                    k = K_HL;
                    break;
                default:  // selector
                    if (f <= p.sr_f_max)
                        k = K_SR;
                    else if (p.phase == 0)
                        k = dw_fit ? K_DW : (hw_fit ? K_HW : (dg_fit ? K_DG : K_HL));
                    else if (p.plan_cap > 0 && p.sym_kind[i] == K_DW && words <= p.plan_len[i] &&
                             nw <= PL_NW_MAX && bound <= PL_R_MAX)
                        k = K_PL;  // the symbolic phase stored this row's structure
                    else
                        k = wh_fit ? K_WH : (hw_fit ? K_HW : (dg_fit ? K_DG : K_HL));
            }
            // heavy rows in segments: the symbolic bit window of a workgroup
            // row cuts them, so rows that may exceed one segment go there
            const long long eb = min(f, 32 * nw);  // entries bound
            if (sg && p.phase == 0 && dg_fit &&
                ((k == K_DW && eb > SG_CAP) || (k == K_HW && eb > p.hw_keys_max)))
                k = K_DG;  // (a word-keyed hash row may still hold more entries than a numeric hash row)
            if (sg && p.phase == 1 && k == K_DG && p.sym_kind[i] != K_DG && (bound > SG_CAP || nw > SG_NW))
                k = hw_fit ? K_HW : K_HL;  // no segment list for this row
            if (p.phase == 0 && p.plan_len) {
                int room = 0;
                if (k == K_DW && p.plan_cap > 0) room = (int)min(words, (long long)p.plan_cap);
                if (k == K_DG && sg && (eb > SG_CAP || nw > SG_NW))
                    room = (int)((eb + SG_CUT - 1) / SG_CUT + (nw + SG_NW - 1) / SG_NW + 2);
                p.plan_len[i] = room;
            }
            if (k == K_SR) bound = f;  // a short row's team size follows its multiplications
            a = (int)min(nw, (long long)INT_MAX);
            bnd = (int)min(bound, (long long)INT_MAX);
            tw = (int)min(words, (long long)INT_MAX);
        } else if (valid && p.phase == 0) {
            row_nnz_out[i] = 0;
            if (p.plan_len) p.plan_len[i] = 0;
        }
        if (valid) kind[i] = (uint8_t)k;
        if (valid && p.words_out) p.words_out[i] = 0;  // the structure kernels fill it for their rows
        for (int kk = 0; kk < NK; ++kk) {
            const unsigned long long bal = __ballot(k == kk);
            if (!bal) continue;
            const int ma = wave_max(k == kk ? a : 0), mb = wave_max(k == kk ? bnd : 0);
            const int mc = wave_max(k == kk ? tw : 0);
            if (l == 0) {
                atomicMax(&smax[kk][0], ma);
                atomicMax(&smax[kk][1], mb);
                atomicMax(&smax[kk][2], mc);
                atomicAdd(&scnt[kk], __popcll(bal));
            }
        }
    }
    __syncthreads();
    if (t < NK) {
        int32_t *q = blk + 4 * ((int64_t)blockIdx.x * NK + t);
        q[0] = smax[t][0];
        q[1] = smax[t][1];
        q[2] = smax[t][2];
        q[3] = scnt[t];
        blk[4 * gridDim.x * NK + (int64_t)blockIdx.x * NK + t] = scnt[t];  // compact counts, read by every partition workgroup
    }
}

// Inclusive max-scan over the 64 lanes (values >= 0) with DPP lane moves;
// lane 63 holds the wavefront maximum.
__device__ __forceinline__ int wave_maxscan_dpp(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false));  // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return v;
}

// One workgroup over the nb classify workgroups: per kind the row total and
// the maxima (into the phase's statistics), the kind offsets koff, and each
// workgroup's count replaced by its exclusive offset (kinds in order, row order
// within a kind).  Counts and offsets fit int32 (rows are int32).
// ------------------------------------------------------------------ partition
// Beyond PF_FEW classify workgroups, the compact counts are folded once by
// one workgroup (k_part_fold) instead of by every partition workgroup, whose
// reads would grow with the square of the workgroup count.
constexpr int64_t PF_FEW = 1024;

// One workgroup: the compact per-workgroup kind counts become exclusive
// prefixes in place (row order within a kind), the kind totals follow them.
__global__ __launch_bounds__(CB) void k_part_fold(int64_t nb, int32_t *cnt) {
    constexpr int NW = CB / WAVE;
    __shared__ int wsum[NK][NW];
    __shared__ int carry[NK];
    const int t = threadIdx.x, l = lane_id(), wv = t / WAVE;
    if (t < NK) carry[t] = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += CB) {
        const int64_t u = c0 + t;
        int c[NK], inc[NK];
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            c[k] = u < nb ? cnt[u * NK + k] : 0;
            inc[k] = wave_scan_dpp(c[k]);
            if (l == WAVE - 1) wsum[k][wv] = inc[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            int off = carry[k];
            for (int w = 0; w < wv; ++w) off += wsum[k][w];
            if (u < nb) cnt[u * NK + k] = off + inc[k] - c[k];
        }
        __syncthreads();
        if (t < NK) {
            int tt = 0;
            for (int w = 0; w < NW; ++w) tt += wsum[t][w];
            carry[t] += tt;
        }
        __syncthreads();
    }
    if (t < NK) cnt[nb * NK + t] = carry[t];
}

// Stable partition of rows by kind.  Every workgroup folds the classify
// workgroups' compact counts itself (a few KB: kind totals give the kind
// bases, the workgroups before it its offset inside each kind), so no
// one-workgroup fold kernel runs in between; workgroup 0 also folds the
// maxima and counts into the phase's statistics and writes the kind offsets.
// A row lands at base + offset + its rank among the same kind in the
// workgroup (wavefront ballots).
static_assert(NK == 8, "the partition reads a workgroup's kind counts as two int4");

__global__ __launch_bounds__(CB) void k_part_scatter(int64_t m, int64_t nb, const uint8_t *kind, const int32_t *blk,
                                                      int32_t *perm, int64_t *koff, int phase, int heavy,
                                                      DevStats *st) {
    constexpr int NW = CB / WAVE;
    __shared__ int wcnt[NW][NK];
    __shared__ int wtot[NK][NW], wpre[NK][NW];
    __shared__ int stot[NK], spre[NK], sbase[NK];
    __shared__ int smax[NK][3];
    const int t = threadIdx.x, l = lane_id(), wv = t / WAVE;
    const int64_t b = blockIdx.x;
    const int32_t *cnt = blk + 4 * nb * NK;
    // kind totals over all classify workgroups and over the ones before this
    int tot[NK], pre[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) tot[k] = pre[k] = 0;
    if (nb > PF_FEW) {
        // folded beforehand by k_part_fold: exclusive prefixes per workgroup,
        // kind totals after them (the per-kind sums below see them in lane 0)
        if (t == 0) {
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                tot[k] = cnt[nb * NK + k];
                pre[k] = cnt[b * NK + k];
            }
        }
    }
    for (int64_t u = t; nb <= PF_FEW && u < nb; u += CB) {
        const int4 c0 = *(const int4 *)(cnt + u * NK), c1 = *(const int4 *)(cnt + u * NK + 4);
        const int c[NK] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            tot[k] += c[k];
            pre[k] += u < b ? c[k] : 0;
        }
    }
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const int ts = __builtin_amdgcn_readlane(wave_scan_dpp(tot[k]), 63);
        const int ps = __builtin_amdgcn_readlane(wave_scan_dpp(pre[k]), 63);
        if (l == 0) {
            wtot[k][wv] = ts;
            wpre[k][wv] = ps;
        }
    }
    if (t < NK) smax[t][0] = smax[t][1] = smax[t][2] = 0;
    __syncthreads();
    if (t < NK) {
        int T = 0, P = 0;
        for (int u = 0; u < NW; ++u) {
            T += wtot[t][u];
            P += wpre[t][u];
        }
        stot[t] = T;
        spre[t] = P;
    }
    __syncthreads();
    if (t < NK) {
        int base = 0;
        for (int k = 0; k < t; ++k) base += stot[k];
        sbase[t] = base;
        if (b == 0 && koff) {
            koff[t] = base;
            if (t == NK - 1) koff[NK] = base + stot[t];
        }
    }
    // workgroup 0: the per-kind maxima into the phase's statistics
    if (b == 0) {
        int mx[NK][3];
#pragma unroll
        for (int k = 0; k < NK; ++k) mx[k][0] = mx[k][1] = mx[k][2] = 0;
        for (int64_t u = t; u < nb; u += CB) {
#pragma unroll
            for (int k = 0; k < NK; ++k) {
                const int4 v = *(const int4 *)(blk + 4 * (u * NK + k));
                mx[k][0] = max(mx[k][0], v.x);
                mx[k][1] = max(mx[k][1], v.y);
                mx[k][2] = max(mx[k][2], v.z);
            }
        }
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const int m0 = __builtin_amdgcn_readlane(wave_maxscan_dpp(mx[k][0]), 63);
            const int m1 = __builtin_amdgcn_readlane(wave_maxscan_dpp(mx[k][1]), 63);
            const int m2 = __builtin_amdgcn_readlane(wave_maxscan_dpp(mx[k][2]), 63);
            if (l == 0) {
                atomicMax(&smax[k][0], m0);
                atomicMax(&smax[k][1], m1);
                atomicMax(&smax[k][2], m2);
            }
        }
    }
    __syncthreads();
    if (b == 0 && t < NK && stot[t]) {
        const int k = t;
        int *gm = phase == 0 ? &st->kmax_sym[k][0] : heavy ? &st->kmax_heavy[k][0] : &st->kmax_num[k][0];
        gm[0] = max(gm[0], smax[k][0]);
        gm[1] = max(gm[1], smax[k][1]);
        gm[2] = max(gm[2], smax[k][2]);
        long long *gc = phase == 0 ? &st->kcount_sym[k] : heavy ? &st->kcount_heavy[k] : &st->kcount_num[k];
        *gc += stot[k];
    }
    // rows of this workgroup, stable within each kind
    const int64_t i = b * CB + t;
    const int k = i < m ? kind[i] : -1;
    int rank = 0;
    for (int kk = 0; kk < NK; ++kk) {
        const unsigned long long bal = __ballot(k == kk);
        if (kk == k) rank = mbcnt(bal);
        if (l == 0) wcnt[wv][kk] = __popcll(bal);
    }
    __syncthreads();
    if (i < m) {
        int off = 0;
        for (int u = 0; u < wv; ++u) off += wcnt[u][k];
        perm[sbase[k] + spre[k] + off + rank] = (int32_t)i;
    }
}

// ------------------------------------------------------------------ scans
constexpr int SC_T = 256, SC_E = 8, SC_B = SC_T * SC_E;

// Local scans with block sums, one workgroup scans the block sums (total to
// out[n]), then the block offsets are added.  enable (optional, device): when
// it reads 0 the scan is skipped.
template <typename T>
__global__ __launch_bounds__(SC_T) void k_scan_local(int64_t n, const T *in, int stride, int64_t *out, int64_t *bsum,
                                                      const int *enable) {
    if (enable && !*enable) return;
    __shared__ long long wsum[SC_T / WAVE];
    const int t = threadIdx.x, l = lane_id(), wv = t / WAVE;
    const int64_t base = (int64_t)blockIdx.x * SC_B + (int64_t)t * SC_E;
    long long v[SC_E];
    long long s = 0;
#pragma unroll
    for (int e = 0; e < SC_E; ++e) {
        v[e] = (base + e < n) ? (long long)in[(base + e) * stride] : 0;
        s += v[e];
    }
    const long long inc = wave_incl_scan64(s);
    if (l == WAVE - 1) wsum[wv] = inc;
    __syncthreads();
    long long off = 0;
    for (int u = 0; u < wv; ++u) off += wsum[u];
    long long run = off + inc - s;
#pragma unroll
    for (int e = 0; e < SC_E; ++e) {
        if (base + e < n) out[base + e] = run;
        run += v[e];
    }
    if (t == SC_T - 1) bsum[blockIdx.x] = off + inc;
}

// Exclusive scan of the block totals in one workgroup (many blocks only).
__global__ __launch_bounds__(SC_T) void k_scan_top(int64_t nb, int64_t *bsum, const int *enable) {
    if (enable && !*enable) return;
    __shared__ long long wsum[SC_T / WAVE];
    __shared__ long long carry;
    const int t = threadIdx.x, l = lane_id(), wv = t / WAVE;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += SC_T) {
        const int64_t b = c0 + t;
        const long long v = b < nb ? bsum[b] : 0;
        const long long inc = wave_incl_scan64(v);
        if (l == WAVE - 1) wsum[wv] = inc;
        __syncthreads();
        long long off = 0, tot = 0;
        for (int u = 0; u < SC_T / WAVE; ++u) {
            if (u < wv) off += wsum[u];
            tot += wsum[u];
        }
        if (b < nb) bsum[b] = carry + off + inc - v;
        __syncthreads();
        if (t == 0) carry += tot;
        __syncthreads();
    }
    if (t == 0) bsum[nb] = carry;
}

// Each block adds the totals of all earlier blocks to its local scan and the
// last block stores the grand total at out[n].  With few blocks (SC_FEW) every
// block reduces its own prefix of the raw totals, saving the one-workgroup
// scan launch; with more, k_scan_top has replaced them by their exclusive
// scan (and the grand total at bsum[nb]).
constexpr int64_t SC_FEW = 1024;
__global__ __launch_bounds__(SC_T) void k_scan_add(int64_t n, int64_t nb, int64_t *out, const int64_t *bsum,
                                                    const int *enable) {
    if (enable && !*enable) return;
    __shared__ long long wsum[SC_T / WAVE];
    const int t = threadIdx.x, l = lane_id(), wv = t / WAVE;
    const int64_t b = blockIdx.x;
    long long add = 0;
    if (nb <= SC_FEW) {
        long long part = 0;
        for (int64_t u = t; u < b; u += SC_T) part += bsum[u];
        part = wave_sum64(part);
        if (l == 0) wsum[wv] = part;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < SC_T / WAVE; ++u) add += wsum[u];
    } else {
        add = bsum[b];
    }
    const int64_t base = b * SC_B;
    for (int e = t; e < SC_B; e += SC_T)
        if (base + e < n) out[base + e] += add;
    if (b == nb - 1 && t == 0) out[n] = nb <= SC_FEW ? add + bsum[b] : bsum[nb];
}

__global__ __launch_bounds__(BLK) void k_store_rp32(int64_t n1, const int64_t *src, int32_t *dst) {
    for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n1; i += (int64_t)gridDim.x * BLK)
        dst[i] = (int32_t)src[i];
}
__global__ __launch_bounds__(BLK) void k_store_rp64(int64_t n1, const int64_t *src, int64_t *dst) {
    for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n1; i += (int64_t)gridDim.x * BLK)
        dst[i] = src[i];
}
__global__ __launch_bounds__(BLK) void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) p[i] = v;
}

// Per kind, the slice of the (row-sorted) kind list holding rows in [rb, re).
__global__ void k_kind_ranges(const int32_t *perm, const int64_t *koff, int64_t rb, int64_t re, int64_t *range) {
    const int k = threadIdx.x;
    if (k >= NK) return;
    int64_t lo = koff[k], hi = koff[k + 1];
    int64_t a = lo, b = hi;  // first index with perm >= rb
    while (a < b) {
        const int64_t m = (a + b) >> 1;
        if (perm[m] < rb) a = m + 1; else b = m;
    }
    const int64_t first = a;
    a = first;
    b = hi;  // first index with perm >= re
    while (a < b) {
        const int64_t m = (a + b) >> 1;
        if (perm[m] < re) a = m + 1; else b = m;
    }
    range[2 * k] = first;
    range[2 * k + 1] = a;
}

inline int grid_for(int64_t work, int per_block, int cap = 65536) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

hipError_t launch_copy_rp(int64_t n1a, const void *srca, int is64a, int64_t nnza, int64_t *dsta, int64_t n1b,
                          const void *srcb, int is64b, int64_t nnzb, int64_t *dstb, int *bad, hipStream_t s) {
    const RpCopy a{srca, is64a, n1a, nnza, dsta}, b{srcb, is64b, n1b, nnzb, dstb};
    hipLaunchKernelGGL(k_copy_rp, dim3(grid_for(n1a + n1b, BLK)), dim3(BLK), 0, s, a, b, bad);
    return hipGetLastError();
}

hipError_t launch_brow(int64_t n, int64_t nnz, int64_t ncols, const int64_t *brp, const int32_t *bci, BRow *out,
                       int32_t *ulist, uint8_t *uflag, DevStats *st, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (nnz <= BR_SHORT * n)
        hipLaunchKernelGGL(k_brow_short, dim3(grid_for(n, BLK, 4096)), dim3(BLK), 0, s, n, ncols, brp, bci, out, ulist,
                           uflag, st);
    else
        hipLaunchKernelGGL(k_brow, dim3(grid_for(n * BR_GS, BLK, 8192)), dim3(BLK), 0, s, n, ncols, brp, bci, out,
                           ulist, uflag, st);
    return hipGetLastError();
}

// The unsorted-row kernels read their row count from device memory, so they
// are enqueued without a host round trip; surplus workgroups exit at once.
constexpr int UB_GRID = 512;  // two 64 KB-LDS workgroups per CU are resident: one round of workgroups

hipError_t launch_brow_unsorted(const int32_t *list, const int *count, const int64_t *brp, const int32_t *bci,
                                BRow *out, DevStats *st, hipStream_t s) {
    hipLaunchKernelGGL(k_brow_unsorted, dim3(UB_GRID), dim3(WAVE), 0, s, list, count, brp, bci, out,
                       (const int64_t *)nullptr, (uint2 *)nullptr, 0, st, (const int *)nullptr);
    return hipGetLastError();
}

hipError_t launch_compress_unsorted(const int32_t *list, const int *count, const int64_t *brp,
                                    const int32_t *bci, const BRow *bi, const int64_t *bcrp, uint2 *bcw,
                                    const int *enable, hipStream_t s) {
    hipLaunchKernelGGL(k_brow_unsorted, dim3(UB_GRID), dim3(WAVE), 0, s, list, count, brp, bci, (BRow *)bi, bcrp,
                       bcw, 1, (DevStats *)nullptr, enable);
    return hipGetLastError();
}

hipError_t launch_compress_sorted_flags(int64_t n, int64_t nnz, const int64_t *brp, const int32_t *bci, const BRow *bi,
                                        const uint8_t *unsorted, const int64_t *bcrp, uint2 *bcw,
                                        const int *enable, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (nnz <= BR_SHORT * n)
        hipLaunchKernelGGL(k_compress_short, dim3(grid_for(n, BLK, 4096)), dim3(BLK), 0, s, n, brp, bci, unsorted,
                           bcrp, bcw, enable);
    else
        hipLaunchKernelGGL(k_compress_sorted, dim3(grid_for(n * BR_GS, BLK, 8192)), dim3(BLK), 0, s, n, brp, bci, bi,
                           unsorted, bcrp, bcw, enable);
    return hipGetLastError();
}

hipError_t launch_rowinfo(int64_t m, int64_t n, const int64_t *arp, const int32_t *aci, const BRow *bi, int64_t *rflops,
                          int64_t *rflopsc, int2 *rwin, DevStats *st, long long *part, int comp_opt, int selector,
                          double cf_threshold, hipStream_t s) {
    const CompRule rule{comp_opt, selector, cf_threshold};
    const int g = m > 0 ? grid_for(m * RI_GS, BLK, RI_GRID) : 1;
    hipLaunchKernelGGL(k_rowinfo, dim3(g), dim3(BLK), 0, s, m, n, arp, aci, bi, rflops, rflopsc, rwin, part, st);
    hipLaunchKernelGGL(k_rowinfo_fin, dim3(1), dim3(BLK), 0, s, g, (const long long *)part, st, rule);
    return hipGetLastError();
}

// tmp: block sums
int64_t scan_tmp_elems(int64_t n) { return (n + SC_B - 1) / SC_B + 1; }

template <typename T>
static hipError_t scan_impl(int64_t n, const T *in, int stride, int64_t *out, int64_t *tmp, const int *enable,
                            hipStream_t s) {
    const int64_t nb = (n + SC_B - 1) / SC_B;
    if (nb > 0) {
        hipLaunchKernelGGL(k_scan_local<T>, dim3((unsigned)nb), dim3(SC_T), 0, s, n, in, stride, out, tmp, enable);
        if (nb > SC_FEW) hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SC_T), 0, s, nb, tmp, enable);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(SC_T), 0, s, n, nb, out, tmp, enable);
    } else {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(BLK), 0, s, (int32_t *)out, (int64_t)2, 0);
    }
    return hipGetLastError();
}

hipError_t launch_scan_i32s(int64_t n, const int32_t *in, int stride, int64_t *out, int64_t *tmp, const int *enable,
                            hipStream_t s) {
    return scan_impl<int32_t>(n, in, stride, out, tmp, enable, s);
}
hipError_t launch_scan_i32(int64_t n, const int32_t *in, int64_t *out, int64_t *tmp, hipStream_t s) {
    return scan_impl<int32_t>(n, in, 1, out, tmp, nullptr, s);
}

hipError_t launch_store_rp(int64_t n1, const int64_t *src, void *dst, int is64, hipStream_t s) {
    const int g = grid_for(n1, BLK);
    if (is64)
        hipLaunchKernelGGL(k_store_rp64, dim3(g), dim3(BLK), 0, s, n1, src, (int64_t *)dst);
    else
        hipLaunchKernelGGL(k_store_rp32, dim3(g), dim3(BLK), 0, s, n1, src, (int32_t *)dst);
    return hipGetLastError();
}

hipError_t launch_classify(int64_t m, const int64_t *rflops, const int64_t *rflopsc, const int2 *rwin,
                           const int32_t *row_nnz, const int32_t *row_words, ClassParams p, uint8_t *kind,
                           int32_t *row_nnz_out, DevStats *st, int64_t *tmp, int64_t *koff, hipStream_t s) {
    const int64_t nb = (m + CB - 1) / CB;
    if (nb == 0) {
        if (koff) hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(BLK), 0, s, (int32_t *)koff, (int64_t)(2 * (NK + 1)), 0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_classify, dim3((unsigned)nb), dim3(CB), 0, s, m, rflops, rflopsc, rwin, row_nnz, row_words,
                       p, kind, row_nnz_out, (int32_t *)tmp);
    return hipGetLastError();
}

// tmp: per classify workgroup and kind, three maxima and the row count (then
// offset), int32
// per classify workgroup: NK int4 records (maxima, count), then NK compact counts
// (and NK kind totals after them when k_part_fold runs)
int64_t part_tmp_elems(int64_t m) { return (5 * ((m + CB - 1) / CB) * NK + NK + 1) / 2 + 1; }

hipError_t launch_partition(int64_t m, const uint8_t *kind, int32_t *perm, const int64_t *tmp, int64_t *koff,
                            int phase, int heavy, DevStats *st, hipStream_t s) {
    const int64_t nb = (m + CB - 1) / CB;
    if (nb == 0) return hipSuccess;
    if (nb > PF_FEW)
        hipLaunchKernelGGL(k_part_fold, dim3(1), dim3(CB), 0, s, nb, (int32_t *)tmp + 4 * nb * NK);
    hipLaunchKernelGGL(k_part_scatter, dim3((unsigned)nb), dim3(CB), 0, s, m, nb, kind, (const int32_t *)tmp, perm,
                       koff, phase, heavy, st);
    return hipGetLastError();
}

hipError_t launch_kind_ranges(const int32_t *perm, const int64_t *koff, int64_t rb, int64_t re, int64_t *range,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_kind_ranges, dim3(1), dim3(64), 0, s, perm, koff, rb, re, range);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, BLK, 4096)), dim3(BLK), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace spg
