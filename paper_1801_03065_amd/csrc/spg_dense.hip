// Bit-window dense accumulator kernels (the "dense accumulator" of the
// Accumulators subsection, re-cut for gfx950 LDS).
//
// A row i of C only touches columns inside a window of words
// [wlo, whi] (word = column >> 5), known from the analysis pass.  The
// structure of row i is the union of the column-set words of the B rows it
// reads (Compression subsection): OR-ing them into an LDS bit array over the
// window gives the row's pattern; a second-level summary bit per word marks
// the touched words, so counting, ordering and resetting cost the touched
// words only, never the whole window.
//
//  symbolic: row size = sum of popcounts of the touched words (Algorithm 3,
//            symbolic branch).
//  numeric:  the touched words in increasing order get prefix popcounts; the
//            rank of column c in the row is then pre[word] + popcount of the
//            lower bits of its word.  Products are added into vals[rank]
//            (LDS, Algorithm 1's accumulation), and the sorted row is written
//            with coalesced stores.  Output columns come out sorted for free.
//
// K_DW: one 64-lane wavefront per row, Thread-Parallel lane groups (a group
//       of 2^lg_gs lanes walks one B row, several groups per wavefront),
//       window up to 2048 words, row up to 1024 entries.
// K_DG: one 1024-lane workgroup per row, Thread-Flat-Parallel (each lane takes
//       one multiplication of the flattened row; Partitioning Schemes
//       subsection), window up to 32768 words in LDS, values in an HBM array
//       over the window (one slice per resident workgroup: the memory pool of
//       the Accumulators subsection in one-to-one mode).
#include "spg_accum.hpp"
#include "spg_internal.hpp"

namespace spg {

namespace {

// ============================================================ wavefront / row

struct DwLayout {
    size_t bits, summ, pre, wlist, vals, st_bs, st_len, st_cbs, st_clen, st_a, total;
};

__host__ __device__ inline DwLayout dw_layout(int nwm, int rm, int acc_bytes, bool numeric) {
    DwLayout L{};
    const int nsm = (nwm + 31) >> 5;
    size_t o = 0;
    L.bits = o;
    o += align16(4 * (size_t)nwm);
    L.summ = o;
    o += align16(4 * (size_t)nsm);
    L.st_cbs = o;
    o += 8 * WAVE;
    L.st_clen = o;
    o += 4 * WAVE;
    if (numeric) {
        L.st_bs = o;
        o += 8 * WAVE;
        L.st_len = o;
        o += 4 * WAVE;
        L.st_a = o;
        o += 8 * WAVE;
        L.pre = o;
        o += align16(2 * (size_t)nwm);
        L.wlist = o;
        o += align16(2 * (size_t)rm);
        L.vals = o;
        o += align16((size_t)acc_bytes * rm);
    }
    L.total = o;
    return L;
}

constexpr int DW_U = 8;  // B rows per lane group kept in flight

// Stage up to 64 entries of A's row: per entry the extent of B(j,:) in the
// structure source (compressed B when present) and, for the numeric phase,
// in raw B plus the A value.  All extents load in one dependent step.
template <typename VT>
__device__ __forceinline__ int dw_stage(int64_t cb, int64_t ae, const int32_t *aci, const VT *aval,
                                        const int64_t *srp, const int64_t *brp, int64_t *st_cbs,
                                        int32_t *st_clen, int64_t *st_bs, int32_t *st_len, double *st_a) {
    const int l = lane_id();
    const int cn = (int)min((int64_t)WAVE, ae - cb);
    if (l < cn) {
        const int j = aci[cb + l];
        const int64_t c0 = srp[j], c1 = srp[j + 1];
        if (st_bs) {
            const int64_t b0 = brp[j], b1 = brp[j + 1];
            st_bs[l] = b0;
            st_len[l] = (int32_t)(b1 - b0);
            st_a[l] = (double)aval[cb + l];
        }
        st_cbs[l] = c0;
        st_clen[l] = (int32_t)(c1 - c0);
    }
    return cn;
}

// One column-set word of the structure source: window-relative word index
// and its bits.  COMP is a template parameter so that the batched loads of
// dw_or_staged stay branch-free and all issue before the first use.
template <bool COMP>
__device__ __forceinline__ void dw_word(int64_t e, int wlo, const int32_t *bci, const uint2 *bcw, uint32_t &d,
                                        uint32_t &cs) {
    if constexpr (COMP) {
        const uint2 v = bcw[e];
        d = v.x - (uint32_t)wlo;
        cs = v.y;
    } else {
        const int c = bci[e];
        d = (uint32_t)((c >> 5) - wlo);
        cs = 1u << (c & 31);
    }
}

__device__ __forceinline__ void dw_or(uint32_t *bits, uint32_t *summ, uint32_t d, uint32_t cs) {
    atomicOr(&bits[d], cs);
    atomicOr(&summ[d >> 5], 1u << (d & 31));
}

// OR the staged entries' column-set words into bits[] / summ[].  Lane group g
// (2^lg_gs lanes) takes entries g, g+ng, ...; DW_U entries per group are
// loaded before any is used, so each lane keeps DW_U loads in flight.
template <bool COMP>
__device__ __forceinline__ void dw_or_batched(int cn, int wlo, const int32_t *bci, const uint2 *bcw,
                                              int lg_gs, const int64_t *st_cbs,
                                              const int32_t *st_clen, uint32_t *bits, uint32_t *summ) {
    const int l = lane_id();
    const int gs = 1 << lg_gs, g = l >> lg_gs, q = l & (gs - 1), ng = WAVE >> lg_gs;
    for (int t0 = g; t0 < cn; t0 += ng * DW_U) {
        uint32_t d[DW_U], cs[DW_U];
        int len[DW_U];
        int64_t bs[DW_U];
        unsigned okm = 0;
#pragma unroll
        for (int u = 0; u < DW_U; ++u) {  // staging reads first (LDS, group-uniform)
            const int t = min(t0 + u * ng, cn - 1);
            len[u] = st_clen[t];
            bs[u] = st_cbs[t];
        }
#pragma unroll
        for (int u = 0; u < DW_U; ++u) {  // then every global load of the batch
            const bool ok = t0 + u * ng < cn && q < len[u];
            okm |= (unsigned)ok << u;
            dw_word<COMP>(ok ? bs[u] + q : 0, wlo, bci, bcw, d[u], cs[u]);
        }
#pragma unroll
        for (int u = 0; u < DW_U; ++u)
            if (okm & (1u << u)) dw_or(bits, summ, d[u], cs[u]);
        for (int u = 0; u < DW_U; ++u) {  // rows of B longer than the group
            const int t = t0 + u * ng;
            if (t >= cn) break;
            const int tl = st_clen[t];
            for (int p = q + gs; p < tl; p += gs) {
                uint32_t dd, cc;
                dw_word<COMP>(st_cbs[t] + p, wlo, bci, bcw, dd, cc);
                dw_or(bits, summ, dd, cc);
            }
        }
    }
}

__device__ __forceinline__ void dw_or_staged(int cn, int wlo, bool comp, const int32_t *bci, const uint2 *bcw,
                                             int lg_gs, const int64_t *st_cbs,
                                             const int32_t *st_clen, uint32_t *bits, uint32_t *summ) {
    if (comp)
        dw_or_batched<true>(cn, wlo, bci, bcw, lg_gs, st_cbs, st_clen, bits, summ);
    else
        dw_or_batched<false>(cn, wlo, bci, bcw, lg_gs, st_cbs, st_clen, bits, summ);
}

struct RowDesc {
    int64_t ab, ae;
    int wlo, ns;
};

__device__ __forceinline__ RowDesc row_desc(int i, const int64_t *arp, const int2 *rwin) {
    RowDesc d;
    d.ab = arp[i];
    d.ae = arp[i + 1];
    const int2 w = rwin[i];
    d.wlo = w.x;
    d.ns = (w.y - w.x + 1 + 31) >> 5;
    return d;
}

// LDS of the symbolic bit-window kernel: the window's bits and summary, and
// two halves (row p, row p+1) of staging and of the row's (word, bits) list.
struct SwLayout {
    size_t bits, summ, half0, hsize, st_cbs, st_clen, pairs, total;
};

__host__ __device__ inline SwLayout sw_layout(int nwm) {
    SwLayout L{};
    const int nsm = (nwm + 31) >> 5;
    size_t o = 0;
    L.bits = o;
    o += align16(4 * (size_t)nwm);
    L.summ = o;
    o += align16(4 * (size_t)nsm);
    L.half0 = o;
    size_t h = 0;
    L.st_cbs = h;
    h += 8 * WAVE;
    L.st_clen = h;
    h += 4 * WAVE;
    L.pairs = h;
    h += 8 * PL_CAP;
    L.hsize = h;
    o += 2 * h;
    L.total = o;
    return L;
}

constexpr int SW_SLOTS = 8;  // B rows per lane group held in registers (fast path)

struct RowDescS {
    int64_t ab, ae, poff;
    int wlo, whi, plen, i;
};

// Symbolic phase, bit-window accumulator, one wavefront per row: the
// compressed-B words of the row's B rows are ORed into an LDS bit array over
// the row's column window, a summary bit per word marks the touched words;
// row size = sum of their popcounts (Algorithm 3, symbolic branch).  The
// touched words, in increasing order, are also kept as (word, bits) pairs
// for the numeric phase.
//
// Software pipeline over the wavefront's rows p, p+s, ...: per row, first the
// loads for later rows (row p+s's compressed extents, row p+2s's A entries,
// row p+3s's descriptor, lane k < 5 holding field k, and row p+4s's index),
// then row p's word gathers, then row p-s's stores (sizes and pairs, from the
// other LDS half).  The memory counter retires in order, so waiting for the
// gathers never waits for those stores, and the values for later rows have
// landed by the time they are used.
template <bool COMP, int LGS>
__global__ __launch_bounds__(WAVE) void k_sym_dw(SymArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const SwLayout L = sw_layout(a.nw_max);
    uint32_t *bits = (uint32_t *)(smem + L.bits);
    uint32_t *summ = (uint32_t *)(smem + L.summ);
    auto half = [&](int b) -> unsigned char * { return smem + L.half0 + (size_t)b * L.hsize; };
    const int l = lane_id();
    const int nsm = (a.nw_max + 31) >> 5;
    for (int w = l; w < a.nw_max; w += WAVE) bits[w] = 0;
    for (int w = l; w < nsm; w += WAVE) summ[w] = 0;
    // compression is a template parameter: a runtime branch between the two
    // word sources inside the unrolled gathers makes the compiler wait for
    // each load before issuing the next
    const int64_t *srp = COMP ? a.bcrp : a.brp;
    constexpr int gs = 1 << LGS, ng = WAVE >> LGS;
    const int g = l >> LGS, q = l & (gs - 1);
    int64_t lo, hi;
    rs_bounds(a.rs, lo, hi);
    const Slice sl = xcd_slice(lo, hi);

    // lanes 0-4: arp[i], arp[i+1], the window (first | last word), plan_off[i],
    // plan_len[i] (its high word unused; the array has a padding element);
    // two dword loads in every lane, no branch and no merge of the halves
    // (either would wait for the loads)
    auto load_desc = [&](int i) -> int64_t {
        const uint32_t *src = (const uint32_t *)(a.arp + i + (l & 1));
        if (l == 2) src = (const uint32_t *)(a.rwin + i);
        if (l == 3 && a.plan) src = (const uint32_t *)(a.plan_off + i);
        if (l == 4 && a.plan) src = (const uint32_t *)(a.plan_len + i);
        const uint32_t vlo = src[0], vhi = src[1];
        return (int64_t)(((uint64_t)vhi << 32) | vlo);
    };
    auto lane64 = [](int64_t v, int k) -> int64_t {
        const uint32_t vlo = __builtin_amdgcn_readlane((uint32_t)v, k);
        const uint32_t vhi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)v >> 32), k);
        return (int64_t)(((uint64_t)vhi << 32) | vlo);
    };
    auto to_uni = [&](int64_t v, int i) -> RowDescS {
        RowDescS d;
        d.ab = lane64(v, 0);
        d.ae = lane64(v, 1);
        const int64_t w = lane64(v, 2);
        d.wlo = (int)(uint32_t)w;
        d.whi = (int)(uint32_t)((uint64_t)w >> 32);
        d.poff = a.plan ? lane64(v, 3) : 0;
        d.plen = a.plan ? (int)__builtin_amdgcn_readlane((uint32_t)v, 4) : 0;
        d.i = i;
        return d;
    };
    // stage a row's first 64 A entries (compressed extent) into half b;
    // returns 0 (slow path), 1 (fast path) or 2 (fast path, and some B row
    // is longer than its lane group: an overflow pass follows)
    auto stage = [&](int b, int64_t na, int64_t c0, uint32_t c1lo) -> int {
        const int cn = (int)min((int64_t)WAVE, na);
        const int len = (int)(c1lo - (uint32_t)c0);
        // B entries below 2^32 (b32): the extent as (low word, length), and
        // length 0 past the row, so the fast path reads both in one 8-byte
        // LDS read; otherwise the 64-bit extent.  The slow paths read the
        // extent's low word when b32 (later chunks store it 64-bit).  (A
        // separate packed array, 512 more LDS bytes per half, made the
        // batched symbolic launch of wide-window products 60% slower; the
        // same launch with its grid cut to as many wavefronts but the
        // smaller LDS was not.)
        if (a.b32)
            ((int2 *)(half(b) + L.st_cbs))[l] = l < cn ? make_int2((int)(uint32_t)c0, len) : make_int2(0, 0);
        else if (l < cn)
            ((int64_t *)(half(b) + L.st_cbs))[l] = c0;
        if (l < cn) ((int32_t *)(half(b) + L.st_clen))[l] = len;
        const bool fast = a.b32 && na <= WAVE && cn <= ng * SW_SLOTS;
        return fast ? 1 + (__ballot(l < cn && len > gs) != 0) : 0;
    };
    const int64_t st1 = sl.step;
    const int64_t p0 = sl.idx, pend = sl.end;
    auto row_at = [&](int64_t pp) -> int { return pp < pend ? read_first(a.rs.rows[pp]) : 0; };

    // ---- prologue (waits here are once per kernel)
    const int i0 = row_at(p0), i1 = row_at(p0 + st1), i2 = row_at(p0 + 2 * st1);
    RowDescS d = p0 < pend ? to_uni(load_desc(i0), i0) : RowDescS{};
    int64_t rn = p0 + st1 < pend ? load_desc(i1) : 0;  // row p+s, raw
    int in1 = i1;
    int64_t r2 = p0 + 2 * st1 < pend ? load_desc(i2) : 0;  // row p+2s, raw
    int in2 = i2;
    int64_t nan = p0 + st1 < pend ? lane64(rn, 1) - lane64(rn, 0) : 0;
    int64_t f2ab = 0, f2na = 0;
    if (p0 + 2 * st1 < pend) {
        f2ab = lane64(r2, 0);
        f2na = lane64(r2, 1) - f2ab;
    }
    int i3u = row_at(p0 + 3 * st1);
    int kc = 0;  // row p: slots per B row (0: slow path)
    if (p0 < pend) {
        const int cn = (int)min((int64_t)WAVE, d.ae - d.ab);
        int64_t c0 = 0, c1 = 0;
        if (l < cn) {
            const int j = a.aci[d.ab + l];
            c0 = srp[j];
            c1 = srp[j + 1];
        }
        kc = stage(0, d.ae - d.ab, c0, (uint32_t)c1);
    }
    int nj = 0;  // row p+s: A column
    if (p0 + st1 < pend && l < min((int64_t)WAVE, nan)) nj = a.aci[lane64(rn, 0) + l];
    // the previous row's outputs, stored during the next row
    int prev_i = -1, prev_cnt = 0, prev_nwt = 0, prev_plen = 0;
    int64_t prev_poff = 0;
    int b = 0;
    wave_lds_sync();
    for (int64_t pp = p0; pp < pend; pp += st1, b ^= 1) {
        const bool has1 = pp + st1 < pend, has2 = pp + 2 * st1 < pend, has3 = pp + 3 * st1 < pend;
        const int wlo = d.wlo;
        const int64_t *st_cbs = (const int64_t *)(half(b) + L.st_cbs);
        const int32_t *st_clen = (const int32_t *)(half(b) + L.st_clen);
        uint2 *pairs = (uint2 *)(half(b) + L.pairs);
        const int cn = (int)min((int64_t)WAVE, d.ae - d.ab);
        const int kk = kc;

        // ---- 1. loads for later rows
        int64_t nc0 = 0;
        uint32_t nc1 = 0;  // low word of srp[j+1]: only the length is needed
        if (has1 && l < min((int64_t)WAVE, nan)) {
            nc0 = srp[nj];
            nc1 = ((const uint32_t *)srp)[2 * (nj + 1)];
        }
        int nnj = 0;
        if (has2 && l < min((int64_t)WAVE, f2na)) nnj = a.aci[f2ab + l];
        const int64_t raw3 = has3 ? load_desc(i3u) : 0;
        const int in3 = i3u;
        const int i4 = pp + 4 * st1 < pend ? a.rs.rows[pp + 4 * st1] : 0;

        // ---- 2. gathers of row p: slot s2 covers B row t = g + s2 * ng, word q
        uint32_t wd[SW_SLOTS], wc[SW_SLOTS];
        int lenv[SW_SLOTS];  // per slot: the B row's length (0: no word for any lane)
        if (kk > 0) {
            // a lane past its B row loads the entry its offset names, clamped
            // to B's last entry, and is masked by the length when the words
            // are ORed
            const uint32_t elast = (uint32_t)max(a.nnzb - 1, (int64_t)0);
            const int2 *st_pk = (const int2 *)st_cbs;  // fast path: packed (b32)
            int2 pk[SW_SLOTS];
#pragma unroll
            for (int s2 = 0; s2 < SW_SLOTS; ++s2)  // staging reads first: one LDS wait for all
                pk[s2] = st_pk[(g + s2 * ng) & (WAVE - 1)];  // entries past the row have length 0
#pragma unroll
            for (int s2 = 0; s2 < SW_SLOTS; ++s2) {
                const uint32_t cb = (uint32_t)pk[s2].x;  // B entries < 2^30 on this path
                const int len = pk[s2].y;
                // entries past the row have length 0; with more than 64
                // slot entries the index wraps and needs its own test
                lenv[s2] = (ng * SW_SLOTS <= WAVE || g + s2 * ng < cn) ? len : 0;
                const uint32_t e = min(cb + (uint32_t)q, elast);
                if constexpr (COMP) {
                    const uint2 v = ld32(a.bcw, e);  // (word, bits): one 8-byte load
                    wd[s2] = v.x;
                    wc[s2] = v.y;
                } else {
                    const int c = ld32(a.bci, e);
                    wd[s2] = (uint32_t)(c >> 5);
                    wc[s2] = 1u << (c & 31);
                }
            }
        }
        // ---- 3. stores of row p-1 (its pairs from the other half)
        if (prev_i >= 0) {
            if (l == 0) {
                a.row_nnz[prev_i] = prev_cnt;
                a.row_words[prev_i] = prev_nwt;
            }
            const uint2 *pp2 = (const uint2 *)(half(b ^ 1) + L.pairs);
            if (l < min(prev_nwt, prev_plen)) a.plan[prev_poff + l] = pp2[l];
        }
        // ---- 4. OR the words into the window
        if (kk > 0) {
#pragma unroll
            for (int s2 = 0; s2 < SW_SLOTS; ++s2)
                if (q < lenv[s2]) dw_or(bits, summ, wd[s2] - (uint32_t)wlo, wc[s2]);
            if (kk == 2) {  // words beyond the lane group of B rows longer than it
                for (int t = g; t < cn; t += ng) {
                    const int64_t cb = (uint32_t)((const int2 *)st_cbs)[t].x;
                    const int len = st_clen[t];
                    for (int w = q + gs; w < len; w += gs) {
                        uint32_t dd, cc;
                        dw_word<COMP>(cb + w, wlo, a.bci, a.bcw, dd, cc);
                        dw_or(bits, summ, dd, cc);
                    }
                }
            }
        } else {
            for (int64_t cb0 = d.ab; cb0 < d.ae; cb0 += WAVE) {
                int ccn = cn;
                const int64_t *scbs = st_cbs;
                const int32_t *sclen = st_clen;
                if (cb0 != d.ab) {  // later chunks: staged into the slow-path area of this half
                    wave_lds_sync();
                    int64_t *wcbs = (int64_t *)(half(b) + L.st_cbs);
                    int32_t *wclen = (int32_t *)(half(b) + L.st_clen);
                    ccn = dw_stage<double>(cb0, d.ae, a.aci, nullptr, srp, nullptr, wcbs, wclen, nullptr, nullptr,
                                           nullptr);
                    wave_lds_sync();
                }
                // rows beyond the fast path's registers: one word per lane at a
                // time (kept light: the kernel's register budget is set by the
                // fast path)
                for (int t = g; t < ccn; t += ng) {
                    const int64_t cb = a.b32 ? (int64_t)(uint32_t)((const int2 *)scbs)[t].x : scbs[t];
                    const int len = sclen[t];
                    for (int w = q; w < len; w += gs) {
                        uint32_t dd, cc;
                        dw_word<COMP>(cb + w, wlo, a.bci, a.bcw, dd, cc);
                        dw_or(bits, summ, dd, cc);
                    }
                }
            }
        }
        wave_lds_sync();
        // ---- 5. count the touched words in increasing order; keep (word, bits)
        const int ns = (d.whi - wlo + 1 + 31) >> 5;
        int cnt = 0, nwt = 0;
        if (ns <= WAVE) {
            // one summary word per lane: list the touched words (writes only),
            // then, if they fit one pass, one word per lane in parallel
            uint32_t m = l < ns ? summ[l] : 0u;
            if (l < ns) summ[l] = 0;
            const int c = __popc(m);
            const int inc = wave_scan_dpp(c);
            nwt = __builtin_amdgcn_readlane(inc, WAVE - 1);
            uint32_t *list = (uint32_t *)pairs;  // word indices, then overwritten by the pairs
            if (nwt <= WAVE) {
                int pos = inc - c;
                while (m) {
                    list[pos++] = (uint32_t)((l << 5) + __ffs(m) - 1);
                    m &= m - 1;
                }
                wave_lds_sync();
                uint32_t w = 0, bw = 0;
                if (l < nwt) {
                    w = list[l];
                    bw = bits[w];
                    bits[w] = 0;
                    cnt = __popc(bw);
                }
                wave_lds_sync();
                if (l < nwt) pairs[l] = make_uint2((uint32_t)wlo + w, bw);
            } else {
                int pos = inc - c;
                while (m) {
                    const int w = (l << 5) + __ffs(m) - 1;
                    m &= m - 1;
                    const uint32_t bw = bits[w];
                    cnt += __popc(bw);
                    bits[w] = 0;
                    if (pos < PL_CAP) pairs[pos] = make_uint2((uint32_t)(wlo + w), bw);
                    ++pos;
                }
            }
        } else {
            for (int s0 = 0; s0 < ns; s0 += WAVE) {
                const int s = s0 + l;
                uint32_t m = s < ns ? summ[s] : 0u;
                if (s < ns) summ[s] = 0;
                const int c = __popc(m);
                const int inc = wave_scan_dpp(c);
                int pos = nwt + inc - c;
                while (m) {
                    const int w = (s << 5) + __ffs(m) - 1;
                    m &= m - 1;
                    const uint32_t bw = bits[w];
                    cnt += __popc(bw);
                    bits[w] = 0;
                    if (pos < PL_CAP) pairs[pos] = make_uint2((uint32_t)(wlo + w), bw);
                    ++pos;
                }
                nwt += __builtin_amdgcn_readlane(inc, WAVE - 1);
            }
        }
        cnt = __builtin_amdgcn_readlane(wave_scan_dpp(cnt), WAVE - 1);
        prev_i = d.i;
        prev_cnt = cnt;
        prev_nwt = nwt;
        prev_poff = d.poff;
        prev_plen = d.plen;
        // ---- 6. next row: stage it, move the landed descriptors to scalars
        if (has1) {
            kc = stage(b ^ 1, nan, nc0, nc1);
            d = to_uni(rn, in1);
        }
        if (has2) nan = lane64(r2, 1) - lane64(r2, 0);
        if (has3) {
            f2ab = lane64(raw3, 0);
            f2na = lane64(raw3, 1) - f2ab;
        }
        i3u = read_first(i4);
        rn = r2;
        in1 = in2;
        r2 = raw3;
        in2 = in3;
        nj = nnj;
        wave_lds_sync();
    }
    // the last row's stores
    if (prev_i >= 0) {
        if (l == 0) {
            a.row_nnz[prev_i] = prev_cnt;
            a.row_words[prev_i] = prev_nwt;
        }
        const uint2 *pp2 = (const uint2 *)(half(b ^ 1) + L.pairs);
        if (l < min(prev_nwt, prev_plen)) a.plan[prev_poff + l] = pp2[l];
    }
}

// Numeric phase, bit-window accumulator, one wavefront per row.  Rows whose A
// entries fit one chunk of 64 are software-pipelined: the next row's A
// entries and B extents load while this row is processed and move into the
// staging arrays once this row no longer reads them.  Columns are written
// straight from the bit window and the word ranks.
template <typename VT, int ACC>
__global__ __launch_bounds__(WAVE) void k_num_dw(NumArgs<VT> a) {
    using A = Accum<VT, ACC>;
    using S = typename A::store_t;
    extern __shared__ __align__(16) unsigned char smem[];
    const DwLayout L = dw_layout(a.nw_max, a.r_max, sizeof(S), true);
    uint32_t *bits = (uint32_t *)(smem + L.bits);
    uint32_t *summ = (uint32_t *)(smem + L.summ);
    uint16_t *pre = (uint16_t *)(smem + L.pre);
    uint16_t *wlist = (uint16_t *)(smem + L.wlist);
    S *vals = (S *)(smem + L.vals);
    int64_t *st_bs = (int64_t *)(smem + L.st_bs);
    int32_t *st_len = (int32_t *)(smem + L.st_len);
    int64_t *st_cbs = (int64_t *)(smem + L.st_cbs);
    int32_t *st_clen = (int32_t *)(smem + L.st_clen);
    double *st_a = (double *)(smem + L.st_a);
    const int l = lane_id();
    const int nsm = (a.nw_max + 31) >> 5;
    for (int w = l; w < a.nw_max; w += WAVE) bits[w] = 0;
    for (int w = l; w < nsm; w += WAVE) summ[w] = 0;
    wave_lds_sync();
    const bool comp = a.bcrp != nullptr;
    const int64_t *srp = comp ? a.bcrp : a.brp;
    const int gs = 1 << a.lg_gs, g = l >> a.lg_gs, q = l & (gs - 1), ng = WAVE >> a.lg_gs;
    int64_t lo, hi;
    rs_bounds(a.rs, lo, hi);
    const int64_t cbase = a.cbase_row >= 0 ? a.coff[a.cbase_row] : 0;
    const Slice sl = xcd_slice(lo, hi);
    int64_t r = sl.idx;
    int i_next = r < sl.end ? a.rs.rows[r] : 0;
    RowDesc dn = r < sl.end ? row_desc(i_next, a.arp, a.rwin) : RowDesc{};
    int64_t c0n = r < sl.end ? a.coff[i_next] : 0, c1n = r < sl.end ? a.coff[i_next + 1] : 0;
    // staging of the next row in registers (lane l: its A entry l), valid when staged_n
    bool staged_n = false;
    int64_t pb0 = 0, pc0 = 0;
    int plen = 0, pclen = 0;
    double pav = 0.0;
    auto load_stage = [&](const RowDesc &dd) {
        // two dependent steps: A entries, then the extents of their B rows
        int j = 0;
        pav = 0.0;
        if (l < dd.ae - dd.ab) {
            j = a.aci[dd.ab + l];
            pav = (double)a.aval[dd.ab + l];
        }
        return j;
    };
    int pj = 0;
    if (r < sl.end && dn.ae - dn.ab <= WAVE) {
        pj = load_stage(dn);
        if (l < dn.ae - dn.ab) {
            pb0 = a.brp[pj];
            plen = (int)(a.brp[pj + 1] - pb0);
            pc0 = srp[pj];
            pclen = (int)(srp[pj + 1] - pc0);
        }
        staged_n = true;
    }
    while (r < sl.end) {
        const int i = i_next;
        const RowDesc d = dn;
        const int64_t cb = c0n, ce = c1n;
        const bool staged = staged_n;
        r += sl.step;
        if (r < sl.end) {  // prefetch the next row's descriptor
            i_next = a.rs.rows[r];
            dn = row_desc(i_next, a.arp, a.rwin);
            c0n = a.coff[i_next];
            c1n = a.coff[i_next + 1];
        }
        const int wlo = d.wlo, ns = d.ns;
        const bool one_chunk = d.ae - d.ab <= WAVE;
        if (staged) {  // this row's staging, loaded during the previous row
            if (l < d.ae - d.ab) {
                st_bs[l] = pb0;
                st_len[l] = plen;
                st_a[l] = pav;
                st_cbs[l] = pc0;
                st_clen[l] = pclen;
            }
            wave_lds_sync();
        }
        // the next row's A entries (first dependent step of its staging)
        staged_n = false;
        if (r < sl.end && dn.ae - dn.ab <= WAVE) {
            pj = load_stage(dn);
            staged_n = true;
        }
        // 1. structure of the row (staging kept for step 4 when the row fits one chunk)
        for (int64_t c0 = d.ab; c0 < d.ae; c0 += WAVE) {
            int cn;
            if (staged) {
                cn = (int)(d.ae - d.ab);
            } else {
                cn = dw_stage<VT>(c0, d.ae, a.aci, a.aval, srp, a.brp, st_cbs, st_clen, st_bs, st_len, st_a);
                wave_lds_sync();
            }
            dw_or_staged(cn, wlo, comp, a.bci, a.bcw, a.lg_gs_or, st_cbs, st_clen, bits, summ);
            wave_lds_sync();
        }
        // the next row's B extents (second step; its A entries have landed)
        if (staged_n && l < dn.ae - dn.ab) {
            pb0 = a.brp[pj];
            plen = (int)(a.brp[pj + 1] - pb0);
            pc0 = srp[pj];
            pclen = (int)(srp[pj + 1] - pc0);
        }
        // 2. touched words in increasing order
        int T = 0;
        for (int s0 = 0; s0 < ns; s0 += WAVE) {
            const int s = s0 + l;
            uint32_t m = (s < ns) ? summ[s] : 0u;
            const int c = __popc(m);
            const int inc = wave_scan_dpp(c);
            int idx = T + inc - c;
            while (m) {
                if (idx < a.r_max) wlist[idx] = (uint16_t)((s << 5) + __ffs(m) - 1);
                ++idx;
                m &= m - 1;
            }
            if (s < ns) summ[s] = 0;
            T += __builtin_amdgcn_readlane(inc, WAVE - 1);
        }
        wave_lds_sync();
        if (T > a.r_max) {  // structure differs from the plan: flag, reset the window, skip the row
            if (l == 0) atomicAdd(&a.st->mismatch, 1);
            for (int w = l; w < ns * 32; w += WAVE) bits[w] = 0;
            wave_lds_sync();
            continue;
        }
        // 3. prefix popcounts of the touched words
        int run = 0;
        for (int r0 = 0; r0 < T; r0 += WAVE) {
            const int rr = r0 + l;
            const int w = rr < T ? wlist[rr] : 0;
            const int c = rr < T ? __popc(bits[w]) : 0;
            const int inc = wave_scan_dpp(c);
            if (rr < T) pre[w] = (uint16_t)(run + inc - c);
            run += __builtin_amdgcn_readlane(inc, WAVE - 1);
        }
        const int rnnz = run;
        const bool ok = (ce - cb == rnnz);
        if (l == 0 && !ok) atomicAdd(&a.st->mismatch, 1);
        for (int t = l; t < rnnz; t += WAVE) vals[t] = A::zero();
        wave_lds_sync();
        // 4. products into vals[rank]
        for (int64_t c0 = d.ab; c0 < d.ae; c0 += WAVE) {
            int cn;
            if (one_chunk) {
                cn = (int)(d.ae - d.ab);
            } else {
                cn = dw_stage<VT>(c0, d.ae, a.aci, a.aval, srp, a.brp, st_cbs, st_clen, st_bs, st_len, st_a);
                wave_lds_sync();
            }
            for (int t0 = g; t0 < cn; t0 += ng * DW_U) {
                int col[DW_U], len[DW_U];
                int64_t bs[DW_U];
                VT bv[DW_U];
                unsigned okm = 0;
#pragma unroll
                for (int u = 0; u < DW_U; ++u) {  // staging reads first
                    const int t = min(t0 + u * ng, cn - 1);
                    len[u] = st_len[t];
                    bs[u] = st_bs[t];
                }
#pragma unroll
                for (int u = 0; u < DW_U; ++u) {  // then every global load of the batch
                    const bool okp = t0 + u * ng < cn && q < len[u];
                    okm |= (unsigned)okp << u;
                    const int64_t e = okp ? bs[u] + q : 0;
                    col[u] = a.bci[e];
                    bv[u] = a.bval[e];
                }
#pragma unroll
                for (int u = 0; u < DW_U; ++u) {
                    if (okm & (1u << u)) {
                        const VT av = (VT)st_a[t0 + u * ng];
                        const int c = col[u];
                        const int w = (c >> 5) - wlo;
                        const int rk = pre[w] + bits_below(bits[w], c & 31);
                        A::add(&vals[rk], av, bv[u]);
                    }
                }
                for (int u = 0; u < DW_U; ++u) {  // rows of B longer than the group
                    const int t = t0 + u * ng;
                    if (t >= cn) break;
                    const int tl = st_len[t];
                    const VT avt = (VT)st_a[t];
                    for (int p = q + gs; p < tl; p += gs) {
                        const int64_t e = st_bs[t] + p;
                        const int c = a.bci[e];
                        const int w = (c >> 5) - wlo;
                        const int rk = pre[w] + bits_below(bits[w], c & 31);
                        A::add(&vals[rk], avt, a.bval[e]);
                    }
                }
            }
            wave_lds_sync();
        }
        // 5. sorted columns straight from the words, values in rank order;
        //    reset of the touched words
        const int64_t ob = cb - cbase;
        for (int t = l; t < T; t += WAVE) {
            const int w = wlist[t];
            uint32_t m = bits[w];
            int p = pre[w];
            const int base = (wlo + w) << 5;
            if (ok) {
                while (m) {
                    a.cci[ob + p++] = base + __ffs(m) - 1;
                    m &= m - 1;
                }
            }
            bits[w] = 0;
        }
        if (ok)
            for (int t = l; t < rnnz; t += WAVE) a.cval[ob + t] = A::fin(vals[t]);
        wave_lds_sync();
    }
}

// ============================================================ workgroup / row

struct DgLayout {
    size_t bits, summ, st_off, st_bs, st_a, red, total;
};

__host__ __device__ inline DgLayout dg_layout(int nwm) {
    DgLayout L{};
    const int nsm = (nwm + 31) >> 5;
    size_t o = 0;
    L.bits = o;
    o += align16(4 * (size_t)nwm);
    L.summ = o;
    o += align16(4 * (size_t)nsm);
    L.st_off = o;
    o += 8 * DG_WG;
    L.st_bs = o;
    o += 8 * DG_WG;
    L.st_a = o;
    o += 8 * DG_WG;
    L.red = o;
    o += 8 * (DG_WG / WAVE + 2);
    L.total = o;
    return L;
}

// Block-wide exclusive scan of v; *total receives the sum.  red holds
// DG_WG/WAVE + 2 longs.
__device__ __forceinline__ long long block_excl_scan(long long v, long long *red, long long *total) {
    const int t = threadIdx.x, l = lane_id(), wv = t / WAVE;
    const long long inc = wave_incl_scan64(v);
    __syncthreads();
    if (l == WAVE - 1) red[wv] = inc;
    __syncthreads();
    long long off = 0, tot = 0;
#pragma unroll
    for (int u = 0; u < DG_WG / WAVE; ++u) {
        const long long x = red[u];
        if (u < wv) off += x;
        tot += x;
    }
    *total = tot;
    return off + inc - v;
}

// Flat-parallel walk over the row's multiplications in chunks of 256 A
// entries: lane f of the chunk's flattened range finds its A entry by binary
// search in the inclusive prefix st_off[] of the B row lengths.
template <typename F>
__device__ __forceinline__ void dg_flat(int64_t ab, int64_t ae, const int32_t *aci, const int64_t *rp,
                                        int64_t *st_off, int64_t *st_bs, long long *red, F &&body) {
    const int t = threadIdx.x;
    for (int64_t cb = ab; cb < ae; cb += DG_WG) {
        const int cn = (int)min((int64_t)DG_WG, ae - cb);
        long long len = 0;
        if (t < cn) {
            const int j = aci[cb + t];
            const int64_t s0 = rp[j], s1 = rp[j + 1];
            st_bs[t] = s0;
            len = s1 - s0;
        }
        long long tot;
        const long long ex = block_excl_scan(len, red, &tot);
        if (t < cn) st_off[t] = ex + len;
        __syncthreads();
        for (long long f = t; f < tot; f += DG_WG) {
            int lo = 0, hi = cn - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (st_off[mid] > f) hi = mid; else lo = mid + 1;
            }
            const long long before = lo ? st_off[lo - 1] : 0;
            body(lo, st_bs[lo] + (f - before), cb);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int dg_next_row(const RowSet &rs, int64_t lo, int64_t hi, int &x, long long *red) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t t = xcd_grab(rs.queue, lo, hi, x);
        red[DG_WG / WAVE] = t < 0 ? -1 : rs.rows[t];
        red[DG_WG / WAVE + 1] = x;
    }
    __syncthreads();
    x = (int)red[DG_WG / WAVE + 1];
    return (int)red[DG_WG / WAVE];
}

// Structure of a heavy row: its B rows' column-set words OR-ed into the LDS
// window, Thread-Flat-Parallel over chunks of 256 A entries.  Each lane keeps
// DG_U words in flight, and finds the B row of its next word from the one it
// had (its words increase), so long rows cost one LDS read per word.
constexpr int DG_U = 8;

template <bool COMP>
__device__ __forceinline__ void dg_or_batched(int64_t ab, int64_t ae, int wlo, const int32_t *aci,
                                              const int64_t *srp, const int32_t *bci, const uint2 *bcw,
                                              uint32_t *bits, uint32_t *summ,
                                              int64_t *st_off, int64_t *st_bs, long long *red) {
    const int t = threadIdx.x;
    for (int64_t cb = ab; cb < ae; cb += DG_WG) {
        const int cn = (int)min((int64_t)DG_WG, ae - cb);
        long long len = 0;
        if (t < cn) {
            const int j = aci[cb + t];
            const int64_t s0 = srp[j], s1 = srp[j + 1];
            st_bs[t] = s0;
            len = s1 - s0;
        }
        long long tot;
        const long long ex = block_excl_scan(len, red, &tot);
        if (t < cn) st_off[t] = ex + len;
        __syncthreads();
        int kc = 0;
        for (long long f0 = 0; f0 < tot; f0 += (long long)DG_WG * DG_U) {
            int64_t e[DG_U];
            bool ok[DG_U];
#pragma unroll
            for (int u = 0; u < DG_U; ++u) {
                const long long f = f0 + u * DG_WG + t;
                ok[u] = f < tot;
                if (ok[u] && st_off[kc] <= f) {  // next B row: binary search over the rest
                    int lo = kc + 1, hi = cn - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (st_off[mid] > f) hi = mid;
                        else lo = mid + 1;
                    }
                    kc = lo;
                }
                e[u] = ok[u] ? st_bs[kc] + (f - (kc ? st_off[kc - 1] : 0)) : 0;
            }
            uint32_t d[DG_U], cs[DG_U];
#pragma unroll
            for (int u = 0; u < DG_U; ++u) {
                if constexpr (COMP) {
                    const uint2 v = bcw[e[u]];
                    d[u] = v.x - (uint32_t)wlo;
                    cs[u] = v.y;
                } else {
                    const int c = bci[e[u]];
                    d[u] = (uint32_t)((c >> 5) - wlo);
                    cs[u] = 1u << (c & 31);
                }
            }
#pragma unroll
            for (int u = 0; u < DG_U; ++u) {
                if (ok[u]) {
                    atomicOr(&bits[d[u]], cs[u]);
                    atomicOr(&summ[d[u] >> 5], 1u << (d[u] & 31));
                }
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void dg_or_pass(int i, int wlo, const int64_t *arp, const int32_t *aci,
                                           const int64_t *brp, const int32_t *bci, const int64_t *bcrp,
                                           const uint2 *bcw, uint32_t *bits,
                                           uint32_t *summ, int64_t *st_off, int64_t *st_bs, long long *red) {
    if (bcrp)
        dg_or_batched<true>(arp[i], arp[i + 1], wlo, aci, bcrp, bci, bcw, bits, summ, st_off, st_bs, red);
    else
        dg_or_batched<false>(arp[i], arp[i + 1], wlo, aci, brp, bci, bcw, bits, summ, st_off, st_bs, red);
}

// Segment list of a heavy row (the row's bit window is complete in bits /
// summ): a segment starts at the touched word that holds entry q*SG_CUT for
// each q, and at the first touched word of each aligned group of SG_NW words.
// So a segment holds at most SG_CUT + 31 < SG_CAP entries and its words lie in
// one group.  list[0] = (S, 0), list[1..S] = (first word, entries before it),
// list[S+1] = (window words, row size).  Clears bits / summ; returns the row
// size (low half) and touched words (high half).
__device__ long long dg_segments(int nw, int ns, uint32_t *bits, uint32_t *summ, int *gfirst, long long *red,
                                 uint2 *list, int cap, DevStats *st) {
    const int t = threadIdx.x;
    const int ng = (nw + SG_NW - 1) / SG_NW;
    if (t < ng) gfirst[t] = INT_MAX;
    __syncthreads();
    for (int s = t; s < ns; s += DG_WG) {
        const uint32_t m = summ[s];
        if (m) atomicMin(&gfirst[(s << 5) / SG_NW], (s << 5) + __ffs(m) - 1);
    }
    __syncthreads();
    long long run = 0, words = 0, cuts = 0;
    for (int s0 = 0; s0 < ns; s0 += DG_WG) {
        const int s = s0 + t;
        const uint32_t m = s < ns ? summ[s] : 0u;
        long long c = 0;
        for (uint32_t mm = m; mm; mm &= mm - 1) c += __popc(bits[(s << 5) + __ffs(mm) - 1]);
        long long tot;
        const long long ex = block_excl_scan(c + ((long long)__popc(m) << 32), red, &tot);
        const int pbeg = (int)(run + (ex & 0xffffffffll));
        int p = pbeg, nc = 0;
        for (uint32_t mm = m; mm; mm &= mm - 1) {
            const int d = (s << 5) + __ffs(mm) - 1;
            const int cd = __popc(bits[d]);
            const int mult = ((p + SG_CUT - 1) / SG_CUT) * SG_CUT;  // first multiple of SG_CUT >= p
            nc += (mult < p + cd || d == gfirst[d / SG_NW]) ? 1 : 0;
            p += cd;
        }
        long long ctot;
        long long idx = cuts + block_excl_scan(nc, red, &ctot);
        p = pbeg;
        for (uint32_t mm = m; mm; mm &= mm - 1) {
            const int d = (s << 5) + __ffs(mm) - 1;
            const int cd = __popc(bits[d]);
            const int mult = ((p + SG_CUT - 1) / SG_CUT) * SG_CUT;
            if (mult < p + cd || d == gfirst[d / SG_NW]) {
                if (idx + 2 < cap) list[1 + idx] = make_uint2((uint32_t)d, (uint32_t)p);
                ++idx;
            }
            p += cd;
            bits[d] = 0;
        }
        if (s < ns) summ[s] = 0;
        run += tot & 0xffffffffll;
        words += tot >> 32;
        cuts += ctot;
    }
    if (t == 0) {
        if (cuts + 2 <= cap) {
            list[0] = make_uint2((uint32_t)cuts, 0u);
            list[1 + cuts] = make_uint2((uint32_t)nw, (uint32_t)run);
        } else {
            atomicAdd(&st->overflow, 1);
        }
    }
    return run | (words << 32);
}

__global__ __launch_bounds__(DG_WG) void k_sym_dg(SymArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const DgLayout L = dg_layout(a.nw_max);
    uint32_t *bits = (uint32_t *)(smem + L.bits);
    uint32_t *summ = (uint32_t *)(smem + L.summ);
    int64_t *st_off = (int64_t *)(smem + L.st_off);
    int64_t *st_bs = (int64_t *)(smem + L.st_bs);
    long long *red = (long long *)(smem + L.red);
    __shared__ int gfirst[DG_NW_MAX / SG_NW];
    const int t = threadIdx.x;
    const int nsm = (a.nw_max + 31) >> 5;
    for (int w = t; w < a.nw_max; w += DG_WG) bits[w] = 0;
    for (int w = t; w < nsm; w += DG_WG) summ[w] = 0;
    int64_t lo, hi;
    rs_bounds(a.rs, lo, hi);
    int x = blockIdx.x % XCDS;
    for (;;) {
        const int i = dg_next_row(a.rs, lo, hi, x, red);
        if (i < 0) break;
        const int2 win = a.rwin[i];
        const int ns = (win.y - win.x + 1 + 31) >> 5;
        dg_or_pass(i, win.x, a.arp, a.aci, a.brp, a.bci, a.bcrp, a.bcw, bits, summ, st_off, st_bs, red);
        const int cap = a.plan ? a.plan_len[i] : 0;
        if (cap > 0) {
            const long long r = dg_segments(win.y - win.x + 1, ns, bits, summ, gfirst, red, a.plan + a.plan_off[i],
                                            cap, a.st);
            if (t == 0) {
                a.row_nnz[i] = (int32_t)(r & 0xffffffffll);
                a.row_words[i] = (int32_t)(r >> 32);
            }
            continue;
        }
        long long cnt = 0;
        for (int s = t; s < ns; s += DG_WG) {
            uint32_t m = summ[s];
            summ[s] = 0;
            cnt += (long long)__popc(m) << 32;  // touched words in the high half
            while (m) {
                const int d = (s << 5) + __ffs(m) - 1;
                m &= m - 1;
                cnt += __popc(bits[d]);
                bits[d] = 0;
            }
        }
        long long tot;
        block_excl_scan(cnt, red, &tot);
        if (t == 0) {
            a.row_nnz[i] = (int32_t)(tot & 0xffffffffll);
            a.row_words[i] = (int32_t)(tot >> 32);
        }
    }
}

template <typename VT, int ACC>
__global__ __launch_bounds__(DG_WG) void k_num_dg(NumArgs<VT> a) {
    using A = Accum<VT, ACC>;
    using S = typename A::store_t;
    extern __shared__ __align__(16) unsigned char smem[];
    const DgLayout L = dg_layout(a.nw_max);
    uint32_t *bits = (uint32_t *)(smem + L.bits);
    uint32_t *summ = (uint32_t *)(smem + L.summ);
    int64_t *st_off = (int64_t *)(smem + L.st_off);
    int64_t *st_bs = (int64_t *)(smem + L.st_bs);
    long long *red = (long long *)(smem + L.red);
    S *gv = (S *)a.arena + (int64_t)blockIdx.x * a.arena_cap;  // this workgroup's window of values
    const int t = threadIdx.x;
    const int nsm = (a.nw_max + 31) >> 5;
    for (int w = t; w < a.nw_max; w += DG_WG) bits[w] = 0;
    for (int w = t; w < nsm; w += DG_WG) summ[w] = 0;
    int64_t lo, hi;
    rs_bounds(a.rs, lo, hi);
    const int64_t cbase = a.cbase_row >= 0 ? a.coff[a.cbase_row] : 0;
    int x = blockIdx.x % XCDS;
    for (;;) {
        const int i = dg_next_row(a.rs, lo, hi, x, red);
        if (i < 0) break;
        const int2 win = a.rwin[i];
        const int wlo = win.x;
        const int ns = (win.y - win.x + 1 + 31) >> 5;
        const int64_t colbase = (int64_t)wlo << 5;  // first column of the row's window
        dg_or_pass(i, wlo, a.arp, a.aci, a.brp, a.bci, a.bcrp, a.bcw, bits, summ, st_off, st_bs, red);
        const int64_t ab = a.arp[i], ae = a.arp[i + 1];
        dg_flat(ab, ae, a.aci, a.brp, st_off, st_bs, red, [&](int k, int64_t e, int64_t cb) {
            const VT av = a.aval[cb + k];
            A::add(&gv[a.bci[e] - colbase], av, a.bval[e]);
        });
        __threadfence();  // the HBM atomics above complete before any lane reads a slot
        __syncthreads();
        // sorted write-out: summary words in chunks of 256
        const int64_t c0 = a.coff[i];
        const int64_t cend = a.coff[i + 1];
        long long run = 0;
        for (int s0 = 0; s0 < ns; s0 += DG_WG) {
            const int s = s0 + t;
            const uint32_t m = (s < ns) ? summ[s] : 0u;
            long long cnt = 0;
            for (uint32_t mm = m; mm; mm &= mm - 1) cnt += __popc(bits[(s << 5) + __ffs(mm) - 1]);
            long long tot;
            const long long ex = block_excl_scan(cnt, red, &tot);
            int64_t pos = c0 + run + ex;
            for (uint32_t mm = m; mm; mm &= mm - 1) {
                const int d = (s << 5) + __ffs(mm) - 1;
                uint32_t w = bits[d];
                const int base = (wlo + d) << 5;
                while (w) {
                    const int col = base + __ffs(w) - 1;
                    w &= w - 1;
                    S *slot = &gv[col - colbase];
                    const S v = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(slot, A::zero(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (pos < cend) {
                        a.cci[pos - cbase] = col;
                        a.cval[pos - cbase] = A::fin(v);
                    }
                    ++pos;
                }
                bits[d] = 0;
            }
            if (s < ns) summ[s] = 0;
            run += tot;
        }
        if (t == 0 && cend - c0 != run) atomicAdd(&a.st->mismatch, 1);
        __threadfence();
    }
}

template <typename K>
inline int resident_grid(K kernel, int block, size_t lds, int cus) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int g = per_cu * cus;
    g = (g / XCDS) * XCDS;
    return g < XCDS ? XCDS : g;
}

}  // namespace

size_t lds_sym_dw(int nw_max) { return sw_layout(nw_max).total; }
size_t lds_num_dw(int nw_max, int r_max, int acc_bytes, int) { return dw_layout(nw_max, r_max, acc_bytes, true).total; }
size_t lds_sym_dg(int nw_max) { return dg_layout(nw_max).total; }
size_t lds_num_dg(int nw_max) { return dg_layout(nw_max).total; }

// At most SW_WAVES_PER_CU resident wavefronts per CU: with small windows the
// LDS would admit 21, and the 27-point A*A symbolic launch is fastest at 18
// (1.01 ms against 1.17 at 21, 1.05 at 16, 1.14 at 12): more rows in flight
// per CU than its L1 holds the B records of.
constexpr int SW_WAVES_PER_CU = 18;

template <bool COMP, int LGS>
hipError_t sym_dw_lg(const SymArgs &a, const LaunchCfg &c) {
    const size_t lds = lds_sym_dw(a.nw_max);
    const int grid = c.grid > 0 ? c.grid
                                : std::min(SW_WAVES_PER_CU * c.cus, resident_grid(k_sym_dw<COMP, LGS>, WAVE, lds, c.cus));
    hipLaunchKernelGGL((k_sym_dw<COMP, LGS>), dim3(grid), dim3(WAVE), lds, c.stream, a);
    return hipGetLastError();
}

template <bool COMP>
hipError_t sym_dw_impl(const SymArgs &a, const LaunchCfg &c) {
    switch (a.lg_gs) {
    case 0: return sym_dw_lg<COMP, 0>(a, c);
    case 1: return sym_dw_lg<COMP, 1>(a, c);
    case 2: return sym_dw_lg<COMP, 2>(a, c);
    case 3: return sym_dw_lg<COMP, 3>(a, c);
    case 4: return sym_dw_lg<COMP, 4>(a, c);
    case 5: return sym_dw_lg<COMP, 5>(a, c);
    case 6: return sym_dw_lg<COMP, 6>(a, c);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sym_dw(const SymArgs &a, const LaunchCfg &c) {
    return a.bcrp ? sym_dw_impl<true>(a, c) : sym_dw_impl<false>(a, c);
}

hipError_t launch_sym_dg(const SymArgs &a, const LaunchCfg &c) {
    const size_t lds = lds_sym_dg(a.nw_max);
    const int grid = c.grid > 0 ? c.grid : resident_grid(k_sym_dg, DG_WG, lds, c.cus);
    hipLaunchKernelGGL(k_sym_dg, dim3(grid), dim3(DG_WG), lds, c.stream, a);
    return hipGetLastError();
}

template <typename VT, int ACC>
static hipError_t num_dw_impl(const NumArgs<VT> &a, const LaunchCfg &c) {
    const size_t lds = lds_num_dw(a.nw_max, a.r_max, sizeof(typename Accum<VT, ACC>::store_t), sizeof(VT));
    const int grid = c.grid > 0 ? c.grid : resident_grid(k_num_dw<VT, ACC>, WAVE, lds, c.cus);
    hipLaunchKernelGGL((k_num_dw<VT, ACC>), dim3(grid), dim3(WAVE), lds, c.stream, a);
    return hipGetLastError();
}

template <typename VT, int ACC>
static hipError_t num_dg_impl(const NumArgs<VT> &a, const LaunchCfg &c) {
    const size_t lds = lds_num_dg(a.nw_max);
    const int grid = c.grid > 0 ? c.grid : resident_grid(k_num_dg<VT, ACC>, DG_WG, lds, c.cus);
    hipLaunchKernelGGL((k_num_dg<VT, ACC>), dim3(grid), dim3(DG_WG), lds, c.stream, a);
    return hipGetLastError();
}

template <>
hipError_t launch_num_dw<double>(const NumArgs<double> &a, int, const LaunchCfg &c) {
    return num_dw_impl<double, ACC_NATIVE>(a, c);
}
template <>
hipError_t launch_num_dw<float>(const NumArgs<float> &a, int acc, const LaunchCfg &c) {
    if (acc == ACC_COMP) return num_dw_impl<float, ACC_COMP>(a, c);
    if (acc == ACC_WIDE) return num_dw_impl<float, ACC_WIDE>(a, c);
    return num_dw_impl<float, ACC_NATIVE>(a, c);
}
template <>
hipError_t launch_num_dg<double>(const NumArgs<double> &a, int, const LaunchCfg &c) {
    return num_dg_impl<double, ACC_NATIVE>(a, c);
}
template <>
hipError_t launch_num_dg<float>(const NumArgs<float> &a, int acc, const LaunchCfg &c) {
    if (acc == ACC_COMP) return num_dg_impl<float, ACC_COMP>(a, c);
    if (acc == ACC_WIDE) return num_dg_impl<float, ACC_WIDE>(a, c);
    return num_dg_impl<float, ACC_NATIVE>(a, c);
}

// Grid of the persistent kernels: resident workgroups of the concrete kernel.
int dg_resident_grid(int acc, bool dbl, size_t lds, int cus) {
    if (dbl) return resident_grid(k_num_dg<double, ACC_NATIVE>, DG_WG, lds, cus);
    if (acc == ACC_COMP) return resident_grid(k_num_dg<float, ACC_COMP>, DG_WG, lds, cus);
    if (acc == ACC_WIDE) return resident_grid(k_num_dg<float, ACC_WIDE>, DG_WG, lds, cus);
    return resident_grid(k_num_dg<float, ACC_NATIVE>, DG_WG, lds, cus);
}

}  // namespace spg
