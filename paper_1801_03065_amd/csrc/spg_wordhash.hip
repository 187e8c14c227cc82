// Word-hash accumulator, one wavefront per row (numeric phase).
//
// The structure of a row of C is the union of column-set words (column >> 5
// with a 32-bit mask; Compression subsection).  Instead of a bit array over
// the row's whole column window, the touched words live in a small
// linear-probing table in LDS (LP hashmap, Accumulators subsection: power-of-two
// size, at most 50% occupancy), plus a one-bit-per-word summary over the
// window that yields the touched words in increasing order.  Each table slot
// holds (bits, pre) where pre is the number of row entries in lower words, so
// the rank of column c in the sorted row is pre + popcount(bits below c).
// Products are added into vals[rank] (Algorithm 1's accumulation), and the row
// leaves sorted, with coalesced stores.
//
// LDS per row is set by the row's touched words and size, not by its column
// window, so many rows are in flight per CU; window-sized state is only the
// summary (window / 1024 words).
//
// Work split (Partitioning Schemes subsection): Thread-Parallel lane groups,
// 2^lg_gs lanes per B row, several B rows per wavefront.  Fast path: when the
// row's A entries fit WH_U entries per group and every B row fits one group,
// all products (column, value) are loaded once into registers, inserted into
// the table, then ranked and accumulated from registers.  Other rows take a
// two-pass batched path (structure pass, then product pass).
#include "spg_accum.hpp"
#include "spg_internal.hpp"

namespace spg {

namespace {

constexpr int WH_U = 16;  // A entries per lane group held in registers (fast path)

struct WhLayout {
    size_t tkey, tbp, summ, wlist, vals, colbuf, st_bs, st_len, st_a, total;
};

__host__ __device__ inline WhLayout wh_layout(int ts, int nsm, int rm, int tm, int acc_bytes) {
    WhLayout L{};
    size_t o = 0;
    L.tbp = o;  // 64-bit slots: low word bits, high word prefix count
    o += 8 * (size_t)ts;
    L.tkey = o;
    o += align16(4 * (size_t)ts);
    L.summ = o;
    o += align16(4 * (size_t)nsm);
    L.wlist = o;  // touched words in order: (word << 16) | slot is too narrow; keep slot only
    o += align16(4 * (size_t)tm);
    L.vals = o;
    o += align16((size_t)acc_bytes * rm);
    L.colbuf = o;
    o += align16(4 * (size_t)rm);
    L.st_bs = o;
    o += 8 * WAVE;
    L.st_a = o;
    o += 8 * WAVE;
    L.st_len = o;
    o += 4 * WAVE;
    L.total = o;
    return L;
}

__device__ __forceinline__ uint32_t wh_hash(uint32_t d, int lg_ts) { return (d * 2654435761u) >> (32 - lg_ts); }

// Slot of window-relative word d, inserted if absent (first insert sets the
// summary bit).  The table never fills: size >= 2 * touched words.
__device__ __forceinline__ uint32_t wh_insert(int32_t *tkey, uint32_t *summ, uint32_t d, int lg_ts) {
    const uint32_t mask = (1u << lg_ts) - 1;
    uint32_t h = wh_hash(d, lg_ts);
    for (;;) {
        const int32_t k = tkey[h];
        if (k == (int32_t)d) return h;
        if (k == -1) {
            const int32_t old = atomicCAS(&tkey[h], -1, (int32_t)d);
            if (old == -1) {
                atomicOr(&summ[d >> 5], 1u << (d & 31));
                return h;
            }
            if (old == (int32_t)d) return h;
        }
        h = (h + 1) & mask;
    }
}

// Slot of a word known to be present.
__device__ __forceinline__ uint32_t wh_find(const int32_t *tkey, uint32_t d, int lg_ts) {
    const uint32_t mask = (1u << lg_ts) - 1;
    uint32_t h = wh_hash(d, lg_ts);
    while (tkey[h] != (int32_t)d) h = (h + 1) & mask;
    return h;
}

struct RowDescW {
    int64_t ab, ae, cb, ce;
    int wlo, ns;
};

__device__ __forceinline__ RowDescW row_desc_w(int i, const int64_t *arp, const int2 *rwin, const int64_t *coff) {
    RowDescW d;
    d.ab = arp[i];
    d.ae = arp[i + 1];
    d.cb = coff[i];
    d.ce = coff[i + 1];
    const int2 w = rwin[i];
    d.wlo = w.x;
    d.ns = (w.y - w.x + 1 + 31) >> 5;
    return d;
}

template <typename VT, int ACC>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_num_wh(NumArgs<VT> a) {
    using A = Accum<VT, ACC>;
    using S = typename A::store_t;
    extern __shared__ __align__(16) unsigned char smem[];
    const int nsm = (a.nw_max + 31) >> 5;
    const int tm = a.ts / 2;
    const WhLayout L = wh_layout(a.ts, nsm, a.r_max, tm, sizeof(S));
    unsigned long long *tbp = (unsigned long long *)(smem + L.tbp);
    uint32_t *tbits = (uint32_t *)(smem + L.tbp);  // low words of tbp (slot h at index 2h)
    int32_t *tkey = (int32_t *)(smem + L.tkey);
    uint32_t *summ = (uint32_t *)(smem + L.summ);
    uint32_t *wlist = (uint32_t *)(smem + L.wlist);
    S *vals = (S *)(smem + L.vals);
    int32_t *colbuf = (int32_t *)(smem + L.colbuf);
    int64_t *st_bs = (int64_t *)(smem + L.st_bs);
    double *st_a = (double *)(smem + L.st_a);
    int32_t *st_len = (int32_t *)(smem + L.st_len);
    const int l = lane_id();
    const int lg_ts = __ffs(a.ts) - 1;
    for (int s = l; s < a.ts; s += WAVE) {
        tkey[s] = -1;
        tbp[s] = 0ull;
    }
    for (int s = l; s < nsm; s += WAVE) summ[s] = 0;
    wave_lds_sync();
    const int gs = 1 << a.lg_gs, g = l >> a.lg_gs, q = l & (gs - 1), ng = WAVE >> a.lg_gs;
    int64_t lo, hi;
    rs_bounds(a.rs, lo, hi);
    const int64_t cbase = a.cbase_row >= 0 ? a.coff[a.cbase_row] : 0;
    const Slice sl = xcd_slice(lo, hi);
    // Software pipeline across rows: while row r is processed, row r+1's A
    // entries (first level) and B row extents (second level) are already in
    // flight, and row r+2's descriptor; only the product loads of a row are
    // exposed latency.
    int64_t r = sl.idx;
    RowDescW dcur = r < sl.end ? row_desc_w(a.rs.rows[r], a.arp, a.rwin, a.coff) : RowDescW{};
    int64_t sb0 = 0, sb1 = 0;  // staged extents / value of this lane's A entry (first chunk)
    double sav = 0.0;
    if (r < sl.end && l < min((int64_t)WAVE, dcur.ae - dcur.ab)) {
        const int j = a.aci[dcur.ab + l];
        sav = (double)a.aval[dcur.ab + l];
        sb0 = a.brp[j];
        sb1 = a.brp[j + 1];
    }
    RowDescW dn = r + sl.step < sl.end ? row_desc_w(a.rs.rows[r + sl.step], a.arp, a.rwin, a.coff) : RowDescW{};
    while (r < sl.end) {
        const RowDescW d = dcur;
        r += sl.step;
        const bool has_next = r < sl.end;
        const int wlo = d.wlo;
        const int64_t na = d.ae - d.ab;
        // ---- stage the first chunk of A's row from the prefetched registers
        int cn = (int)min((int64_t)WAVE, na);
        int mylen = 0;
        if (l < cn) {
            st_bs[l] = sb0;
            st_a[l] = sav;
            mylen = (int)(sb1 - sb0);
            st_len[l] = mylen;
        }
        const bool fast = na <= WAVE && cn <= ng * WH_U && wave_max(mylen) <= gs;
        // next row, first level: its A entries
        const int ncn = has_next ? (int)min((int64_t)WAVE, dn.ae - dn.ab) : 0;
        int nj = 0;
        if (l < ncn) {
            nj = a.aci[dn.ab + l];
            sav = (double)a.aval[dn.ab + l];
        }
        wave_lds_sync();

        // ---- structure: insert every product's word, keep its slot / bit
        uint32_t pk[WH_U];  // slot << 5 | bit, or ~0u for no product
        VT pv[WH_U];
        unsigned okm = 0;
        if (fast) {
            int col[WH_U];
#pragma unroll
            for (int u = 0; u < WH_U; ++u) {
                const int t = g + u * ng;
                const int tt = t < cn ? t : 0;
                const int len = st_len[tt];
                const bool ok = t < cn && q < len;
                okm |= (unsigned)ok << u;
                col[u] = a.bci[ok ? st_bs[tt] + q : 0];
            }
#pragma unroll
            for (int u = 0; u < WH_U; ++u) {
                pk[u] = ~0u;
                if (okm & (1u << u)) {
                    const int c = col[u];
                    const uint32_t dw = (uint32_t)((c >> 5) - wlo);
                    const uint32_t h = wh_insert(tkey, summ, dw, lg_ts);
                    atomicOr(&tbits[2 * h], 1u << (c & 31));
                    pk[u] = (h << 5) | (uint32_t)(c & 31);
                }
            }
            // the values load now and arrive during the scans below
#pragma unroll
            for (int u = 0; u < WH_U; ++u) {
                const int t = g + u * ng;
                const int tt = t < cn ? t : 0;
                pv[u] = a.bval[(okm & (1u << u)) ? st_bs[tt] + q : 0];
            }
        } else {
            for (int64_t c0 = d.ab; c0 < d.ae; c0 += WAVE) {
                if (c0 != d.ab) {
                    wave_lds_sync();
                    cn = (int)min((int64_t)WAVE, d.ae - c0);
                    if (l < cn) {
                        const int j = a.aci[c0 + l];
                        const int64_t b0 = a.brp[j], b1 = a.brp[j + 1];
                        st_bs[l] = b0;
                        st_len[l] = (int)(b1 - b0);
                    }
                    wave_lds_sync();
                }
                for (int t = g; t < cn; t += ng) {
                    const int64_t bs = st_bs[t];
                    const int len = st_len[t];
                    for (int p = q; p < len; p += gs) {
                        const int c = a.bci[bs + p];
                        const uint32_t h = wh_insert(tkey, summ, (uint32_t)((c >> 5) - wlo), lg_ts);
                        atomicOr(&tbits[2 * h], 1u << (c & 31));
                    }
                }
            }
        }
        // next row, second level: its B row extents; the row after: descriptor
        if (l < ncn) {
            sb0 = a.brp[nj];
            sb1 = a.brp[nj + 1];
        }
        dcur = dn;
        if (r + sl.step < sl.end) dn = row_desc_w(a.rs.rows[r + sl.step], a.arp, a.rwin, a.coff);
        wave_lds_sync();

        // ---- touched words in increasing order (summary), prefix counts per slot
        int T = 0;
        for (int s0 = 0; s0 < d.ns; s0 += WAVE) {
            const int s = s0 + l;
            uint32_t m = (s < d.ns) ? summ[s] : 0u;
            const int c = __popc(m);
            const int inc = wave_incl_scan(c);
            int idx = T + inc - c;
            while (m) {
                const uint32_t dw = (uint32_t)((s << 5) + __ffs(m) - 1);
                m &= m - 1;
                if (idx < tm) wlist[idx] = wh_find(tkey, dw, lg_ts);
                ++idx;
            }
            if (s < d.ns) summ[s] = 0;
            T += __shfl(inc, WAVE - 1);
        }
        wave_lds_sync();
        int run = 0;
        for (int r0 = 0; r0 < T; r0 += WAVE) {
            const int rr = r0 + l;
            const uint32_t h = rr < T ? wlist[rr] : 0u;
            const int c = rr < T ? __popc(tbits[2 * h]) : 0;
            const int inc = wave_incl_scan(c);
            if (rr < T) tbits[2 * h + 1] = (uint32_t)(run + inc - c);
            run += __shfl(inc, WAVE - 1);
        }
        const int rnnz = run;
        const bool ok = (d.ce - d.cb == rnnz) && rnnz <= a.r_max && T <= tm;
        if (l == 0 && !ok) atomicAdd(&a.st->mismatch, 1);
        for (int t = l; t < min(rnnz, a.r_max); t += WAVE) vals[t] = A::zero();
        wave_lds_sync();

        // ---- products into vals[rank]
        if (ok) {
            if (fast) {
#pragma unroll
                for (int u = 0; u < WH_U; ++u) {
                    if (pk[u] != ~0u) {
                        const unsigned long long e = tbp[pk[u] >> 5];
                        const uint32_t bits = (uint32_t)e, pre = (uint32_t)(e >> 32);
                        const int rk = (int)pre + __popc(bits & ((1u << (pk[u] & 31)) - 1u));
                        A::add(&vals[rk], (VT)st_a[g + u * ng], pv[u]);
                    }
                }
            } else {
                for (int64_t c0 = d.ab; c0 < d.ae; c0 += WAVE) {
                    wave_lds_sync();
                    cn = (int)min((int64_t)WAVE, d.ae - c0);
                    if (l < cn) {
                        const int j = a.aci[c0 + l];
                        const int64_t b0 = a.brp[j], b1 = a.brp[j + 1];
                        st_bs[l] = b0;
                        st_len[l] = (int)(b1 - b0);
                        st_a[l] = (double)a.aval[c0 + l];
                    }
                    wave_lds_sync();
                    for (int t = g; t < cn; t += ng) {
                        const int64_t bs = st_bs[t];
                        const int len = st_len[t];
                        const VT av = (VT)st_a[t];
                        for (int p = q; p < len; p += gs) {
                            const int c = a.bci[bs + p];
                            const uint32_t h = wh_find(tkey, (uint32_t)((c >> 5) - wlo), lg_ts);
                            const unsigned long long e = tbp[h];
                            const int rk = (int)(uint32_t)(e >> 32) + bits_below((uint32_t)e, c & 31);
                            A::add(&vals[rk], av, a.bval[bs + p]);
                        }
                    }
                }
            }
        }
        wave_lds_sync();

        // ---- sorted columns, table reset
        for (int t = l; t < min(T, tm); t += WAVE) {
            const uint32_t h = wlist[t];
            const int32_t dw = tkey[h];
            const unsigned long long e = tbp[h];
            uint32_t m = (uint32_t)e;
            int p = (int)(uint32_t)(e >> 32);
            const int base = (wlo + dw) << 5;
            if (ok) {
                while (m) {
                    colbuf[p++] = base + __ffs(m) - 1;
                    m &= m - 1;
                }
            }
            tkey[h] = -1;
            tbp[h] = 0ull;
        }
        if (T > tm) {  // inconsistent row: clear the whole table
            for (int s = l; s < a.ts; s += WAVE) {
                tkey[s] = -1;
                tbp[s] = 0ull;
            }
        }
        wave_lds_sync();
        if (ok) {
            const int64_t ob = d.cb - cbase;
            for (int t = l; t < rnnz; t += WAVE) {
                a.cci[ob + t] = colbuf[t];
                a.cval[ob + t] = A::fin(vals[t]);
            }
        }
        wave_lds_sync();
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

template <typename VT, int ACC>
hipError_t num_wh_impl(const NumArgs<VT> &a, const LaunchCfg &c) {
    const size_t lds = lds_num_wh(a.ts, a.nw_max, a.r_max, sizeof(typename Accum<VT, ACC>::store_t));
    const int grid = c.grid > 0 ? c.grid : resident_grid(k_num_wh<VT, ACC>, WAVE, lds, c.cus);
    hipLaunchKernelGGL((k_num_wh<VT, ACC>), dim3(grid), dim3(WAVE), lds, c.stream, a);
    return hipGetLastError();
}

}  // namespace

size_t lds_num_wh(int ts, int nw_max, int r_max, int acc_bytes) {
    return wh_layout(ts, (nw_max + 31) >> 5, r_max, ts / 2, acc_bytes).total;
}

template <>
hipError_t launch_num_wh<double>(const NumArgs<double> &a, int, const LaunchCfg &c) {
    return num_wh_impl<double, ACC_NATIVE>(a, c);
}
template <>
hipError_t launch_num_wh<float>(const NumArgs<float> &a, int acc, const LaunchCfg &c) {
    if (acc == ACC_COMP) return num_wh_impl<float, ACC_COMP>(a, c);
    if (acc == ACC_WIDE) return num_wh_impl<float, ACC_WIDE>(a, c);
    return num_wh_impl<float, ACC_NATIVE>(a, c);
}

}  // namespace spg
