// Numeric phase on the symbolic phase's row structure, one wavefront per row.
//
// The bit-window symbolic kernel ends each row with the row's pattern as the
// union of column-set words (Compression subsection): word index + 32-bit
// mask per touched word, in increasing word order.  For rows whose touched
// words fit the per-row plan (at most 64), it stores these (word, bits)
// pairs.  The numeric phase (Algorithm 3, numeric branch) then needs no
// structure pass: per row it loads the pairs, a wavefront scan of their
// popcounts gives pre(word), a direct LDS map window-word -> pair index
// replaces the hash lookup, and each product (i, k, j) lands at
//     rank(j) = pre(word(j)) + popcount(bits(word(j)) below j)
// in the row's sorted value array (Algorithm 1's accumulation, sorted output).
//
// Work split as in the other wavefront kernels: Thread-Parallel lane groups
// of 2^lg_gs lanes per B row; a fast path keeps up to PL_U products per lane
// in registers (loads issued before the plan is decoded, so their latency
// overlaps it); rows that do not fit walk A's row in chunks.  Rows are
// software-pipelined: the next row's A entries, B extents and plan pairs load
// while the current row is processed.
#include "spg_accum.hpp"
#include "spg_internal.hpp"

namespace spg {

namespace {

constexpr int PL_U = 16;  // products per lane held in registers (fast path)

struct PlLayout {
    size_t map, bp, vals, colbuf, st_bs, st_a, st_len, total;
};

__host__ __device__ inline PlLayout pl_layout(int nw_max, int r_max, int acc_bytes) {
    PlLayout L{};
    size_t o = 0;
    L.bp = o;  // per plan pair: bits | pre << 32
    o += 8 * (size_t)PL_CAP;
    L.st_bs = o;
    o += 8 * WAVE;
    L.st_a = o;
    o += 8 * WAVE;
    L.vals = o;
    o += align16((size_t)acc_bytes * r_max);
    L.colbuf = o;
    o += align16(4 * (size_t)r_max);
    L.st_len = o;
    o += 4 * WAVE;
    L.map = o;  // window word -> pair index (uint8)
    o += align16((size_t)nw_max);
    L.total = o;
    return L;
}

struct RowDescP {
    int64_t ab, ae, cb, ce, po;
    int wlo, nw;  // nw: touched words (plan pairs)
};

template <typename VT, int ACC>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_num_pl(NumArgs<VT> a) {
    using A = Accum<VT, ACC>;
    using S = typename A::store_t;
    extern __shared__ __align__(16) unsigned char smem[];
    const PlLayout L = pl_layout(a.nw_max, a.r_max, sizeof(S));
    unsigned long long *bp = (unsigned long long *)(smem + L.bp);
    uint8_t *map = smem + L.map;
    S *vals = (S *)(smem + L.vals);
    int32_t *colbuf = (int32_t *)(smem + L.colbuf);
    int64_t *st_bs = (int64_t *)(smem + L.st_bs);
    double *st_a = (double *)(smem + L.st_a);
    int32_t *st_len = (int32_t *)(smem + L.st_len);
    const int l = lane_id();
    for (int t = l; t < a.r_max; t += WAVE) vals[t] = A::zero();
    wave_lds_sync();
    const int gs = 1 << a.lg_gs, g = l >> a.lg_gs, q = l & (gs - 1), ng = WAVE >> a.lg_gs;
    int64_t lo, hi;
    rs_bounds(a.rs, lo, hi);
    const int64_t cbase = a.cbase_row >= 0 ? a.coff[a.cbase_row] : 0;
    const Slice sl = xcd_slice(lo, hi);

    // row descriptor: wavefront-uniform, kept in scalar registers
    auto desc = [&](int64_t rr) -> RowDescP {
        const int i = read_first(a.rs.rows[rr]);
        RowDescP d;
        d.ab = uni64(a.arp[i]);
        d.ae = uni64(a.arp[i + 1]);
        d.cb = uni64(a.coff[i]);
        d.ce = uni64(a.coff[i + 1]);
        d.po = uni64(a.plan_off[i]);
        d.wlo = read_first(a.rwin[i].x);
        d.nw = read_first(a.row_words[i]);
        return d;
    };

    int64_t r = sl.idx;
    RowDescP dcur = r < sl.end ? desc(r) : RowDescP{};
    int64_t sb0 = 0, sb1 = 0;
    double sav = 0.0;
    uint2 pw = make_uint2(0u, 0u);
    if (r < sl.end) {
        if (l < min((int64_t)WAVE, dcur.ae - dcur.ab)) {
            const int j = a.aci[dcur.ab + l];
            sav = (double)a.aval[dcur.ab + l];
            sb0 = a.brp[j];
            sb1 = a.brp[j + 1];
        }
        if (l < dcur.nw) pw = a.plan[dcur.po + l];
    }
    RowDescP dn = r + sl.step < sl.end ? desc(r + sl.step) : RowDescP{};
    while (r < sl.end) {
        const RowDescP d = dcur;
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
        const bool fast = a.b32 && na <= WAVE && cn <= ng * PL_U && wave_max(mylen) <= gs;
        wave_lds_sync();

        // ---- fast path: every product's column and value load now
        int col[PL_U];
        VT pv[PL_U];
        unsigned okm = 0;
        if (fast) {
#pragma unroll
            for (int u = 0; u < PL_U; ++u) {
                const int t = g + u * ng;
                const int tt = t < cn ? t : 0;
                const bool ok = t < cn && q < st_len[tt];
                okm |= (unsigned)ok << u;
                const uint32_t e = ok ? (uint32_t)st_bs[tt] + q : 0u;  // nnz(B) * 8 < 2^32 on this path
                col[u] = ld32(a.bci, e);
                pv[u] = ld32(a.bval, e);
            }
        }
        // ---- decode the plan while they are in flight: pre(word), word -> pair
        const bool have = l < d.nw;
        const int pc = have ? __popc(pw.y) : 0;
        const int inc = wave_incl_scan(pc);
        const int pre = inc - pc;
        const int rnnz = __shfl(inc, WAVE - 1);
        const uint2 mypw = pw;
        if (have) {
            map[(int)mypw.x - wlo] = (uint8_t)l;
            bp[l] = (unsigned long long)mypw.y | ((unsigned long long)(uint32_t)pre << 32);
        }
        const bool ok = (d.ce - d.cb == rnnz) && rnnz <= a.r_max && d.nw <= PL_CAP;
        if (l == 0 && !ok) atomicAdd(&a.st->mismatch, 1);
        // next row, first level: its A entries and plan pairs
        const int ncn = has_next ? (int)min((int64_t)WAVE, dn.ae - dn.ab) : 0;
        int nj = 0;
        if (l < ncn) {
            nj = a.aci[dn.ab + l];
            sav = (double)a.aval[dn.ab + l];
        }
        pw = make_uint2(0u, 0u);
        if (has_next && l < dn.nw) pw = a.plan[dn.po + l];
        wave_lds_sync();

        // ---- products into vals[rank]
        if (ok) {
            if (fast) {
#pragma unroll
                for (int u = 0; u < PL_U; ++u) {
                    if (okm & (1u << u)) {
                        const int c = col[u];
                        const int s = map[(c >> 5) - wlo];
                        const unsigned long long e = bp[s];
                        const int rk = (int)(uint32_t)(e >> 32) + __popc((uint32_t)e & ((1u << (c & 31)) - 1u));
                        A::add(&vals[rk < rnnz ? rk : 0], (VT)st_a[g + u * ng], pv[u]);
                    }
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
                            st_a[l] = (double)a.aval[c0 + l];
                        }
                        wave_lds_sync();
                    }
                    for (int t = g; t < cn; t += ng) {
                        const int64_t bs = st_bs[t];
                        const int len = st_len[t];
                        const VT av = (VT)st_a[t];
                        for (int p = q; p < len; p += gs) {
                            const int c = a.bci[bs + p];
                            const int s = map[(c >> 5) - wlo];
                            const unsigned long long e = bp[s];
                            const int rk =
                                (int)(uint32_t)(e >> 32) + __popc((uint32_t)e & ((1u << (c & 31)) - 1u));
                            A::add(&vals[rk < rnnz ? rk : 0], av, a.bval[bs + p]);
                        }
                    }
                }
            }
        }
        // sorted columns of the row from its pairs
        if (ok && have) {
            uint32_t m = mypw.y;
            int p = pre;
            const int base = (int)(mypw.x << 5);
            while (m) {
                colbuf[p++] = base + __ffs(m) - 1;
                m &= m - 1;
            }
        }
        // next row, second level: B extents; the row after next: descriptor
        if (l < ncn) {
            sb0 = a.brp[nj];
            sb1 = a.brp[nj + 1];
        }
        dcur = dn;
        if (r + sl.step < sl.end) dn = desc(r + sl.step);
        wave_lds_sync();
        if (ok) {
            const int64_t ob = d.cb - cbase;
            for (int t = l; t < rnnz; t += WAVE) {
                a.cci[ob + t] = colbuf[t];
                a.cval[ob + t] = A::fin(vals[t]);
                vals[t] = A::zero();
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
hipError_t num_pl_impl(const NumArgs<VT> &a, const LaunchCfg &c) {
    const size_t lds = lds_num_pl(a.nw_max, a.r_max, sizeof(typename Accum<VT, ACC>::store_t));
    const int grid = c.grid > 0 ? c.grid : resident_grid(k_num_pl<VT, ACC>, WAVE, lds, c.cus);
    hipLaunchKernelGGL((k_num_pl<VT, ACC>), dim3(grid), dim3(WAVE), lds, c.stream, a);
    return hipGetLastError();
}

}  // namespace

size_t lds_num_pl(int nw_max, int r_max, int acc_bytes) { return pl_layout(nw_max, r_max, acc_bytes).total; }

template <>
hipError_t launch_num_pl<double>(const NumArgs<double> &a, int, const LaunchCfg &c) {
    return num_pl_impl<double, ACC_NATIVE>(a, c);
}
template <>
hipError_t launch_num_pl<float>(const NumArgs<float> &a, int acc, const LaunchCfg &c) {
    if (acc == ACC_COMP) return num_pl_impl<float, ACC_COMP>(a, c);
    if (acc == ACC_WIDE) return num_pl_impl<float, ACC_WIDE>(a, c);
    return num_pl_impl<float, ACC_NATIVE>(a, c);
}

}  // namespace spg
