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
constexpr int PL_CH = 4;  // consecutive rows per chunk of a wavefront's rows

// Staged A entry: one 16-byte LDS record, so a product reads its A value and
// its B row's length (which masks the lanes past the row) in one LDS read,
// and a gather its B row's offset and length in another.  Entries past the
// row have length 0.
struct StRec {
    double av;
    uint32_t x8;  // 8 * (B row start): byte offset into FP64 values (fast path: nnz(B) * 8 < 2^32)
    int32_t len;
};

// LDS of one wavefront.  Staging, values and sorted columns are double
// buffered: row p's results leave from one half while row p+1 is staged into
// the other.  Half b starts at half0 + b * hsize; offsets inside a half are
// the same for both.
struct PlLayout {
    size_t bp, map, half0, hsize, st_bs, st_rec, vals, colbuf, total;
};

__host__ __device__ inline PlLayout pl_layout(int nw_max, int r_max, int acc_bytes) {
    PlLayout L{};
    size_t o = 0;
    L.bp = o;  // per plan pair: bits | pre << 32
    o += 8 * (size_t)PL_CAP;
    L.half0 = o;
    size_t h = 0;
    L.st_bs = h;  // B row start per A entry (64-bit)
    h += 8 * WAVE;
    L.st_rec = h;  // per A entry: A value, byte offset of its B row's values (fast path), B row length
    h += sizeof(StRec) * WAVE;
    L.vals = h;
    h += align16((size_t)acc_bytes * r_max);
    L.colbuf = h;
    h += align16(4 * (size_t)r_max);
    L.hsize = h;
    o += 2 * h;
    L.map = o;  // window word -> pair index (uint8)
    o += align16((size_t)nw_max);
    L.total = o;
    return L;
}

struct RowDescP {
    int64_t ab, ae, cb, ce, po;
    int wlo, nw;  // nw: touched words (plan pairs)
};

// LGS: lanes per B row as a compile-time power of two (the launch's lg_gs),
// so the staging offsets of a lane's products are immediates; NU products per
// lane cover the fast path (NU * NG >= 64 or NU = PL_U), and every staged
// index g + u * NG stays below 64.
template <typename VT, int ACC, int LGS>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_num_pl(NumArgs<VT> a) {
    using A = Accum<VT, ACC>;
    using S = typename A::store_t;
    extern __shared__ __align__(16) unsigned char smem[];
    const PlLayout L = pl_layout(a.nw_max, a.r_max, sizeof(S));
    unsigned long long *bp = (unsigned long long *)(smem + L.bp);
    uint8_t *map = smem + L.map;
    const int l = lane_id();
    auto half = [&](int b) -> unsigned char * { return smem + L.half0 + (size_t)b * L.hsize; };
    for (int b = 0; b < 2; ++b)
        for (int t = l; t < a.r_max; t += WAVE) ((S *)(half(b) + L.vals))[t] = A::zero();
    constexpr int gs = 1 << LGS, ng = WAVE >> LGS;
    constexpr int NU = PL_U < WAVE / ng ? PL_U : WAVE / ng;
    const int g = l >> LGS, q = l & (gs - 1);
    int64_t lo, hi;
    rs_bounds(a.rs, lo, hi);
    const int64_t cbase = a.cbase_row >= 0 ? a.coff[a.cbase_row] : 0;
    // The wavefront takes its die's rows in chunks of PL_CH consecutive rows,
    // chunk after chunk at the stride of all the die's wavefronts: neighbouring
    // rows of C share most of their B rows (a stencil's rows i and i+1 share
    // two thirds), so a chunk finds them in the CU's L1 and the die's L2
    // (27-point A*A on 100^3: 44% less traffic beyond L2 than row by row).
    const Slice sl = xcd_slice(lo, hi, PL_CH, 0);

    // Software pipeline over the wavefront's rows p, p+s, p+2s, ... (p+s: the
    // next row of its sequence, pos(t + 1)): while row p is processed, row
    // p+s's B extents (second level) and row p+2s's A entries and plan pairs
    // (first level) load; lane k < 7 loads field k of
    // row p+3s's descriptor (moved to scalar registers a row later) and the
    // row index of p+4s loads a row before that.  Memory operations are
    // issued in the order gathers of row p, pipeline loads, stores of row
    // p-1: the vector-memory counter retires in order, so waiting for a load
    // never waits for the previous row's stores.
    auto load_desc = [&](int i) -> int64_t {
        // lanes 0-4: arp[i], arp[i+1], coff[i], coff[i+1], plan_off[i] (64-bit);
        // lane 5: the window's first word; lane 6: touched words (the row_words
        // array has a padding element).  Two dword loads in every lane, no branch.
        const uint32_t *src = (const uint32_t *)(a.arp + i + (l & 1));
        if (l >= 2 && l < 4) src = (const uint32_t *)(a.coff + i + (l - 2));
        if (l == 4) src = (const uint32_t *)(a.plan_off + i);
        if (l == 5) src = (const uint32_t *)(a.rwin + i);
        if (l == 6) src = (const uint32_t *)(a.row_words + i);
        const uint32_t vlo = src[0], vhi = src[1];
        return (int64_t)(((uint64_t)vhi << 32) | vlo);
    };
    auto lane64 = [](int64_t v, int k) -> int64_t {
        const uint32_t vlo = __builtin_amdgcn_readlane((uint32_t)v, k);
        const uint32_t vhi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)v >> 32), k);
        return (int64_t)(((uint64_t)vhi << 32) | vlo);
    };
    auto to_uni = [&](int64_t v) -> RowDescP {
        RowDescP d;
        d.ab = lane64(v, 0);
        d.ae = lane64(v, 1);
        d.cb = lane64(v, 2);
        d.ce = lane64(v, 3);
        d.po = lane64(v, 4);
        d.wlo = (int)__builtin_amdgcn_readlane((uint32_t)v, 5);
        d.nw = (int)__builtin_amdgcn_readlane((uint32_t)v, 6);
        return d;
    };
    // stage up to 64 A entries of a row into half b; returns the fast-path test
    auto stage = [&](int b, int cn, int64_t na, int64_t b0, int64_t b1, double av) -> bool {
        const int len = (int)(b1 - b0);
        unsigned char *hb = half(b);
        if (l < cn) ((int64_t *)(hb + L.st_bs))[l] = b0;
        ((StRec *)(hb + L.st_rec))[l] = StRec{av, (uint32_t)b0 * 8u, l < cn ? len : 0};
        return a.b32 && na <= WAVE && cn <= ng * NU && __ballot(l < cn && len > gs) == 0;
    };
    const int64_t step = sl.step;
    const int64_t p0 = sl.idx, pend = sl.end;
    auto pos = [&](int64_t t) -> int64_t { return p0 + (t / PL_CH) * step + (t % PL_CH); };  // t-th row
    auto row_at = [&](int64_t pp) -> int { return pp < pend ? read_first(a.rs.rows[pp]) : 0; };

    // ---- prologue: fill the pipeline (waits here are once per kernel).
    // Naming by distance from the current row p: *_m = row p+s, *_l = row
    // p+2s; rn, r2, r3 = raw descriptors of rows p+s, p+2s, p+3s.
    RowDescP d = p0 < pend ? to_uni(load_desc(row_at(p0))) : RowDescP{};      // row p
    int64_t rn = pos(1) < pend ? load_desc(row_at(pos(1))) : 0;
    int64_t r2 = pos(2) < pend ? load_desc(row_at(pos(2))) : 0;
    int64_t r3 = pos(3) < pend ? load_desc(row_at(pos(3))) : 0;
    int i4 = pos(4) < pend ? a.rs.rows[pos(4)] : 0;            // row index of p+4s
    bool fast_c = false;
    uint2 cpw = make_uint2(0u, 0u), npw_m = make_uint2(0u, 0u), npw_l = make_uint2(0u, 0u);
    int64_t nb0n = 0, nb1n = 0;  // row p+s: B extents per A entry
    double nav_m = 0.0, nav_l = 0.0;
    int nj_l = 0;                // row p+2s: A columns
    if (p0 < pend) {  // row p: staged into half 0; its plan pair in a register
        const int cn = (int)min((int64_t)WAVE, d.ae - d.ab);
        int64_t b0 = 0, b1 = 0;
        double av = 0.0;
        if (l < cn) {
            const int j = a.aci[d.ab + l];
            av = (double)a.aval[d.ab + l];
            b0 = a.brp[j];
            b1 = a.brp[j + 1];
        }
        fast_c = stage(0, cn, d.ae - d.ab, b0, b1, av);
        if (l < d.nw) cpw = a.plan[d.po + l];
    }
    if (pos(1) < pend) {
        const RowDescP d1 = to_uni(rn);
        if (l < min((int64_t)WAVE, d1.ae - d1.ab)) {
            const int j = a.aci[d1.ab + l];
            nav_m = (double)a.aval[d1.ab + l];
            nb0n = a.brp[j];
            nb1n = a.brp[j + 1];
        }
        if (l < d1.nw) npw_m = a.plan[d1.po + l];
    }
    if (pos(2) < pend) {
        const RowDescP d2 = to_uni(r2);
        if (l < min((int64_t)WAVE, d2.ae - d2.ab)) {
            nj_l = a.aci[d2.ab + l];
            nav_l = (double)a.aval[d2.ab + l];
        }
        if (l < d2.nw) npw_l = a.plan[d2.po + l];
    }
    // gathers of a staged row (fast path): every product's column and value,
    // issued a row ahead of the products that use them.  A lane past its B
    // row loads the entry its offset names, clamped to B's last entry; the
    // length test masks it when the products are added.
    int col[NU];
    VT pv[NU];
    const uint32_t q8 = 8u * (uint32_t)q, elast8 = 8u * (uint32_t)max(a.nnzb - 1, (int64_t)0);
    auto gather = [&](int hb_i) {
        const StRec *rec = (const StRec *)(half(hb_i) + L.st_rec);
        uint2 xl[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) xl[u] = *(const uint2 *)&rec[g + u * ng].x8;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const uint32_t e8 = min(xl[u].x + q8, elast8);
            col[u] = *(const int *)((const char *)a.bci + (e8 >> 1));
            pv[u] = *(const VT *)((const char *)a.bval + (sizeof(VT) == 8 ? e8 : e8 >> 1));
        }
    };
    wave_lds_sync();
    if (p0 < pend && fast_c) gather(0);

    // Per row p: plan decode and products of p, p's stores, pipeline loads
    // (p+2s B extents, p+3s A entries and plan pairs, p+4s descriptor, p+5s
    // index), then the staging and gathers of p+s, issued last.  The
    // vector-memory counter retires in order: when the products of p+s wait
    // for its gathers, every earlier load has landed too, so a loaded value
    // is only read (or copied) a row after its load, without a stall.
    int b = 0;  // half of the current row
    for (int64_t t = 0; pos(t) < pend; ++t, b ^= 1) {
        const bool has1 = pos(t + 1) < pend, has2 = pos(t + 2) < pend, has3 = pos(t + 3) < pend,
                   has4 = pos(t + 4) < pend;
        const int wlo = d.wlo;
        unsigned char *hb = half(b);
        int64_t *st_bs = (int64_t *)(hb + L.st_bs);
        StRec *rec = (StRec *)(hb + L.st_rec);
        S *vals = (S *)(hb + L.vals);
        int32_t *colbuf = (int32_t *)(hb + L.colbuf);
        const bool fast = fast_c;
        int cn = (int)min((int64_t)WAVE, d.ae - d.ab);
        const int64_t ob = d.cb - cbase;

        // ---- 1. decode the plan of row p: pre(word), word -> pair
        const uint2 mypw = cpw;
        const bool have = l < d.nw;
        const int pc = have ? __popc(mypw.y) : 0;
        const int inc = wave_scan_dpp(pc);
        const int pre = inc - pc;
        const int rnnz = __builtin_amdgcn_readlane(inc, WAVE - 1);
        if (have) {
            map[(int)mypw.x - wlo] = (uint8_t)l;
            bp[l] = (unsigned long long)mypw.y | ((unsigned long long)(uint32_t)pre << 32);
        }
        const bool ok = (d.ce - d.cb == rnnz) && rnnz <= a.r_max && d.nw <= PL_CAP;
        const int rlast = rnnz > 0 ? rnnz - 1 : 0;  // ranks past the row (bad input) stay inside it
        const uint8_t *mapw = map - wlo;              // indexed by absolute word (32-bit LDS addresses)
        if (l == 0 && !ok) atomicAdd(&a.st->mismatch, 1);
        wave_lds_sync();

        // ---- 2. products into vals[rank]
        if (ok) {
            if (fast) {
                int lenv[NU];  // every length first: one LDS wait, not one per product
#pragma unroll
                for (int u = 0; u < NU; ++u) lenv[u] = rec[g + u * ng].len;
#pragma unroll
                for (int u = 0; u < NU; ++u) {
                    if (q < lenv[u]) {
                        const int c = col[u];
                        const VT av = (VT)rec[g + u * ng].av;  // issued with the word-map read
                        const int s = mapw[c >> 5];
                        const unsigned long long e = bp[s];
                        const int rk = (int)(uint32_t)(e >> 32) + bits_below((uint32_t)e, c & 31);
                        A::add(&vals[min(rk, rlast)], av, pv[u]);
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
                            rec[l].len = (int)(b1 - b0);
                            rec[l].av = (double)a.aval[c0 + l];
                        }
                        wave_lds_sync();
                    }
                    for (int t = g; t < cn; t += ng) {
                        const int64_t bs = st_bs[t];
                        const int len = rec[t].len;
                        const VT av = (VT)rec[t].av;
                        for (int p = q; p < len; p += gs) {
                            const int c = a.bci[bs + p];
                            const int s = map[(c >> 5) - wlo];
                            const unsigned long long e = bp[s];
                            const int rk =
                                (int)(uint32_t)(e >> 32) + bits_below((uint32_t)e, c & 31);
                            A::add(&vals[min(rk, rlast)], av, a.bval[bs + p]);
                        }
                    }
                }
            }
        }
        // ---- 3. sorted columns of row p from its pairs, then p's stores
        if (ok && have && !a.values_only) {
            uint32_t m = mypw.y;
            int p = pre;
            const int base = (int)(mypw.x << 5);
            while (m) {
                colbuf[p++] = base + __ffs(m) - 1;
                m &= m - 1;
            }
        }
        // ---- 4. pipeline: values loaded a row ago move on; the addresses of
        //      the new loads are formed before p's stores, so reading those
        //      values never waits for the stores
        const RowDescP dn = has1 ? to_uni(rn) : RowDescP{};  // row p+s
        const int64_t nan1 = dn.ae - dn.ab;
        const int64_t nan2 = has2 ? lane64(r2, 1) - lane64(r2, 0) : 0;
        const int64_t nb0 = nb0n, nb1 = nb1n;
        const double nav1 = nav_m;
        const uint2 cpw_next = npw_m;
        nav_m = nav_l;
        npw_m = npw_l;
        const bool ld_ext = has2 && l < min((int64_t)WAVE, nan2);
        const int64_t *ext_p = a.brp + nj_l;                 // row p+2s: B extents
        int64_t f3ab = 0, f3na = 0, f3po = 0;
        int f3nw = 0;
        if (has3) {
            f3ab = lane64(r3, 0);
            f3na = lane64(r3, 1) - f3ab;
            f3po = lane64(r3, 4);
            f3nw = (int)__builtin_amdgcn_readlane((uint32_t)r3, 6);
        }
        const bool ld_a = has3 && l < min((int64_t)WAVE, f3na), ld_pw = has3 && l < f3nw;
        const int i4s = read_first(i4);                      // row p+4s
        wave_lds_sync();
        if (ok) {  // row p's stores
            for (int t = l; t < rnnz; t += WAVE) {
                if (!a.values_only) a.cci[ob + t] = colbuf[t];
                a.cval[ob + t] = A::fin(vals[t]);
                vals[t] = A::zero();
            }
        }
        nb0n = ld_ext ? ext_p[0] : 0;
        nb1n = ld_ext ? ext_p[1] : 0;
        if (ld_a) {
            nj_l = a.aci[f3ab + l];
            nav_l = (double)a.aval[f3ab + l];
        }
        if (ld_pw) npw_l = a.plan[f3po + l];
        rn = r2;
        r2 = r3;
        r3 = has4 ? load_desc(i4s) : 0;                                 // row p+4s
        i4 = pos(t + 5) < pend ? a.rs.rows[pos(t + 5)] : 0;      // row p+5s
        // ---- 5. row p+s: staged, then its gathers (the last memory
        //      operations before its products)
        if (has1) {
            fast_c = stage(b ^ 1, (int)min((int64_t)WAVE, nan1), nan1, nb0, nb1, nav1);
            d = dn;
            cpw = cpw_next;
        }
        wave_lds_sync();
        // (issued even when there is no next fast row: a fixed count of loads
        // after the pipeline loads lets their wait at the loop's end skip the
        // gathers; the offsets are clamped into B whatever the records hold)
        gather(b ^ 1);
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

template <typename VT, int ACC, int LGS>
hipError_t num_pl_lg(const NumArgs<VT> &a, const LaunchCfg &c) {
    const size_t lds = lds_num_pl(a.nw_max, a.r_max, sizeof(typename Accum<VT, ACC>::store_t));
    const int grid = c.grid > 0 ? c.grid : resident_grid(k_num_pl<VT, ACC, LGS>, WAVE, lds, c.cus);
    hipLaunchKernelGGL((k_num_pl<VT, ACC, LGS>), dim3(grid), dim3(WAVE), lds, c.stream, a);
    return hipGetLastError();
}

template <typename VT, int ACC>
hipError_t num_pl_impl(const NumArgs<VT> &a, const LaunchCfg &c) {
    switch (a.lg_gs) {
    case 0: return num_pl_lg<VT, ACC, 0>(a, c);
    case 1: return num_pl_lg<VT, ACC, 1>(a, c);
    case 2: return num_pl_lg<VT, ACC, 2>(a, c);
    case 3: return num_pl_lg<VT, ACC, 3>(a, c);
    case 4: return num_pl_lg<VT, ACC, 4>(a, c);
    case 5: return num_pl_lg<VT, ACC, 5>(a, c);
    case 6: return num_pl_lg<VT, ACC, 6>(a, c);
    default: return hipErrorInvalidValue;
    }
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
