// Heavy rows in column segments: the dense accumulator of the Accumulators
// subsection, cut to the size of LDS.
//
// A heavy row of C (thousands to a million entries spread over up to 2^20
// columns) does not fit in LDS as a whole.  The symbolic phase, which holds
// the row's complete bit window, cuts it into segments: runs of consecutive
// column-set words with at most SG_CAP entries that stay inside one aligned
// group of SG_NW words.  The numeric phase then walks the segments in column
// order, one 512-lane workgroup per row (a launch may hold two row sets, the
// second taken first and accumulated with its own accumulator):
//
//   1. the part of each B row that falls in the segment (B's columns are
//      sorted, so it is one run; each A entry keeps a cursor into its B row
//      from segment to segment, in a register for rows of one chunk of A
//      entries, in HBM scratch for longer rows, else binary search); the
//      nonempty runs are staged back to back,
//   2. structure: the run's columns OR-ed into an LDS bit array over the
//      segment's words, Thread-Flat-Parallel over the segment's products
//      (neighbouring lanes on neighbouring products, so a run's loads
//      coalesce; each wavefront finds the run of every product of its
//      window from run starts marked in LDS and a forward fill),
//   3. ranks: prefix popcounts of the words give every column its place in
//      the row,
//   4. values: each product added at its rank in LDS (Algorithm 1's
//      accumulation), Thread-Flat-Parallel again,
//   5. write-out: values in rank order, then columns expanded from the bits
//      into LDS and stored in rank order (both coalesced), at the segment's
//      offset in the row, which the symbolic phase recorded.
//
// Nothing lives in HBM but the inputs and C; a row with one segment (its
// entries and window fit) runs the same steps once, with whole B rows.
#include "spg_accum.hpp"
#include "spg_internal.hpp"

namespace spg {
namespace {

constexpr int SG_U = 8;  // products per lane per round of the flat walks (loads in flight)
// The staging scan adds (run length) + (1 << SG_SHIFT if the run is nonempty):
// products below the shift, the nonempty run's slot above it.
constexpr int SG_SHIFT = 48;
constexpr long long SG_ONE = 1ll << SG_SHIFT, SG_LEN = SG_ONE - 1;
// Lanes per workgroup (one heavy row).  LDS (~76 KB) allows two workgroups
// per CU; 512 lanes rather than 256 double the loads in flight per CU for the
// same LDS, with registers held to 128 (4 waves per SIMD).
constexpr int SG_WG = 512;

__device__ __forceinline__ long long sg_block_excl_scan(long long v, long long *red, long long *total) {
    const int t = threadIdx.x, l = lane_id(), wv = t / WAVE;
    const long long inc = wave_incl_scan64(v);
    __syncthreads();
    if (l == WAVE - 1) red[wv] = inc;
    __syncthreads();
    long long off = 0, tot = 0;
#pragma unroll
    for (int u = 0; u < SG_WG / WAVE; ++u) {
        const long long x = red[u];
        if (u < wv) off += x;
        tot += x;
    }
    *total = tot;
    return off + inc - v;
}

__device__ __forceinline__ int sg_next_row(const RowSet &rs, int64_t lo, int64_t hi, int &x, long long *red) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t t = xcd_grab(rs.queue, lo, hi, x);
        red[SG_WG / WAVE] = t < 0 ? -1 : rs.rows[t];
        red[SG_WG / WAVE + 1] = x;
    }
    __syncthreads();
    x = (int)red[SG_WG / WAVE + 1];
    return (int)red[SG_WG / WAVE];
}

// First index in [lo, hi) whose column is >= key (hi when none); the row's
// columns are sorted.  The two ends are tested first: runs that start at the
// row's start or end at its end need no search.
__device__ __forceinline__ int64_t sg_lower_bound(const int32_t *bci, int64_t lo, int64_t hi, int64_t key) {
    if (lo >= hi || (int64_t)bci[lo] >= key) return lo;
    if ((int64_t)bci[hi - 1] < key) return hi;
    ++lo;  // bci[lo] < key
    --hi;  // bci[hi] >= key
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)bci[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// First index in [lo, hi) whose column is >= key, searched from lo (the run
// is usually short): the row's end first, then probes at lo + 1, 3, 7, ...
// and a binary search in the last gap.
__device__ __forceinline__ int64_t sg_gallop(const int32_t *bci, int64_t lo, int64_t hi, int64_t key) {
    if (lo >= hi) return lo;
    const int32_t first = bci[lo], last = bci[hi - 1];
    if ((int64_t)first >= key) return lo;
    if ((int64_t)last < key) return hi;
    int64_t below = lo, step = 1;  // bci[below] < key, bci[hi - 1] >= key
    while (below + step < hi - 1 && (int64_t)bci[below + step] < key) {
        below += step;
        step <<= 1;
    }
    int64_t a = below + 1, b = min(below + step, hi - 1);  // answer in [a, b]
    while (a < b) {
        const int64_t mid = a + ((b - a) >> 1);
        if ((int64_t)bci[mid] < key) a = mid + 1;
        else b = mid;
    }
    return a;
}

// Index k of the run that holds flat product f: the first k >= kc with
// st_off[k] > f (run ends, increasing: only nonempty runs are staged).  The
// wavefront's window starts increase, so its previous run kc is a lower bound
// and often the answer; otherwise a binary search over the rest.
__device__ __forceinline__ int sg_find(const int64_t *st_off, int cn, long long f, int kc) {
    if (st_off[kc] > f) return kc;
    int lo = kc + 1, hi = cn - 1;  // st_off[cn - 1] > f for every product f of the chunk
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (st_off[mid] > f) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// ACC accumulates the rows of a.rs, ACC2 those of a.rs2 (FP32 values: the
// heaviest rows in FP64); the value array holds either kind of entry.
template <typename VT, int ACC, int ACC2>
__global__ __launch_bounds__(SG_WG) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_num_sg(NumArgs<VT> a) {
    using A = Accum<VT, ACC>;
    using S = typename A::store_t;
    using A2 = Accum<VT, ACC2>;
    using S2 = typename A2::store_t;
    constexpr int VB = sizeof(S) > sizeof(S2) ? sizeof(S) : sizeof(S2);
    __shared__ __align__(16) uint32_t bits[SG_NW];
    __shared__ uint16_t pre[SG_NW];
    __shared__ __align__(16) unsigned char vals_raw[SG_CAP * VB];
    S *vals = (S *)vals_raw;
    S2 *vals2 = (S2 *)vals_raw;
    __shared__ int64_t st_lo[SG_WG];   // run start (B entry) per A entry of the chunk
    __shared__ int64_t st_off[SG_WG];  // inclusive prefix of the run lengths
    __shared__ VT st_a[SG_WG];
    __shared__ long long red[SG_WG / WAVE + 2];
    // per wavefront: the run of each product of its window (relative to the
    // window's first run), so that neighbouring lanes take neighbouring products
    __shared__ __align__(16) uint16_t widx[SG_WG / WAVE][SG_U * WAVE];
    const int t = threadIdx.x;
    for (int w = t; w < SG_NW; w += SG_WG) bits[w] = 0;
    for (int r = t; r < SG_CAP * VB / 4; r += SG_WG) ((uint32_t *)vals_raw)[r] = 0u;  // every kind of zero
    int64_t qlo, qhi;
    rs_bounds(a.rs, qlo, qhi);
    const int64_t cbase = a.cbase_row >= 0 ? a.coff[a.cbase_row] : 0;
    int x = blockIdx.x % XCDS;
    // a second row set (the heaviest rows) is drained first, then the first set
    bool second = a.rs2.rows != nullptr;
    int64_t qlo2 = 0, qhi2 = 0;
    if (second) rs_bounds(a.rs2, qlo2, qhi2);
    int x2 = x;
    for (;;) {
        int i;
        if (second) {
            i = sg_next_row(a.rs2, qlo2, qhi2, x2, red);
            if (i < 0) {
                second = false;
                continue;
            }
        } else {
            i = sg_next_row(a.rs, qlo, qhi, x, red);
            if (i < 0) break;
        }
        const bool acc2 = ACC2 != ACC && second;  // this row accumulates with ACC2
        const int2 win = a.rwin[i];
        const int wlo = win.x, nw = win.y - win.x + 1;
        const int64_t c0 = a.coff[i], nnz = a.coff[i + 1] - c0;
        const int64_t ab = a.arp[i], ae = a.arp[i + 1];
        const bool has_list = a.plan_len != nullptr && a.sym_kind[i] == K_DG && a.plan_len[i] > 0;
        const uint2 *list = has_list ? a.plan + a.plan_off[i] : nullptr;
        const int nseg = has_list ? (int)list[0].x : 1;
        const bool single = nseg == 1;
        const bool one_chunk = ae - ab <= SG_WG;
        // several chunks: per A entry, in this workgroup's scratch, the B
        // entry where its run in the segment starts (cursor), where that run
        // ends, and the end of its B row (absolute positions: nnz(B) < 2^31),
        // so that a chunk's staging loads no A column and no B row extent
        int32_t *cur_g = nullptr, *nxt_g = nullptr, *end_g = nullptr;
        if (!one_chunk && !single && a.sg_cur != nullptr && ae - ab <= a.sg_cap) {
            cur_g = a.sg_cur + (int64_t)blockIdx.x * 3 * a.sg_cap;
            nxt_g = cur_g + a.sg_cap;
            end_g = nxt_g + a.sg_cap;
            for (int64_t k = t; k < ae - ab; k += SG_WG) {
                const int j = a.aci[ab + k];
                cur_g[k] = (int32_t)a.brp[j];
                end_g[k] = (int32_t)a.brp[j + 1];
            }
            __syncthreads();
        }
        // one chunk: lane t keeps A entry t for the whole row, with a cursor
        // into its B row that moves from segment to segment
        int64_t cur = 0, bend = 0;
        int cn1 = 0;
        VT av1 = VT(0);
        if (one_chunk) {
            cn1 = (int)(ae - ab);
            if (t < cn1) {
                const int j = a.aci[ab + t];
                cur = a.brp[j];
                bend = a.brp[j + 1];
                av1 = a.aval[ab + t];
            }
        }
        int bad = 0;
        for (int sg = 0; sg < nseg; ++sg) {
            int w1 = 0, w2 = nw;
            int64_t p1 = 0, p2 = nnz;
            if (has_list) {
                const uint2 d1 = list[1 + sg], d2 = list[2 + sg];
                w1 = (int)d1.x;
                p1 = d1.y;
                w2 = (int)d2.x;
                p2 = d2.y;
            }
            const int cnt = (int)(p2 - p1);
            const int64_t col_lo = (int64_t)(wlo + w1) << 5, col_hi = (int64_t)(wlo + w2) << 5;
            const int span = min(w2 - w1, SG_NW);
            const int dbase = wlo + w1;  // column-set word of bits[0]
            long long tot1 = 0;
            int nz1 = 0;
            if (one_chunk) {
                long long len = 0;
                int64_t s0 = cur;
                if (t < cn1) {
                    const int64_t e = single ? bend : sg_gallop(a.bci, cur, bend, col_hi);
                    len = e - cur;
                    cur = e;
                }
                long long pt;
                const long long ex = sg_block_excl_scan(len + (len > 0 ? SG_ONE : 0), red, &pt);
                tot1 = pt & SG_LEN;
                nz1 = (int)(pt >> SG_SHIFT);
                if (len > 0) {
                    const int k = (int)(ex >> SG_SHIFT);
                    st_lo[k] = s0;
                    st_off[k] = (ex & SG_LEN) + len;
                    st_a[k] = av1;
                }
                __syncthreads();
            }
            // pass 1 (structure) and pass 2 (values) walk the same runs
            for (int pass = 0; pass < 2; ++pass) {
                for (int64_t cb = ab; cb < ae; cb += SG_WG) {
                    int cn = nz1;
                    long long tot = tot1;
                    if (!one_chunk) {
                        const int cnc = (int)min((int64_t)SG_WG, ae - cb);
                        long long len = 0;
                        int64_t lo_t = 0;
                        VT av_t = VT(0);
                        if (t < cnc) {
                            const int64_t k = cb - ab + t;
                            int64_t s0, s1;
                            if (cur_g) {
                                s0 = cur_g[k];
                                if (pass == 0) {
                                    s1 = sg_gallop(a.bci, s0, (int64_t)end_g[k], col_hi);
                                    nxt_g[k] = (int32_t)s1;
                                } else {
                                    s1 = nxt_g[k];
                                    cur_g[k] = (int32_t)s1;  // the next segment starts where this run ends
                                }
                            } else {
                                const int j = a.aci[cb + t];
                                s0 = a.brp[j];
                                s1 = a.brp[j + 1];
                                if (!single) {
                                    s0 = sg_lower_bound(a.bci, s0, s1, col_lo);
                                    s1 = sg_lower_bound(a.bci, s0, s1, col_hi);
                                }
                            }
                            lo_t = s0;
                            av_t = a.aval[cb + t];
                            len = s1 - s0;
                        }
                        long long pt;
                        const long long ex = sg_block_excl_scan(len + (len > 0 ? SG_ONE : 0), red, &pt);
                        tot = pt & SG_LEN;
                        cn = (int)(pt >> SG_SHIFT);
                        if (len > 0) {
                            const int k = (int)(ex >> SG_SHIFT);
                            st_lo[k] = lo_t;
                            st_off[k] = (ex & SG_LEN) + len;
                            st_a[k] = av_t;
                        }
                        __syncthreads();
                    }
                    // Flat walk: per round, wavefront wv takes the SG_U * 64
                    // products from F = f0 + wv * SG_U * 64 on, lane l the
                    // products F + l + 64 u (neighbouring lanes, neighbouring
                    // B entries).  The run of each product comes from a
                    // per-wavefront index: run starts marked in LDS, then a
                    // forward fill (max-scan) over the window.
                    const int wv = t / WAVE, l = t % WAVE;
                    uint16_t *wi = widx[wv];
                    int kc = 0;  // the run of the wavefront's previous window start
                    for (long long f0 = 0; f0 < tot; f0 += (long long)SG_WG * SG_U) {
                        int64_t e[SG_U];
                        bool ok[SG_U];
                        const long long F = f0 + (long long)wv * (SG_U * WAVE);
                        int klo = 0;
                        if (F < tot) {  // the same for the whole wavefront
                            klo = sg_find(st_off, cn, F, kc);
                            kc = klo;
                            *(uint4 *)&wi[l * SG_U] = make_uint4(0u, 0u, 0u, 0u);
                            wave_lds_sync();
                            const long long Fe = min(F + (long long)(SG_U * WAVE), tot);
                            for (int k = klo + 1 + l; k < cn; k += WAVE) {
                                const long long st = st_off[k - 1];  // run k's first product
                                if (st >= Fe) break;                  // starts increase with k
                                wi[st - F] = (uint16_t)(k - klo);
                            }
                            wave_lds_sync();
                            const uint4 q4 = *(const uint4 *)&wi[l * SG_U];
                            uint32_t w4[4] = {q4.x, q4.y, q4.z, q4.w};
                            int m[SG_U];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                m[2 * u] = (int)(w4[u] & 0xFFFFu);
                                m[2 * u + 1] = (int)(w4[u] >> 16);
                            }
#pragma unroll
                            for (int u = 1; u < SG_U; ++u) m[u] = max(m[u], m[u - 1]);
                            int incl = m[SG_U - 1];  // inclusive max-scan of the lanes' maxima
                            incl = max(incl, __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xF, 0xF, false));
                            incl = max(incl, __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xF, 0xF, false));
                            incl = max(incl, __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xF, 0xF, false));
                            incl = max(incl, __builtin_amdgcn_update_dpp(0, incl, 0x118, 0xF, 0xF, false));
                            incl = max(incl, __builtin_amdgcn_update_dpp(0, incl, 0x142, 0xA, 0xF, false));
                            incl = max(incl, __builtin_amdgcn_update_dpp(0, incl, 0x143, 0xC, 0xF, false));
                            const int before = __shfl_up(incl, 1);
                            const int pm = l ? before : 0;
#pragma unroll
                            for (int u = 0; u < 4; ++u)
                                w4[u] = (uint32_t)max(m[2 * u], pm) | ((uint32_t)max(m[2 * u + 1], pm) << 16);
                            *(uint4 *)&wi[l * SG_U] = make_uint4(w4[0], w4[1], w4[2], w4[3]);
                            wave_lds_sync();
#pragma unroll
                            for (int u = 0; u < SG_U; ++u) {
                                const long long f = F + l + u * WAVE;
                                ok[u] = f < tot;
                                const int k = klo + (int)wi[l + u * WAVE];
                                e[u] = st_lo[k] + (f - (k ? st_off[k - 1] : 0));
                            }
                        } else {
#pragma unroll
                            for (int u = 0; u < SG_U; ++u) {
                                ok[u] = false;
                                e[u] = 0;
                            }
                        }
                        int c[SG_U];
#pragma unroll
                        for (int u = 0; u < SG_U; ++u) c[u] = ok[u] ? a.bci[e[u]] : 0;
                        if (pass == 0) {
#pragma unroll
                            for (int u = 0; u < SG_U; ++u) {
                                const int d = (c[u] >> 5) - dbase;
                                if (ok[u] && (unsigned)d < (unsigned)SG_NW) atomicOr(&bits[d], 1u << (c[u] & 31));
                            }
                        } else {
                            VT v[SG_U];
#pragma unroll
                            for (int u = 0; u < SG_U; ++u) v[u] = ok[u] ? a.bval[e[u]] : VT(0);
#pragma unroll
                            for (int u = 0; u < SG_U; ++u) {
                                const int d = (c[u] >> 5) - dbase;
                                if (!ok[u] || (unsigned)d >= (unsigned)SG_NW) continue;
                                const int r = (int)pre[d] + bits_below(bits[d], c[u] & 31);
                                if (r < SG_CAP) {
                                    if (acc2) A2::add(&vals2[r], st_a[klo + (int)wi[l + u * WAVE]], v[u]);
                                    else A::add(&vals[r], st_a[klo + (int)wi[l + u * WAVE]], v[u]);
                                }
                            }
                        }
                    }
                    if (!one_chunk) __syncthreads();  // st_* are refilled for the next chunk
                }
                __syncthreads();
                if (pass == 0) {
                    // ranks: lane t scans words [t*SG_NW/SG_WG, ...) of the segment
                    constexpr int WPL = SG_NW / SG_WG;
                    const int wb = t * WPL;
                    uint32_t wv[WPL];
                    int sum = 0;
#pragma unroll
                    for (int u = 0; u < WPL; u += 4) {
                        const uint4 q = *(const uint4 *)&bits[wb + u];
                        wv[u] = q.x;
                        wv[u + 1] = q.y;
                        wv[u + 2] = q.z;
                        wv[u + 3] = q.w;
                    }
#pragma unroll
                    for (int u = 0; u < WPL; ++u) sum += __popc(wv[u]);
                    long long tot;
                    int run = (int)sg_block_excl_scan(sum, red, &tot);
#pragma unroll
                    for (int u = 0; u < WPL; ++u) {
                        pre[wb + u] = (uint16_t)min(run, 65535);
                        run += __popc(wv[u]);
                    }
                    if (tot != cnt) bad = 1;
                    __syncthreads();
                }
            }
            // write-out at the segment's offset, both arrays in rank order with
            // coalesced stores: first the values; then the columns, expanded
            // from the bits (one word per lane) into the freed value array;
            // the bits and values are cleared for the next segment
            const int64_t o = c0 + p1 - cbase;
            const int cw = min(cnt, SG_CAP);
            for (int r = t; r < cw; r += SG_WG) a.cval[o + r] = acc2 ? A2::fin(vals2[r]) : A::fin(vals[r]);
            __syncthreads();
            int32_t *colbuf = (int32_t *)vals_raw;  // SG_CAP * VB >= 4 * SG_CAP bytes
            for (int w = t; w < span; w += SG_WG) {
                uint32_t m = bits[w];
                int r = pre[w];
                const int colb = (dbase + w) << 5;
                while (m) {
                    const int b = __ffs(m) - 1;
                    m &= m - 1;
                    if (r < cw) colbuf[r] = colb + b;
                    ++r;
                }
                bits[w] = 0;
            }
            __syncthreads();
            for (int r = t; r < cw; r += SG_WG) a.cci[o + r] = colbuf[r];
            __syncthreads();
            for (int r = t; r < cw; r += SG_WG) {  // all-zero bytes either way
                if (acc2) vals2[r] = A2::zero();
                else vals[r] = A::zero();
            }
            __syncthreads();
        }
        if (t == 0 && bad) atomicAdd(&a.st->mismatch, 1);
    }
}

template <typename VT, int ACC, int ACC2>
hipError_t num_sg_impl(const NumArgs<VT> &a, const LaunchCfg &c) {
    int grid = c.grid;
    if (grid <= 0) grid = sg_resident_grid(ACC, ACC2, sizeof(VT) == 8, c.cus);
    hipLaunchKernelGGL((k_num_sg<VT, ACC, ACC2>), dim3(grid), dim3(SG_WG), 0, c.stream, a);
    return hipGetLastError();
}

template <typename K>
int resident(K kernel, int cus) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, SG_WG, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int g = per_cu * cus;
    g = (g / XCDS) * XCDS;
    return g < XCDS ? XCDS : g;
}

}  // namespace

int sg_resident_grid(int acc, int acc2, bool dbl, int cus) {
    if (dbl) return resident(k_num_sg<double, ACC_NATIVE, ACC_NATIVE>, cus);
    if (acc2 == ACC_WIDE && acc == ACC_NATIVE) return resident(k_num_sg<float, ACC_NATIVE, ACC_WIDE>, cus);
    if (acc2 == ACC_WIDE && acc == ACC_COMP) return resident(k_num_sg<float, ACC_COMP, ACC_WIDE>, cus);
    if (acc == ACC_COMP) return resident(k_num_sg<float, ACC_COMP, ACC_COMP>, cus);
    if (acc == ACC_WIDE) return resident(k_num_sg<float, ACC_WIDE, ACC_WIDE>, cus);
    return resident(k_num_sg<float, ACC_NATIVE, ACC_NATIVE>, cus);
}

template <>
hipError_t launch_num_sg<double>(const NumArgs<double> &a, int, int, const LaunchCfg &c) {
    return num_sg_impl<double, ACC_NATIVE, ACC_NATIVE>(a, c);
}
template <>
hipError_t launch_num_sg<float>(const NumArgs<float> &a, int acc, int acc2, const LaunchCfg &c) {
    if (acc2 == ACC_WIDE && acc == ACC_NATIVE) return num_sg_impl<float, ACC_NATIVE, ACC_WIDE>(a, c);
    if (acc2 == ACC_WIDE && acc == ACC_COMP) return num_sg_impl<float, ACC_COMP, ACC_WIDE>(a, c);
    if (acc == ACC_COMP) return num_sg_impl<float, ACC_COMP, ACC_COMP>(a, c);
    if (acc == ACC_WIDE) return num_sg_impl<float, ACC_WIDE, ACC_WIDE>(a, c);
    return num_sg_impl<float, ACC_NATIVE, ACC_NATIVE>(a, c);
}

}  // namespace spg
