// Numeric phase on a known structure: the Reuse case of the Experiments
// section (symbolic once, numeric repeated with new values on the same
// structure), taken one step further.
//
// After a numeric call has written C's sorted columns, every multiplication
// (i, k, j) of Algorithm 1 has a fixed place in row i of C: the rank of j
// among the row's columns.  A position map -- one 16-bit rank per
// multiplication, in the row's product order (A entries in stored order, each
// B row in stored order) -- is taken once from C's columns by binary search.
// A later numeric call on new values then needs no accumulator structure at
// all (no hash, no bit window, no sort): each product is added at its rank
// in an LDS copy of the row, and only C's values are written.
//
// Work split: teams of T = 2^LGT lanes per row (WAVE / T rows per
// wavefront); a team stages its row's A entries T at a time (B row start and
// length, the prefix of the lengths, A's value), then groups of G = 2^LGS
// lanes walk one staged B row each.
#include "spg_accum.hpp"
#include "spg_internal.hpp"

namespace spg {

namespace {

struct MapLayout {
    size_t b0, a, len, pre, vals, total;
};
__host__ __device__ inline MapLayout map_layout(int r_max, int teams, int acc_bytes) {
    MapLayout L{};
    L.b0 = 0;
    L.a = 8 * WAVE;
    L.len = 16 * WAVE;
    L.pre = 20 * WAVE;
    L.vals = 24 * WAVE;
    L.total = L.vals + align16((size_t)acc_bytes * r_max * teams);
    return L;
}

// Rows of this wavefront and team: the wavefront takes NT consecutive rows of
// its die's slice per step; the loop runs while the wavefront's first row is
// in the slice (uniform), a team whose row is past the end idles.
struct TeamRow {
    bool valid;
    int i;
    int64_t ab, ae, cb, ce, mo;
};

template <int LGT>
__device__ __forceinline__ int team_total(int inc) {
    constexpr int T = 1 << LGT;
    return __shfl(inc, T - 1, T);
}

template <int LGT, typename F>
__device__ __forceinline__ void map_rows(const RowSet &rs, const int64_t *arp, const int64_t *coff,
                                         const int64_t *moff, F &&body) {
    constexpr int T = 1 << LGT, NT = WAVE / T;
    const int l = lane_id(), team = l >> LGT;
    int64_t lo, hi;
    rs_bounds(rs, lo, hi);
    const Slice sl = xcd_slice(lo, hi, NT, 0);
    for (int64_t r0 = sl.idx; r0 < sl.end; r0 += sl.step) {
        TeamRow tr{};
        const int64_t r = r0 + team;
        tr.valid = r < sl.end;
        if (tr.valid) {
            tr.i = rs.rows[r];
            tr.ab = arp[tr.i];
            tr.ae = arp[tr.i + 1];
            tr.cb = coff[tr.i];
            tr.ce = coff[tr.i + 1];
            tr.mo = moff[tr.i];
        }
        body(tr);
    }
}

// Stage the team's A entries [e0, e0 + T) of the row: returns the team's
// total product count of the chunk; st_* hold, per lane, the entry's B row
// start, length, product offset inside the row (carry + exclusive prefix)
// and A value.
template <int LGT, typename VT>
__device__ __forceinline__ int stage_chunk(const TeamRow &tr, int64_t e0, int carry, const int32_t *aci,
                                           const VT *aval, const int64_t *brp, int64_t *st_b0, double *st_a,
                                           int *st_len, int *st_pre) {
    const int l = lane_id(), t = l & ((1 << LGT) - 1);
    const int64_t e = e0 + t;
    int64_t b0 = 0;
    int len = 0;
    double av = 0.0;
    if (tr.valid && e < tr.ae) {
        const int j = aci[e];
        b0 = brp[j];
        len = (int)(brp[j + 1] - b0);
        if (aval) av = (double)aval[e];
    }
    const int inc = team_scan<LGT>(len, t);
    st_b0[l] = b0;
    st_len[l] = len;
    st_pre[l] = carry + inc - len;
    st_a[l] = av;
    return team_total<LGT>(inc);
}

// Position map of the rows of one kind (one-time, from C's sorted columns).
template <int LGT, int LGS>
__global__ __launch_bounds__(WAVE) void k_posmap(NumArgs<double> a, const int32_t *cci) {
    constexpr int T = 1 << LGT, G = 1 << LGS, NG = T / G;
    __shared__ int64_t st_b0[WAVE];
    __shared__ double st_a[WAVE];
    __shared__ int st_len[WAVE], st_pre[WAVE];
    const int l = lane_id(), team = l >> LGT, t = l & (T - 1), g = t >> LGS, q = t & (G - 1);
    map_rows<LGT>(a.rs, a.arp, a.coff, a.map_off, [&](const TeamRow &tr) {
        const int64_t na = tr.valid ? tr.ae - tr.ab : 0;
        const int nch = wave_max((int)((na + T - 1) / T));
        int carry = 0;
        for (int c = 0; c < nch; ++c) {
            const int tot = stage_chunk<LGT, double>(tr, tr.ab + (int64_t)c * T, carry, a.aci, nullptr, a.brp,
                                                      st_b0, st_a, st_len, st_pre);
            wave_lds_sync();
            for (int s = g; s < T; s += NG) {
                const int u = team * T + s, len = st_len[u];
                const int64_t b0 = st_b0[u];
                const int64_t mb = tr.mo + st_pre[u];
                for (int p = q; p < len; p += G) {
                    const int col = a.bci[b0 + p];
                    int64_t lo2 = tr.cb, n2 = tr.ce - tr.cb;  // lower bound of col in C's row
                    while (n2 > 0) {
                        const int64_t h2 = n2 >> 1;
                        if (cci[lo2 + h2] < col) {
                            lo2 += h2 + 1;
                            n2 -= h2 + 1;
                        } else {
                            n2 = h2;
                        }
                    }
                    if (lo2 >= tr.ce || cci[lo2] != col) {
                        atomicAdd(&a.st->mismatch, 1);  // C's columns are not this product's
                        lo2 = tr.cb;
                    }
                    a.map[mb + p] = (uint16_t)(lo2 - tr.cb);
                }
            }
            carry += tot;
            wave_lds_sync();
        }
    });
}

// Values of the rows of one kind on their position maps.
template <typename VT, int ACC, int LGT, int LGS>
__global__ __launch_bounds__(WAVE) void k_num_map(NumArgs<VT> a) {
    using Acc = Accum<VT, ACC>;
    using S = typename Acc::store_t;
    constexpr int T = 1 << LGT, NT = WAVE / T, G = 1 << LGS, NG = T / G;
    extern __shared__ __align__(16) unsigned char smem[];
    const MapLayout L = map_layout(a.r_max, NT, sizeof(S));
    int64_t *st_b0 = (int64_t *)(smem + L.b0);
    double *st_a = (double *)(smem + L.a);
    int *st_len = (int *)(smem + L.len), *st_pre = (int *)(smem + L.pre);
    const int l = lane_id(), team = l >> LGT, t = l & (T - 1), g = t >> LGS, q = t & (G - 1);
    S *tv = (S *)(smem + L.vals) + (size_t)team * a.r_max;
    for (int u = t; u < a.r_max; u += T) tv[u] = Acc::zero();
    const int64_t cbase = a.cbase_row >= 0 ? a.coff[a.cbase_row] : 0;
    wave_lds_sync();
    map_rows<LGT>(a.rs, a.arp, a.coff, a.map_off, [&](const TeamRow &tr) {
        const int64_t na = tr.valid ? tr.ae - tr.ab : 0;
        const int rs = tr.valid ? (int)(tr.ce - tr.cb) : 0;
        const int rlast = rs > 0 ? rs - 1 : 0;
        const int nch = wave_max((int)((na + T - 1) / T));
        int carry = 0;
        for (int c = 0; c < nch; ++c) {
            const int tot = stage_chunk<LGT, VT>(tr, tr.ab + (int64_t)c * T, carry, a.aci, a.aval, a.brp, st_b0,
                                                  st_a, st_len, st_pre);
            wave_lds_sync();
            if (rs > 0) {
                for (int s = g; s < T; s += NG) {
                    const int u = team * T + s, len = st_len[u];
                    const int64_t b0 = st_b0[u];
                    const int64_t mb = tr.mo + st_pre[u];
                    const VT av = (VT)st_a[u];
                    for (int p = q; p < len; p += G) {
                        const int rk = min((int)a.map[mb + p], rlast);
                        Acc::add(&tv[rk], av, a.bval[b0 + p]);
                    }
                }
            }
            carry += tot;
            wave_lds_sync();
        }
        for (int u = t; u < rs; u += T) {
            a.cval[tr.cb - cbase + u] = Acc::fin(tv[u]);
            tv[u] = Acc::zero();
        }
        wave_lds_sync();
    });
}

template <typename K>
inline int resident_grid(K kernel, size_t lds, int cus) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, WAVE, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int g = (per_cu * cus / XCDS) * XCDS;
    return g < XCDS ? XCDS : g;
}

template <int LGT, int LGS>
hipError_t posmap_ts(const NumArgs<double> &a, const int32_t *cci, const LaunchCfg &c, int64_t rows) {
    constexpr int NT = WAVE >> LGT;
    int grid = resident_grid(k_posmap<LGT, LGS>, 0, c.cus);
    const int64_t need = (rows + NT - 1) / NT;
    grid = (int)std::min<int64_t>(grid, std::max<int64_t>(XCDS, ((need + XCDS - 1) / XCDS) * XCDS));
    hipLaunchKernelGGL((k_posmap<LGT, LGS>), dim3(grid), dim3(WAVE), 0, c.stream, a, cci);
    return hipGetLastError();
}

template <typename VT, int ACC, int LGT, int LGS>
hipError_t num_map_ts(const NumArgs<VT> &a, const LaunchCfg &c, int64_t rows) {
    using S = typename Accum<VT, ACC>::store_t;
    constexpr int NT = WAVE >> LGT;
    const size_t lds = map_layout(a.r_max, NT, sizeof(S)).total;
    int grid = resident_grid(k_num_map<VT, ACC, LGT, LGS>, lds, c.cus);
    const int64_t need = (rows + NT - 1) / NT;
    grid = (int)std::min<int64_t>(grid, std::max<int64_t>(XCDS, ((need + XCDS - 1) / XCDS) * XCDS));
    hipLaunchKernelGGL((k_num_map<VT, ACC, LGT, LGS>), dim3(grid), dim3(WAVE), lds, c.stream, a);
    return hipGetLastError();
}

// lanes per B row: 1 .. T
template <int LGT, typename F>
hipError_t by_lgs(int lgs, F &&f) {
    lgs = std::max(0, std::min(lgs, LGT));
    switch (lgs) {
    case 0: return f(std::integral_constant<int, 0>{});
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, (LGT >= 3 ? 3 : 2)>{});
    case 4: return f(std::integral_constant<int, (LGT >= 4 ? 4 : 2)>{});
    case 5: return f(std::integral_constant<int, (LGT >= 5 ? 5 : 2)>{});
    default: return f(std::integral_constant<int, (LGT >= 6 ? 6 : 2)>{});
    }
}

template <typename F>
hipError_t by_lgt(int lgt, F &&f) {
    switch (std::max(3, std::min(lgt, 6))) {
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    default: return f(std::integral_constant<int, 6>{});
    }
}

template <typename VT, int ACC>
hipError_t num_map_acc(const NumArgs<VT> &a, int lgt, int lgs, const LaunchCfg &c, int64_t rows) {
    return by_lgt(lgt, [&](auto T) {
        constexpr int LT = decltype(T)::value;
        return by_lgs<LT>(lgs, [&](auto S) {
            constexpr int LS = decltype(S)::value;
            return num_map_ts<VT, ACC, LT, LS>(a, c, rows);
        });
    });
}

}  // namespace

size_t lds_num_map(int r_max, int lgt, int acc_bytes) { return map_layout(r_max, WAVE >> lgt, acc_bytes).total; }

hipError_t launch_posmap(const NumArgs<double> &a, const int32_t *cci, int lgt, int lgs, const LaunchCfg &c,
                         int64_t rows) {
    return by_lgt(lgt, [&](auto T) {
        constexpr int LT = decltype(T)::value;
        return by_lgs<LT>(lgs, [&](auto S) {
            constexpr int LS = decltype(S)::value;
            return posmap_ts<LT, LS>(a, cci, c, rows);
        });
    });
}

template <>
hipError_t launch_num_map<double>(const NumArgs<double> &a, int, int lgt, int lgs, const LaunchCfg &c, int64_t rows) {
    return num_map_acc<double, ACC_NATIVE>(a, lgt, lgs, c, rows);
}
template <>
hipError_t launch_num_map<float>(const NumArgs<float> &a, int acc, int lgt, int lgs, const LaunchCfg &c, int64_t rows) {
    if (acc == ACC_COMP) return num_map_acc<float, ACC_COMP>(a, lgt, lgs, c, rows);
    if (acc == ACC_WIDE) return num_map_acc<float, ACC_WIDE>(a, lgt, lgs, c, rows);
    return num_map_acc<float, ACC_NATIVE>(a, lgt, lgs, c, rows);
}

}  // namespace spg

namespace spg {

namespace {

// Multiplications per row of the rows that get a position map (rows of the
// wavefront and team kinds in the plan's main or FP64-accumulated lists),
// 0 for the others.
__global__ __launch_bounds__(256) void k_map_rows(int64_t m, const uint8_t *kind, const uint8_t *kind_heavy,
                                                  const int64_t *rflops, int32_t *out) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
        const int k = kind[i], kh = kind_heavy ? kind_heavy[i] : 0;
        const bool mapped = map_kind(k) || map_kind(kh);
        out[i] = mapped ? (int32_t)rflops[i] : 0;
    }
}

}  // namespace

hipError_t launch_map_rows(int64_t m, const uint8_t *kind, const uint8_t *kind_heavy, const int64_t *rflops,
                           int32_t *out, hipStream_t s) {
    if (m == 0) return hipSuccess;
    const int g = (int)std::min<int64_t>(4096, (m + 255) / 256);
    hipLaunchKernelGGL(k_map_rows, dim3(g), dim3(256), 0, s, m, kind, kind_heavy, rflops, out);
    return hipGetLastError();
}

}  // namespace spg
