// Short rows: several rows of C per wavefront (Partitioning Schemes
// subsection, Thread-Parallel with a team of lanes per row).
//
// A row whose multiplication count f_m(i) is at most T = 2^lg_t lanes is
// handled by a team of T lanes, WAVE / T rows at once.  The row's products
// are spread one per lane (expansion: prefix sum of the B row lengths over
// the row of A, then each lane finds the A entry that owns its product), and
// go into a team-private linear-probing hash in LDS keyed by column (LP
// hashmap, Accumulators subsection: 2T slots, so at most 50% occupancy).
//   symbolic: row size = number of first insertions.
//   numeric:  the team compacts its occupied slots, sorts the (column, slot)
//             pairs with a bitonic network across its lanes and writes the
//             sorted row.
// The per-row cost of a whole wavefront (stage, scans, summary) is what this
// avoids: for rows of a few dozen multiplications it dominates.  Like the
// wavefront kernels, the loop is software-pipelined across rows: the next
// row's A entries and B extents load while the current row is processed.
#include "spg_accum.hpp"
#include "spg_internal.hpp"

namespace spg {

namespace {

template <typename VT>
struct SrArgs {
    const int64_t *arp;
    const int32_t *aci;
    const VT *aval;  // numeric only
    const int64_t *brp;
    const int32_t *bci;
    const VT *bval;  // numeric only
    const int64_t *coff;
    int32_t *cci;
    VT *cval;
    int64_t cbase_row;
    int32_t *row_nnz;    // symbolic only
    int32_t *row_words;  // symbolic only (row size as the word bound)
    RowSet rs;
    int lg_t;
    DevStats *st;
};

// Slot of column c in a table of 2^lg slots (Fibonacci hash of the low 24 bits).
__device__ __forceinline__ uint32_t sr_hash(int c, int lg) {
    return (__umul24((uint32_t)c & 0xFFFFFFu, 0x9E3779u) >> (24 - lg)) & ((1u << lg) - 1u);
}

template <bool NUM, typename VT, int ACC>
__global__ __launch_bounds__(WAVE) void k_sr(SrArgs<VT> a) {
    using A = Accum<VT, ACC>;
    using S = typename A::store_t;
    __shared__ int32_t keys_all[2 * WAVE];
    __shared__ S vals_all[NUM ? 2 * WAVE : 1];
    __shared__ int32_t own_all[WAVE];
    __shared__ int32_t uslot_all[NUM ? WAVE : 1];
    const int l = lane_id();
    const int lgT = a.lg_t, T = 1 << lgT, q = l & (T - 1), team = l >> lgT, nteam = WAVE >> lgT;
    int32_t *keys = keys_all + 2 * T * team;
    S *vals = vals_all + (NUM ? 2 * T * team : 0);
    int32_t *own = own_all + T * team;
    int32_t *uslot = uslot_all + (NUM ? T * team : 0);
    keys_all[l] = -1;
    keys_all[l + WAVE] = -1;
    if (NUM) {
        vals_all[l] = A::zero();
        vals_all[l + WAVE] = A::zero();
    }
    wave_lds_sync();
    int64_t lo, hi;
    rs_bounds(a.rs, lo, hi);
    const int64_t ngroups = (hi - lo + nteam - 1) / nteam;
    const Slice sl = xcd_slice(0, ngroups);
    const int64_t cbase = (NUM && a.cbase_row >= 0) ? a.coff[a.cbase_row] : 0;
    const uint32_t tmask = 2u * T - 1u;

    // this team's row in group gg, or -1
    auto row_of = [&](int64_t gg) -> int {
        const int64_t r = lo + gg * nteam + team;
        return (gg < sl.end && r < hi) ? a.rs.rows[r] : -1;
    };

    int64_t g = sl.idx;
    int ic = row_of(g);
    int64_t abc = 0, aec = 0;
    if (ic >= 0) {
        abc = a.arp[ic];
        aec = a.arp[ic + 1];
    }
    int jc = 0, lenc = 0;
    int64_t b0c = 0;
    VT avc = VT(0);
    if (q < aec - abc) {
        jc = a.aci[abc + q];
        if (NUM) avc = a.aval[abc + q];
        b0c = a.brp[jc];
        lenc = (int)(a.brp[jc + 1] - b0c);
    }
    int in = row_of(g + sl.step);
    int64_t abn = 0, aen = 0;
    if (in >= 0) {
        abn = a.arp[in];
        aen = a.arp[in + 1];
    }
    int i2 = row_of(g + 2 * sl.step);  // row indices load two groups ahead
    while (g < sl.end) {
        // next row, first level: its A entries (first chunk)
        int jn = 0;
        VT avn = VT(0);
        if (q < aen - abn) {
            jn = a.aci[abn + q];
            if (NUM) avn = a.aval[abn + q];
        }
        int64_t cb = 0, ce = 0;
        if (NUM && ic >= 0) {
            cb = a.coff[ic];
            ce = a.coff[ic + 1];
        }
        // ---- expansion + insertion, T A entries at a time (team-uniform loop)
        int nins = 0;
        for (int64_t c0 = abc; c0 < aec; c0 += T) {
            int j = jc, len = lenc;
            int64_t b0 = b0c;
            VT av = avc;
            if (c0 != abc) {
                j = 0;
                len = 0;
                b0 = 0;
                av = VT(0);
                if (c0 + q < aec) {
                    j = a.aci[c0 + q];
                    if (NUM) av = a.aval[c0 + q];
                    b0 = a.brp[j];
                    len = (int)(a.brp[j + 1] - b0);
                }
            }
            int inc = len;
#pragma unroll
            for (int d = 1; d < WAVE; d <<= 1) {
                if (d >= T) break;
                const int t = __shfl_up(inc, d, T);
                if (q >= d) inc += t;
            }
            const int F = __shfl(inc, T - 1, T);  // products of this chunk (<= T for a short row)
            const int off = inc - len;
            own[q] = -1;
            wave_lds_sync();
            if (len > 0 && off < T) own[off] = q;
            wave_lds_sync();
            int k = own[q];  // owner of product q: the last A entry starting at or before q
#pragma unroll
            for (int d = 1; d < WAVE; d <<= 1) {
                if (d >= T) break;
                const int t = __shfl_up(k, d, T);
                if (q >= d) k = max(k, t);
            }
            k = max(k, 0);
            const int offk = __shfl(off, k, T);
            const int64_t b0k = __shfl(b0, k, T);
            VT avk = VT(0);
            if (NUM) avk = __shfl(av, k, T);
            if (q == 0 && F > T) atomicAdd(&a.st->mismatch, 1);  // not a short row: plan inconsistent
            if (q < F) {
                const int64_t e = b0k + (q - offk);
                const int col = a.bci[e];
                VT bv = VT(0);
                if (NUM) bv = a.bval[e];
                uint32_t h = sr_hash(col, lgT + 1);
                for (;;) {
                    const int32_t old = atomicCAS(&keys[h], -1, col);
                    if (old == -1) {
                        ++nins;
                        break;
                    }
                    if (old == col) break;
                    h = (h + 1) & tmask;
                }
                if (NUM) A::add(&vals[h], avk, bv);
            }
            wave_lds_sync();
        }
        int cnt = nins;
#pragma unroll
        for (int d = WAVE / 2; d >= 1; d >>= 1)
            if (d < T) cnt += __shfl_xor(cnt, d, T);

        if (!NUM) {
            if (q == 0 && ic >= 0) {
                a.row_nnz[ic] = cnt;
                a.row_words[ic] = cnt;
            }
            keys[q] = -1;
            keys[q + T] = -1;
        } else {
            // ---- compact the occupied slots, sort by column, write the row
            const int k0 = keys[q], k1 = keys[q + T];
            const int c = (k0 >= 0) + (k1 >= 0);
            int pin = c;
#pragma unroll
            for (int d = 1; d < WAVE; d <<= 1) {
                if (d >= T) break;
                const int t = __shfl_up(pin, d, T);
                if (q >= d) pin += t;
            }
            int p = pin - c;
            if (k0 >= 0) {
                own[p] = k0;
                uslot[p] = q;
                ++p;
            }
            if (k1 >= 0) {
                own[p] = k1;
                uslot[p] = q + T;
            }
            wave_lds_sync();
            int key = q < cnt ? own[q] : INT_MAX;
            int slot = q < cnt ? uslot[q] : 0;
            // bitonic sort of (key, slot) across the team, ascending
            for (int kk = 2; kk <= T; kk <<= 1) {
                for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                    const int ok = __shfl_xor(key, jj, T);
                    const int os = __shfl_xor(slot, jj, T);
                    const bool up = (q & kk) == 0, lower = (q & jj) == 0;
                    if (lower == up ? ok < key : ok > key) {
                        key = ok;
                        slot = os;
                    }
                }
            }
            const bool okrow = ic < 0 || ce - cb == cnt;
            if (q == 0 && !okrow) atomicAdd(&a.st->mismatch, 1);
            if (okrow && q < cnt) {
                a.cci[cb - cbase + q] = key;
                a.cval[cb - cbase + q] = A::fin(vals[slot]);
            }
            wave_lds_sync();
            keys[q] = -1;
            keys[q + T] = -1;
            vals[q] = A::zero();
            vals[q + T] = A::zero();
        }
        // next row, second level: B extents of its first chunk
        int64_t b0n = 0;
        int lenn = 0;
        if (q < aen - abn) {
            b0n = a.brp[jn];
            lenn = (int)(a.brp[jn + 1] - b0n);
        }
        // the row after next: its A extent (its index loaded a group ago)
        g += sl.step;
        const int inn = i2;
        int64_t abnn = 0, aenn = 0;
        if (inn >= 0) {
            abnn = a.arp[inn];
            aenn = a.arp[inn + 1];
        }
        i2 = row_of(g + 2 * sl.step);
        ic = in;
        abc = abn;
        aec = aen;
        jc = jn;
        avc = avn;
        b0c = b0n;
        lenc = lenn;
        in = inn;
        abn = abnn;
        aen = aenn;
        wave_lds_sync();
    }
}

template <typename K>
int sr_grid(K kernel, int cus, int64_t groups) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, WAVE, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int64_t g = (int64_t)per_cu * cus;
    g = std::min<int64_t>(g, ((groups + XCDS - 1) / XCDS) * XCDS);
    g = (g / XCDS) * XCDS;
    return (int)(g < XCDS ? XCDS : g);
}

template <typename VT, int ACC>
hipError_t num_sr_impl(const NumArgs<VT> &n, int lg_t, const LaunchCfg &c, int64_t rows) {
    SrArgs<VT> a{};
    a.arp = n.arp;
    a.aci = n.aci;
    a.aval = n.aval;
    a.brp = n.brp;
    a.bci = n.bci;
    a.bval = n.bval;
    a.coff = n.coff;
    a.cci = n.cci;
    a.cval = n.cval;
    a.cbase_row = n.cbase_row;
    a.rs = n.rs;
    a.lg_t = lg_t;
    a.st = n.st;
    const int grid = c.grid > 0 ? c.grid : sr_grid(k_sr<true, VT, ACC>, c.cus, rows >> (6 - lg_t));
    hipLaunchKernelGGL((k_sr<true, VT, ACC>), dim3(grid), dim3(WAVE), 0, c.stream, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sym_sr(const SymArgs &s, int lg_t, const LaunchCfg &c, int64_t rows) {
    if (lg_t < 0 || lg_t > 6) return hipErrorInvalidValue;
    SrArgs<double> a{};
    a.arp = s.arp;
    a.aci = s.aci;
    a.brp = s.brp;
    a.bci = s.bci;
    a.row_nnz = s.row_nnz;
    a.row_words = s.row_words;
    a.rs = s.rs;
    a.lg_t = lg_t;
    a.st = s.st;
    a.cbase_row = -1;
    const int grid = c.grid > 0 ? c.grid : sr_grid(k_sr<false, double, ACC_NATIVE>, c.cus, rows >> (6 - lg_t));
    hipLaunchKernelGGL((k_sr<false, double, ACC_NATIVE>), dim3(grid), dim3(WAVE), 0, c.stream, a);
    return hipGetLastError();
}

template <>
hipError_t launch_num_sr<double>(const NumArgs<double> &a, int, int lg_t, const LaunchCfg &c, int64_t rows) {
    if (lg_t < 0 || lg_t > 6) return hipErrorInvalidValue;
    return num_sr_impl<double, ACC_NATIVE>(a, lg_t, c, rows);
}
template <>
hipError_t launch_num_sr<float>(const NumArgs<float> &a, int acc, int lg_t, const LaunchCfg &c, int64_t rows) {
    if (lg_t < 0 || lg_t > 6) return hipErrorInvalidValue;
    if (acc == ACC_COMP) return num_sr_impl<float, ACC_COMP>(a, lg_t, c, rows);
    if (acc == ACC_WIDE) return num_sr_impl<float, ACC_WIDE>(a, lg_t, c, rows);
    return num_sr_impl<float, ACC_NATIVE>(a, lg_t, c, rows);
}

}  // namespace spg
