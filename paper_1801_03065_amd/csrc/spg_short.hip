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

// The same with max (values >= 0 after the first step; lanes without a
// source read 0).
template <int LG>
__device__ __forceinline__ int team_maxscan(int v, int q) {
    if (LG >= 1) { const int t = __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false); v = (LG >= 4 || q >= 1) ? max(v, t) : v; }
    if (LG >= 2) { const int t = __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false); v = (LG >= 4 || q >= 2) ? max(v, t) : v; }
    if (LG >= 3) { const int t = __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false); v = (LG >= 4 || q >= 4) ? max(v, t) : v; }
    if (LG >= 4) v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false));
    if (LG >= 5) v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false));
    if (LG >= 6) v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false));
    return v;
}
// Value of lane (lane ^ J): DPP quad permutes for 1 and 2, a row rotation
// for 8, swizzles inside 32 lanes for 4 and 16, a lane permute for 32.
template <int J>
__device__ __forceinline__ int lane_xor(int v) {
    if (J == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    if (J == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    if (J == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);  // row_ror:8
    if (J == 4) return __builtin_amdgcn_ds_swizzle(v, 0x1F | (4 << 10));
    if (J == 16) return __builtin_amdgcn_ds_swizzle(v, 0x1F | (16 << 10));
    return __shfl_xor(v, J);
}
// One compare-exchange step of the bitonic network (block size KK, distance J).
template <int KK, int J>
__device__ __forceinline__ void bitonic_step(int &key, int &slot, int q) {
    const int ok = lane_xor<J>(key), os = lane_xor<J>(slot);
    const bool up = (q & KK) == 0, lower = (q & J) == 0;
    if (lower == up ? ok < key : ok > key) {
        key = ok;
        slot = os;
    }
}
// Sort (key, slot) ascending inside blocks of P lanes (P <= 2^LG, a power of
// two, wavefront-uniform): the stages for blocks above P are skipped.
template <int LG>
__device__ __forceinline__ void team_sort(int &key, int &slot, int q, int P) {
#define SR_STAGE(KK, J) \
    if (KK <= (1 << LG) && KK <= P) bitonic_step<KK, J>(key, slot, q);
    SR_STAGE(2, 1)
    SR_STAGE(4, 2) SR_STAGE(4, 1)
    SR_STAGE(8, 4) SR_STAGE(8, 2) SR_STAGE(8, 1)
    SR_STAGE(16, 8) SR_STAGE(16, 4) SR_STAGE(16, 2) SR_STAGE(16, 1)
    SR_STAGE(32, 16) SR_STAGE(32, 8) SR_STAGE(32, 4) SR_STAGE(32, 2) SR_STAGE(32, 1)
    SR_STAGE(64, 32) SR_STAGE(64, 16) SR_STAGE(64, 8) SR_STAGE(64, 4) SR_STAGE(64, 2) SR_STAGE(64, 1)
#undef SR_STAGE
}

template <bool NUM, typename VT, int ACC, int LG>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_sr(SrArgs<VT> a) {
    using A = Accum<VT, ACC>;
    using S = typename A::store_t;
    __shared__ int32_t keys_all[2 * WAVE];
    __shared__ S vals_all[NUM ? 2 * WAVE : 1];
    __shared__ int32_t own_all[WAVE];
    __shared__ int32_t uslot_all[NUM ? WAVE : 1];
    const int l = lane_id();
    constexpr int lgT = LG, T = 1 << LG;
    const int q = l & (T - 1), team = l >> lgT;
    constexpr int nteam = WAVE >> LG;
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
            // B rows of at most one entry (every A entry makes at most one
            // product, e.g. aggregation or injection operators): each lane
            // forms its own product, no expansion
            const bool unit = __ballot(len > 1) == 0;
            int64_t e = b0;
            VT avk = av;
            bool mine = len > 0;
            if (!unit) {
                const int inc = team_scan<LG>(len, q);
                const int F = __shfl(inc, T - 1, T);  // products of this chunk (<= T for a short row)
                const int off = inc - len;
                own[q] = -1;
                wave_lds_sync();
                if (len > 0 && off < T) own[off] = q;
                wave_lds_sync();
                // owner of product q: the last A entry starting at or before q
                const int k = max(team_maxscan<LG>(own[q], q), 0);
                const int offk = __shfl(off, k, T);
                const int64_t b0k = __shfl(b0, k, T);
                if (NUM) avk = __shfl(av, k, T);
                if (q == 0 && F > T) atomicAdd(&a.st->mismatch, 1);  // not a short row: plan inconsistent
                e = b0k + (q - offk);
                mine = q < F;
            }
            if (mine) {
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
        const int cnt = __shfl(team_scan<LG>(nins, q), T - 1, T);

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
            int p = team_scan<LG>(c, q) - c;
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
            // bitonic sort of (key, slot) across the team, ascending, over the
            // next power of two of the wavefront's largest row
            int P = 2;
            {
                const int mc = __builtin_amdgcn_readfirstlane(wave_max(cnt));
                while (P < mc) P <<= 1;
            }
            team_sort<LG>(key, slot, q, P);
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

template <typename VT, int ACC, int LG>
hipError_t num_sr_lg(const SrArgs<VT> &a, const LaunchCfg &c, int64_t rows) {
    const int grid = c.grid > 0 ? c.grid : sr_grid(k_sr<true, VT, ACC, LG>, c.cus, rows >> (6 - LG));
    hipLaunchKernelGGL((k_sr<true, VT, ACC, LG>), dim3(grid), dim3(WAVE), 0, c.stream, a);
    return hipGetLastError();
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
    if (lg_t <= 3) return num_sr_lg<VT, ACC, 3>(a, c, rows);
    if (lg_t == 4) return num_sr_lg<VT, ACC, 4>(a, c, rows);
    if (lg_t == 5) return num_sr_lg<VT, ACC, 5>(a, c, rows);
    return num_sr_lg<VT, ACC, 6>(a, c, rows);
}

template <int LG>
hipError_t sym_sr_lg(const SrArgs<double> &a, const LaunchCfg &c, int64_t rows) {
    const int grid = c.grid > 0 ? c.grid : sr_grid(k_sr<false, double, ACC_NATIVE, LG>, c.cus, rows >> (6 - LG));
    hipLaunchKernelGGL((k_sr<false, double, ACC_NATIVE, LG>), dim3(grid), dim3(WAVE), 0, c.stream, a);
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
    if (lg_t <= 3) return sym_sr_lg<3>(a, c, rows);
    if (lg_t == 4) return sym_sr_lg<4>(a, c, rows);
    if (lg_t == 5) return sym_sr_lg<5>(a, c, rows);
    return sym_sr_lg<6>(a, c, rows);
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
