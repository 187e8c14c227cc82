// Numeric phase with the paper's linked-list hashmap and unsorted rows
// (Accumulators subsection, LL hashmap; the kkmem method of the Meta-
// algorithm section: Thread-Sequential partitioning + LL accumulators).
//
// A group of G = 2^LGG lanes owns one row of C (WAVE / G rows per
// wavefront) and walks the row's A entries in order; for each it takes the
// B row with its G lanes, one column per lane.  The keys inserted at once are
// then distinct (one B row has no duplicate column), which is the condition
// the LL map is built on: a key found in its bucket's chain is updated in
// place without atomics, a new key takes the next free slot from the group's
// counter and is pushed on its bucket's list with a compare-and-swap (a lane
// walking the chain while another pushes can only miss the other lane's key,
// never its own).  The map's arrays follow the paper's names: begins (bucket
// heads, key AND (size-1)), nexts, ids, values.  The row leaves in slot
// order, i.e. unsorted (the paper's output order); its size is known from
// the symbolic phase, so the map never fills.
#include "spg_accum.hpp"
#include "spg_internal.hpp"

namespace spg {

namespace {

struct LlLayout {
    size_t b0, a, len, group, begins, nexts, ids, vals, total;
};

// per wavefront: staging of 64 A entries; per group: count, begins[hb],
// nexts[cap], ids[cap], values[cap]
__host__ __device__ inline LlLayout ll_layout(int hb, int cap, int groups, int acc_bytes) {
    LlLayout L{};
    L.b0 = 0;
    L.a = 8 * WAVE;
    L.len = 16 * WAVE;
    size_t o = 20 * WAVE;
    size_t g = 0;
    L.begins = g;
    g += 4 * (size_t)hb;
    L.nexts = g;
    g += 4 * (size_t)cap;
    L.ids = g;
    g += 4 * (size_t)cap;
    g = align16(g + 4);  // count after ids
    L.vals = g;
    g += align16((size_t)acc_bytes * cap);
    L.group = g;
    L.total = o + g * groups;
    return L;
}

template <typename VT, int ACC, int LGG>
__global__ __launch_bounds__(WAVE) void k_num_ll(NumArgs<VT> a) {
    using Acc = Accum<VT, ACC>;
    using S = typename Acc::store_t;
    constexpr int G = 1 << LGG, NG = WAVE / G;
    extern __shared__ __align__(16) unsigned char smem[];
    const int hb = a.ts, cap = a.r_max;  // buckets (power of two), slots
    const LlLayout L = ll_layout(hb, cap, NG, sizeof(S));
    int64_t *st_b0 = (int64_t *)(smem + L.b0);
    double *st_a = (double *)(smem + L.a);
    int *st_len = (int *)(smem + L.len);
    const int l = lane_id(), grp = l >> LGG, q = l & (G - 1);
    unsigned char *gb = smem + 20 * WAVE + (size_t)grp * L.group;
    int *begins = (int *)(gb + L.begins);
    int *nexts = (int *)(gb + L.nexts);
    int *ids = (int *)(gb + L.ids);
    int *count = ids + cap;
    S *vals = (S *)(gb + L.vals);
    for (int s = q; s < hb; s += G) begins[s] = -1;
    if (q == 0) *count = 0;
    const uint32_t hmask = (uint32_t)hb - 1;
    const int64_t cbase = a.cbase_row >= 0 ? a.coff[a.cbase_row] : 0;
    int64_t lo, hi;
    rs_bounds(a.rs, lo, hi);
    const Slice sl = xcd_slice(lo, hi, NG, 0);
    wave_lds_sync();
    for (int64_t r0 = sl.idx; r0 < sl.end; r0 += sl.step) {
        const int64_t r = r0 + grp;
        const bool valid = r < sl.end;
        int i = 0;
        int64_t ab = 0, ae = 0;
        if (valid) {
            i = a.rs.rows[r];
            ab = a.arp[i];
            ae = a.arp[i + 1];
        }
        const int nch = wave_max((int)((ae - ab + G - 1) / G));
        for (int c = 0; c < nch; ++c) {
            // stage G A entries of the group's row: B row start and length, A value
            const int64_t e = ab + (int64_t)c * G + q;
            int64_t b0 = 0;
            int len = 0;
            double av = 0.0;
            if (valid && e < ae) {
                const int j = a.aci[e];
                b0 = a.brp[j];
                len = (int)(a.brp[j + 1] - b0);
                av = (double)a.aval[e];
            }
            st_b0[l] = b0;
            st_len[l] = len;
            st_a[l] = av;
            wave_lds_sync();
            // Thread-Sequential: the group's B rows one after another
            for (int s = 0; s < G; ++s) {
                const int u = grp * G + s;
                const int n = st_len[u];
                const int64_t bs = st_b0[u];
                const VT avs = (VT)st_a[u];
                for (int p = q; p < n; p += G) {
                    const int key = a.bci[bs + p];
                    const VT bv = a.bval[bs + p];
                    const uint32_t hsh = (uint32_t)key & hmask;
                    int slot = __hip_atomic_load(&begins[hsh], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    while (slot >= 0 &&
                           __hip_atomic_load(&ids[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != key)
                        slot = __hip_atomic_load(&nexts[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (slot < 0) {  // a new key: next free slot, pushed on the bucket's list
                        slot = atomicAdd(count, 1);
                        if (slot >= cap) {  // more keys than the symbolic row size: not this plan's structure
                            atomicAdd(&a.st->mismatch, 1);
                            continue;
                        }
                        __hip_atomic_store(&ids[slot], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        vals[slot] = Acc::zero();
                        int head = __hip_atomic_load(&begins[hsh], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        for (;;) {
                            __hip_atomic_store(&nexts[slot], head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                            const int seen = atomicCAS(&begins[hsh], head, slot);
                            if (seen == head) break;
                            head = seen;
                        }
                    }
                    Acc::add(&vals[slot], avs, bv);
                }
            }
            wave_lds_sync();
        }
        // the row in slot order (unsorted), then the map is reset
        const int n = *count;
        int64_t cb = 0;
        if (valid) {
            cb = a.coff[i];
            const int64_t want = a.coff[i + 1] - cb;
            if (q == 0 && want != n) atomicAdd(&a.st->mismatch, 1);
            const int w = (int)min((int64_t)n, want);
            for (int t = q; t < w; t += G) {
                a.cci[cb - cbase + t] = ids[t];
                a.cval[cb - cbase + t] = Acc::fin(vals[t]);
            }
        }
        for (int t = q; t < n && t < cap; t += G) begins[(uint32_t)ids[t] & hmask] = -1;
        wave_lds_sync();
        if (q == 0) *count = 0;
        wave_lds_sync();
    }
}

template <typename K>
inline int resident_grid(K kernel, size_t lds, int cus) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, WAVE, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int g = (per_cu * cus / XCDS) * XCDS;
    return g < XCDS ? XCDS : g;
}

template <typename VT, int ACC, int LGG>
hipError_t num_ll_g(const NumArgs<VT> &a, const LaunchCfg &c, int64_t rows) {
    using S = typename Accum<VT, ACC>::store_t;
    constexpr int NG = WAVE >> LGG;
    const size_t lds = ll_layout(a.ts, a.r_max, NG, sizeof(S)).total;
    int grid = c.grid > 0 ? c.grid : resident_grid(k_num_ll<VT, ACC, LGG>, lds, c.cus);
    const int64_t need = (rows + NG - 1) / NG;
    grid = (int)std::min<int64_t>(grid, std::max<int64_t>(XCDS, ((need + XCDS - 1) / XCDS) * XCDS));
    hipLaunchKernelGGL((k_num_ll<VT, ACC, LGG>), dim3(grid), dim3(WAVE), lds, c.stream, a);
    return hipGetLastError();
}

template <typename VT, int ACC>
hipError_t num_ll_acc(const NumArgs<VT> &a, int lgg, const LaunchCfg &c, int64_t rows) {
    switch (std::max(2, std::min(lgg, 6))) {
    case 2: return num_ll_g<VT, ACC, 2>(a, c, rows);
    case 3: return num_ll_g<VT, ACC, 3>(a, c, rows);
    case 4: return num_ll_g<VT, ACC, 4>(a, c, rows);
    case 5: return num_ll_g<VT, ACC, 5>(a, c, rows);
    default: return num_ll_g<VT, ACC, 6>(a, c, rows);
    }
}

}  // namespace

size_t lds_num_ll(int hb, int cap, int lgg, int acc_bytes) {
    return ll_layout(hb, cap, WAVE >> lgg, acc_bytes).total;
}

template <>
hipError_t launch_num_ll<double>(const NumArgs<double> &a, int, int lgg, const LaunchCfg &c, int64_t rows) {
    return num_ll_acc<double, ACC_NATIVE>(a, lgg, c, rows);
}
template <>
hipError_t launch_num_ll<float>(const NumArgs<float> &a, int acc, int lgg, const LaunchCfg &c, int64_t rows) {
    if (acc == ACC_COMP) return num_ll_acc<float, ACC_COMP>(a, lgg, c, rows);
    if (acc == ACC_WIDE) return num_ll_acc<float, ACC_WIDE>(a, lgg, c, rows);
    return num_ll_acc<float, ACC_NATIVE>(a, lgg, c, rows);
}

}  // namespace spg
