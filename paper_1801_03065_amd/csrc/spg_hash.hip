// Linear-probing hash accumulators (LP hashmap of the Accumulators
// subsection): parallel arrays of keys (-1 = empty) and values; the slot of a
// key is key AND (size - 1) with a power-of-two size; a taken slot sends the
// insert to the next slot.  Inserts from different lanes may carry the same
// key (Thread-Parallel / Thread-Flat-Parallel partitioning), so keys are
// claimed with compare-and-swap and values accumulated atomically.
//
// K_HW: one wavefront per row, the whole table in LDS (sized 2x the row's
//       bound: at most 50% occupancy, the paper's cut-off), sorted output by
//       an LDS bitonic sort of the occupied slots.
// K_HL: one 256-lane workgroup per row, two levels (Algorithm 3): the level-1
//       table lives in LDS and stops taking new keys at 50% occupancy; the
//       inserts it refuses go to a level-2 table in HBM sized for the whole
//       row (a slice of an arena owned by the workgroup: the memory pool in
//       one-to-one mode).  At the end of the row the level-1 entries are merged
//       into level 2, so a key that reached both levels is summed once, and the
//       row is compacted and sorted.
#include "spg_accum.hpp"
#include "spg_internal.hpp"

namespace spg {

namespace {

__device__ __forceinline__ uint32_t slot_of(uint32_t key, uint32_t mask) { return key & mask; }

// ------------------------------------------------------------ LDS bitonic sort
// Sort n (power of two) (key, value) pairs ascending by key; `nthreads` lanes
// cooperate, all of them call this.
template <typename S>
__device__ __forceinline__ void bitonic_lds(int32_t *key, S *val, int n, int nthreads) {
    const int t = threadIdx.x;
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int p = t; p < (n >> 1); p += nthreads) {
                const int i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
                const int o = i + j;
                const bool up = (i & k) == 0;
                const int32_t ki = key[i], ko = key[o];
                if ((ki > ko) == up) {
                    key[i] = ko;
                    key[o] = ki;
                    const S vi = val[i];
                    val[i] = val[o];
                    val[o] = vi;
                }
            }
            wave_lds_sync();
        }
    }
}

// ============================================================ wavefront / row

struct HwLayout {
    size_t keys, vals, sk, sv, st_bs, st_len, st_a, total;
};

__host__ __device__ inline HwLayout hw_layout(int ts, int acc_bytes, bool numeric) {
    HwLayout L{};
    size_t o = 0;
    L.keys = o;
    o += align16(4 * (size_t)ts);
    L.vals = o;
    o += align16((size_t)(numeric ? acc_bytes : 4) * ts);
    if (numeric) {
        L.sk = o;
        o += align16(4 * (size_t)(ts / 2));
        L.sv = o;
        o += align16((size_t)acc_bytes * (ts / 2));
    }
    L.st_bs = o;
    o += 8 * WAVE;
    L.st_len = o;
    o += 4 * WAVE;
    L.st_a = o;
    o += 8 * WAVE;
    L.total = o;
    return L;
}

template <typename VT>
__device__ __forceinline__ int hw_stage(int64_t cb, int64_t ae, const int32_t *aci, const VT *aval,
                                        const int64_t *rp, int64_t *st_bs, int32_t *st_len, double *st_a) {
    const int l = lane_id();
    const int cn = (int)min((int64_t)WAVE, ae - cb);
    if (l < cn) {
        const int j = aci[cb + l];
        const int64_t s0 = rp[j], s1 = rp[j + 1];
        st_bs[l] = s0;
        st_len[l] = (int32_t)(s1 - s0);
        if (aval) st_a[l] = (double)aval[cb + l];
    }
    return cn;
}

// Claim (or find) the slot of `key`; the table never fills (occupancy <= 50%).
__device__ __forceinline__ uint32_t lp_find_or_insert(int32_t *keys, uint32_t mask, int32_t key) {
    uint32_t h = slot_of((uint32_t)key, mask);
    for (;;) {
        const int32_t k = keys[h];
        if (k == key) return h;
        if (k == -1) {
            const int32_t old = atomicCAS(&keys[h], -1, key);
            if (old == -1 || old == key) return h;
        }
        h = (h + 1) & mask;
    }
}

__global__ __launch_bounds__(WAVE) void k_sym_hw(SymArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const HwLayout L = hw_layout(a.ts, 4, false);
    int32_t *keys = (int32_t *)(smem + L.keys);
    uint32_t *masks = (uint32_t *)(smem + L.vals);
    int64_t *st_bs = (int64_t *)(smem + L.st_bs);
    int32_t *st_len = (int32_t *)(smem + L.st_len);
    double *st_a = (double *)(smem + L.st_a);
    const int l = lane_id();
    const uint32_t mask = (uint32_t)a.ts - 1;
    for (int s = l; s < a.ts; s += WAVE) {
        keys[s] = -1;
        masks[s] = 0;
    }
    wave_lds_sync();
    const bool comp = a.bcrp != nullptr;
    const int gs = 1 << a.lg_gs, g = l >> a.lg_gs, q = l & (gs - 1), ng = WAVE >> a.lg_gs;
    int64_t lo, hi;
    rs_bounds(a.rs, lo, hi);
    const Slice sl = xcd_slice(lo, hi);
    for (int64_t r = sl.idx; r < sl.end; r += sl.step) {
        const int i = a.rs.rows[r];
        const int64_t ab = a.arp[i], ae = a.arp[i + 1];
        for (int64_t cb = ab; cb < ae; cb += WAVE) {
            const int cn = hw_stage<double>(cb, ae, a.aci, nullptr, comp ? a.bcrp : a.brp, st_bs, st_len, st_a);
            wave_lds_sync();
            for (int t = g; t < cn; t += ng) {
                const int64_t bs = st_bs[t];
                const int len = st_len[t];
                for (int p = q; p < len; p += gs) {
                    int32_t key;
                    uint32_t cs;
                    if (comp) {
                        const uint2 v = a.bcw[bs + p];
                        key = (int)v.x;
                        cs = v.y;
                    } else {
                        key = a.bci[bs + p];
                        cs = 1u;
                    }
                    atomicOr(&masks[lp_find_or_insert(keys, mask, key)], cs);
                }
            }
            wave_lds_sync();
        }
        int cnt = 0, occ = 0;
        for (int s = l; s < a.ts; s += WAVE) {
            if (keys[s] != -1) {
                cnt += __popc(masks[s]);
                ++occ;
                keys[s] = -1;
                masks[s] = 0;
            }
        }
        cnt = wave_sum(cnt);
        occ = wave_sum(occ);
        if (l == 0) {
            a.row_nnz[i] = cnt;
            // compressed keys are the touched words; column keys bound them by the window
            const int2 win = a.rwin[i];
            a.row_words[i] = comp ? occ : min(cnt, win.y - win.x + 1);
        }
        wave_lds_sync();
    }
}

template <typename VT, int ACC>
__global__ __launch_bounds__(WAVE) void k_num_hw(NumArgs<VT> a) {
    using A = Accum<VT, ACC>;
    using S = typename A::store_t;
    extern __shared__ __align__(16) unsigned char smem[];
    const HwLayout L = hw_layout(a.ts, sizeof(S), true);
    int32_t *keys = (int32_t *)(smem + L.keys);
    S *vals = (S *)(smem + L.vals);
    int32_t *sk = (int32_t *)(smem + L.sk);
    S *sv = (S *)(smem + L.sv);
    int64_t *st_bs = (int64_t *)(smem + L.st_bs);
    int32_t *st_len = (int32_t *)(smem + L.st_len);
    double *st_a = (double *)(smem + L.st_a);
    const int l = lane_id();
    const uint32_t mask = (uint32_t)a.ts - 1;
    for (int s = l; s < a.ts; s += WAVE) {
        keys[s] = -1;
        vals[s] = A::zero();
    }
    wave_lds_sync();
    const int gs = 1 << a.lg_gs, g = l >> a.lg_gs, q = l & (gs - 1), ng = WAVE >> a.lg_gs;
    int64_t lo, hi;
    rs_bounds(a.rs, lo, hi);
    const int64_t cbase = a.cbase_row >= 0 ? a.coff[a.cbase_row] : 0;
    const Slice sl = xcd_slice(lo, hi);
    for (int64_t r = sl.idx; r < sl.end; r += sl.step) {
        const int i = a.rs.rows[r];
        const int64_t ab = a.arp[i], ae = a.arp[i + 1];
        for (int64_t cb = ab; cb < ae; cb += WAVE) {
            const int cn = hw_stage<VT>(cb, ae, a.aci, a.aval, a.brp, st_bs, st_len, st_a);
            wave_lds_sync();
            for (int t = g; t < cn; t += ng) {
                const int64_t bs = st_bs[t];
                const int len = st_len[t];
                const VT av = (VT)st_a[t];
                for (int p = q; p < len; p += gs) {
                    const int32_t c = a.bci[bs + p];
                    const VT bv = a.bval[bs + p];
                    A::add(&vals[lp_find_or_insert(keys, mask, c)], av, bv);
                }
            }
            wave_lds_sync();
        }
        // compact the occupied slots (in slot order), reset the table
        int n = 0;
        for (int s0 = 0; s0 < a.ts; s0 += WAVE) {
            const int s = s0 + l;
            const bool occ = s < a.ts && keys[s] != -1;
            const unsigned long long bal = __ballot(occ);
            if (occ) {
                const int pos = n + mbcnt(bal);
                if (pos < a.ts / 2) {
                    sk[pos] = keys[s];
                    sv[pos] = vals[s];
                }
                keys[s] = -1;
                vals[s] = A::zero();
            }
            n += __popcll(bal);
        }
        const int64_t cb = a.coff[i];
        const bool ok = (a.coff[i + 1] - cb == n) && n <= a.ts / 2;
        if (l == 0 && !ok) atomicAdd(&a.st->mismatch, 1);
        int np = 1;
        while (np < n) np <<= 1;
        if (np > a.ts / 2) np = a.ts / 2;
        for (int p = n + l; p < np; p += WAVE) sk[p] = INT_MAX;
        wave_lds_sync();
        if (ok) {
            bitonic_lds(sk, sv, np, WAVE);
            for (int t = l; t < n; t += WAVE) {
                a.cci[cb - cbase + t] = sk[t];
                a.cval[cb - cbase + t] = A::fin(sv[t]);
            }
        }
        wave_lds_sync();
    }
}

// ============================================================ workgroup / row, two levels

struct HlLayout {
    size_t keys, vals, st_off, st_bs, red, misc, total;
};

__host__ __device__ inline HlLayout hl_layout(int l1, int acc_bytes) {
    HlLayout L{};
    size_t o = 0;
    L.keys = o;
    o += align16(4 * (size_t)l1);
    L.vals = o;
    o += align16((size_t)acc_bytes * l1);
    L.st_off = o;
    o += 8 * WG_BIG;
    L.st_bs = o;
    o += 8 * WG_BIG;
    L.red = o;
    o += 8 * (WG_BIG / WAVE + 2);
    L.misc = o;
    o += 16;
    L.total = o;
    return L;
}

__device__ __forceinline__ long long hl_block_excl_scan(long long v, long long *red, long long *total) {
    const int t = threadIdx.x, l = lane_id(), wv = t / WAVE;
    const long long inc = wave_incl_scan64(v);
    __syncthreads();
    if (l == WAVE - 1) red[wv] = inc;
    __syncthreads();
    long long off = 0, tot = 0;
#pragma unroll
    for (int u = 0; u < WG_BIG / WAVE; ++u) {
        const long long x = red[u];
        if (u < wv) off += x;
        tot += x;
    }
    *total = tot;
    return off + inc - v;
}

template <typename F>
__device__ __forceinline__ void hl_flat(int64_t ab, int64_t ae, const int32_t *aci, const int64_t *rp,
                                        int64_t *st_off, int64_t *st_bs, long long *red, F &&body) {
    const int t = threadIdx.x;
    for (int64_t cb = ab; cb < ae; cb += WG_BIG) {
        const int cn = (int)min((int64_t)WG_BIG, ae - cb);
        long long len = 0;
        if (t < cn) {
            const int j = aci[cb + t];
            const int64_t s0 = rp[j], s1 = rp[j + 1];
            st_bs[t] = s0;
            len = s1 - s0;
        }
        long long tot;
        const long long ex = hl_block_excl_scan(len, red, &tot);
        if (t < cn) st_off[t] = ex + len;
        __syncthreads();
        for (long long f = t; f < tot; f += WG_BIG) {
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

__device__ __forceinline__ int hl_next_row(const RowSet &rs, int64_t lo, int64_t hi, int &x, long long *red) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t t = xcd_grab(rs.queue, lo, hi, x);
        red[WG_BIG / WAVE] = t < 0 ? -1 : rs.rows[t];
        red[WG_BIG / WAVE + 1] = x;
    }
    __syncthreads();
    x = (int)red[WG_BIG / WAVE + 1];
    return (int)red[WG_BIG / WAVE];
}

// Level-2 (HBM) find-or-insert; cap2 is a power of two >= 2 * row bound, so a
// free slot always exists.  Keys are device-coherent atomics.
__device__ __forceinline__ uint32_t l2_find_or_insert(int32_t *keys2, uint32_t mask2, int32_t key) {
    uint32_t h = slot_of((uint32_t)key * 2654435761u, mask2);
    for (;;) {
        const int32_t k = __hip_atomic_load(&keys2[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == key) return h;
        if (k == -1) {
            const int32_t old = atomicCAS(&keys2[h], -1, key);
            if (old == -1 || old == key) return h;
        }
        h = (h + 1) & mask2;
    }
}

// Level-1 find-or-insert with the occupancy cut-off; returns -1 if the key
// must go to level 2.  Probing stops after l1 slots, so it always ends.
__device__ __forceinline__ int l1_find_or_insert(int32_t *keys, uint32_t mask, int32_t key, int *used, int cap) {
    uint32_t h = slot_of((uint32_t)key, mask);
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        const int32_t k = keys[h];
        if (k == key) return (int)h;
        if (k == -1) {
            if (*(volatile int *)used >= cap) return -1;
            const int32_t old = atomicCAS(&keys[h], -1, key);
            if (old == -1) {
                atomicAdd(used, 1);
                return (int)h;
            }
            if (old == key) return (int)h;
        }
        h = (h + 1) & mask;
    }
    return -1;
}

__global__ __launch_bounds__(WG_BIG) void k_sym_hl(SymArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int l1 = a.l1_slots;
    const HlLayout L = hl_layout(l1, 4);
    int32_t *keys = (int32_t *)(smem + L.keys);
    uint32_t *masks = (uint32_t *)(smem + L.vals);
    int64_t *st_off = (int64_t *)(smem + L.st_off);
    int64_t *st_bs = (int64_t *)(smem + L.st_bs);
    long long *red = (long long *)(smem + L.red);
    int *used = (int *)(smem + L.misc);
    int32_t *keys2 = (int32_t *)a.l2_keys + (int64_t)blockIdx.x * a.l2_cap;
    uint32_t *masks2 = a.l2_vals + (int64_t)blockIdx.x * a.l2_cap;
    const int t = threadIdx.x;
    const uint32_t mask = (uint32_t)l1 - 1;
    const int cap = l1 / 2;
    for (int s = t; s < l1; s += WG_BIG) {
        keys[s] = -1;
        masks[s] = 0;
    }
    const bool comp = a.bcrp != nullptr;
    int64_t lo, hi;
    rs_bounds(a.rs, lo, hi);
    int x = blockIdx.x % XCDS;
    for (;;) {
        const int i = hl_next_row(a.rs, lo, hi, x, red);
        if (i < 0) break;
        if (t == 0) *used = 0;
        // level-2 table size: power of two >= 2 * bound (bound from the analysis)
        const int2 win = a.rwin[i];
        const int64_t ab = a.arp[i], ae = a.arp[i + 1];
        __syncthreads();
        // row bound: distinct keys <= min(inserts, window keys)
        long long ins = 0;
        for (int64_t e = ab + t; e < ae; e += WG_BIG) {
            const int j = a.aci[e];
            ins += comp ? (a.bcrp[j + 1] - a.bcrp[j]) : (a.brp[j + 1] - a.brp[j]);
        }
        long long tot_ins;
        hl_block_excl_scan(ins, red, &tot_ins);
        const long long wkeys = comp ? ((long long)win.y - win.x + 1) : 32ll * ((long long)win.y - win.x + 1);
        const long long bound = min(tot_ins, wkeys);
        int64_t cap2 = 1;
        while (cap2 < 2 * bound) cap2 <<= 1;
        if (cap2 > a.l2_cap) {
            if (t == 0) {
                atomicAdd(&a.st->overflow, 1);
                a.row_nnz[i] = 0;
                a.row_words[i] = 0;
            }
            continue;
        }
        const uint32_t mask2 = (uint32_t)(cap2 - 1);
        for (int64_t s = t; s < cap2; s += WG_BIG) {
            keys2[s] = -1;
            masks2[s] = 0;
        }
        __threadfence();
        __syncthreads();
        hl_flat(ab, ae, a.aci, comp ? a.bcrp : a.brp, st_off, st_bs, red, [&](int, int64_t e, int64_t) {
            int32_t key;
            uint32_t cs;
            if (comp) {
                const uint2 v = a.bcw[e];
                key = (int)v.x;
                cs = v.y;
            } else {
                key = a.bci[e];
                cs = 1u;
            }
            const int h = l1_find_or_insert(keys, mask, key, used, cap);
            if (h >= 0)
                atomicOr(&masks[h], cs);
            else
                atomicOr(&masks2[l2_find_or_insert(keys2, mask2, key)], cs);
        });
        // merge level 1 into level 2, reset level 1
        for (int s = t; s < l1; s += WG_BIG) {
            const int32_t k = keys[s];
            if (k != -1) {
                atomicOr(&masks2[l2_find_or_insert(keys2, mask2, k)], masks[s]);
                keys[s] = -1;
                masks[s] = 0;
            }
        }
        __threadfence();
        __syncthreads();
        long long cnt = 0;
        for (int64_t s = t; s < cap2; s += WG_BIG) {
            if (__hip_atomic_load(&keys2[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != -1)
                cnt += __popc(__hip_atomic_load(&masks2[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) +
                       (1ll << 32);
        }
        long long tot;
        hl_block_excl_scan(cnt, red, &tot);
        if (t == 0) {
            const int rn = (int32_t)(tot & 0xffffffffll), occ = (int32_t)(tot >> 32);
            a.row_nnz[i] = rn;
            a.row_words[i] = comp ? occ : (int)min((long long)rn, (long long)win.y - win.x + 1);
        }
    }
}

template <typename VT, int ACC>
__global__ __launch_bounds__(WG_BIG) void k_num_hl(NumArgs<VT> a) {
    using A = Accum<VT, ACC>;
    using S = typename A::store_t;
    extern __shared__ __align__(16) unsigned char smem[];
    const int l1 = a.l1_slots;
    const HlLayout L = hl_layout(l1, sizeof(S));
    int32_t *keys = (int32_t *)(smem + L.keys);
    S *vals = (S *)(smem + L.vals);
    int64_t *st_off = (int64_t *)(smem + L.st_off);
    int64_t *st_bs = (int64_t *)(smem + L.st_bs);
    long long *red = (long long *)(smem + L.red);
    int *used = (int *)(smem + L.misc);
    // arena slice: keys2[cap] | vals2[cap] | sort keys[cap/2] | sort vals[cap/2]
    unsigned char *base = (unsigned char *)a.arena + (int64_t)blockIdx.x * a.arena_cap * (8 + 2 * sizeof(S));
    int32_t *keys2 = (int32_t *)base;
    S *vals2 = (S *)(base + 4 * a.arena_cap);
    int32_t *sk = (int32_t *)(base + (4 + sizeof(S)) * a.arena_cap);
    S *sv = (S *)(base + (4 + sizeof(S)) * a.arena_cap + 4 * (a.arena_cap / 2));
    const int t = threadIdx.x;
    const uint32_t mask = (uint32_t)l1 - 1;
    const int cap = l1 / 2;
    for (int s = t; s < l1; s += WG_BIG) {
        keys[s] = -1;
        vals[s] = A::zero();
    }
    int64_t lo, hi;
    rs_bounds(a.rs, lo, hi);
    const int64_t cbase = a.cbase_row >= 0 ? a.coff[a.cbase_row] : 0;
    int x = blockIdx.x % XCDS;
    for (;;) {
        const int i = hl_next_row(a.rs, lo, hi, x, red);
        if (i < 0) break;
        if (t == 0) *used = 0;
        const int64_t c0 = a.coff[i];
        const int64_t rn = a.coff[i + 1] - c0;
        int64_t cap2 = 1;
        while (cap2 < 2 * rn) cap2 <<= 1;
        if (cap2 > a.arena_cap) {
            if (t == 0) atomicAdd(&a.st->overflow, 1);
            continue;
        }
        const uint32_t mask2 = (uint32_t)(cap2 - 1);
        for (int64_t s = t; s < cap2; s += WG_BIG) {
            keys2[s] = -1;
            vals2[s] = A::zero();
        }
        __threadfence();
        __syncthreads();
        const int64_t ab = a.arp[i], ae = a.arp[i + 1];
        hl_flat(ab, ae, a.aci, a.brp, st_off, st_bs, red, [&](int k, int64_t e, int64_t cb) {
            const int32_t c = a.bci[e];
            const VT av = a.aval[cb + k], bv = a.bval[e];
            const int h = l1_find_or_insert(keys, mask, c, used, cap);
            if (h >= 0)
                A::add(&vals[h], av, bv);
            else
                A::add(&vals2[l2_find_or_insert(keys2, mask2, c)], av, bv);
        });
        // merge level 1 into level 2 as one more accumulation of each entry
        for (int s = t; s < l1; s += WG_BIG) {
            const int32_t k = keys[s];
            if (k != -1) {
                S *dst = &vals2[l2_find_or_insert(keys2, mask2, k)];
                if constexpr (ACC == ACC_COMP) {
                    // fold the (s, c) pair in as two compensated additions of value*1
                    const S v = vals[s];
                    A::add(dst, __uint_as_float((uint32_t)v), 1.0f);
                    A::add(dst, __uint_as_float((uint32_t)(v >> 32)), 1.0f);
                } else {
                    atomicAdd(dst, vals[s]);
                }
                keys[s] = -1;
                vals[s] = A::zero();
            }
        }
        __threadfence();
        __syncthreads();
        // compact level 2 into the sort buffer (slot order)
        long long run = 0;
        for (int64_t s0 = 0; s0 < cap2; s0 += WG_BIG) {
            const int64_t s = s0 + t;
            const int32_t k = s < cap2 ? __hip_atomic_load(&keys2[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : -1;
            long long tot;
            const long long ex = hl_block_excl_scan(k != -1 ? 1 : 0, red, &tot);
            if (k != -1 && run + ex < cap2 / 2) {
                sk[run + ex] = k;
                sv[run + ex] = __hip_atomic_load(&vals2[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            run += tot;
        }
        const bool ok = (run == rn);
        if (t == 0 && !ok) atomicAdd(&a.st->mismatch, 1);
        int64_t np = 1;
        while (np < run) np <<= 1;
        if (np > cap2 / 2) np = cap2 / 2;
        for (int64_t p = run + t; p < np; p += WG_BIG) sk[p] = INT_MAX;
        __threadfence();
        __syncthreads();
        if (ok) {
            // bitonic sort in HBM (rows here are the rare very large, very wide ones)
            for (int64_t k = 2; k <= np; k <<= 1) {
                for (int64_t j = k >> 1; j > 0; j >>= 1) {
                    for (int64_t p = t; p < (np >> 1); p += WG_BIG) {
                        const int64_t ii = ((p & ~(j - 1)) << 1) | (p & (j - 1));
                        const int64_t o = ii + j;
                        const bool up = (ii & k) == 0;
                        const int32_t ki = sk[ii], ko = sk[o];
                        if ((ki > ko) == up) {
                            sk[ii] = ko;
                            sk[o] = ki;
                            const S vi = sv[ii];
                            sv[ii] = sv[o];
                            sv[o] = vi;
                        }
                    }
                    __threadfence();
                    __syncthreads();
                }
            }
            for (int64_t p = t; p < rn; p += WG_BIG) {
                a.cci[c0 - cbase + p] = sk[p];
                a.cval[c0 - cbase + p] = A::fin(sv[p]);
            }
        }
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

size_t lds_sym_hw(int ts) { return hw_layout(ts, 4, false).total; }
size_t lds_num_hw(int ts, int acc_bytes) { return hw_layout(ts, acc_bytes, true).total; }
size_t lds_sym_hl(int l1) { return hl_layout(l1, 4).total; }
size_t lds_num_hl(int l1, int acc_bytes) { return hl_layout(l1, acc_bytes).total; }

hipError_t launch_sym_hw(const SymArgs &a, const LaunchCfg &c) {
    const size_t lds = lds_sym_hw(a.ts);
    const int grid = c.grid > 0 ? c.grid : resident_grid(k_sym_hw, WAVE, lds, c.cus);
    hipLaunchKernelGGL(k_sym_hw, dim3(grid), dim3(WAVE), lds, c.stream, a);
    return hipGetLastError();
}

hipError_t launch_sym_hl(const SymArgs &a, const LaunchCfg &c) {
    const size_t lds = lds_sym_hl(a.l1_slots);
    const int grid = c.grid;  // fixed by the arena slices
    hipLaunchKernelGGL(k_sym_hl, dim3(grid), dim3(WG_BIG), lds, c.stream, a);
    return hipGetLastError();
}

template <typename VT, int ACC>
static hipError_t num_hw_impl(const NumArgs<VT> &a, const LaunchCfg &c) {
    const size_t lds = lds_num_hw(a.ts, sizeof(typename Accum<VT, ACC>::store_t));
    const int grid = c.grid > 0 ? c.grid : resident_grid(k_num_hw<VT, ACC>, WAVE, lds, c.cus);
    hipLaunchKernelGGL((k_num_hw<VT, ACC>), dim3(grid), dim3(WAVE), lds, c.stream, a);
    return hipGetLastError();
}

template <typename VT, int ACC>
static hipError_t num_hl_impl(const NumArgs<VT> &a, const LaunchCfg &c) {
    const size_t lds = lds_num_hl(a.l1_slots, sizeof(typename Accum<VT, ACC>::store_t));
    hipLaunchKernelGGL((k_num_hl<VT, ACC>), dim3(c.grid), dim3(WG_BIG), lds, c.stream, a);
    return hipGetLastError();
}

template <>
hipError_t launch_num_hw<double>(const NumArgs<double> &a, int, const LaunchCfg &c) {
    return num_hw_impl<double, ACC_NATIVE>(a, c);
}
template <>
hipError_t launch_num_hw<float>(const NumArgs<float> &a, int acc, const LaunchCfg &c) {
    if (acc == ACC_COMP) return num_hw_impl<float, ACC_COMP>(a, c);
    if (acc == ACC_WIDE) return num_hw_impl<float, ACC_WIDE>(a, c);
    return num_hw_impl<float, ACC_NATIVE>(a, c);
}
template <>
hipError_t launch_num_hl<double>(const NumArgs<double> &a, int, const LaunchCfg &c) {
    return num_hl_impl<double, ACC_NATIVE>(a, c);
}
template <>
hipError_t launch_num_hl<float>(const NumArgs<float> &a, int acc, const LaunchCfg &c) {
    if (acc == ACC_COMP) return num_hl_impl<float, ACC_COMP>(a, c);
    if (acc == ACC_WIDE) return num_hl_impl<float, ACC_WIDE>(a, c);
    return num_hl_impl<float, ACC_NATIVE>(a, c);
}

int hl_resident_grid(int acc, bool dbl, size_t lds, int cus) {
    if (dbl) return resident_grid(k_num_hl<double, ACC_NATIVE>, WG_BIG, lds, cus);
    if (acc == ACC_COMP) return resident_grid(k_num_hl<float, ACC_COMP>, WG_BIG, lds, cus);
    if (acc == ACC_WIDE) return resident_grid(k_num_hl<float, ACC_WIDE>, WG_BIG, lds, cus);
    return resident_grid(k_num_hl<float, ACC_NATIVE>, WG_BIG, lds, cus);
}

}  // namespace spg
