// Masked product C = (A * B) on the pattern of a mask M, and its structural
// form (path counts): the graph-analytics use of SpGEMM the paper names in
// its Background section (triangle counting works on the structure of
// L * L restricted to L, Compression subsection).  No symbolic phase is
// needed: C's structure is M's.
//
// Rows of M with at most MW_MAX entries: one wavefront per row.  M's row
// goes into an LDS linear-probing table (column -> position in M's row, at
// most 50% occupancy); the row's products are formed as in the other
// wavefront kernels (Thread-Parallel groups of lanes per B row) and each one
// whose column is in the table is added at its position in an LDS row of
// FP64 accumulators (FP32 inputs accumulate in FP64: the products of two FP32
// numbers are exact there).  Longer mask rows: one 256-lane workgroup per
// row with the table and the accumulators in a slice of an HBM arena.
#include "spg_accum.hpp"
#include "spg_internal.hpp"

namespace spg {

namespace {

constexpr int MK_CB = 256;

__device__ __forceinline__ uint32_t mk_hash(int c, uint32_t lg) {
    return ((uint32_t)c * 0x9E3779B1u) >> (32 - lg);
}

template <typename VT>
__device__ __forceinline__ double mk_term(VT a, VT b, int structural) {
    return structural ? 1.0 : (double)a * (double)b;
}

// LP insert of key c at position pos into keys/posv (size 2^lg); returns the slot.
__device__ __forceinline__ int mk_insert(int *keys, int *posv, uint32_t lg, int c, int pos) {
    const uint32_t mask = (1u << lg) - 1u;
    uint32_t s = mk_hash(c, lg);
    for (;;) {
        const int prev = atomicCAS(&keys[s], -1, c);
        if (prev == -1 || prev == c) {
            posv[s] = pos;
            return (int)s;
        }
        s = (s + 1) & mask;
    }
}

__device__ __forceinline__ int mk_find(const int *keys, const int *posv, uint32_t lg, int c) {
    const uint32_t mask = (1u << lg) - 1u;
    uint32_t s = mk_hash(c, lg);
    for (;;) {
        const int k = keys[s];
        if (k == c) return posv[s];
        if (k == -1) return -1;
        s = (s + 1) & mask;
    }
}

struct MkLayout {
    size_t b0, a, len, keys, posv, slotof, acc, total;
};
__host__ __device__ inline MkLayout mk_layout(int lg, int mmax) {
    MkLayout L{};
    L.b0 = 0;
    L.a = 8 * WAVE;
    L.len = 16 * WAVE;
    size_t o = 20 * WAVE;
    L.keys = o;
    o += 4 * ((size_t)1 << lg);
    L.posv = o;
    o += 4 * ((size_t)1 << lg);
    L.slotof = o;
    o += align16(4 * (size_t)mmax);
    L.acc = o;
    o += 8 * (size_t)mmax;
    L.total = o;
    return L;
}

template <typename VT>
__global__ __launch_bounds__(WAVE) void k_mask_w(MaskArgs<VT> a, int lg, int mmax) {
    extern __shared__ __align__(16) unsigned char smem[];
    const MkLayout L = mk_layout(lg, mmax);
    int64_t *st_b0 = (int64_t *)(smem + L.b0);
    double *st_a = (double *)(smem + L.a);
    int *st_len = (int *)(smem + L.len);
    int *keys = (int *)(smem + L.keys), *posv = (int *)(smem + L.posv), *slotof = (int *)(smem + L.slotof);
    double *acc = (double *)(smem + L.acc);
    const int l = lane_id(), ts = 1 << lg;
    for (int s = l; s < ts; s += WAVE) keys[s] = -1;
    for (int t = l; t < mmax; t += WAVE) acc[t] = 0.0;
    const int gs = 1 << a.lg_gs, g = l >> a.lg_gs, q = l & (gs - 1), ng = WAVE >> a.lg_gs;
    int badc = 0;
    wave_lds_sync();
    const Slice sl = xcd_slice(0, a.nrows);
    for (int64_t r = sl.idx; r < sl.end; r += sl.step) {
        const int i = a.rows[r];
        const int64_t mb = a.mrp[i], ml = a.mrp[i + 1] - mb;
        const int64_t ab = a.arp[i], ae = a.arp[i + 1];
        for (int t = l; t < ml; t += WAVE) {
            const int c = a.mci[mb + t];
            const bool okc = c >= 0 && c < a.k;
            badc |= !okc;
            slotof[t] = okc ? mk_insert(keys, posv, lg, c, t) : -1;
        }
        wave_lds_sync();
        for (int64_t c0 = ab; c0 < ae; c0 += WAVE) {
            const int cn = (int)min((int64_t)WAVE, ae - c0);
            if (l < cn) {
                const int j = a.aci[c0 + l];
                const bool okj = j >= 0 && j < a.n;
                badc |= !okj;
                const int64_t b0 = okj ? a.brp[j] : 0;
                st_b0[l] = b0;
                st_len[l] = okj ? (int)(a.brp[j + 1] - b0) : 0;
                st_a[l] = a.aval ? (double)a.aval[c0 + l] : 0.0;
            }
            wave_lds_sync();
            for (int t = g; t < cn; t += ng) {
                const int64_t bs = st_b0[t];
                const int len = st_len[t];
                const VT av = (VT)st_a[t];
                for (int p = q; p < len; p += gs) {
                    const int c = a.bci[bs + p];
                    const int pos = mk_find(keys, posv, lg, c);
                    if (pos >= 0) atomicAdd(&acc[pos], mk_term<VT>(av, a.bval ? a.bval[bs + p] : VT(0), a.structural));
                }
            }
            wave_lds_sync();
        }
        for (int t = l; t < ml; t += WAVE) {
            a.out[mb + t] = (VT)acc[t];
            acc[t] = 0.0;
            if (slotof[t] >= 0) keys[slotof[t]] = -1;
        }
        wave_lds_sync();
    }
    if (__ballot(badc) && l == 0) atomicOr(a.bad, 1);
}

// One heavy mask row per 256-lane workgroup; table (keys, positions) and FP64
// accumulators in this workgroup's arena slice: keys[cap] | posv[cap] | acc[cap / 2].
template <typename VT>
__global__ __launch_bounds__(MK_CB) void k_mask_g(MaskArgs<VT> a) {
    __shared__ int64_t st_b0[MK_CB];
    __shared__ double st_a[MK_CB];
    __shared__ int st_len[MK_CB];
    const int t = threadIdx.x, l = lane_id(), wv = t / WAVE;
    unsigned char *base = (unsigned char *)a.arena + (size_t)blockIdx.x * (size_t)a.arena_cap * 12;
    int *keys = (int *)base, *posv = (int *)(base + 4 * a.arena_cap);
    double *acc = (double *)(base + 8 * a.arena_cap);
    for (int64_t s = t; s < a.arena_cap; s += MK_CB) keys[s] = -1;
    for (int64_t s = t; s < a.arena_cap / 2; s += MK_CB) acc[s] = 0.0;
    __syncthreads();
    const int gs = 1 << a.lg_gs, g = l >> a.lg_gs, q = l & (gs - 1), ng = WAVE >> a.lg_gs;
    int badc = 0;
    for (int64_t r = blockIdx.x; r < a.nrows; r += gridDim.x) {
        const int i = a.rows[r];
        const int64_t mb = a.mrp[i], ml = a.mrp[i + 1] - mb;
        const int64_t ab = a.arp[i], ae = a.arp[i + 1];
        uint32_t lg = 4;
        while (((int64_t)1 << lg) < 2 * ml) ++lg;
        if (((int64_t)1 << lg) > a.arena_cap) {  // sized by the launch's longest mask row: cannot happen
            if (t == 0) atomicOr(a.bad, 2);
            continue;
        }
        for (int64_t e = t; e < ml; e += MK_CB) {
            const int c = a.mci[mb + e];
            const bool okc = c >= 0 && c < a.k;
            badc |= !okc;
            if (okc) mk_insert(keys, posv, lg, c, (int)e);
        }
        __syncthreads();
        for (int64_t c0 = ab; c0 < ae; c0 += MK_CB) {
            const int cn = (int)min((int64_t)MK_CB, ae - c0);
            if (t < cn) {
                const int j = a.aci[c0 + t];
                const bool okj = j >= 0 && j < a.n;
                badc |= !okj;
                const int64_t b0 = okj ? a.brp[j] : 0;
                st_b0[t] = b0;
                st_len[t] = okj ? (int)(a.brp[j + 1] - b0) : 0;
                st_a[t] = a.aval ? (double)a.aval[c0 + t] : 0.0;
            }
            __syncthreads();
            // wavefront wv takes staged entries wv*ng + g, then every 4*ng-th
            for (int u = wv * ng + g; u < cn; u += (MK_CB / WAVE) * ng) {
                const int64_t bs = st_b0[u];
                const int len = st_len[u];
                const VT av = (VT)st_a[u];
                for (int p = q; p < len; p += gs) {
                    const int c = a.bci[bs + p];
                    const int pos = mk_find(keys, posv, lg, c);
                    if (pos >= 0) atomicAdd(&acc[pos], mk_term<VT>(av, a.bval ? a.bval[bs + p] : VT(0), a.structural));
                }
            }
            __syncthreads();
        }
        for (int64_t e = t; e < ml; e += MK_CB) {
            a.out[mb + e] = (VT)acc[e];
            acc[e] = 0.0;
        }
        for (int64_t s = t; s < ((int64_t)1 << lg); s += MK_CB) keys[s] = -1;
        __syncthreads();
    }
    if (__ballot(badc) && l == 0) atomicOr(a.bad, 1);
}

// Rows by mask length: kind 1 (wavefront) 0 < len <= mw_max, kind 2
// (workgroup) beyond; rows with an empty mask row or an empty A row need no
// kernel (their outputs are zero-filled).  Per workgroup: counts by ballot,
// one atomic per kind for the base; longest mask row per kind.
__global__ __launch_bounds__(MK_CB) void k_mask_class(int64_t m, const int64_t *arp, const int64_t *mrp, int mw_max,
                                                      int32_t *rows1, int32_t *rows2, int *cnt) {
    __shared__ int sc[2], sb[2], smx[2];
    const int t = threadIdx.x;
    if (t < 2) {
        sc[t] = 0;
        smx[t] = 0;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * MK_CB + t;
    int k = 0, ml = 0;
    if (i < m) {
        const int64_t len = mrp[i + 1] - mrp[i];
        ml = (int)min(len, (int64_t)INT_MAX);
        if (len > 0 && arp[i + 1] > arp[i]) k = len <= mw_max ? 1 : 2;
    }
    int my = 0;
    if (k) {
        my = atomicAdd(&sc[k - 1], 1);
        atomicMax(&smx[k - 1], ml);
    }
    __syncthreads();
    if (t < 2) {
        sb[t] = sc[t] ? atomicAdd(&cnt[t], sc[t]) : 0;
        if (smx[t]) atomicMax(&cnt[2 + t], smx[t]);
    }
    __syncthreads();
    if (k == 1) rows1[sb[0] + my] = (int32_t)i;
    if (k == 2) rows2[sb[1] + my] = (int32_t)i;
}

template <typename K>
inline int resident(K kernel, int block, size_t lds, int cus) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int g = (per_cu * cus / XCDS) * XCDS;
    return g < XCDS ? XCDS : g;
}

}  // namespace

size_t lds_mask_w(int lg, int mmax) { return mk_layout(lg, mmax).total; }

hipError_t launch_mask_class(int64_t m, const int64_t *arp, const int64_t *mrp, int mw_max, int32_t *rows1,
                             int32_t *rows2, int *cnt, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mask_class, dim3((unsigned)((m + MK_CB - 1) / MK_CB)), dim3(MK_CB), 0, s, m, arp, mrp, mw_max,
                       rows1, rows2, cnt);
    return hipGetLastError();
}

template <typename VT>
hipError_t launch_mask_w(const MaskArgs<VT> &a, int lg, int mmax, const LaunchCfg &c) {
    const size_t lds = mk_layout(lg, mmax).total;
    int grid = resident(k_mask_w<VT>, WAVE, lds, c.cus);
    grid = (int)std::min<int64_t>(grid, std::max<int64_t>(XCDS, ((a.nrows + XCDS - 1) / XCDS) * XCDS));
    hipLaunchKernelGGL(k_mask_w<VT>, dim3(grid), dim3(WAVE), lds, c.stream, a, lg, mmax);
    return hipGetLastError();
}

template <typename VT>
hipError_t launch_mask_g(const MaskArgs<VT> &a, const LaunchCfg &c) {
    hipLaunchKernelGGL(k_mask_g<VT>, dim3(c.grid), dim3(MK_CB), 0, c.stream, a);
    return hipGetLastError();
}

template hipError_t launch_mask_w<double>(const MaskArgs<double> &, int, int, const LaunchCfg &);
template hipError_t launch_mask_w<float>(const MaskArgs<float> &, int, int, const LaunchCfg &);
template hipError_t launch_mask_g<double>(const MaskArgs<double> &, const LaunchCfg &);
template hipError_t launch_mask_g<float>(const MaskArgs<float> &, const LaunchCfg &);

}  // namespace spg
