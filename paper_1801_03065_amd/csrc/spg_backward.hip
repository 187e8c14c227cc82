// Backward of C = A * B restricted to the stored entries of A and B.
//
// For L with dL/dC = G on pattern(C), each multiplication (i, k, j) of the
// numeric phase (A(i,k) and B(k,j) stored) contributes
//     dA(i,k) += G(i,j) * B(k,j)        dB(k,j) += A(i,k) * G(i,j)
// so dA = (G * B^T) masked to pattern(A) and dB = (A^T * G) masked to
// pattern(B).  The kernel walks the same multiplications as the numeric phase
// (Gustavson rows of A, Thread-Parallel lane groups over B rows), finds
// G(i,j) by binary search in the sorted row i of C (staged in LDS when it
// fits), reduces dA(i,k) inside the lane group (no atomics) and adds dB(k,j)
// with hardware floating-point atomics in HBM.
#include "spg_accum.hpp"
#include "spg_internal.hpp"

namespace spg {

namespace {

constexpr int BW_LDS = 4096;  // C row entries staged in LDS

template <typename VT>
__global__ __launch_bounds__(WAVE) void k_bwd(BwdArgs<VT> a) {
    __shared__ int32_t ccol[BW_LDS];
    __shared__ int64_t st_bs[WAVE];
    __shared__ int32_t st_len[WAVE];
    __shared__ double st_a[WAVE];
    const int l = lane_id();
    const int gs = 1 << a.lg_gs, g = l >> a.lg_gs, q = l & (gs - 1), ng = WAVE >> a.lg_gs;
    const Slice sl = xcd_slice(0, a.m);
    for (int64_t r = sl.idx; r < sl.end; r += sl.step) {
        const int i = (int)r;
        const int64_t ab = a.arp[i], ae = a.arp[i + 1];
        if (ab == ae) continue;
        const int64_t cb = a.coff[i], ce = a.coff[i + 1];
        const int rn = (int)(ce - cb);
        const bool in_lds = rn <= BW_LDS;
        if (in_lds)
            for (int t = l; t < rn; t += WAVE) ccol[t] = a.gci[cb + t];
        const int32_t *row = in_lds ? ccol : a.gci + cb;
        for (int64_t c0 = ab; c0 < ae; c0 += WAVE) {
            const int cn = (int)min((int64_t)WAVE, ae - c0);
            if (l < cn) {
                const int j = a.aci[c0 + l];
                const int64_t b0 = a.brp[j], b1 = a.brp[j + 1];
                st_bs[l] = b0;
                st_len[l] = (int32_t)(b1 - b0);
                st_a[l] = (double)a.aval[c0 + l];
            }
            wave_lds_sync();
            // every group runs the same number of rounds, so the group-wide
            // reduction below always sees all its lanes
            const int rounds = (cn + ng - 1) / ng;
            for (int k = 0; k < rounds; ++k) {
                const int t = g + k * ng;
                const bool have = t < cn;
                const int len = have ? st_len[t] : 0;
                const int64_t bs = have ? st_bs[t] : 0;
                const VT av = have ? (VT)st_a[t] : VT(0);
                VT s = VT(0);
                for (int p = q; p < len; p += gs) {
                    const int col = a.bci[bs + p];
                    int lo = 0, hi = rn - 1;  // first position with row[pos] >= col
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (row[mid] < col) lo = mid + 1; else hi = mid;
                    }
                    if (row[lo] != col) {
                        atomicAdd(&a.st->mismatch, 1);
                        continue;
                    }
                    const VT gv = a.gval[cb + lo];
                    s += gv * a.bval[bs + p];
                    if (a.dB) atomicAdd(&a.dB[bs + p], av * gv);
                }
                for (int d = gs >> 1; d >= 1; d >>= 1) s += __shfl_xor(s, d, gs);
                if (have && q == 0 && a.dA) a.dA[c0 + t] = s;
            }
            wave_lds_sync();
        }
    }
}

template <typename VT>
__global__ void k_zero(VT *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = VT(0);
}

template <typename VT>
hipError_t bwd_impl(const BwdArgs<VT> &a, const LaunchCfg &c) {
    if (a.dB && a.nnzb > 0) {
        const int64_t blocks = std::min<int64_t>((a.nnzb + 255) / 256, 8192);
        hipLaunchKernelGGL(k_zero<VT>, dim3((unsigned)blocks), dim3(256), 0, c.stream, a.dB, a.nnzb);
    }
    if (a.dA && a.nnza > 0) {
        const int64_t blocks = std::min<int64_t>((a.nnza + 255) / 256, 8192);
        hipLaunchKernelGGL(k_zero<VT>, dim3((unsigned)blocks), dim3(256), 0, c.stream, a.dA, a.nnza);
    }
    if (a.m == 0) return hipGetLastError();
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bwd<VT>, WAVE, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int grid = ((per_cu * c.cus) / XCDS) * XCDS;
    if (grid < XCDS) grid = XCDS;
    hipLaunchKernelGGL(k_bwd<VT>, dim3(grid), dim3(WAVE), 0, c.stream, a);
    return hipGetLastError();
}

}  // namespace

template <>
hipError_t launch_backward<double>(const BwdArgs<double> &a, const LaunchCfg &c) {
    return bwd_impl<double>(a, c);
}
template <>
hipError_t launch_backward<float>(const BwdArgs<float> &a, const LaunchCfg &c) {
    return bwd_impl<float>(a, c);
}

}  // namespace spg
