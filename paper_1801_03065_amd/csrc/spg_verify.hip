// Structure fingerprint of a product's operands: a 64-bit digest of A's and
// B's row pointers and column indices, taken at the symbolic phase and
// checked again before a numeric (or backward) call when the handle asks for
// it.  The numeric phase reuses the symbolic phase's structure (the reuse
// case of the paper's two-phase method), so a structure changed in place
// behind unchanged pointers and sizes would otherwise give silently wrong
// values.  The digest is a sum (mod 2^64) of a mixed hash of (array, index,
// value) per element, so it is order-free to reduce and any single changed
// element changes it.
#include "spg_internal.hpp"

namespace spg {

namespace {

constexpr int VB = 256;
constexpr int VGRID = 1024;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

struct HashArr {
    const void *p;
    int64_t n;
    int is64;
};

__device__ __forceinline__ uint64_t elem_hash(const HashArr &a, int id, int64_t i) {
    const uint64_t v = a.is64 ? (uint64_t)((const int64_t *)a.p)[i] : (uint64_t)(uint32_t)((const int32_t *)a.p)[i];
    return mix64(((uint64_t)id << 60) ^ ((uint64_t)i * 0x9E3779B97F4A7C15ull) ^ mix64(v + (uint64_t)id));
}

__global__ __launch_bounds__(VB) void k_hash_part(HashArr a0, HashArr a1, HashArr a2, HashArr a3,
                                                   unsigned long long *part) {
    __shared__ unsigned long long ws[VB / WAVE];
    uint64_t s = 0;
    const int64_t stride = (int64_t)gridDim.x * VB;
    const int64_t t0 = (int64_t)blockIdx.x * VB + threadIdx.x;
    for (int64_t i = t0; i < a0.n; i += stride) s += elem_hash(a0, 0, i);
    for (int64_t i = t0; i < a1.n; i += stride) s += elem_hash(a1, 1, i);
    for (int64_t i = t0; i < a2.n; i += stride) s += elem_hash(a2, 2, i);
    for (int64_t i = t0; i < a3.n; i += stride) s += elem_hash(a3, 3, i);
    s = (uint64_t)wave_sum64((long long)s);
    if (lane_id() == 0) ws[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < VB / WAVE; ++w) t += ws[w];
        part[blockIdx.x] = t;
    }
}

// mode 0: store the digest in *ref; mode 1: compare with *ref and count a
// mismatch.
__global__ __launch_bounds__(VB) void k_hash_fin(int nb, const unsigned long long *part,
                                                  unsigned long long *ref, int mode, int *mismatch) {
    __shared__ unsigned long long ws[VB / WAVE];
    uint64_t s = 0;
    for (int i = threadIdx.x; i < nb; i += VB) s += part[i];
    s = (uint64_t)wave_sum64((long long)s);
    if (lane_id() == 0) ws[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < VB / WAVE; ++w) t += ws[w];
        if (mode == 0)
            *ref = t;
        else if (*ref != t)
            atomicAdd(mismatch, 1);
    }
}

}  // namespace

hipError_t launch_struct_digest(const StructRef &s, unsigned long long *part, unsigned long long *ref, int check,
                                int *mismatch, hipStream_t st) {
    const HashArr a0{s.arp, s.m + 1, s.arp64}, a1{s.aci, s.nnza, 0}, a2{s.brp, s.n + 1, s.brp64},
        a3{s.bci, s.nnzb, 0};
    const int64_t most = std::max(std::max(a0.n, a1.n), std::max(a2.n, a3.n));
    int g = (int)std::min<int64_t>(VGRID, std::max<int64_t>(1, (most + 8 * VB - 1) / (8 * VB)));
    hipLaunchKernelGGL(k_hash_part, dim3(g), dim3(VB), 0, st, a0, a1, a2, a3, part);
    hipLaunchKernelGGL(k_hash_fin, dim3(1), dim3(VB), 0, st, g, (const unsigned long long *)part, ref, check,
                       mismatch);
    return hipGetLastError();
}

}  // namespace spg
