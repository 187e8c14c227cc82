// Accumulator arithmetic shared by the numeric kernels.
//
// Three forms of "C(i,j) += A(i,k) * B(k,j)":
//   ACC_NATIVE: product and sum in the value type (FP64 for the plain method,
//               FP32 for the single-precision form); hardware atomic add.
//   ACC_COMP:   FP32 values, compensated pair (s, c) per entry: TwoProduct of
//               the operands (exact error by fused multiply-add), TwoSum into s,
//               both errors into c; the pair is one 64-bit word updated by
//               compare-and-swap.  Result s + c (Ogita, Rump, Oishi, "Accurate
//               sum and dot product", 2005, algorithm Dot2).
//   ACC_WIDE:   FP32 values, FP64 accumulation (the product of two FP32 numbers
//               is exact in FP64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spg {

enum { ACC_NATIVE = 0, ACC_COMP = 1, ACC_WIDE = 2 };

template <typename VT, int ACC>
struct Accum;

template <typename VT>
struct Accum<VT, ACC_NATIVE> {
    using store_t = VT;
    static __device__ __forceinline__ void add(store_t *p, VT a, VT b) { atomicAdd(p, a * b); }
    static __device__ __forceinline__ VT fin(store_t v) { return v; }
    static __device__ __forceinline__ store_t zero() { return VT(0); }
};

template <>
struct Accum<float, ACC_WIDE> {
    using store_t = double;
    static __device__ __forceinline__ void add(store_t *p, float a, float b) {
        atomicAdd(p, (double)a * (double)b);
    }
    static __device__ __forceinline__ float fin(store_t v) { return (float)v; }
    static __device__ __forceinline__ store_t zero() { return 0.0; }
};

template <>
struct Accum<float, ACC_COMP> {
    using store_t = unsigned long long;  // low word s, high word c
    static __device__ __forceinline__ void add(store_t *p, float a, float b) {
        const float x = a * b;
        const float ex = __builtin_fmaf(a, b, -x);  // a*b == x + ex exactly
        store_t old = *(volatile store_t *)p, assumed;
        do {
            assumed = old;
            const float s = __uint_as_float((uint32_t)assumed);
            const float c = __uint_as_float((uint32_t)(assumed >> 32));
            const float s2 = s + x;  // TwoSum(s, x) = (s2, e), s + x == s2 + e exactly
            const float bv = s2 - s;
            const float e = (s - (s2 - bv)) + (x - bv);
            const float c2 = c + (e + ex);
            const store_t nv = (store_t)__float_as_uint(s2) | ((store_t)__float_as_uint(c2) << 32);
            old = atomicCAS(p, assumed, nv);
        } while (old != assumed);
    }
    static __device__ __forceinline__ float fin(store_t v) {
        return __uint_as_float((uint32_t)v) + __uint_as_float((uint32_t)(v >> 32));
    }
    static __device__ __forceinline__ store_t zero() { return 0ull; }
};

__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

}  // namespace spg
