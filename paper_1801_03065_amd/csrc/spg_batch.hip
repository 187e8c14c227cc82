// Batch support: many independent products C_i = A_i * B_i run as one
// block-diagonal product diag(A_i) * diag(B_i) = diag(C_i).  The structure of
// the batch is concatenated once (symbolic phase): rows of A_i follow each
// other, A_i's column j becomes row (B offset of i) + j of the stacked B, and
// B_i keeps its own (local) columns, so every row of the stacked product is a
// row of its own C_i with local column indices.  All the kernels of the single
// product then serve the batch unchanged: one persistent launch per row kind
// over the rows of every product, with a work queue that is binned by flops.
#include "spg_internal.hpp"

namespace spg {

namespace {

constexpr int BB = 256;

__global__ __launch_bounds__(BB) void k_batch_struct(const BatchDesc *d, int64_t *dst_rp, int32_t *dst_ci,
                                                     int *bad) {
    const BatchDesc m = d[blockIdx.y];
    const int64_t n1 = m.nrows + 1;
    for (int64_t r = (int64_t)blockIdx.x * BB + threadIdx.x; r < n1; r += (int64_t)gridDim.x * BB) {
        const int64_t v = m.rp64 ? ((const int64_t *)m.rp)[r] : (int64_t)((const int32_t *)m.rp)[r];
        dst_rp[m.row_off + r] = v + m.nnz_off;
        if ((r == 0 && v != 0) || (r == n1 - 1 && v != m.nnz)) atomicOr(bad, 1);
        if (r > 0) {
            const int64_t p = m.rp64 ? ((const int64_t *)m.rp)[r - 1] : (int64_t)((const int32_t *)m.rp)[r - 1];
            if (v < p) atomicOr(bad, 1);
        }
    }
    int b = 0;
    for (int64_t e = (int64_t)blockIdx.x * BB + threadIdx.x; e < m.nnz; e += (int64_t)gridDim.x * BB) {
        const int32_t c = m.ci[e];
        b |= (c < 0) | ((int64_t)c >= m.ncols);
        dst_ci[m.nnz_off + e] = c + m.col_add;
    }
    if (b) atomicOr(bad, 1);
}

template <typename T>
__global__ __launch_bounds__(BB) void k_batch_gather(const BatchDesc *d, T *dst) {
    const BatchDesc m = d[blockIdx.y];
    const T *src = (const T *)m.vals;
    for (int64_t e = (int64_t)blockIdx.x * BB + threadIdx.x; e < m.nnz; e += (int64_t)gridDim.x * BB)
        dst[m.nnz_off + e] = src[e];
}

template <typename T>
__global__ __launch_bounds__(BB) void k_batch_scatter(const BatchDesc *d, const T *src) {
    const BatchDesc m = d[blockIdx.y];
    T *dst = (T *)m.vals;
    for (int64_t e = (int64_t)blockIdx.x * BB + threadIdx.x; e < m.nnz; e += (int64_t)gridDim.x * BB)
        dst[e] = src[m.nnz_off + e];
}

// C_i.row_ptr[r] = coff[row_off_i + r] - coff[row_off_i]
__global__ __launch_bounds__(BB) void k_batch_rp_out(const BatchDesc *d, const int64_t *coff) {
    const BatchDesc m = d[blockIdx.y];
    const int64_t base = coff[m.row_off];
    for (int64_t r = (int64_t)blockIdx.x * BB + threadIdx.x; r <= m.nrows; r += (int64_t)gridDim.x * BB) {
        const int64_t v = coff[m.row_off + r] - base;
        if (m.rp64)
            ((int64_t *)m.rp)[r] = v;
        else
            ((int32_t *)m.rp)[r] = (int32_t)v;
    }
}

__global__ __launch_bounds__(BB) void k_batch_bounds(const BatchDesc *d, int count, const int64_t *coff,
                                                     int64_t *out) {
    for (int i = blockIdx.x * BB + threadIdx.x; i < count; i += gridDim.x * BB) {
        out[2 * i] = coff[d[i].row_off];
        out[2 * i + 1] = coff[d[i].row_off + d[i].nrows];
    }
}

__global__ __launch_bounds__(BB) void k_batch_row_class(const BatchDesc *d, uint8_t *row_cls) {
    const BatchDesc m = d[blockIdx.y];
    for (int64_t r = (int64_t)blockIdx.x * BB + threadIdx.x; r < m.nrows; r += (int64_t)gridDim.x * BB)
        row_cls[m.row_off + r] = (uint8_t)m.cls;
}

__global__ __launch_bounds__(BB) void k_kind_merge(int64_t m, const uint8_t *row_cls, const uint8_t *kind_cls,
                                                   uint8_t *kind) {
    for (int64_t i = (int64_t)blockIdx.x * BB + threadIdx.x; i < m; i += (int64_t)gridDim.x * BB)
        kind[i] = kind_cls[(int64_t)row_cls[i] * m + i];
}

inline dim3 batch_grid(int64_t max_work, int count) {
    int64_t gx = (max_work + BB - 1) / BB;
    gx = gx < 1 ? 1 : (gx > 64 ? 64 : gx);
    return dim3((unsigned)gx, (unsigned)count);
}

}  // namespace

hipError_t launch_batch_struct(const BatchDesc *d, int count, int64_t max_work, int64_t *dst_rp, int32_t *dst_ci,
                               int *bad, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_struct, batch_grid(max_work, count), dim3(BB), 0, s, d, dst_rp, dst_ci, bad);
    return hipGetLastError();
}

hipError_t launch_batch_gather(const BatchDesc *d, int count, int64_t max_nnz, void *dst, int bytes,
                               hipStream_t s) {
    if (count == 0) return hipSuccess;
    if (bytes == 8)
        hipLaunchKernelGGL(k_batch_gather<double>, batch_grid(max_nnz, count), dim3(BB), 0, s, d, (double *)dst);
    else
        hipLaunchKernelGGL(k_batch_gather<float>, batch_grid(max_nnz, count), dim3(BB), 0, s, d, (float *)dst);
    return hipGetLastError();
}

hipError_t launch_batch_scatter(const BatchDesc *d, int count, int64_t max_nnz, const void *src, int bytes,
                                hipStream_t s) {
    if (count == 0) return hipSuccess;
    if (bytes == 8)
        hipLaunchKernelGGL(k_batch_scatter<double>, batch_grid(max_nnz, count), dim3(BB), 0, s, d,
                           (const double *)src);
    else if (bytes == 4)
        hipLaunchKernelGGL(k_batch_scatter<float>, batch_grid(max_nnz, count), dim3(BB), 0, s, d,
                           (const float *)src);
    return hipGetLastError();
}

hipError_t launch_batch_rp_out(const BatchDesc *d, int count, int64_t max_rows, const int64_t *coff,
                               hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_rp_out, batch_grid(max_rows + 1, count), dim3(BB), 0, s, d, coff);
    return hipGetLastError();
}

hipError_t launch_batch_bounds(const BatchDesc *d, int count, const int64_t *coff, int64_t *out, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_bounds, dim3((count + BB - 1) / BB), dim3(BB), 0, s, d, count, coff, out);
    return hipGetLastError();
}

hipError_t launch_batch_row_class(const BatchDesc *d, int count, int64_t max_rows, uint8_t *row_cls, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_row_class, batch_grid(max_rows, count), dim3(BB), 0, s, d, row_cls);
    return hipGetLastError();
}

hipError_t launch_kind_merge(int64_t m, const uint8_t *row_cls, const uint8_t *kind_cls, uint8_t *kind, hipStream_t s) {
    if (m == 0) return hipSuccess;
    const int64_t g = std::min<int64_t>(4096, (m + BB - 1) / BB);
    hipLaunchKernelGGL(k_kind_merge, dim3((unsigned)g), dim3(BB), 0, s, m, row_cls, kind_cls, kind);
    return hipGetLastError();
}

}  // namespace spg
