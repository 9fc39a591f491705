// Level-1 vector kernels: inner products with FP64 accumulation and a fixed
// reduction order (grid-stride partial sums per workgroup, then one workgroup
// sums the partials in index order), so results are reproducible run to run.
#include "solver.h"

namespace hdcr {

namespace {

template <typename T>
__global__ void __launch_bounds__(REDUCE_THREADS) dot_partial_kernel(int64_t n, const C2<T>* __restrict__ x,
                                                                     const C2<T>* __restrict__ y,
                                                                     double2* __restrict__ partials) {
    double v[2] = {0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const C2<T> a = x[i];
        const C2<T> b = y[i];
        v[0] += (double)a.x * (double)b.x + (double)a.y * (double)b.y;
        v[1] += (double)a.x * (double)b.y - (double)a.y * (double)b.x;
    }
    block_reduce<2>(v);
    if (threadIdx.x == 0) partials[blockIdx.x] = make_double2(v[0], v[1]);
}

__global__ void __launch_bounds__(REDUCE_THREADS) finalize_kernel(const double2* __restrict__ partials, int np,
                                                                  double2* __restrict__ result) {
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        v[0] += partials[i].x;
        v[1] += partials[i].y;
    }
    block_reduce<2>(v);
    if (threadIdx.x == 0) *result = make_double2(v[0], v[1]);
}

__global__ void __launch_bounds__(REDUCE_THREADS) finalize_real_kernel(const double* __restrict__ partials, int nq,
                                                                       double* __restrict__ S, int d0, int d1,
                                                                       int csrc, int cdst) {
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < REDUCE_BLOCKS; i += blockDim.x) {
        v[0] += partials[i];
        if (nq > 1) v[1] += partials[REDUCE_BLOCKS + i];
    }
    block_reduce<2>(v);
    if (threadIdx.x == 0) {
        if (csrc >= 0) S[cdst] = S[csrc];
        S[d0] = v[0];
        if (nq > 1) S[d1] = v[1];
    }
}

}  // namespace

void launch_finalize_real(const double* partials, int nq, double* S, int d0, int d1, int csrc, int cdst,
                          hipStream_t s) {
    hipLaunchKernelGGL(finalize_real_kernel, dim3(1), dim3(REDUCE_THREADS), 0, s, partials, nq, S, d0, d1, csrc,
                       cdst);
}

void launch_finalize(const double2* partials, int np, double2* result, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(REDUCE_THREADS), 0, s, partials, np, result);
}

template <typename T>
void launch_dot(int64_t n, const C2<T>* x, const C2<T>* y, double2* partials, double2* result, hipStream_t s) {
    hipLaunchKernelGGL(dot_partial_kernel<T>, dim3(REDUCE_BLOCKS), dim3(REDUCE_THREADS), 0, s, n, x, y, partials);
    launch_finalize(partials, REDUCE_BLOCKS, result, s);
}

namespace {
// Plain streaming copy: each workgroup moves one contiguous 64 KiB chunk, every
// work-item issuing its sixteen 16-byte loads before its first store.
constexpr int COPY_UNROLL = 16;
__global__ void __launch_bounds__(256) stream_copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                          size_t n) {
    const size_t base = (size_t)blockIdx.x * (256 * COPY_UNROLL) + threadIdx.x;
    uint4 v[COPY_UNROLL];
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) {
        const size_t i = base + (size_t)u * 256;
        if (i < n) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) {
        const size_t i = base + (size_t)u * 256;
        if (i < n) dst[i] = v[u];
    }
}
}  // namespace

void launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 16;
    if (n == 0) return;
    const size_t per = (size_t)256 * COPY_UNROLL;
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)((n + per - 1) / per)), dim3(256), 0, s,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), n);
}

template void launch_dot<double>(int64_t, const double2*, const double2*, double2*, double2*, hipStream_t);
template void launch_dot<float>(int64_t, const float2*, const float2*, double2*, double2*, hipStream_t);

}  // namespace hdcr
