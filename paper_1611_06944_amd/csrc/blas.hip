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
// work-item issuing its sixteen 16-byte loads before its first store.  It uses
// the memory instructions of the library's field kernels (raw buffer loads and
// non-temporal buffer stores through a descriptor of the workgroup's chunk), so
// that the memory-traffic counters, whose request-size accounting differs
// between instruction types, read it as they read those kernels.  Loads past the
// descriptor's range return zero and stores past it are dropped, so the last,
// partial chunk needs no per-load test (a guarded load in an unrolled loop ends
// in a wait for it at the branch's join, which would serialise the loads).
constexpr int COPY_UNROLL = 16;
constexpr uint32_t COPY_CHUNK = 256u * COPY_UNROLL * 16u;  // bytes per workgroup
__global__ void __launch_bounds__(256) stream_copy_kernel(const unsigned char* __restrict__ src,
                                                          unsigned char* __restrict__ dst, size_t bytes) {
    const size_t off = (size_t)blockIdx.x * COPY_CHUNK;
    const size_t left = bytes - off;
    const uint32_t range = left < COPY_CHUNK ? (uint32_t)left : COPY_CHUNK;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(src + off, range), rd = make_rsrc(dst + off, range);
    typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
    u32x4_t v[COPY_UNROLL];
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u)
        v[u] = __builtin_amdgcn_raw_buffer_load_b128(rs, (threadIdx.x + u * 256u) * 16u, 0, 0);
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) store_b128<CPOL_NT>(v[u], rd, (threadIdx.x + u * 256u) * 16u, 0u);
}
}  // namespace

void launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    if (bytes == 0) return;
    hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)((bytes + COPY_CHUNK - 1) / COPY_CHUNK)), dim3(256), 0, s,
                       static_cast<const unsigned char*>(src), static_cast<unsigned char*>(dst), bytes);
}

template void launch_dot<double>(int64_t, const double2*, const double2*, double2*, double2*, hipStream_t);
template void launch_dot<float>(int64_t, const float2*, const float2*, double2*, double2*, hipStream_t);

}  // namespace hdcr
