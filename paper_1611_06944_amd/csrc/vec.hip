// Vector kernels used by the two-level solver: precision conversion, linear
// combinations with scalars from the host or from device memory, fused
// Chebyshev recurrence steps, and multi-vector inner products (FP64
// accumulation, fixed reduction order).
#include "vec.h"
#include "solver.h"

namespace hdcr {

namespace {

constexpr int VWG = 256;

int vgrid(int64_t n) {
    int64_t b = (n + VWG - 1) / VWG;
    if (b > 8192) b = 8192;
    return (int)(b < 1 ? 1 : b);
}

template <typename A, typename B>
__global__ void __launch_bounds__(VWG) convert_kernel(int64_t n, const A* __restrict__ x, B* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * VWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * VWG) {
        const A v = x[i];
        B o;
        o.x = v.x;
        o.y = v.y;
        y[i] = o;
    }
}

// y = a x + b y (real a, b)
template <typename T>
__global__ void __launch_bounds__(VWG) axpby_kernel(int64_t n, T a, const C2<T>* __restrict__ x, T b,
                                                    C2<T>* __restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * VWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * VWG) {
        const C2<T> xv = x[i];
        C2<T> yv = y[i];
        yv.x = a * xv.x + b * yv.x;
        yv.y = a * xv.y + b * yv.y;
        y[i] = yv;
    }
}

// out = x - y
template <typename T>
__global__ void __launch_bounds__(VWG) sub_kernel(int64_t n, const C2<T>* __restrict__ x, const C2<T>* __restrict__ y,
                                                  C2<T>* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * VWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * VWG)
        out[i] = csub<T>(x[i], y[i]);
}

// out = a x (real a)
template <typename T>
__global__ void __launch_bounds__(VWG) scale_kernel(int64_t n, T a, const C2<T>* __restrict__ x,
                                                    C2<T>* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * VWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * VWG) {
        const C2<T> v = x[i];
        out[i] = mk<T>(a * v.x, a * v.y);
    }
}

// Entries 2k and 2k+1 of an array of complex values: one 16-byte load for FP32
// storage, two for FP64.
template <typename T>
__device__ __forceinline__ void ld_two(const C2<T>* p, int64_t k, C2<T>& a, C2<T>& b) {
    if constexpr (sizeof(T) == 4) {
        const float4 q = reinterpret_cast<const float4*>(p)[k];
        a = make_float2(q.x, q.y);
        b = make_float2(q.z, q.w);
    } else {
        a = p[2 * k];
        b = p[2 * k + 1];
    }
}
template <typename T> __device__ __forceinline__ void st_two(C2<T>* p, int64_t k, C2<T> a, C2<T> b) {
    if constexpr (sizeof(T) == 4) {
        reinterpret_cast<float4*>(p)[k] = make_float4(a.x, a.y, b.x, b.y);
    } else {
        p[2 * k] = a;
        p[2 * k + 1] = b;
    }
}

// acc[2j], acc[2j+1] += <v_j, y> (re, im) for j < nv; acc[2 MAXV] += |y|^2
template <typename TV>
__device__ __forceinline__ void dot_terms(const C2<TV> (&vt)[MAXV], int nv, double2 yv, double (&acc)[2 * MAXV + 1]) {
#pragma unroll
    for (int j = 0; j < MAXV; ++j) {
        if (j < nv) {
            const double2 v = make_double2(vt[j].x, vt[j].y);
            acc[2 * j] += v.x * yv.x + v.y * yv.y;
            acc[2 * j + 1] += v.x * yv.y - v.y * yv.x;
        }
    }
    acc[2 * MAXV] += yv.x * yv.x + yv.y * yv.y;
}

// partial sums of <V[j], y> for j < nv and |y|^2 into part[q * REDUCE_BLOCKS + blk]
// (V and y in FP64 or FP32 storage, FP64 accumulation).  PAIR (FP32 y, n even,
// 16-byte aligned arrays): a work-item takes entries 2k and 2k+1 per step, so
// FP32 storage is read in 16-byte runs, twice the bytes per load of one entry at
// a time (which kept the kernel below 4 TB/s at 4 waves per SIMD).
template <typename TV, typename TY, bool PAIR>
__global__ void __launch_bounds__(REDUCE_THREADS) multidot_kernel(int64_t n, PtrListT<TV> V, int nv,
                                                                  const C2<TY>* __restrict__ y,
                                                                  double* __restrict__ part) {
    double acc[2 * MAXV + 1];
#pragma unroll
    for (int q = 0; q < 2 * MAXV + 1; ++q) acc[q] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if constexpr (PAIR) {
        for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n / 2; k += stride) {
            C2<TY> y0, y1;
            ld_two<TY>(y, k, y0, y1);
            C2<TV> v0[MAXV], v1[MAXV];
#pragma unroll
            for (int j = 0; j < MAXV; ++j)
                if (j < nv) ld_two<TV>(V.p[j], k, v0[j], v1[j]);
            dot_terms<TV>(v0, nv, make_double2(y0.x, y0.y), acc);
            dot_terms<TV>(v1, nv, make_double2(y1.x, y1.y), acc);
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
            const C2<TY> yt = y[i];
            C2<TV> vt[MAXV];
#pragma unroll
            for (int j = 0; j < MAXV; ++j)
                if (j < nv) vt[j] = V.p[j][i];
            dot_terms<TV>(vt, nv, make_double2(yt.x, yt.y), acc);
        }
    }
    block_reduce<2 * MAXV + 1>(acc);
    if (threadIdx.x == 0) {
        for (int q = 0; q < 2 * MAXV + 1; ++q) part[(int64_t)q * REDUCE_BLOCKS + blockIdx.x] = acc[q];
    }
}

__global__ void __launch_bounds__(REDUCE_THREADS) multidot_finalize_kernel(const double* __restrict__ part, int nq,
                                                                           double* __restrict__ out) {
    // one workgroup per quantity
    const int q = blockIdx.x;
    if (q >= nq) return;
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < REDUCE_BLOCKS; i += blockDim.x) v[0] += part[(int64_t)q * REDUCE_BLOCKS + i];
    block_reduce<1>(v);
    if (threadIdx.x == 0) out[q] = v[0];
}

// y <- y - sum_j coef[j] V[j]   (coef: complex, device memory; FP64 arithmetic, one rounding to TV)
template <typename TV>
__global__ void __launch_bounds__(VWG) multi_axpy_kernel(int64_t n, PtrListT<TV> V, int nv,
                                                         const double* __restrict__ coef, C2<TV>* __restrict__ y,
                                                         const double* __restrict__ sc) {
    double2 cf[MAXV];
#pragma unroll
    for (int j = 0; j < MAXV; ++j) {
        const double f = (j < nv && sc) ? sc[j] : 1.0;
        cf[j] = (j < nv) ? make_double2(f * coef[2 * j], f * coef[2 * j + 1]) : make_double2(0, 0);
    }
    for (int64_t i = (int64_t)blockIdx.x * VWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * VWG) {
        const C2<TV> yt = y[i];
        double2 yv = make_double2(yt.x, yt.y);
#pragma unroll
        for (int j = 0; j < MAXV; ++j) {
            if (j < nv) {
                const C2<TV> vt = V.p[j][i];
                yv = cfma<double>(cneg<double>(cf[j]), make_double2(vt.x, vt.y), yv);
            }
        }
        y[i] = mk<TV>((TV)yv.x, (TV)yv.y);
    }
}

// y <- y - sum_j coef[j] sc[j] V[j] as multi_axpy_kernel, and the partial sums of
// <V[j], y> and |y|^2 of the stored result as multidot_kernel: same grid, same
// entries per work-item (PAIR as there) and same reduction, so the sums are
// bitwise those of a separate multidot pass over the updated y
template <typename TV, bool PAIR>
__global__ void __launch_bounds__(REDUCE_THREADS) multi_axpy_dot_kernel(int64_t n, PtrListT<TV> V, int nv,
                                                                        const double* __restrict__ coef,
                                                                        C2<TV>* __restrict__ y,
                                                                        double* __restrict__ part,
                                                                        const double* __restrict__ sc) {
    double2 cf[MAXV];
#pragma unroll
    for (int j = 0; j < MAXV; ++j) {
        const double f = (j < nv && sc) ? sc[j] : 1.0;
        cf[j] = (j < nv) ? make_double2(f * coef[2 * j], f * coef[2 * j + 1]) : make_double2(0, 0);
    }
    auto update = [&](C2<TV> yt, const C2<TV> (&vt)[MAXV]) {
        double2 yv = make_double2(yt.x, yt.y);
#pragma unroll
        for (int j = 0; j < MAXV; ++j)
            if (j < nv) yv = cfma<double>(cneg<double>(cf[j]), make_double2(vt[j].x, vt[j].y), yv);
        return mk<TV>((TV)yv.x, (TV)yv.y);
    };
    double acc[2 * MAXV + 1];
#pragma unroll
    for (int q = 0; q < 2 * MAXV + 1; ++q) acc[q] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if constexpr (PAIR) {
        for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n / 2; k += stride) {
            C2<TV> y0, y1;
            ld_two<TV>(y, k, y0, y1);
            C2<TV> v0[MAXV], v1[MAXV];
#pragma unroll
            for (int j = 0; j < MAXV; ++j)
                if (j < nv) ld_two<TV>(V.p[j], k, v0[j], v1[j]);
            const C2<TV> o0 = update(y0, v0), o1 = update(y1, v1);
            st_two<TV>(y, k, o0, o1);
            dot_terms<TV>(v0, nv, make_double2(o0.x, o0.y), acc);
            dot_terms<TV>(v1, nv, make_double2(o1.x, o1.y), acc);
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
            C2<TV> vt[MAXV];
#pragma unroll
            for (int j = 0; j < MAXV; ++j)
                if (j < nv) vt[j] = V.p[j][i];
            const C2<TV> yo = update(y[i], vt);
            y[i] = yo;
            dot_terms<TV>(vt, nv, make_double2(yo.x, yo.y), acc);
        }
    }
    block_reduce<2 * MAXV + 1>(acc);
    if (threadIdx.x == 0) {
        for (int q = 0; q < 2 * MAXV + 1; ++q) part[(int64_t)q * REDUCE_BLOCKS + blockIdx.x] = acc[q];
    }
}

// x <- x + sum_j g[j] Z[j]   (g: complex, kernel arguments; x FP64)
struct Coefs {
    double2 g[MAXV];
};
template <typename TV>
__global__ void __launch_bounds__(VWG) multi_update_kernel(int64_t n, PtrListT<TV> Z, int nz, Coefs g,
                                                           double2* __restrict__ x) {
    for (int64_t i = (int64_t)blockIdx.x * VWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * VWG) {
        double2 xv = x[i];
#pragma unroll
        for (int j = 0; j < MAXV; ++j) {
            if (j < nz) {
                const C2<TV> zt = Z.p[j][i];
                xv = cfma<double>(g.g[j], make_double2(zt.x, zt.y), xv);
            }
        }
        x[i] = xv;
    }
}

// r <- r - (conj(c) / nn) w with c = (S[ic], S[ic+1]) = <r, w> and nn = S[inn] = |w|^2
// (so the step is <w, r>/|w|^2); partial |r|^2.  r FP64, w FP64 or FP32; r32, if
// not null, receives r rounded to FP32 (the inner cycle's copy).
template <typename TV>
__global__ void __launch_bounds__(REDUCE_THREADS) r_update_kernel(int64_t n, const double* __restrict__ S, int ic,
                                                                  int inn, const C2<TV>* __restrict__ w,
                                                                  double2* __restrict__ r, double* __restrict__ part,
                                                                  float2* __restrict__ r32) {
    const double nn = S[inn];
    const double2 a = make_double2(S[ic] / nn, -S[ic + 1] / nn);
    double v[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const C2<TV> wt = w[i];
        double2 rv = cfma<double>(cneg<double>(a), make_double2(wt.x, wt.y), r[i]);
        r[i] = rv;
        if (r32) r32[i] = make_float2((float)rv.x, (float)rv.y);
        v[0] += rv.x * rv.x + rv.y * rv.y;
    }
    block_reduce<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// partial |x|^2 (FP64 accumulation)
template <typename T>
__global__ void __launch_bounds__(REDUCE_THREADS) norm2_kernel(int64_t n, const C2<T>* __restrict__ x,
                                                               double* __restrict__ part) {
    double v[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const C2<T> a = x[i];
        v[0] += (double)a.x * a.x + (double)a.y * a.y;
    }
    block_reduce<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// x <- x / sqrt(S[idx])  (S[idx] > 0)
template <typename T>
__global__ void __launch_bounds__(VWG) scale_inv_sqrt_kernel(int64_t n, C2<T>* __restrict__ x,
                                                             const double* __restrict__ S, int idx) {
    const T f = (T)(1.0 / sqrt(S[idx]));
    for (int64_t i = (int64_t)blockIdx.x * VWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * VWG) {
        const C2<T> v = x[i];
        x[i] = mk<T>(f * v.x, f * v.y);
    }
}

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

__global__ void __launch_bounds__(VWG) to_h16_scaled_kernel(int64_t n, const float2* __restrict__ x,
                                                            const double* __restrict__ S, int idx,
                                                            uint32_t* __restrict__ y) {
    const double nn = S[idx];
    const float f = nn > 0.0 ? (float)sqrt((double)n / nn) : 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * VWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * VWG) {
        const float2 v = x[i];
        const half2_t h = {(_Float16)(f * v.x), (_Float16)(f * v.y)};
        y[i] = __builtin_bit_cast(uint32_t, h);
    }
}

__global__ void __launch_bounds__(VWG) from_h16_scaled_kernel(int64_t n, const uint32_t* __restrict__ y,
                                                              const double* __restrict__ S, int idx,
                                                              float2* __restrict__ out, int accumulate) {
    const float f = (float)sqrt(S[idx] / (double)n);
    for (int64_t i = (int64_t)blockIdx.x * VWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * VWG) {
        const half2_t h = __builtin_bit_cast(half2_t, y[i]);
        float2 o = make_float2(f * (float)h.x, f * (float)h.y);
        if (accumulate) {
            const float2 a = out[i];
            o.x += a.x;
            o.y += a.y;
        }
        out[i] = o;
    }
}

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef unsigned uint2_t __attribute__((ext_vector_type(2)));
struct H16Combine {
    const uint2_t* z[4];
    float g[4];
};
// two complex entries (8 bytes) per work-item and step
template <int NY>
__global__ void __launch_bounds__(VWG) h16_combine_kernel(int64_t n2, float beta, const uint2_t* x, H16Combine c,
                                                          uint2_t* y) {
    for (int64_t i = (int64_t)blockIdx.x * VWG + threadIdx.x; i < n2; i += (int64_t)gridDim.x * VWG) {
        const half4_t hx = __builtin_bit_cast(half4_t, x[i]);
        float o[4] = {beta * (float)hx.x, beta * (float)hx.y, beta * (float)hx.z, beta * (float)hx.w};
#pragma unroll
        for (int q = 0; q < NY; ++q) {
            const half4_t hz = __builtin_bit_cast(half4_t, c.z[q][i]);
            o[0] = fmaf(c.g[q], (float)hz.x, o[0]);
            o[1] = fmaf(c.g[q], (float)hz.y, o[1]);
            o[2] = fmaf(c.g[q], (float)hz.z, o[2]);
            o[3] = fmaf(c.g[q], (float)hz.w, o[3]);
        }
        const half4_t ho = {(_Float16)o[0], (_Float16)o[1], (_Float16)o[2], (_Float16)o[3]};
        y[i] = __builtin_bit_cast(uint2_t, ho);
    }
}

// partial |x|^2 over pairs of complex entries (FP64 accumulation)
__global__ void __launch_bounds__(REDUCE_THREADS) h16_norm2_kernel(int64_t n2, const uint2_t* __restrict__ x,
                                                                   double* __restrict__ part) {
    double v[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) {
        const half4_t h = __builtin_bit_cast(half4_t, x[i]);
        const double a = (float)h.x, b = (float)h.y, c = (float)h.z, d = (float)h.w;
        v[0] += a * a + b * b + c * c + d * d;
    }
    block_reduce<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(VWG) h16_scale_rms_kernel(int64_t n2, uint2_t* __restrict__ x,
                                                            const double* __restrict__ S, int idx) {
    const double nn = S[idx];
    const float f = nn > 0.0 ? (float)sqrt((double)(2 * n2) / nn) : 1.0f;
    for (int64_t i = (int64_t)blockIdx.x * VWG + threadIdx.x; i < n2; i += (int64_t)gridDim.x * VWG) {
        const half4_t h = __builtin_bit_cast(half4_t, x[i]);
        const half4_t o = {(_Float16)(f * (float)h.x), (_Float16)(f * (float)h.y), (_Float16)(f * (float)h.z),
                           (_Float16)(f * (float)h.w)};
        x[i] = __builtin_bit_cast(uint2_t, o);
    }
}

__global__ void __launch_bounds__(VWG) h16_to_c128_kernel(int64_t n, const uint32_t* __restrict__ x,
                                                          double2* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * VWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * VWG) {
        const half2_t h = __builtin_bit_cast(half2_t, x[i]);
        out[i] = make_double2((float)h.x, (float)h.y);
    }
}

}  // namespace

void launch_h16_norm2(int64_t n, const void* x, double* part, double* S, int idx, hipStream_t s) {
    hipLaunchKernelGGL(h16_norm2_kernel, dim3(REDUCE_BLOCKS), dim3(REDUCE_THREADS), 0, s, n / 2,
                       static_cast<const uint2_t*>(x), part);
    launch_finalize_real(part, 1, S, idx, -1, -1, -1, s);
}
void launch_h16_scale_rms(int64_t n, void* x, const double* S, int idx, hipStream_t s) {
    hipLaunchKernelGGL(h16_scale_rms_kernel, dim3(vgrid(n / 2)), dim3(VWG), 0, s, n / 2, static_cast<uint2_t*>(x), S,
                       idx);
}
void launch_h16_to_c128(int64_t n, const void* x, double2* out, hipStream_t s) {
    hipLaunchKernelGGL(h16_to_c128_kernel, dim3(vgrid(n)), dim3(VWG), 0, s, n, static_cast<const uint32_t*>(x), out);
}

void launch_h16_combine(int64_t n, float beta, const void* x, const void* const z[4], const float g[4], int ny, void* y,
                        hipStream_t s) {
    // n complex entries = n / 2 eight-byte pairs (n is even: 12 components per site)
    const int64_t n2 = n / 2;
    H16Combine c{};
    for (int q = 0; q < 4; ++q) {
        c.z[q] = q < ny ? static_cast<const uint2_t*>(z[q]) : nullptr;
        c.g[q] = q < ny ? g[q] : 0.0f;
    }
    const uint2_t* xp = static_cast<const uint2_t*>(x);
    uint2_t* yp = static_cast<uint2_t*>(y);
    switch (ny) {
        case 0: hipLaunchKernelGGL(h16_combine_kernel<0>, dim3(vgrid(n2)), dim3(VWG), 0, s, n2, beta, xp, c, yp); break;
        case 1: hipLaunchKernelGGL(h16_combine_kernel<1>, dim3(vgrid(n2)), dim3(VWG), 0, s, n2, beta, xp, c, yp); break;
        case 2: hipLaunchKernelGGL(h16_combine_kernel<2>, dim3(vgrid(n2)), dim3(VWG), 0, s, n2, beta, xp, c, yp); break;
        case 3: hipLaunchKernelGGL(h16_combine_kernel<3>, dim3(vgrid(n2)), dim3(VWG), 0, s, n2, beta, xp, c, yp); break;
        default: hipLaunchKernelGGL(h16_combine_kernel<4>, dim3(vgrid(n2)), dim3(VWG), 0, s, n2, beta, xp, c, yp); break;
    }
}

void launch_to_h16_scaled(int64_t n, const float2* x, const double* S, int idx, void* y, hipStream_t s) {
    hipLaunchKernelGGL(to_h16_scaled_kernel, dim3(vgrid(n)), dim3(VWG), 0, s, n, x, S, idx, static_cast<uint32_t*>(y));
}
void launch_from_h16_scaled(int64_t n, const void* y, const double* S, int idx, float2* out, bool accumulate,
                            hipStream_t s) {
    hipLaunchKernelGGL(from_h16_scaled_kernel, dim3(vgrid(n)), dim3(VWG), 0, s, n, static_cast<const uint32_t*>(y), S,
                       idx, out, accumulate ? 1 : 0);
}

template <typename T>
void launch_norm2(int64_t n, const C2<T>* x, double* part, double* S, int idx, hipStream_t s) {
    hipLaunchKernelGGL(norm2_kernel<T>, dim3(REDUCE_BLOCKS), dim3(REDUCE_THREADS), 0, s, n, x, part);
    launch_finalize_real(part, 1, S, idx, -1, -1, -1, s);
}
template <typename T>
void launch_scale_inv_sqrt(int64_t n, C2<T>* x, const double* S, int idx, hipStream_t s) {
    hipLaunchKernelGGL(scale_inv_sqrt_kernel<T>, dim3(vgrid(n)), dim3(VWG), 0, s, n, x, S, idx);
}
template void launch_norm2<double>(int64_t, const double2*, double*, double*, int, hipStream_t);
template void launch_norm2<float>(int64_t, const float2*, double*, double*, int, hipStream_t);
template void launch_scale_inv_sqrt<double>(int64_t, double2*, const double*, int, hipStream_t);
template void launch_scale_inv_sqrt<float>(int64_t, float2*, const double*, int, hipStream_t);

template <typename A, typename B>
void launch_convert(int64_t n, const A* x, B* y, hipStream_t s) {
    hipLaunchKernelGGL((convert_kernel<A, B>), dim3(vgrid(n)), dim3(VWG), 0, s, n, x, y);
}
template void launch_convert<double2, float2>(int64_t, const double2*, float2*, hipStream_t);
template void launch_convert<float2, double2>(int64_t, const float2*, double2*, hipStream_t);
template void launch_convert<double2, double2>(int64_t, const double2*, double2*, hipStream_t);
template void launch_convert<float2, float2>(int64_t, const float2*, float2*, hipStream_t);

template <typename T>
void launch_axpby(int64_t n, T a, const C2<T>* x, T b, C2<T>* y, hipStream_t s) {
    hipLaunchKernelGGL(axpby_kernel<T>, dim3(vgrid(n)), dim3(VWG), 0, s, n, a, x, b, y);
}
template <typename T>
void launch_sub(int64_t n, const C2<T>* x, const C2<T>* y, C2<T>* out, hipStream_t s) {
    hipLaunchKernelGGL(sub_kernel<T>, dim3(vgrid(n)), dim3(VWG), 0, s, n, x, y, out);
}
template <typename T>
void launch_scale(int64_t n, T a, const C2<T>* x, C2<T>* out, hipStream_t s) {
    hipLaunchKernelGGL(scale_kernel<T>, dim3(vgrid(n)), dim3(VWG), 0, s, n, a, x, out);
}
#define HDCR_VEC_INST(T)                                                                                      \
    template void launch_axpby<T>(int64_t, T, const C2<T>*, T, C2<T>*, hipStream_t);                           \
    template void launch_sub<T>(int64_t, const C2<T>*, const C2<T>*, C2<T>*, hipStream_t);                     \
    template void launch_scale<T>(int64_t, T, const C2<T>*, C2<T>*, hipStream_t);
HDCR_VEC_INST(double)
HDCR_VEC_INST(float)
#undef HDCR_VEC_INST

// entries taken two at a time: FP32 y (FP64 entries are 16 bytes already), n
// even and every array 16-byte aligned
template <typename TV, typename TY>
static bool pair_ok(int64_t n, const PtrListT<TV>& V, int nv, const C2<TY>* y) {
    if (sizeof(TY) != 4 || n % 2 || reinterpret_cast<uintptr_t>(y) % 16) return false;
    for (int j = 0; j < nv; ++j)
        if (reinterpret_cast<uintptr_t>(V.p[j]) % 16) return false;
    return true;
}

template <typename TV, typename TY>
void launch_multidot(int64_t n, const PtrListT<TV>& V, int nv, const C2<TY>* y, double* part, double* out,
                     hipStream_t s) {
    if (pair_ok<TV, TY>(n, V, nv, y))
        hipLaunchKernelGGL((multidot_kernel<TV, TY, true>), dim3(REDUCE_BLOCKS), dim3(REDUCE_THREADS), 0, s, n, V, nv,
                           y, part);
    else
        hipLaunchKernelGGL((multidot_kernel<TV, TY, false>), dim3(REDUCE_BLOCKS), dim3(REDUCE_THREADS), 0, s, n, V,
                           nv, y, part);
    hipLaunchKernelGGL(multidot_finalize_kernel, dim3(2 * MAXV + 1), dim3(REDUCE_THREADS), 0, s, part, 2 * MAXV + 1,
                       out);
}

template <typename TV>
void launch_multi_axpy(int64_t n, const PtrListT<TV>& V, int nv, const double* coef, C2<TV>* y, hipStream_t s,
                       const double* sc) {
    hipLaunchKernelGGL(multi_axpy_kernel<TV>, dim3(vgrid(n)), dim3(VWG), 0, s, n, V, nv, coef, y, sc);
}

template <typename TV>
void launch_multi_axpy_dot(int64_t n, const PtrListT<TV>& V, int nv, const double* coef, C2<TV>* y, double* part,
                           double* out, hipStream_t s, const double* sc) {
    if (pair_ok<TV, TV>(n, V, nv, y))
        hipLaunchKernelGGL((multi_axpy_dot_kernel<TV, true>), dim3(REDUCE_BLOCKS), dim3(REDUCE_THREADS), 0, s, n, V,
                           nv, coef, y, part, sc);
    else
        hipLaunchKernelGGL((multi_axpy_dot_kernel<TV, false>), dim3(REDUCE_BLOCKS), dim3(REDUCE_THREADS), 0, s, n, V,
                           nv, coef, y, part, sc);
    hipLaunchKernelGGL(multidot_finalize_kernel, dim3(2 * MAXV + 1), dim3(REDUCE_THREADS), 0, s, part, 2 * MAXV + 1,
                       out);
}

template <typename TV>
void launch_multi_update(int64_t n, const PtrListT<TV>& Z, int nz, const double2* g, double2* x, hipStream_t s) {
    Coefs c;
    for (int j = 0; j < MAXV; ++j) c.g[j] = (j < nz) ? g[j] : make_double2(0, 0);
    hipLaunchKernelGGL(multi_update_kernel<TV>, dim3(vgrid(n)), dim3(VWG), 0, s, n, Z, nz, c, x);
}

template <typename TV>
void launch_r_update(int64_t n, const double* S, int ic, int inn, const C2<TV>* w, double2* r, double* part,
                     hipStream_t s, float2* r32) {
    hipLaunchKernelGGL(r_update_kernel<TV>, dim3(REDUCE_BLOCKS), dim3(REDUCE_THREADS), 0, s, n, S, ic, inn, w, r,
                       part, r32);
}

__global__ void inv_copy_kernel(double* S, int src, int dst) {
    if (threadIdx.x == 0) S[dst] = 1.0 / S[src];
}
void launch_inv_copy(double* S, int src, int dst, hipStream_t s) {
    hipLaunchKernelGGL(inv_copy_kernel, dim3(1), dim3(64), 0, s, S, src, dst);
}

template void launch_multidot<double, double>(int64_t, const PtrListT<double>&, int, const double2*, double*, double*,
                                              hipStream_t);
template void launch_multidot<float, float>(int64_t, const PtrListT<float>&, int, const float2*, double*, double*,
                                            hipStream_t);
template void launch_multidot<double, float>(int64_t, const PtrListT<double>&, int, const float2*, double*, double*,
                                             hipStream_t);
template void launch_multi_axpy<double>(int64_t, const PtrListT<double>&, int, const double*, double2*, hipStream_t,
                                        const double*);
template void launch_multi_axpy<float>(int64_t, const PtrListT<float>&, int, const double*, float2*, hipStream_t,
                                       const double*);
template void launch_multi_axpy_dot<double>(int64_t, const PtrListT<double>&, int, const double*, double2*, double*,
                                            double*, hipStream_t, const double*);
template void launch_multi_axpy_dot<float>(int64_t, const PtrListT<float>&, int, const double*, float2*, double*,
                                           double*, hipStream_t, const double*);
template void launch_multi_update<double>(int64_t, const PtrListT<double>&, int, const double2*, double2*,
                                          hipStream_t);
template void launch_multi_update<float>(int64_t, const PtrListT<float>&, int, const double2*, double2*, hipStream_t);
template void launch_r_update<double>(int64_t, const double*, int, int, const double2*, double2*, double*,
                                      hipStream_t, float2*);
template void launch_r_update<float>(int64_t, const double*, int, int, const float2*, double2*, double*, hipStream_t,
                                     float2*);

}  // namespace hdcr
