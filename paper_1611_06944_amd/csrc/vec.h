// Vector kernels of the two-level solver (vec.hip).
#pragma once

#include "internal.h"

namespace hdcr {

// up to MAXV vectors combined by one multi-vector kernel
constexpr int MAXV = 8;
template <typename TV> struct PtrListT {
    const C2<TV>* p[MAXV];
};
typedef PtrListT<double> PtrList;

template <typename A, typename B> void launch_convert(int64_t n, const A* x, B* y, hipStream_t s);
// y = a x + b y
template <typename T> void launch_axpby(int64_t n, T a, const C2<T>* x, T b, C2<T>* y, hipStream_t s);
// out = x - y
template <typename T> void launch_sub(int64_t n, const C2<T>* x, const C2<T>* y, C2<T>* out, hipStream_t s);
// out = a x
template <typename T> void launch_scale(int64_t n, T a, const C2<T>* x, C2<T>* out, hipStream_t s);

// out[2j], out[2j+1] = <V[j], y> (j < nv), out[2*MAXV] = |y|^2 (FP64 accumulation whatever the
// storage of V and y); part: (2*MAXV+1)*REDUCE_BLOCKS doubles
template <typename TV, typename TY>
void launch_multidot(int64_t n, const PtrListT<TV>& V, int nv, const C2<TY>* y, double* part, double* out,
                     hipStream_t s);
// y <- y - sum_j (coef[2j] + i coef[2j+1]) sc[j] V[j]   (sc: real scales, null for 1)
template <typename TV>
void launch_multi_axpy(int64_t n, const PtrListT<TV>& V, int nv, const double* coef, C2<TV>* y, hipStream_t s,
                       const double* sc = nullptr);
// y <- y - sum_j (coef[2j] + i coef[2j+1]) sc[j] V[j], then out as launch_multidot(V, y) of the
// stored result (bitwise the same sums), in one pass over V and y
template <typename TV>
void launch_multi_axpy_dot(int64_t n, const PtrListT<TV>& V, int nv, const double* coef, C2<TV>* y, double* part,
                           double* out, hipStream_t s, const double* sc = nullptr);
// x <- x + sum_j g[j] Z[j]   (g on the host, x FP64)
template <typename TV>
void launch_multi_update(int64_t n, const PtrListT<TV>& Z, int nz, const double2* g, double2* x, hipStream_t s);
// r <- r - ((S[ic] - i S[ic+1]) / S[inn]) w, partial |r|^2 in part[0..REDUCE_BLOCKS)  (r FP64);
// r32, if not null, receives r rounded to FP32
template <typename TV>
void launch_r_update(int64_t n, const double* S, int ic, int inn, const C2<TV>* w, double2* r, double* part,
                     hipStream_t s, float2* r32 = nullptr);

// FP16 field storage, (fp16 re, fp16 im) per complex entry: y = fp16(f x) with
// f = sqrt(n / S[idx]), so that y has unit RMS per entry (f = 0 when S[idx] = 0;
// S[idx] = |x|^2 from launch_norm2), and back: out = float(y) / f (+ out when
// accumulate).  Rounding to nearest.
void launch_to_h16_scaled(int64_t n, const float2* x, const double* S, int idx, void* y, hipStream_t s);
void launch_from_h16_scaled(int64_t n, const void* y, const double* S, int idx, float2* out, bool accumulate,
                            hipStream_t s);

// y = beta x + sum_{i < ny} g[i] z[i] on FP16-stored fields (0 <= ny <= 4; FP32
// arithmetic, one rounding per entry); y may be one of the z[i], not x
void launch_h16_combine(int64_t n, float beta, const void* x, const void* const z[4], const float g[4], int ny, void* y,
                        hipStream_t s);

// FP16-stored fields: S[idx] = |x|^2 (FP64 accumulation, fixed order; part:
// REDUCE_BLOCKS doubles); x <- sqrt(n / S[idx]) x (unit RMS per entry; unchanged
// when S[idx] is 0); out (C128) = x
void launch_h16_norm2(int64_t n, const void* x, double* part, double* S, int idx, hipStream_t s);
void launch_h16_scale_rms(int64_t n, void* x, const double* S, int idx, hipStream_t s);
void launch_h16_to_c128(int64_t n, const void* x, double2* out, hipStream_t s);

// S[idx] = |x|^2 (FP64 accumulation, fixed order); part: REDUCE_BLOCKS doubles
template <typename T> void launch_norm2(int64_t n, const C2<T>* x, double* part, double* S, int idx, hipStream_t s);
// x <- x / sqrt(S[idx])
template <typename T> void launch_scale_inv_sqrt(int64_t n, C2<T>* x, const double* S, int idx, hipStream_t s);
// S[dst] = 1 / S[src] (one work-item)
void launch_inv_copy(double* S, int src, int dst, hipStream_t s);

}  // namespace hdcr
