// Vector kernels of the two-level solver (vec.hip).
#pragma once

#include "internal.h"

namespace hdcr {

// up to MAXV vectors combined by one multi-vector kernel
constexpr int MAXV = 8;
struct PtrList {
    const double2* p[MAXV];
};

template <typename A, typename B> void launch_convert(int64_t n, const A* x, B* y, hipStream_t s);
// y = a x + b y
template <typename T> void launch_axpby(int64_t n, T a, const C2<T>* x, T b, C2<T>* y, hipStream_t s);
// out = x - y
template <typename T> void launch_sub(int64_t n, const C2<T>* x, const C2<T>* y, C2<T>* out, hipStream_t s);
// t0 <- a w + b t1 - t0;  acc <- acc + c t0  (acc may be null)
template <typename T>
void launch_cheb_step(int64_t n, T a, const C2<T>* w, T b, const C2<T>* t1, C2<T>* t0, T c, C2<T>* acc,
                      hipStream_t s);
// out = a x
template <typename T> void launch_scale(int64_t n, T a, const C2<T>* x, C2<T>* out, hipStream_t s);

// out[2j], out[2j+1] = <V[j], y> (j < nv), out[2*MAXV] = |y|^2; part: (2*MAXV+1)*REDUCE_BLOCKS doubles
void launch_multidot(int64_t n, const PtrList& V, int nv, const double2* y, double* part, double* out,
                     hipStream_t s);
// y <- y - sum_j (coef[2j] + i coef[2j+1]) V[j]
void launch_multi_axpy(int64_t n, const PtrList& V, int nv, const double* coef, double2* y, hipStream_t s);
// x <- x + sum_j g[j] Z[j]   (g on the host)
void launch_multi_update(int64_t n, const PtrList& Z, int nz, const double2* g, double2* x, hipStream_t s);
// r <- r - ((S[ic] - i S[ic+1]) / S[inn]) w, partial |r|^2 in part[0..REDUCE_BLOCKS)
void launch_r_update(int64_t n, const double* S, int ic, int inn, const double2* w, double2* r, double* part,
                     hipStream_t s);

// S[idx] = |x|^2 (FP64 accumulation, fixed order); part: REDUCE_BLOCKS doubles
template <typename T> void launch_norm2(int64_t n, const C2<T>* x, double* part, double* S, int idx, hipStream_t s);
// x <- x / sqrt(S[idx])
template <typename T> void launch_scale_inv_sqrt(int64_t n, C2<T>* x, const double* S, int idx, hipStream_t s);

}  // namespace hdcr
