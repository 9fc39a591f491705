// Coarse space of the two-level method (Sec. 4) on gfx950: chiral split and
// block orthonormalisation of the subspace vectors, restriction P^dag and
// prolongation P, the little Dirac operator A = P^dag H P and its 9-point
// coarse apply.  Layouts are described in coarse.h.
#include <algorithm>
#include <type_traits>
#include <atomic>
#include <cmath>

#include <cstdlib>

#include "coarse.h"

namespace hdcr {

namespace {

constexpr int CWG = 256;
constexpr double RSQRT2 = 0.70710678118654752440;

// block-local site sl of coarse site a -> lexicographic 4d site index
__device__ __forceinline__ int block_site(const CoarseGeom& c, int a, int sl) {
    int x[4];
    int r = sl;
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
        x[mu] = r % c.B[mu];
        r /= c.B[mu];
    }
    x[3] = r;
    int ca = a;
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
        x[mu] += (ca % c.C[mu]) * c.B[mu];
        ca /= c.C[mu];
    }
    x[3] += ca * c.B[3];
    return ((x[3] * c.f.L[2] + x[2]) * c.f.L[1] + x[1]) * c.f.L[0] + x[0];
}

// coarse neighbour a + d (coarse-periodic), d in D9 = (0,+x,+y,+z,+t,-x,-y,-z,-t)
__device__ __forceinline__ int coarse_nbr(const CoarseGeom& c, int a, int d) {
    if (d == 0) return a;
    const int mu = (d - 1) & 3;
    const int xm = (a / c.cstride[mu]) % c.C[mu];
    if (d <= 4) return (xm == c.C[mu] - 1) ? a - (c.C[mu] - 1) * c.cstride[mu] : a + c.cstride[mu];
    return (xm == 0) ? a + (c.C[mu] - 1) * c.cstride[mu] : a - c.cstride[mu];
}

template <typename T> __device__ __forceinline__ C2<T> shfl_xor_c(C2<T> v, int m) {
    return mk<T>(__shfl_xor(v.x, m), __shfl_xor(v.y, m));
}

// sum of v over the 256 work-items; every work-item gets the result.
// sh must hold 4 * N entries.
template <typename T, int N>
__device__ __forceinline__ void wg_sum(C2<T> (&v)[N], C2<T>* sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < N; ++q) {
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) v[q] = cadd<T>(v[q], shfl_xor_c<T>(v[q], m));
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < N; ++q) sh[wave * N + q] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = cadd<T>(cadd<T>(sh[q], sh[N + q]), cadd<T>(sh[2 * N + q], sh[3 * N + q]));
}

// ---------------------------------------------------------------------------
// basis construction
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(CWG) basis_fold_kernel(CoarseGeom c, const double2* __restrict__ vecs,
                                                         double2* __restrict__ b64) {
    const size_t total = (size_t)c.nvec * c.Nc * c.nhalf;
    for (size_t e = (size_t)blockIdx.x * CWG + threadIdx.x; e < total; e += (size_t)gridDim.x * CWG) {
        const int i = (int)(e % c.nhalf);
        const size_t rest = e / c.nhalf;
        const int a = (int)(rest % c.Nc);
        const int k = (int)(rest / c.Nc);
        const int s = i % c.Lh;
        const int sl = (i / c.Lh) % c.bvol;
        const int comp = i / (c.Lh * c.bvol);
        const int site = block_site(c, a, sl);
        const size_t fb = (((size_t)k * 12 + comp) * c.f.V4 + site) * c.f.Ls;
        const double2 v1 = vecs[fb + s];
        const double2 v2 = vecs[fb + c.f.Ls - 1 - s];
        const double g = (comp < 6) ? 1.0 : -1.0;
        // compressed sqrt(2) * (v +- Gamma5 v)/2 on s < Ls/2
        const double2 wp = make_double2((v1.x + g * v2.x) * RSQRT2, (v1.y + g * v2.y) * RSQRT2);
        const double2 wm = make_double2((v1.x - g * v2.x) * RSQRT2, (v1.y - g * v2.y) * RSQRT2);
        b64[(((size_t)a * 2 + 0) * c.nvec + k) * c.nhalf + i] = wp;
        b64[(((size_t)a * 2 + 1) * c.nvec + k) * c.nhalf + i] = wm;
    }
}

// One workgroup per (block, chirality): the vectors are orthonormalised in
// index order, a panel of ORTH_P at a time (block classical Gram-Schmidt
// applied twice).  Each round projects the panel against all finished vectors,
// ORTH_Q of them per sweep, so a finished vector is read once per panel and
// round rather than once per vector and pass, then orthogonalises the panel
// in index order and normalises it.  The result is the Q factor of the thin
// QR in index order with a positive real R diagonal, as for vector-by-vector
// Gram-Schmidt.  Rank test: a vector whose squared norm after the first round
// is at most 1e-24 of its squared norm before any projection sets the flag
// and is left unnormalised.  Every work-item owns the same indices i of all
// vectors, so only the reductions cross work-items.
constexpr int ORTH_P = 4;
constexpr int ORTH_Q = 4;

__global__ void __launch_bounds__(CWG) block_orth_kernel(CoarseGeom c, double2* __restrict__ b64,
                                                         int* __restrict__ rank_flag) {
    __shared__ double2 sh[4 * ORTH_P * ORTH_Q];
    double2* base = b64 + (size_t)blockIdx.x * c.nvec * c.nhalf;
    const int n = c.nhalf;
    for (int k0 = 0; k0 < c.nvec; k0 += ORTH_P) {
        const int kp = min(ORTH_P, c.nvec - k0);
        double2* W = base + (size_t)k0 * n;
        double2 n0[ORTH_P];
#pragma unroll
        for (int p = 0; p < ORTH_P; ++p) n0[p] = make_double2(0, 0);
        for (int i = threadIdx.x; i < n; i += CWG) {
#pragma unroll
            for (int p = 0; p < ORTH_P; ++p)
                if (p < kp) {
                    const double2 w = W[(size_t)p * n + i];
                    n0[p].x += w.x * w.x + w.y * w.y;
                }
        }
        wg_sum<double, ORTH_P>(n0, sh);
        bool bad[ORTH_P];
#pragma unroll
        for (int p = 0; p < ORTH_P; ++p) bad[p] = false;
        for (int round = 0; round < 2; ++round) {
            // W -= Q (Q^dag W) over the k0 finished vectors Q
            for (int j0 = 0; j0 < k0; j0 += ORTH_Q) {
                const int jn = min(ORTH_Q, k0 - j0);
                double2 r[ORTH_P * ORTH_Q];
#pragma unroll
                for (int e = 0; e < ORTH_P * ORTH_Q; ++e) r[e] = make_double2(0, 0);
                for (int i = threadIdx.x; i < n; i += CWG) {
                    double2 wv[ORTH_P];
#pragma unroll
                    for (int p = 0; p < ORTH_P; ++p) wv[p] = (p < kp) ? W[(size_t)p * n + i] : make_double2(0, 0);
#pragma unroll
                    for (int q = 0; q < ORTH_Q; ++q)
                        if (q < jn) {
                            const double2 qv = base[(size_t)(j0 + q) * n + i];
#pragma unroll
                            for (int p = 0; p < ORTH_P; ++p) r[p * ORTH_Q + q] = cjfma<double>(qv, wv[p], r[p * ORTH_Q + q]);
                        }
                }
                wg_sum<double, ORTH_P * ORTH_Q>(r, sh);
                for (int i = threadIdx.x; i < n; i += CWG) {
                    double2 qv[ORTH_Q];
#pragma unroll
                    for (int q = 0; q < ORTH_Q; ++q) qv[q] = (q < jn) ? base[(size_t)(j0 + q) * n + i] : make_double2(0, 0);
#pragma unroll
                    for (int p = 0; p < ORTH_P; ++p)
                        if (p < kp) {
                            double2 wv = W[(size_t)p * n + i];
#pragma unroll
                            for (int q = 0; q < ORTH_Q; ++q)
                                if (q < jn) wv = cfma<double>(cneg<double>(r[p * ORTH_Q + q]), qv[q], wv);
                            W[(size_t)p * n + i] = wv;
                        }
                }
            }
            // the panel itself in index order, then normalisation
#pragma unroll
            for (int p = 0; p < ORTH_P; ++p) {
                if (p >= kp) break;
                double2* w = W + (size_t)p * n;
                if (p > 0) {
                    double2 r[ORTH_P];
#pragma unroll
                    for (int q = 0; q < ORTH_P; ++q) r[q] = make_double2(0, 0);
                    for (int i = threadIdx.x; i < n; i += CWG) {
                        const double2 wi = w[i];
#pragma unroll
                        for (int q = 0; q < ORTH_P; ++q)
                            if (q < p) r[q] = cjfma<double>(W[(size_t)q * n + i], wi, r[q]);
                    }
                    wg_sum<double, ORTH_P>(r, sh);
                    for (int i = threadIdx.x; i < n; i += CWG) {
                        double2 wi = w[i];
#pragma unroll
                        for (int q = 0; q < ORTH_P; ++q)
                            if (q < p) wi = cfma<double>(cneg<double>(r[q]), W[(size_t)q * n + i], wi);
                        w[i] = wi;
                    }
                }
                double2 nn[1] = {make_double2(0, 0)};
                for (int i = threadIdx.x; i < n; i += CWG) nn[0].x += w[i].x * w[i].x + w[i].y * w[i].y;
                wg_sum<double, 1>(nn, sh);
                if (round == 0 && !(nn[0].x > 1e-24 * n0[p].x)) {
                    if (threadIdx.x == 0) rank_flag[0] = 1;
                    bad[p] = true;
                }
                if (bad[p]) continue;
                const double inv = 1.0 / sqrt(nn[0].x);
                for (int i = threadIdx.x; i < n; i += CWG) w[i] = make_double2(w[i].x * inv, w[i].y * inv);
            }
        }
    }
}

// The same Q by Cholesky QR applied twice (nvec <= 32): per block and
// chirality the Gram matrix G = V^dag V, its Cholesky factor R (G = R^dag R,
// R upper triangular with a positive real diagonal, so V = Q R is the thin QR
// in index order) and Q = V R^-1; the second round repeats this on Q, which
// restores orthogonality to rounding.  It reads the vectors 6 times instead of
// about 2 nvec times.  A pivot of the first round at most 1e-8 of its diagonal
// entry (a vector whose part outside the span of the previous ones is below
// 1e-4 of its norm) is out of reach of Cholesky QR in FP64; the caller then
// runs the Gram-Schmidt kernel above, whose rank test stays the reference.
constexpr int CHQ_MAXV = 32;   // vectors per block and chirality
constexpr int CHQ_CH = 64;     // indices staged per step of the Gram kernel
constexpr int CHQ_R = 2;       // Gram entries per work-item in each direction (16 x 16 work-items)

// partial Gram matrices: grid (2 Nc, parts); part z sums the indices of its
// contiguous range, Gp[(ah * parts + z)][j][k] = sum_i conj(V_j[i]) V_k[i]
__global__ void __launch_bounds__(CWG) chq_gram_kernel(CoarseGeom c, const double2* __restrict__ b64,
                                                       double2* __restrict__ Gp) {
    __shared__ double2 S[CHQ_MAXV][CHQ_CH + 1];
    const int ah = blockIdx.x, n = c.nvec, nh = c.nhalf;
    const double2* V = b64 + (size_t)ah * n * nh;
    const int nchunk = (nh + CHQ_CH - 1) / CHQ_CH;
    const int cb = (int)(((long long)nchunk * blockIdx.y) / gridDim.y);
    const int ce = (int)(((long long)nchunk * (blockIdx.y + 1)) / gridDim.y);
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    double2 acc[CHQ_R][CHQ_R];
#pragma unroll
    for (int r = 0; r < CHQ_R; ++r)
#pragma unroll
        for (int q = 0; q < CHQ_R; ++q) acc[r][q] = make_double2(0, 0);
    for (int ch = cb; ch < ce; ++ch) {
        const int i0 = ch * CHQ_CH;
        __syncthreads();  // the previous chunk has been read
        for (int e = threadIdx.x; e < CHQ_MAXV * CHQ_CH; e += CWG) {
            const int j = e / CHQ_CH, ii = e - j * CHQ_CH;
            S[j][ii] = (j < n && i0 + ii < nh) ? V[(size_t)j * nh + i0 + ii] : make_double2(0, 0);
        }
        __syncthreads();
        for (int ii = 0; ii < CHQ_CH; ++ii) {
            double2 a[CHQ_R], b[CHQ_R];
#pragma unroll
            for (int r = 0; r < CHQ_R; ++r) {
                a[r] = S[ty * CHQ_R + r][ii];
                b[r] = S[tx * CHQ_R + r][ii];
            }
#pragma unroll
            for (int r = 0; r < CHQ_R; ++r)
#pragma unroll
                for (int q = 0; q < CHQ_R; ++q) acc[r][q] = cjfma<double>(a[r], b[q], acc[r][q]);
        }
    }
    double2* G = Gp + ((size_t)ah * gridDim.y + blockIdx.y) * n * n;
#pragma unroll
    for (int r = 0; r < CHQ_R; ++r)
#pragma unroll
        for (int q = 0; q < CHQ_R; ++q) {
            const int j = ty * CHQ_R + r, k = tx * CHQ_R + q;
            if (j < n && k < n) G[j * n + k] = acc[r][q];
        }
}

// one wavefront per block and chirality: G = sum of the partials in part
// order, its Cholesky factor R and Rinv = R^-1 (upper triangular; zeros below
// the diagonal).  First pass (pass = 0): a pivot d_k <= 1e-8 G_kk sets flag[1]
// (Cholesky QR out of reach: use Gram-Schmidt); second pass (pass = 1): a pivot
// <= G_kk / 4, impossible for the nearly orthonormal output of the first, sets
// flag[2].
__global__ void __launch_bounds__(64) chq_chol_kernel(CoarseGeom c, const double2* __restrict__ Gp, int parts,
                                                      int pass, double2* __restrict__ Rinv, int* __restrict__ flag) {
    __shared__ double2 G[CHQ_MAXV][CHQ_MAXV + 1];
    __shared__ double2 Rm[CHQ_MAXV][CHQ_MAXV + 1];
    __shared__ double2 X[CHQ_MAXV][CHQ_MAXV + 1];
    const int ah = blockIdx.x, n = c.nvec, l = threadIdx.x;
    for (int e = l; e < n * n; e += 64) {
        double2 g = make_double2(0, 0);
        for (int z = 0; z < parts; ++z) g = cadd<double>(g, Gp[((size_t)ah * parts + z) * n * n + e]);
        G[e / n][e % n] = g;
    }
    __syncthreads();
    const double thr = (pass == 0) ? 1e-8 : 0.25;
    for (int k = 0; k < n; ++k) {
        if (l == k) {
            double d = G[k][k].x;
            for (int j = 0; j < k; ++j) d -= Rm[j][k].x * Rm[j][k].x + Rm[j][k].y * Rm[j][k].y;
            if (!(d > thr * G[k][k].x)) {
                flag[pass == 0 ? 1 : 2] = 1;
                d = 1.0;  // keep the factor finite; the caller discards it
            }
            Rm[k][k] = make_double2(sqrt(d), 0.0);
        }
        __syncthreads();
        if (l > k && l < n) {
            double2 sacc = G[k][l];
            for (int j = 0; j < k; ++j) sacc = cjfma<double>(cneg<double>(Rm[j][k]), Rm[j][l], sacc);
            const double inv = 1.0 / Rm[k][k].x;
            Rm[k][l] = make_double2(sacc.x * inv, sacc.y * inv);
        }
        __syncthreads();
    }
    // column l of R^-1 by back substitution
    if (l < n) {
        X[l][l] = make_double2(1.0 / Rm[l][l].x, 0.0);
        for (int k = l - 1; k >= 0; --k) {
            double2 sacc = make_double2(0, 0);
            for (int j = k + 1; j <= l; ++j) sacc = cfma<double>(Rm[k][j], X[j][l], sacc);
            const double inv = -1.0 / Rm[k][k].x;
            X[k][l] = make_double2(sacc.x * inv, sacc.y * inv);
        }
    }
    __syncthreads();
    for (int e = l; e < n * n; e += 64) {
        const int k = e / n, q = e % n;
        Rinv[(size_t)ah * n * n + e] = (k <= q) ? X[k][q] : make_double2(0, 0);
    }
}

// V <- V Rinv in place: grid (2 Nc, parts); a workgroup stages 64 indices of
// all nvec vectors in LDS, then work-item (i, g) forms columns 8 g .. 8 g + 7 of
// index i (column q sums rows k <= q) and writes them back
constexpr int CHQ_TI = 64;
__global__ void __launch_bounds__(CWG) chq_apply_kernel(CoarseGeom c, double2* __restrict__ b64,
                                                        const double2* __restrict__ Rinv) {
    __shared__ double2 Ri[CHQ_MAXV * CHQ_MAXV];
    __shared__ double2 S[CHQ_MAXV][CHQ_TI + 1];
    const int ah = blockIdx.x, n = c.nvec, nh = c.nhalf;
    for (int e = threadIdx.x; e < n * n; e += CWG) Ri[e] = Rinv[(size_t)ah * n * n + e];
    double2* V = b64 + (size_t)ah * n * nh;
    const int ii = threadIdx.x % CHQ_TI, g = threadIdx.x / CHQ_TI;  // 4 groups of 8 columns
    const int ntile = (nh + CHQ_TI - 1) / CHQ_TI;
    for (int t = blockIdx.y; t < ntile; t += gridDim.y) {
        const int i0 = t * CHQ_TI;
        __syncthreads();  // Ri staged; the previous tile has been read
        for (int e = threadIdx.x; e < n * CHQ_TI; e += CWG) {
            const int k = e / CHQ_TI, x = e - k * CHQ_TI;
            S[k][x] = (i0 + x < nh) ? V[(size_t)k * nh + i0 + x] : make_double2(0, 0);
        }
        __syncthreads();
        double2 w[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) w[q] = make_double2(0, 0);
        const int q0 = 8 * g;
        const int kmax = min(n, q0 + 8);
        for (int k = 0; k < kmax; ++k) {
            const double2 v = S[k][ii];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (k <= q0 + q) w[q] = cfma<double>(v, Ri[k * n + min(q0 + q, n - 1)], w[q]);
        }
        if (i0 + ii < nh) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q0 + q < n) V[(size_t)(q0 + q) * nh + i0 + ii] = w[q];
        }
    }
}

__global__ void __launch_bounds__(CWG) basis_to_f32_kernel(size_t n, const double2* __restrict__ a,
                                                           float2* __restrict__ b) {
    for (size_t e = (size_t)blockIdx.x * CWG + threadIdx.x; e < n; e += (size_t)gridDim.x * CWG)
        b[e] = make_float2((float)a[e].x, (float)a[e].y);
}

// FP16 copy of the basis: HBASIS_SCALE * phi, rounded to nearest even
__global__ void __launch_bounds__(CWG) basis_to_f16_kernel(size_t n, const double2* __restrict__ a,
                                                           uint32_t* __restrict__ b) {
    for (size_t e = (size_t)blockIdx.x * CWG + threadIdx.x; e < n; e += (size_t)gridDim.x * CWG) {
        const _Float16 re = (_Float16)((float)(a[e].x * (double)HBASIS_SCALE));
        const _Float16 im = (_Float16)((float)(a[e].y * (double)HBASIS_SCALE));
        b[e] = (uint32_t)__builtin_bit_cast(unsigned short, re) | ((uint32_t)__builtin_bit_cast(unsigned short, im) << 16);
    }
}

// fields[kk][comp][site][s] = basis vector k0+kk as a full fine field
__global__ void __launch_bounds__(CWG) basis_expand_kernel(CoarseGeom c, const double2* __restrict__ b64, int k0,
                                                           int nk, double2* __restrict__ fields) {
    const size_t per = (size_t)12 * c.f.N5;
    const size_t total = per * nk;
    for (size_t e = (size_t)blockIdx.x * CWG + threadIdx.x; e < total; e += (size_t)gridDim.x * CWG) {
        const int kk = (int)(e / per);
        size_t r = e % per;
        const int s = (int)(r % c.f.Ls);
        r /= c.f.Ls;
        const int site = (int)(r % c.f.V4);
        const int comp = (int)(r / c.f.V4);
        // coordinates -> block and block-local site
        int x[4], t = site;
        x[0] = t % c.f.L[0];
        t /= c.f.L[0];
        x[1] = t % c.f.L[1];
        t /= c.f.L[1];
        x[2] = t % c.f.L[2];
        x[3] = t / c.f.L[2];
        int a = 0, sl = 0;
#pragma unroll
        for (int mu = 3; mu >= 0; --mu) {
            a = a * c.C[mu] + x[mu] / c.B[mu];
            sl = sl * c.B[mu] + x[mu] % c.B[mu];
        }
        const int k = k0 + kk;
        const int h = (k < c.nvec) ? 0 : 1;
        const int kh = k - h * c.nvec;
        const bool upper_s = s < c.Lh;
        const int sc = upper_s ? s : c.f.Ls - 1 - s;
        const int i = (comp * c.bvol + sl) * c.Lh + sc;
        double2 v = b64[(((size_t)a * 2 + h) * c.nvec + kh) * c.nhalf + i];
        double f = RSQRT2;
        if (!upper_s) f *= (h == 0 ? 1.0 : -1.0) * (comp < 6 ? 1.0 : -1.0);
        fields[e] = make_double2(v.x * f, v.y * f);
    }
}

// ---------------------------------------------------------------------------
// restriction and prolongation
// ---------------------------------------------------------------------------

// two consecutive complex entries (s and s+1 of one component)
template <typename T> struct Pair {
    C2<T> a, b;
};
template <typename T> __device__ __forceinline__ Pair<T> ld_pair(const C2<T>* p) {
    Pair<T> r;
    if constexpr (sizeof(T) == 4) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        r.a = mk<T>(q.x, q.y);
        r.b = mk<T>(q.z, q.w);
    } else {
        r.a = p[0];
        r.b = p[1];
    }
    return r;
}

// W consecutive basis entries starting at p, as complex T: the FP64 / FP32
// regions directly, the FP16 copy ((fp16 re, fp16 im) words holding
// HBASIS_SCALE * phi) decoded and rescaled.
__device__ __forceinline__ float2 dec_h(uint32_t w) {
    const float re = (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
    const float im = (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
    constexpr float inv = 1.0f / HBASIS_SCALE;
    return make_float2(re * inv, im * inv);
}
template <typename T, int W> __device__ __forceinline__ void ld_basis(const C2<T>* p, C2<T> (&o)[W]) {
    if constexpr (W >= 4) {
#pragma unroll
        for (int u = 0; u < W / 2; ++u) {
            const Pair<T> q = ld_pair<T>(p + 2 * u);
            o[2 * u] = q.a;
            o[2 * u + 1] = q.b;
        }
    } else if constexpr (W == 2) {
        const Pair<T> q = ld_pair<T>(p);
        o[0] = q.a;
        o[1] = q.b;
    } else {
        o[0] = *p;
    }
}
template <typename T, int W> __device__ __forceinline__ void ld_basis(const uint32_t* p, float2 (&o)[W]) {
    if constexpr (W >= 4) {
#pragma unroll
        for (int u = 0; u < W / 4; ++u) {
            const uint4 q = *reinterpret_cast<const uint4*>(p + 4 * u);
            o[4 * u] = dec_h(q.x);
            o[4 * u + 1] = dec_h(q.y);
            o[4 * u + 2] = dec_h(q.z);
            o[4 * u + 3] = dec_h(q.w);
        }
    } else if constexpr (W == 2) {
        const uint2 q = *reinterpret_cast<const uint2*>(p);
        o[0] = dec_h(q.x);
        o[1] = dec_h(q.y);
    } else {
        o[0] = dec_h(*p);
    }
}

// basis vectors per restriction workgroup: all 32 at nvec >= 32 (psi is then
// read by two workgroups per coarse site), else 16
constexpr int RKG_MAX = 32;

// grid (Nc, 2 chiralities, ceil(nvec / RKG)): v[a][h*nvec + k] = <phi^{a,h}_k, psi - psi2>
// for the RKG vectors k of the workgroup.  Work-item = (row slot, W consecutive s):
// a row is (component, block site), so the loads of the compressed basis (index
// row * Lh + s) and of psi are contiguous; W = 2 (Lh even) makes them 16-byte
// pairs in FP32.
template <typename T, typename B, bool SUB, int W, int RKG>
__global__ void __launch_bounds__(CWG) restrict_kernel(CoarseGeom c, const B* __restrict__ basis,
                                                       const C2<T>* __restrict__ psi, const C2<T>* __restrict__ psi2,
                                                       C2<T>* __restrict__ v) {
    __shared__ C2<T> sh[4 * RKG];
    // one-dimensional grid of Nc x 2 x (vector groups) workgroups, remapped
    // so that the workgroups of one coarse site (both chiralities, every
    // vector group) are consecutive on one XCD: the site's psi block is then
    // read from memory once and served from that XCD's L2 to the others
    const int ng = (c.nvec + RKG - 1) / RKG;
    const int lb = logical_block(blockIdx.x, gridDim.x);
    const int a = lb / (2 * ng), h = (lb / ng) % 2;
    const int k0 = (lb % ng) * RKG;
    const int kn = min(RKG, c.nvec - k0);
    const int nsp = c.Lh / W;                 // s slots per row
    const int slots = CWG / nsp;              // rows processed per sweep
    const int sp = threadIdx.x % nsp, q0 = threadIdx.x / nsp;
    const int s = W * sp;
    const int nrows = 12 * c.bvol;
    const B* bh = basis + (((size_t)a * 2 + h) * c.nvec + k0) * c.nhalf;
    const T r2 = (T)RSQRT2;
    C2<T> acc[RKG];
#pragma unroll
    for (int q = 0; q < RKG; ++q) acc[q] = mk<T>(0, 0);
    if (q0 < slots) {
        for (int row = q0; row < nrows; row += slots) {
            const int comp = row / c.bvol, sl = row - comp * c.bvol;
            const size_t fb = ((size_t)comp * c.f.V4 + block_site(c, a, sl)) * c.f.Ls;
            // slot s + w pairs with the mirrored Ls-1-s-w
            C2<T> p1[W], p2[W];
            if constexpr (W >= 4) {
                // pairs from both ends: slot s + w and its mirror Ls-1-s-w
#pragma unroll
                for (int u = 0; u < W / 2; ++u) {
                    const Pair<T> lo = ld_pair<T>(psi + fb + s + 2 * u);
                    const Pair<T> hi = ld_pair<T>(psi + fb + c.f.Ls - 2 - s - 2 * u);
                    p1[2 * u] = lo.a;
                    p1[2 * u + 1] = lo.b;
                    p2[2 * u] = hi.b;
                    p2[2 * u + 1] = hi.a;
                }
            } else if constexpr (W == 2) {
                const Pair<T> lo = ld_pair<T>(psi + fb + s), hi = ld_pair<T>(psi + fb + c.f.Ls - 2 - s);
                p1[0] = lo.a;
                p1[1] = lo.b;
                p2[0] = hi.b;
                p2[1] = hi.a;
            } else {
                p1[0] = psi[fb + s];
                p2[0] = psi[fb + c.f.Ls - 1 - s];
            }
            if constexpr (SUB) {
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    p1[w] = csub<T>(p1[w], psi2[fb + s + w]);
                    p2[w] = csub<T>(p2[w], psi2[fb + c.f.Ls - 1 - s - w]);
                }
            }
            const T sg = ((comp < 6) == (h == 0)) ? (T)1 : (T)-1;
            C2<T> f[W];
#pragma unroll
            for (int w = 0; w < W; ++w) f[w] = mk<T>((p1[w].x + sg * p2[w].x) * r2, (p1[w].y + sg * p2[w].y) * r2);
            const size_t i = (size_t)row * c.Lh + s;
#pragma unroll
            for (int q = 0; q < RKG; ++q) {
                if (q < kn) {
                    C2<T> bv[W];
                    ld_basis<T, W>(bh + (size_t)q * c.nhalf + i, bv);
#pragma unroll
                    for (int w = 0; w < W; ++w) acc[q] = cjfma<T>(bv[w], f[w], acc[q]);
                }
            }
        }
    }
    wg_sum<T, RKG>(acc, sh);
#pragma unroll
    for (int q = 0; q < RKG; ++q)
        if ((int)threadIdx.x == q && q < kn) v[(size_t)a * c.Nb + h * c.nvec + k0 + q] = acc[q];
}

// Vectors whose basis entries a prolongation work-item requests together: 8
// (108 VGPRs, 4 waves per SIMD) took 1.73 ms at 24^4 x 16 against 1.87 ms for
// one vector at a time, timed in one process (2 and 4 lay in between).
constexpr int PKU = 8;

// psi = y + P v for coarse site a (workgroups blockIdx.y = 0 .. gridDim.y - 1
// take consecutive parts of its compressed indices, each part a multiple of NI
// long).  A work-item handles NI consecutive compressed indices (4 when nhalf is
// a multiple of 4, else 2; nhalf is even), so the basis loads are 16-byte (FP16
// at NI = 4, FP32 at NI = 2) or 8-byte runs; each index yields the pair of
// outputs at s and its mirror Ls-1-s.
template <typename T, typename B, int NI>
__global__ void __launch_bounds__(CWG) prolong_kernel(CoarseGeom c, const B* __restrict__ basis,
                                                      const C2<T>* __restrict__ v, const C2<T>* __restrict__ y,
                                                      C2<T>* __restrict__ psi) {
    extern __shared__ unsigned char smem_raw[];
    C2<T>* vs = reinterpret_cast<C2<T>*>(smem_raw);
    const int a = blockIdx.x;
    for (int j = threadIdx.x; j < c.Nb; j += CWG) vs[j] = v[(size_t)a * c.Nb + j];
    __syncthreads();
    const B* bp = basis + ((size_t)a * 2 + 0) * c.nvec * c.nhalf;
    const B* bm = basis + ((size_t)a * 2 + 1) * c.nvec * c.nhalf;
    const T r2 = (T)RSQRT2;
    const int part = NI * ((c.nhalf / NI + (int)gridDim.y - 1) / (int)gridDim.y);
    const int beg = (int)blockIdx.y * part;
    const int end = min(c.nhalf, beg + part);
    for (int i0 = beg + NI * threadIdx.x; i0 < end; i0 += NI * CWG) {
        C2<T> tp[NI], tm[NI];
#pragma unroll
        for (int q = 0; q < NI; ++q) tp[q] = tm[q] = mk<T>(0, 0);
        // PKU vectors' basis entries are requested before the first of them is
        // used; the products are summed in vector order as one at a time would
        int k = 0;
        for (; k + PKU <= c.nvec; k += PKU) {
            C2<T> ep[PKU][NI], em[PKU][NI];
#pragma unroll
            for (int u = 0; u < PKU; ++u) {
                ld_basis<T, NI>(bp + (size_t)(k + u) * c.nhalf + i0, ep[u]);
                ld_basis<T, NI>(bm + (size_t)(k + u) * c.nhalf + i0, em[u]);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < PKU; ++u) {
                const C2<T> xp = vs[k + u], xm = vs[c.nvec + k + u];
#pragma unroll
                for (int q = 0; q < NI; ++q) {
                    tp[q] = cfma<T>(ep[u][q], xp, tp[q]);
                    tm[q] = cfma<T>(em[u][q], xm, tm[q]);
                }
            }
        }
        for (; k < c.nvec; ++k) {
            C2<T> ep[NI], em[NI];
            ld_basis<T, NI>(bp + (size_t)k * c.nhalf + i0, ep);
            ld_basis<T, NI>(bm + (size_t)k * c.nhalf + i0, em);
            const C2<T> xp = vs[k], xm = vs[c.nvec + k];
#pragma unroll
            for (int q = 0; q < NI; ++q) {
                tp[q] = cfma<T>(ep[q], xp, tp[q]);
                tm[q] = cfma<T>(em[q], xm, tm[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < NI; ++q) {
            const int i = i0 + q;
            const int s = i % c.Lh;
            const int sl = (i / c.Lh) % c.bvol;
            const int comp = i / (c.Lh * c.bvol);
            const size_t fb = ((size_t)comp * c.f.V4 + block_site(c, a, sl)) * c.f.Ls;
            const T g = (comp < 6) ? (T)1 : (T)-1;
            C2<T> o1 = mk<T>((tp[q].x + tm[q].x) * r2, (tp[q].y + tm[q].y) * r2);
            C2<T> o2 = mk<T>(g * (tp[q].x - tm[q].x) * r2, g * (tp[q].y - tm[q].y) * r2);
            if (y) {
                o1 = cadd<T>(o1, y[fb + s]);
                o2 = cadd<T>(o2, y[fb + c.f.Ls - 1 - s]);
            }
            psi[fb + s] = o1;
            psi[fb + c.f.Ls - 1 - s] = o2;
        }
    }
}

// ---------------------------------------------------------------------------
// coarse apply (column-major blocks: A[a][d][k][j], a lane owns row j)
// ---------------------------------------------------------------------------

template <typename T, typename S> __device__ __forceinline__ C2<T> ldA(const S* A, size_t idx);
template <> __device__ __forceinline__ float2 ldA<float, float2>(const float2* A, size_t idx) { return A[idx]; }
template <> __device__ __forceinline__ float2 ldA<float, uint32_t>(const uint32_t* A, size_t idx) {
    const uint32_t w = A[idx];  // (bf16 re, bf16 im)
    return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
}

// E consecutive entries A[.][k][j..j+E) with one 16-byte load (E = 16 / entry
// size; E = 1 falls back to single-entry loads)
template <typename T, typename S, int E> struct WideA;
template <typename T, typename S> struct WideA<T, S, 1> {
    static __device__ __forceinline__ void ld(const S* p, C2<T> (&e)[1]) { e[0] = ldA<T, S>(p, 0); }
};
template <> struct WideA<double, double2, 1> {
    static __device__ __forceinline__ void ld(const double2* p, double2 (&e)[1]) { e[0] = *p; }
};
template <> struct WideA<float, float2, 2> {
    static __device__ __forceinline__ void ld(const float2* p, float2 (&e)[2]) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        e[0] = make_float2(q.x, q.y);
        e[1] = make_float2(q.z, q.w);
    }
};
template <> struct WideA<float, uint32_t, 4> {
    static __device__ __forceinline__ void ld(const uint32_t* p, float2 (&e)[4]) {
        const uint4 q = *reinterpret_cast<const uint4*>(p);
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) e[i] = make_float2(__uint_as_float(w[i] << 16), __uint_as_float(w[i] & 0xffff0000u));
    }
};
template <typename S> constexpr int wide_entries() { return (int)(16 / sizeof(S)); }

// res[j] = sum_d sum_k A[a][d][k][j] vs[d][k] for one coarse site a (one
// workgroup).  Work-item t covers E consecutive rows j (t % (Nb/E)) and the
// columns k = kk, kk + kg, ... (kk = t / (Nb/E), kg = CWG / (Nb/E) groups), so
// every load of A is a contiguous 16-byte run and a work-item issues
// 9 Nb / kg independent loads; the kg partial sums are added in a fixed order.
// red: LDS of CWG * E complex; ends with a barrier.
template <typename T, typename S, int E>
__device__ __forceinline__ void site_gemv(const CoarseGeom& c, const S* __restrict__ A, int a, const C2<T>* vs,
                                          C2<T>* red, C2<T>* res) {
    const int Nb = c.Nb;
    const int nj = Nb / E;
    const int kg = CWG / nj;
    const int t = threadIdx.x;
    const int jq = t % nj, kk = t / nj;
    C2<T> acc[E];
#pragma unroll
    for (int q = 0; q < E; ++q) acc[q] = mk<T>(0, 0);
    if (kk < kg) {
        const size_t blk = (size_t)Nb * Nb;
        const S* Aa = A + (size_t)a * 9 * blk + (size_t)jq * E;
        for (int d = 0; d < 9; ++d) {
            const S* Ad = Aa + d * blk;
            const C2<T>* vd = vs + d * Nb;
#pragma unroll 4
            for (int k = kk; k < Nb; k += kg) {
                C2<T> e[E];
                WideA<T, S, E>::ld(Ad + (size_t)k * Nb, e);
                const C2<T> x = vd[k];
#pragma unroll
                for (int q = 0; q < E; ++q) acc[q] = cfma<T>(e[q], x, acc[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < E; ++q) red[kk * Nb + jq * E + q] = acc[q];
    }
    __syncthreads();
    for (int j = t; j < Nb; j += CWG) {
        C2<T> sum = red[j];
        for (int g = 1; g < kg; ++g) sum = cadd<T>(sum, red[g * Nb + j]);
        res[j] = sum;
    }
    __syncthreads();
}

// LDS bytes of a coarse-apply workgroup: vs [9][Nb], red [CWG * E], res [Nb]
template <typename T, int E> size_t apply_lds(const CoarseGeom& c) {
    return (size_t)(10 * c.Nb + CWG * E) * sizeof(C2<T>);
}

// one workgroup per (coarse site, right-hand side); the neighbour vectors are
// staged in LDS
template <typename T, typename S, int E>
__global__ void __launch_bounds__(CWG) coarse_apply_kernel(CoarseGeom c, const S* __restrict__ A,
                                                           const C2<T>* __restrict__ v, C2<T>* __restrict__ out) {
    extern __shared__ unsigned char smem_raw[];
    C2<T>* vs = reinterpret_cast<C2<T>*>(smem_raw);   // [9][Nb]
    C2<T>* res = vs + 9 * c.Nb;                        // [Nb]
    C2<T>* red = res + c.Nb;                           // [CWG * E]
    const int a = blockIdx.x;
    const int rhs = blockIdx.y;
    const C2<T>* vr = v + (size_t)rhs * c.Nc * c.Nb;
    for (int e = threadIdx.x; e < 9 * c.Nb; e += CWG) {
        const int d = e / c.Nb, k = e - d * c.Nb;
        vs[e] = vr[(size_t)coarse_nbr(c, a, d) * c.Nb + k];
    }
    __syncthreads();
    site_gemv<T, S, E>(c, A, a, vs, red, res);
    for (int j = threadIdx.x; j < c.Nb; j += CWG) out[((size_t)rhs * c.Nc + a) * c.Nb + j] = res[j];
}

// ---------------------------------------------------------------------------
// coarse conjugate residual
// ---------------------------------------------------------------------------

// After every workgroup has stored its partial sums, true in the workgroup
// that arrived last (which then reduces them in a fixed order).
__device__ __forceinline__ bool last_arrival(int* counters) {
    // Arrivals are counted in ARRIVE_GROUPS group counters (workgroup b in group
    // b % ARRIVE_GROUPS, each on its own cache line) and a master counter that
    // the last workgroup of each group increments: a single counter hit by
    // every workgroup serialises ~Nc device-scope atomics.  Counters return to
    // zero for the next launch.
    __shared__ int is_last;
    const int nb = (int)(gridDim.x * gridDim.y);
    const int b = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const int g = b % ARRIVE_GROUPS;
        const int gsize = (nb - g + ARRIVE_GROUPS - 1) / ARRIVE_GROUPS;
        const int ngroups = nb < ARRIVE_GROUPS ? nb : ARRIVE_GROUPS;
        int last = 0;
        int* cg = counters + (1 + g) * ARRIVE_STRIDE;
        if (atomicAdd(cg, 1) == gsize - 1) {
            atomicExch(cg, 0);
            __threadfence();
            if (atomicAdd(counters, 1) == ngroups - 1) {
                atomicExch(counters, 0);
                last = 1;
            }
        }
        is_last = last;
    }
    __syncthreads();
    return is_last != 0;
}

// fixed-order sum of nq rows of np partials (row q at part + q*np), in the last block
template <int NQ>
__device__ __forceinline__ void reduce_partials(const double* part, int np, double (&out)[NQ]) {
    __threadfence();
    double v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] += __builtin_nontemporal_load(part + (size_t)q * np + i);
    }
    block_reduce<NQ>(v);
#pragma unroll
    for (int q = 0; q < NQ; ++q) out[q] = v[q];
}

// fixed-order sum of nq rows of np partials written by an earlier kernel; every
// workgroup that calls it gets the same values (no cross-workgroup traffic)
template <int NQ>
__device__ __forceinline__ void sum_partials(const double* part, int np, double (&out)[NQ]) {
    double v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = 0.0;
#pragma unroll 4
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] += part[(size_t)q * np + i];
    }
    block_reduce<NQ>(v);
#pragma unroll
    for (int q = 0; q < NQ; ++q) out[q] = v[q];
}

// Near-breakdown test of the coarse CR: <r, Ar> is the numerator of alpha and the
// denominator of the next beta; once |<r, Ar>| < eps |r| |Ar| the recurrence makes
// no progress (alpha ~ 0) or loses its conjugacy (beta unbounded), so the solve
// stops with the iterate it has.  eps = 1e-13 for FP64 vectors (the fine CR's and
// the oracle's threshold) and 1e-6 for FP32 vectors, about 8 units of FP32
// roundoff, below which <r, Ar> of an FP32 apply is rounding noise.
// Returns 0 (go on), 2 (breakdown) or 3 (not finite).
template <typename T> __device__ __forceinline__ int ccr_breakdown(double rar, double rr, double arar) {
    constexpr double eps = sizeof(T) == 8 ? 1e-13 : 1e-6;
    if (!isfinite(rar) || !isfinite(arar)) return 3;
    return (fabs(rar) > eps * sqrt(rr) * sqrt(arar)) ? 0 : 2;
}

template <typename T>
__global__ void __launch_bounds__(CWG) ccr_init_kernel(int n, const C2<T>* __restrict__ b, C2<T>* __restrict__ x,
                                                       C2<T>* __restrict__ r, double* part, double* cs, int* flags,
                                                       int maxiter, double tol2) {
    double v[1] = {0.0};
    for (int i = blockIdx.x * CWG + threadIdx.x; i < n; i += gridDim.x * CWG) {
        const C2<T> bv = b[i];
        r[i] = bv;
        x[i] = mk<T>(0, 0);
        v[0] += (double)bv.x * bv.x + (double)bv.y * bv.y;
    }
    block_reduce<1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
    if (last_arrival(flags + CCR_COUNTERS)) {
        double s[1];
        reduce_partials<1>(part, gridDim.x, s);
        if (threadIdx.x == 0) {
            cs[4] = s[0];
            cs[3] = s[0];
            cs[5] = tol2;
            flags[3] = maxiter;
            flags[1] = 0;
            flags[4] = 0;
            flags[0] = (s[0] == 0.0 || maxiter <= 0 || !isfinite(s[0])) ? 1 : 0;
        }
    }
}

// Partial sums of <V_j, b> for the eight deflation vectors j = 8*blockIdx.y + jj:
// dpart[(16*blockIdx.y + 2*jj (+1)) * DEFL_BLOCKS + blockIdx.x] (re, im).
template <typename T>
__global__ void __launch_bounds__(CWG) defl_dot_kernel(int n, DeflView<T> d, const C2<T>* __restrict__ b,
                                                       double* __restrict__ dpart) {
    const int j0 = blockIdx.y * 8;
    const int nv = min(8, d.k - j0);
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    for (int i = blockIdx.x * CWG + threadIdx.x; i < n; i += gridDim.x * CWG) {
        const C2<T> bv = b[i];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            if (jj < nv) {
                const C2<T> v = d.V[(size_t)(j0 + jj) * n + i];
                acc[2 * jj] += (double)v.x * bv.x + (double)v.y * bv.y;
                acc[2 * jj + 1] += (double)v.x * bv.y - (double)v.y * bv.x;
            }
        }
    }
    block_reduce<16>(acc);
    if (threadIdx.x == 0) {
        for (int q = 0; q < 16; ++q) dpart[((size_t)blockIdx.y * 16 + q) * DEFL_BLOCKS + blockIdx.x] = acc[q];
    }
}

// coef[q] = (sum of the dot partials of row q, fixed order) / theta_{q/2}: one
// work-group per real or imaginary part q < 2k
template <typename T>
__global__ void __launch_bounds__(CWG) defl_coef_kernel(DeflView<T> d, const double* __restrict__ dpart,
                                                        double* __restrict__ coef) {
    const int q = blockIdx.x, j = q >> 1;
    const double* row = dpart + ((size_t)(j >> 3) * 16 + 2 * (j & 7) + (q & 1)) * DEFL_BLOCKS;
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < DEFL_BLOCKS; i += CWG) v[0] += row[i];
    block_reduce<1>(v);
    if (threadIdx.x == 0) coef[q] = v[0] / d.theta[j];
}

// x = sum_j g_j V_j, r = b - sum_j g_j W_j with g_j = <V_j, b> / theta_j (from
// defl_coef_kernel); then as ccr_init with cs[3] = |r|^2 and cs[4] = |b|^2
template <typename T>
__global__ void __launch_bounds__(CWG) ccr_init_defl_kernel(int n, const C2<T>* __restrict__ b, C2<T>* __restrict__ x,
                                                            C2<T>* __restrict__ r, DeflView<T> d,
                                                            const double* __restrict__ coef, double* part,
                                                            double* cs, int* flags, int maxiter, double tol2) {
    __shared__ double gs[2 * DEFL_KMAX];
    for (int q = threadIdx.x; q < 2 * d.k; q += CWG) gs[q] = coef[q];
    __syncthreads();
    double v[2] = {0.0, 0.0};
    for (int i = blockIdx.x * CWG + threadIdx.x; i < n; i += gridDim.x * CWG) {
        const C2<T> bv = b[i];
        double2 xa = make_double2(0.0, 0.0), ra = make_double2(bv.x, bv.y);
#pragma unroll 8
        for (int j = 0; j < d.k; ++j) {
            const double2 g = make_double2(gs[2 * j], gs[2 * j + 1]);
            const C2<T> vv = d.V[(size_t)j * n + i], wv = d.W[(size_t)j * n + i];
            xa = cfma<double>(g, make_double2(vv.x, vv.y), xa);
            ra = cfma<double>(cneg<double>(g), make_double2(wv.x, wv.y), ra);
        }
        const C2<T> xo = mk<T>((T)xa.x, (T)xa.y), ro = mk<T>((T)ra.x, (T)ra.y);
        x[i] = xo;
        r[i] = ro;
        v[0] += (double)bv.x * bv.x + (double)bv.y * bv.y;
        v[1] += (double)ro.x * ro.x + (double)ro.y * ro.y;
    }
    block_reduce<2>(v);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = v[0];
        part[gridDim.x + blockIdx.x] = v[1];
    }
    if (last_arrival(flags + CCR_COUNTERS)) {
        double s[2];
        reduce_partials<2>(part, gridDim.x, s);
        if (threadIdx.x == 0) {
            cs[4] = s[0];
            cs[3] = s[1];
            cs[5] = tol2;
            flags[3] = maxiter;
            flags[1] = 0;
            flags[4] = 0;
            flags[0] = (s[0] == 0.0 || maxiter <= 0 || !isfinite(s[0]) || !isfinite(s[1])) ? 1 : 0;
        }
    }
}

// Ar = A r for coarse site a (one workgroup).  Partial sums per coarse site:
// <r,Ar> to part[a], |Ar|^2 to part[Nc+a] and Re<Ap,Ar> (Ap of the previous
// step; 0 on the first apply, FIRST) to part[2Nc+a].
template <typename T, typename S, int E, bool FIRST>
__global__ void __launch_bounds__(CWG) ccr_apply_kernel(CoarseGeom c, const S* __restrict__ A,
                                                        const C2<T>* __restrict__ r, C2<T>* __restrict__ Ar,
                                                        const C2<T>* __restrict__ Ap, double* part, int* flags) {
    if (flags[0]) return;
    extern __shared__ unsigned char smem_raw[];
    C2<T>* vs = reinterpret_cast<C2<T>*>(smem_raw);   // [9][Nb]
    C2<T>* res = vs + 9 * c.Nb;                        // [Nb]
    C2<T>* red = res + c.Nb;                           // [CWG * E]
    const int a = blockIdx.x;
    for (int e = threadIdx.x; e < 9 * c.Nb; e += CWG) {
        const int d = e / c.Nb, k = e - d * c.Nb;
        vs[e] = r[(size_t)coarse_nbr(c, a, d) * c.Nb + k];
    }
    __syncthreads();
    site_gemv<T, S, E>(c, A, a, vs, red, res);
    double sums[3] = {0.0, 0.0, 0.0};
    for (int j = threadIdx.x; j < c.Nb; j += CWG) {
        const C2<T> o = res[j];
        const size_t idx = (size_t)a * c.Nb + j;
        Ar[idx] = o;
        const C2<T> rv = vs[j];  // d = 0 slot holds r(a)
        sums[0] += (double)rv.x * o.x + (double)rv.y * o.y;
        sums[1] += (double)o.x * o.x + (double)o.y * o.y;
        if (!FIRST) {
            const C2<T> q = Ap[idx];
            sums[2] += (double)q.x * o.x + (double)q.y * o.y;
        }
    }
    block_reduce<3>(sums);
    // partial sums only: the update kernel reduces them in every one of its
    // workgroups (no device-scope fence and atomic per coarse site here)
    if (threadIdx.x == 0) {
        part[a] = sums[0];
        part[c.Nc + a] = sums[1];
        part[2 * c.Nc + a] = sums[2];
    }
}

// CR step k (k >= 1) after the apply of r_k, in a single pass:
//   beta = <r,Ar>_k / <r,Ar>_{k-1}, p = r + beta p, Ap = Ar + beta Ap
//   (step 1: p = r, Ap = Ar),
//   alpha = <r,Ar>_k / |Ap|^2,  x += alpha p,  r -= alpha Ap,
// with |Ap|^2 = |Ar|^2 + 2 beta Re<Ap_old,Ar> + beta^2 |Ap_old|^2 from the
// apply's partials, so no reduction separates the p update from the x, r update.
// The step needs no grid-wide arrival either: it stores its per-work-group
// partials of |r_{k+1}|^2 and |Ap_k|^2 (uout), and step k+1 reduces them
// (uin, the other half of a ping-pong pair) in each of its work-groups, ordered
// by the kernel boundary.  So the convergence test of r_k runs at the start of
// step k (from step 2 on; step 1 runs unconditionally, as the start kernel only
// stops on a zero or non-finite b), and a converged r_k costs one apply that is
// not used.  All work-groups reduce the same partials in the same order and so
// take the same decisions; work-group 0 records them.
template <typename T>
__global__ void __launch_bounds__(CWG) ccr_update_kernel(int n, C2<T>* __restrict__ x, C2<T>* __restrict__ r,
                                                         C2<T>* __restrict__ p, const C2<T>* __restrict__ Ar,
                                                         C2<T>* __restrict__ Ap, const double* apart, int nc,
                                                         const double* uin, double* uout, double* cs, int* flags,
                                                         int step) {
    if (flags[0]) return;
    const bool first = step == 1;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    // the apply's partials (t[0..2]) and the previous step's (t[3..4]) in one
    // pass and one workgroup reduction, each sum in the order of sum_partials
    double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int i = threadIdx.x; i < nc; i += CWG) {
#pragma unroll
        for (int q = 0; q < 3; ++q) t[q] += apart[(size_t)q * nc + i];
    }
    if (!first) {
        const int nu = (int)gridDim.x;
        for (int i = threadIdx.x; i < nu; i += CWG) {
            t[3] += uin[i];
            t[4] += uin[nu + i];
        }
    }
    block_reduce<5>(t);
    double rr = cs[3], apold = 0.0;
    if (!first) {
        rr = t[3];
        apold = t[4];
        if (rr <= cs[5] * cs[4] || !isfinite(rr)) {  // r_k converged (or not finite): x_k is the result
            if (lead) flags[0] = 1;
            return;
        }
    }
    const double rar = t[0];
    const int bd = ccr_breakdown<T>(rar, rr, t[1]);
    const double beta = first ? 0.0 : rar / cs[6 + ((step - 1) & 1)];
    const double apap = first ? t[1] : t[1] + 2.0 * beta * t[2] + beta * beta * apold;
    if (bd || !(apap > 0.0)) {  // (near-)breakdown ends the coarse solve
        if (lead) {
            flags[4] = bd ? bd : 2;
            flags[0] = 1;
        }
        return;
    }
    const T bt = (T)beta, alpha = (T)(rar / apap);
    double v[2] = {0.0, 0.0};
    for (int i = blockIdx.x * CWG + threadIdx.x; i < n; i += gridDim.x * CWG) {
        C2<T> rv = r[i], pv, apv;
        const C2<T> arv = Ar[i];
        if (first) {
            pv = rv;
            apv = arv;
        } else {
            pv = p[i];
            apv = Ap[i];
            pv.x = rv.x + bt * pv.x;
            pv.y = rv.y + bt * pv.y;
            apv.x = arv.x + bt * apv.x;
            apv.y = arv.y + bt * apv.y;
        }
        C2<T> xv = x[i];
        xv.x += alpha * pv.x;
        xv.y += alpha * pv.y;
        rv.x -= alpha * apv.x;
        rv.y -= alpha * apv.y;
        p[i] = pv;
        Ap[i] = apv;
        x[i] = xv;
        r[i] = rv;
        v[0] += (double)rv.x * rv.x + (double)rv.y * rv.y;
        v[1] += (double)apv.x * apv.x + (double)apv.y * apv.y;
    }
    block_reduce<2>(v);
    if (threadIdx.x == 0) {
        uout[blockIdx.x] = v[0];
        uout[gridDim.x + blockIdx.x] = v[1];
    }
    if (lead) {
        cs[6 + (step & 1)] = rar;
        flags[1] = step;
    }
}

// coarse vectors are FP64 with C128 storage and FP32 with C64 / BF16 storage
template <typename T, typename S, bool FIRST>
void ccr_apply_launch(const CoarseGeom& c, const S* A, const CoarseCRWork<T>& w, hipStream_t s) {
    constexpr int E = wide_entries<S>();
    if (c.Nb % E == 0)
        hipLaunchKernelGGL((ccr_apply_kernel<T, S, E, FIRST>), dim3(c.Nc), dim3(CWG), (apply_lds<T, E>(c)), s, c, A,
                           w.r, w.Ar, w.Ap, w.part, w.flags);
    else
        hipLaunchKernelGGL((ccr_apply_kernel<T, S, 1, FIRST>), dim3(c.Nc), dim3(CWG), (apply_lds<T, 1>(c)), s, c, A,
                           w.r, w.Ar, w.Ap, w.part, w.flags);
}

template <typename T, bool FIRST>
void ccr_apply_dispatch(const CoarseGeom& c, hdcr_dtype dt, const void* A, const CoarseCRWork<T>& w, hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        ccr_apply_launch<T, double2, FIRST>(c, static_cast<const double2*>(A), w, s);
    } else if (dt == HDCR_C64) {
        ccr_apply_launch<T, float2, FIRST>(c, static_cast<const float2*>(A), w, s);
    } else {
        ccr_apply_launch<T, uint32_t, FIRST>(c, static_cast<const uint32_t*>(A), w, s);
    }
}

// ---------------------------------------------------------------------------
// coarse build: projection of the class-split fields onto the block basis
// ---------------------------------------------------------------------------

constexpr int PROJ_NK = 4;     // basis vectors (columns) per launch: one per wavefront of the work-group
constexpr int PROJ_ROWS = 64;  // basis rows per work-group
constexpr int PROJ_CHUNK = 16; // compressed indices of the block staged per step
constexpr int PROJ_PARTS = 4;  // work-groups splitting one block's indices

// grid (Nc, ceil(Nb / 64), PROJ_PARTS): the work-group sums conj(phi^a_j) . (H^(d) Phi_k)
// for all nine classes d, 64 rows j and nk <= 4 columns kk over part blockIdx.z of
// block a's compressed indices, and writes the partial sums to
// P[((part * Nc + a) * 9 + d) * PROJ_NK + kk][j].  One pass over the indices
// serves all classes: class 0 takes every site, the face classes only the sites
// on their face (a per-index test, the same for the whole work-group), so every
// basis entry is read once per launch.  Chunks of the 64 basis rows are staged
// in LDS with coalesced loads.
__global__ void __launch_bounds__(CWG) coarse_project_kernel(CoarseGeom c, const double2* __restrict__ b64,
                                                             const double2* __restrict__ Y, int nk,
                                                             double2* __restrict__ P) {
    __shared__ double2 F[2][PROJ_NK][9][PROJ_CHUNK];  // chiral folds of the class fields
    __shared__ double2 Bs[PROJ_ROWS][PROJ_CHUNK + 1];  // basis rows of the chunk
    __shared__ int mask[PROJ_CHUNK];                  // classes of each staged index
    const int a = blockIdx.x;
    const int j0 = blockIdx.y * PROJ_ROWS;
    const int ntot = 12 * c.bvol * c.Lh;
    // this part's index range, in whole chunks
    const int nchunk = (ntot + PROJ_CHUNK - 1) / PROJ_CHUNK;
    const int cb = (int)(((long long)nchunk * blockIdx.z) / gridDim.z);
    const int ce = (int)(((long long)nchunk * (blockIdx.z + 1)) / gridDim.z);
    const int nidx = min(ntot, ce * PROJ_CHUNK);
    const size_t fsz = (size_t)12 * c.f.N5;
    const int jl = threadIdx.x % PROJ_ROWS, kk = threadIdx.x / PROJ_ROWS;
    const int j = j0 + jl;
    const int h = (j < c.nvec) ? 0 : 1;
    double2 acc[9];
#pragma unroll
    for (int d = 0; d < 9; ++d) acc[d] = make_double2(0, 0);
    for (int i0 = cb * PROJ_CHUNK; i0 < nidx; i0 += PROJ_CHUNK) {
        // classes of the staged indices: 0, and the faces the site lies on
        if (threadIdx.x < PROJ_CHUNK) {
            const int idx = i0 + threadIdx.x;
            int m = 0;
            if (idx < nidx) {
                int f = (idx / c.Lh) % c.bvol;
                m = 1;
#pragma unroll
                for (int mu = 0; mu < 4; ++mu) {
                    const int x = f % c.B[mu];
                    f /= c.B[mu];
                    if (x == c.B[mu] - 1) m |= 1 << (1 + mu);
                    if (x == 0) m |= 1 << (5 + mu);
                }
            }
            mask[threadIdx.x] = m;
        }
        // basis rows: 64 rows x 16 consecutive indices, one 256-byte run per row
        for (int e = threadIdx.x; e < PROJ_ROWS * PROJ_CHUNK; e += CWG) {
            const int r = e / PROJ_CHUNK, ii = e % PROJ_CHUNK;
            const int jr = j0 + r, idx = i0 + ii;
            double2 v = make_double2(0, 0);
            if (jr < c.Nb && idx < nidx) {
                const int hr = (jr < c.nvec) ? 0 : 1;
                v = b64[(((size_t)a * 2 + hr) * c.nvec + (jr - hr * c.nvec)) * c.nhalf + idx];
            }
            Bs[r][ii] = v;
        }
        __syncthreads();
        // folds of the class fields at the staged indices (only the classes present)
        for (int e = threadIdx.x; e < nk * 9 * PROJ_CHUNK; e += CWG) {
            const int ii = e % PROJ_CHUNK, dk = e / PROJ_CHUNK;
            const int d = dk % 9, q = dk / 9;
            const int idx = i0 + ii;
            if (idx >= nidx || !((mask[ii] >> d) & 1)) continue;
            const int s = idx % c.Lh;
            const int f = (idx / c.Lh) % c.bvol;
            const int comp = idx / (c.Lh * c.bvol);
            const int site = block_site(c, a, f);
            const size_t fb = (((size_t)q * 9 + d) * fsz) + ((size_t)comp * c.f.V4 + site) * c.f.Ls;
            const double2 p1 = Y[fb + s], p2 = Y[fb + c.f.Ls - 1 - s];
            const double g = (comp < 6) ? 1.0 : -1.0;
            F[0][q][d][ii] = make_double2((p1.x + g * p2.x) * RSQRT2, (p1.y + g * p2.y) * RSQRT2);
            F[1][q][d][ii] = make_double2((p1.x - g * p2.x) * RSQRT2, (p1.y - g * p2.y) * RSQRT2);
        }
        __syncthreads();
        if (j < c.Nb && kk < nk) {
            const int iend = min(PROJ_CHUNK, nidx - i0);
            for (int ii = 0; ii < iend; ++ii) {
                const double2 bv = Bs[jl][ii];
                const int m = mask[ii];
                acc[0] = cjfma<double>(bv, F[h][kk][0][ii], acc[0]);
#pragma unroll
                for (int d = 1; d < 9; ++d)
                    if ((m >> d) & 1) acc[d] = cjfma<double>(bv, F[h][kk][d][ii], acc[d]);
            }
        }
        __syncthreads();
    }
    if (j < c.Nb && kk < nk) {
#pragma unroll
        for (int d = 0; d < 9; ++d)
            P[((((size_t)blockIdx.z * c.Nc + a) * 9 + d) * PROJ_NK + kk) * c.Nb + j] = acc[d];
    }
}

// A64[a][d][k0+kk][j] = sum over the parts, in part order
__global__ void __launch_bounds__(CWG) coarse_project_sum_kernel(CoarseGeom c, const double2* __restrict__ P, int k0,
                                                                 int nk, double2* __restrict__ A64) {
    const size_t n = (size_t)c.Nc * 9 * nk * c.Nb;
    for (size_t e = (size_t)blockIdx.x * CWG + threadIdx.x; e < n; e += (size_t)gridDim.x * CWG) {
        const int j = (int)(e % c.Nb);
        const size_t r = e / c.Nb;
        const int kk = (int)(r % nk);
        const size_t ad = r / nk;  // a * 9 + d
        double2 sum = P[(ad * PROJ_NK + kk) * c.Nb + j];
        for (int q = 1; q < PROJ_PARTS; ++q) sum = cadd<double>(sum, P[(((size_t)q * c.Nc * 9 + ad) * PROJ_NK + kk) * c.Nb + j]);
        A64[(ad * c.Nb + (k0 + kk)) * c.Nb + j] = sum;
    }
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ void __launch_bounds__(CWG) coarse_convert_kernel(size_t n, const double2* __restrict__ A64, int dt,
                                                             void* __restrict__ dst) {
    for (size_t e = (size_t)blockIdx.x * CWG + threadIdx.x; e < n; e += (size_t)gridDim.x * CWG) {
        const double2 v = A64[e];
        if (dt == HDCR_C64) {
            static_cast<float2*>(dst)[e] = make_float2((float)v.x, (float)v.y);
        } else {
            const uint32_t re = f32_to_bf16_rne((float)v.x), im = f32_to_bf16_rne((float)v.y);
            static_cast<uint32_t*>(dst)[e] = re | (im << 16);
        }
    }
}

// logical out[a][d][j][k] from column-major storage [a][d][k][j]
__global__ void __launch_bounds__(CWG) coarse_export_kernel(CoarseGeom c, int dt, const void* __restrict__ A,
                                                            double2* __restrict__ out) {
    const size_t n = coarse_elems(c);
    const size_t nb2 = (size_t)c.Nb * c.Nb;
    for (size_t e = (size_t)blockIdx.x * CWG + threadIdx.x; e < n; e += (size_t)gridDim.x * CWG) {
        const size_t blk = e / nb2;
        const int r = (int)(e % nb2);
        const int j = r / c.Nb, k = r % c.Nb;
        const size_t src = blk * nb2 + (size_t)k * c.Nb + j;
        double2 v;
        if (dt == HDCR_C128) {
            v = static_cast<const double2*>(A)[src];
        } else if (dt == HDCR_C64) {
            const float2 f = static_cast<const float2*>(A)[src];
            v = make_double2(f.x, f.y);
        } else {
            const float2 f = ldA<float, uint32_t>(static_cast<const uint32_t*>(A), src);
            v = make_double2(f.x, f.y);
        }
        out[e] = v;
    }
}

int grid_for(size_t n) {
    size_t b = (n + CWG - 1) / CWG;
    return (int)(b > 65536 ? 65536 : (b == 0 ? 1 : b));
}

}  // namespace

namespace {
__global__ void __launch_bounds__(CWG) zero_i32_kernel(int* __restrict__ p, int n) {
    for (int i = blockIdx.x * CWG + threadIdx.x; i < n; i += gridDim.x * CWG) p[i] = 0;
}
}  // namespace

void launch_zero_i32(int* p, int n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(zero_i32_kernel, dim3((n + CWG - 1) / CWG), dim3(CWG), 0, s, p, n);
}

template <typename T>
void launch_ccr_init(const CoarseGeom& c, const C2<T>* b, C2<T>* x, const CoarseCRWork<T>& w, int maxiter, double tol,
                     hipStream_t s) {
    const double tol2 = tol > 0 ? tol * tol : 0.0;
    hipLaunchKernelGGL(ccr_init_kernel<T>, dim3(CCR_BLOCKS), dim3(CWG), 0, s, c.Nc * c.Nb, b, x, w.r,
                       w.part + 3 * (size_t)c.Nc, w.cs, w.flags, maxiter, tol2);
}

template <typename T>
void launch_ccr_init_defl(const CoarseGeom& c, const C2<T>* b, C2<T>* x, const CoarseCRWork<T>& w,
                          const DeflView<T>& d, int maxiter, double tol, hipStream_t s) {
    const double tol2 = tol > 0 ? tol * tol : 0.0;
    const int n = c.Nc * c.Nb;
    hipLaunchKernelGGL(defl_dot_kernel<T>, dim3(DEFL_BLOCKS, (d.k + 7) / 8), dim3(CWG), 0, s, n, d, b, w.dpart);
    hipLaunchKernelGGL(defl_coef_kernel<T>, dim3(2 * d.k), dim3(CWG), 0, s, d, (const double*)w.dpart, w.dcoef);
    hipLaunchKernelGGL(ccr_init_defl_kernel<T>, dim3(DEFL_INIT_BLOCKS), dim3(CWG), 0, s, n, b, x, w.r, d,
                       (const double*)w.dcoef, w.part + 3 * (size_t)c.Nc, w.cs, w.flags, maxiter, tol2);
}

static int ccr_update_blocks(int n) {
    const int b = (n + CWG - 1) / CWG;
    return b < 1 ? 1 : (b > CCR_UPDATE_MAX ? CCR_UPDATE_MAX : b);
}

template <typename T>
void launch_ccr_step(const CoarseGeom& c, hdcr_dtype A_dtype, const void* A, C2<T>* x, const CoarseCRWork<T>& w,
                     int step, hipStream_t s) {
    const int n = c.Nc * c.Nb;
    if (step == 0) {
        ccr_apply_dispatch<T, true>(c, A_dtype, A, w, s);
        return;
    }
    double* upart = w.part + 3 * (size_t)c.Nc + 2 * (size_t)std::max(CCR_BLOCKS, DEFL_INIT_BLOCKS);
    const size_t half = 2 * (size_t)CCR_UPDATE_MAX;
    hipLaunchKernelGGL(ccr_update_kernel<T>, dim3(ccr_update_blocks(n)), dim3(CWG), 0, s, n, x, w.r, w.p, w.Ar, w.Ap,
                       (const double*)w.part, c.Nc, (const double*)(upart + ((step - 1) & 1) * half),
                       upart + (step & 1) * half, w.cs, w.flags, step);
    ccr_apply_dispatch<T, false>(c, A_dtype, A, w, s);
}

template void launch_ccr_init<double>(const CoarseGeom&, const double2*, double2*, const CoarseCRWork<double>&, int,
                                      double, hipStream_t);
template void launch_ccr_init<float>(const CoarseGeom&, const float2*, float2*, const CoarseCRWork<float>&, int,
                                     double, hipStream_t);
template void launch_ccr_init_defl<double>(const CoarseGeom&, const double2*, double2*, const CoarseCRWork<double>&,
                                           const DeflView<double>&, int, double, hipStream_t);
template void launch_ccr_init_defl<float>(const CoarseGeom&, const float2*, float2*, const CoarseCRWork<float>&,
                                          const DeflView<float>&, int, double, hipStream_t);
template void launch_ccr_step<double>(const CoarseGeom&, hdcr_dtype, const void*, double2*,
                                      const CoarseCRWork<double>&, int, hipStream_t);
template void launch_ccr_step<float>(const CoarseGeom&, hdcr_dtype, const void*, float2*, const CoarseCRWork<float>&,
                                     int, hipStream_t);

size_t coarse_bytes(const CoarseGeom& c, hdcr_dtype dt) {
    return coarse_elems(c) * (dt == HDCR_C128 ? 16 : dt == HDCR_C64 ? 8 : 4);
}

void launch_basis_fold(const CoarseGeom& c, const double2* vecs, double2* b64, hipStream_t s) {
    const size_t total = (size_t)c.nvec * c.Nc * c.nhalf;
    hipLaunchKernelGGL(basis_fold_kernel, dim3(grid_for(total)), dim3(CWG), 0, s, c, vecs, b64);
}

void launch_block_orth(const CoarseGeom& c, double2* b64, int* rank_flag, hipStream_t s) {
    hipLaunchKernelGGL(block_orth_kernel, dim3(c.Nc * 2), dim3(CWG), 0, s, c, b64, rank_flag);
}

bool chq_ok(const CoarseGeom& c) { return c.nvec <= CHQ_MAXV; }
int chq_parts(const CoarseGeom& c) {
    const int want = (2048 + 2 * c.Nc - 1) / (2 * c.Nc);  // about 2048 workgroups in all
    const int chunks = (c.nhalf + CHQ_CH - 1) / CHQ_CH;
    return std::max(1, std::min(std::min(want, 16), chunks));
}
size_t chq_scratch_elems(const CoarseGeom& c) {
    return chq_ok(c) ? (size_t)2 * c.Nc * (chq_parts(c) + 1) * c.nvec * c.nvec : 0;
}
void launch_chq_pass(const CoarseGeom& c, double2* b64, double2* scratch, int pass, int* flag, hipStream_t s) {
    const int parts = chq_parts(c);
    double2* Gp = scratch;
    double2* Rinv = scratch + (size_t)2 * c.Nc * parts * c.nvec * c.nvec;
    hipLaunchKernelGGL(chq_gram_kernel, dim3(c.Nc * 2, parts), dim3(CWG), 0, s, c, b64, Gp);
    hipLaunchKernelGGL(chq_chol_kernel, dim3(c.Nc * 2), dim3(64), 0, s, c, Gp, parts, pass, Rinv, flag);
}
void launch_chq_apply(const CoarseGeom& c, double2* b64, const double2* scratch, hipStream_t s) {
    const int parts = chq_parts(c);
    const double2* Rinv = scratch + (size_t)2 * c.Nc * parts * c.nvec * c.nvec;
    const int ap = std::max(1, std::min(16, (c.nhalf + CHQ_TI - 1) / CHQ_TI));
    hipLaunchKernelGGL(chq_apply_kernel, dim3(c.Nc * 2, ap), dim3(CWG), 0, s, c, b64, Rinv);
}

void launch_basis_to_f32(const CoarseGeom& c, const double2* b64, float2* b32, hipStream_t s) {
    const size_t n = basis_elems(c);
    hipLaunchKernelGGL(basis_to_f32_kernel, dim3(grid_for(n)), dim3(CWG), 0, s, n, b64, b32);
}

void launch_basis_to_f16(const CoarseGeom& c, const double2* b64, uint32_t* b16, hipStream_t s) {
    const size_t n = basis_elems(c);
    hipLaunchKernelGGL(basis_to_f16_kernel, dim3(grid_for(n)), dim3(CWG), 0, s, n, b64, b16);
}

void launch_basis_expand(const CoarseGeom& c, const double2* b64, int k0, int nk, double2* fields, hipStream_t s) {
    const size_t n = (size_t)12 * c.f.N5 * nk;
    hipLaunchKernelGGL(basis_expand_kernel, dim3(grid_for(n)), dim3(CWG), 0, s, c, b64, k0, nk, fields);
}

template <typename T, typename B, int W, int RKG>
void restrict_launch_w(const CoarseGeom& c, const B* basis, const C2<T>* psi, const C2<T>* psi2, C2<T>* v,
                       hipStream_t s) {
    const dim3 grid(c.Nc * 2 * ((c.nvec + RKG - 1) / RKG));
    if (psi2)
        hipLaunchKernelGGL((restrict_kernel<T, B, true, W, RKG>), grid, dim3(CWG), 0, s, c, basis, psi, psi2, v);
    else
        hipLaunchKernelGGL((restrict_kernel<T, B, false, W, RKG>), grid, dim3(CWG), 0, s, c, basis, psi, psi2, v);
}

template <typename T, typename B, int RKG>
void restrict_launch_r(const CoarseGeom& c, int wmax, const B* basis, const C2<T>* psi, const C2<T>* psi2, C2<T>* v,
                       hipStream_t s) {
    // W consecutive s slots per work-item: 8 (on request) or 4 when Ls/2 is a
    // multiple of it (16-byte basis loads in FP16, 16-byte psi pairs in FP32), 2
    // when it is even, and a row must fit the workgroup
    if (wmax >= 8 && c.Lh % 8 == 0 && c.Lh / 8 <= CWG)
        restrict_launch_w<T, B, 8, RKG>(c, basis, psi, psi2, v, s);
    else if (wmax >= 4 && c.Lh % 4 == 0 && c.Lh / 4 <= CWG)
        restrict_launch_w<T, B, 4, RKG>(c, basis, psi, psi2, v, s);
    else if (wmax >= 2 && c.Lh % 2 == 0 && c.Lh / 2 <= CWG)
        restrict_launch_w<T, B, 2, RKG>(c, basis, psi, psi2, v, s);
    else
        restrict_launch_w<T, B, 1, RKG>(c, basis, psi, psi2, v, s);
}

template <typename T, typename B>
void restrict_launch(const CoarseGeom& c, const B* basis, const C2<T>* psi, const C2<T>* psi2, C2<T>* v, hipStream_t s) {
    if (c.Lh > CWG) return;  // not reachable: Ls <= 512 is enforced by the descriptor checks
    // the caller's shape (tune.restrict_w / restrict_rkg; 0 = 16 vectors and 8
    // slots with the FP16 basis copy, 4 with the FP32 and FP64 ones: measured at
    // 24^4 x 16, Nb = 64, 1.45 against 1.93 ms with the FP16 copy, 2.77 against
    // 2.69 ms with the FP32 one)
    const int wmax = c.f.tune.restrict_w > 0 ? c.f.tune.restrict_w : (std::is_same<B, uint32_t>::value ? 8 : 4);
    const int rkg = c.f.tune.restrict_rkg > 0 ? c.f.tune.restrict_rkg : 16;
    if (rkg >= RKG_MAX && c.nvec >= RKG_MAX)
        restrict_launch_r<T, B, RKG_MAX>(c, wmax, basis, psi, psi2, v, s);
    else
        restrict_launch_r<T, B, 16>(c, wmax, basis, psi, psi2, v, s);
}

template <typename T>
void launch_restrict(const CoarseGeom& c, const C2<T>* basis, const C2<T>* psi, const C2<T>* psi2, C2<T>* v,
                     hipStream_t s) {
    restrict_launch<T, C2<T>>(c, basis, psi, psi2, v, s);
}

void launch_restrict_h(const CoarseGeom& c, const uint32_t* basis, const float2* psi, const float2* psi2, float2* v,
                       hipStream_t s) {
    restrict_launch<float, uint32_t>(c, basis, psi, psi2, v, s);
}

// Workgroups per coarse site of the prolongation: tune.prolong_split, else about
// 7800 workgroups in all (six per site at 6^4 coarse sites, the fastest of 1 to
// 8 measured at 24^4 x 16 with Nb = 64: 1.74 ms against 1.86 ms for one), with
// parts of at least one sweep of the workgroup over its indices.  One workgroup
// per site left the grid at 1296 workgroups, about five waves per SIMD with one
// basis load pair in flight per work-item.
static int prolong_parts(const CoarseGeom& c) {
    int p = c.f.tune.prolong_split;
    if (p <= 0) {
        p = (7800 + c.Nc / 2) / c.Nc;
        const int sweeps = c.nhalf / (2 * CWG);
        if (p > sweeps) p = sweeps;
    }
    return p < 1 ? 1 : (p > 16 ? 16 : p);
}

template <typename T>
void launch_prolong(const CoarseGeom& c, const C2<T>* basis, const C2<T>* v, const C2<T>* y, C2<T>* psi,
                    hipStream_t s) {
    hipLaunchKernelGGL((prolong_kernel<T, C2<T>, 2>), dim3(c.Nc, prolong_parts(c)), dim3(CWG), c.Nb * sizeof(C2<T>), s,
                       c, basis, v, y, psi);
}

void launch_prolong_h(const CoarseGeom& c, const uint32_t* basis, const float2* v, const float2* y, float2* psi,
                      hipStream_t s) {
    // two indices per work-item (measured faster at 24^4 x 16 than four with
    // 16-byte FP16 loads: 1.88 against 1.94 ms); tune.prolong_ni = 4 selects four
    const int ni = c.f.tune.prolong_ni > 0 ? c.f.tune.prolong_ni : 2;
    const dim3 grid(c.Nc, prolong_parts(c));
    if (ni >= 4 && c.nhalf % 4 == 0)
        hipLaunchKernelGGL((prolong_kernel<float, uint32_t, 4>), grid, dim3(CWG), c.Nb * sizeof(float2), s, c, basis,
                           v, y, psi);
    else
        hipLaunchKernelGGL((prolong_kernel<float, uint32_t, 2>), grid, dim3(CWG), c.Nb * sizeof(float2), s, c, basis,
                           v, y, psi);
}

namespace {

// The same for R right-hand sides per work-group (blockIdx.y = group of R):
// each A entry is read once for all R vectors.  Every output element takes the
// same products in the same order as site_gemv (over d, then k in steps of kg
// per thread, then the fixed sum over the kg thread groups), so the results
// equal the one-vector kernel's bit for bit.
template <typename T, typename S, int E, int R>
__global__ void __launch_bounds__(CWG) coarse_apply_multi_kernel(CoarseGeom c, const S* __restrict__ A,
                                                                 const C2<T>* __restrict__ v, C2<T>* __restrict__ out,
                                                                 int nrhs) {
    extern __shared__ unsigned char smem_raw[];
    const int Nb = c.Nb;
    C2<T>* vs = reinterpret_cast<C2<T>*>(smem_raw);  // [R][9][Nb]
    C2<T>* red = vs + R * 9 * Nb;                    // [CWG * E]
    const int a = blockIdx.x;
    const int r0 = blockIdx.y * R;
    const int nr = min(R, nrhs - r0);
    const size_t nv = (size_t)c.Nc * Nb;
    for (int e = threadIdx.x; e < R * 9 * Nb; e += CWG) {
        const int r = e / (9 * Nb), rem = e - r * 9 * Nb;
        const int d = rem / Nb, k = rem - d * Nb;
        vs[e] = (r < nr) ? v[(size_t)(r0 + r) * nv + (size_t)coarse_nbr(c, a, d) * Nb + k] : mk<T>(0, 0);
    }
    __syncthreads();
    const int nj = Nb / E;
    const int kg = CWG / nj;
    const int t = threadIdx.x;
    const int jq = t % nj, kk = t / nj;
    C2<T> acc[R][E];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < E; ++q) acc[r][q] = mk<T>(0, 0);
    if (kk < kg) {
        const size_t blk = (size_t)Nb * Nb;
        const S* Aa = A + (size_t)a * 9 * blk + (size_t)jq * E;
        for (int d = 0; d < 9; ++d) {
            const S* Ad = Aa + d * blk;
#pragma unroll 2
            for (int k = kk; k < Nb; k += kg) {
                C2<T> e[E];
                WideA<T, S, E>::ld(Ad + (size_t)k * Nb, e);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const C2<T> x = vs[(r * 9 + d) * Nb + k];
#pragma unroll
                    for (int q = 0; q < E; ++q) acc[r][q] = cfma<T>(e[q], x, acc[r][q]);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (r >= nr) break;  // nr is the same for the whole work-group
        if (kk < kg) {
#pragma unroll
            for (int q = 0; q < E; ++q) red[kk * Nb + jq * E + q] = acc[r][q];
        }
        __syncthreads();
        for (int j = t; j < Nb; j += CWG) {
            C2<T> sum = red[j];
            for (int g = 1; g < kg; ++g) sum = cadd<T>(sum, red[g * Nb + j]);
            out[((size_t)(r0 + r) * c.Nc + a) * Nb + j] = sum;
        }
        __syncthreads();
    }
}

constexpr size_t MULTI_LDS_MAX = 65536;
template <typename T, int E, int R> size_t multi_lds(const CoarseGeom& c) {
    return ((size_t)R * 9 * c.Nb + (size_t)CWG * E) * sizeof(C2<T>);
}

template <typename T, typename S, int E>
bool coarse_apply_multi_launch(const CoarseGeom& c, const S* A, const C2<T>* v, C2<T>* out, int nrhs, hipStream_t s) {
    if (nrhs >= 8 && multi_lds<T, E, 8>(c) <= MULTI_LDS_MAX) {
        hipLaunchKernelGGL((coarse_apply_multi_kernel<T, S, E, 8>), dim3(c.Nc, (nrhs + 7) / 8), dim3(CWG),
                           (multi_lds<T, E, 8>(c)), s, c, A, v, out, nrhs);
        return true;
    }
    if (nrhs >= 4 && multi_lds<T, E, 4>(c) <= MULTI_LDS_MAX) {
        hipLaunchKernelGGL((coarse_apply_multi_kernel<T, S, E, 4>), dim3(c.Nc, (nrhs + 3) / 4), dim3(CWG),
                           (multi_lds<T, E, 4>(c)), s, c, A, v, out, nrhs);
        return true;
    }
    if (nrhs >= 2 && multi_lds<T, E, 2>(c) <= MULTI_LDS_MAX) {
        hipLaunchKernelGGL((coarse_apply_multi_kernel<T, S, E, 2>), dim3(c.Nc, (nrhs + 1) / 2), dim3(CWG),
                           (multi_lds<T, E, 2>(c)), s, c, A, v, out, nrhs);
        return true;
    }
    return false;
}

}  // namespace

template <typename T, typename S>
void coarse_apply_launch(const CoarseGeom& c, const S* A, const C2<T>* v, C2<T>* out, int nrhs, hipStream_t s) {
    constexpr int E = wide_entries<S>();
    if (nrhs > 1) {
        if (c.Nb % E == 0) {
            if (coarse_apply_multi_launch<T, S, E>(c, A, v, out, nrhs, s)) return;
        } else if (coarse_apply_multi_launch<T, S, 1>(c, A, v, out, nrhs, s)) {
            return;
        }
    }
    if (c.Nb % E == 0)
        hipLaunchKernelGGL((coarse_apply_kernel<T, S, E>), dim3(c.Nc, nrhs), dim3(CWG), (apply_lds<T, E>(c)), s, c,
                           A, v, out);
    else
        hipLaunchKernelGGL((coarse_apply_kernel<T, S, 1>), dim3(c.Nc, nrhs), dim3(CWG), (apply_lds<T, 1>(c)), s, c,
                           A, v, out);
}

template <typename T>
void launch_coarse_apply(const CoarseGeom& c, const C2<T>* A, const C2<T>* v, C2<T>* out, int nrhs, hipStream_t s) {
    coarse_apply_launch<T, C2<T>>(c, A, v, out, nrhs, s);
}

void launch_coarse_apply_bf16(const CoarseGeom& c, const uint16_t* A, const float2* v, float2* out, int nrhs,
                              hipStream_t s) {
    coarse_apply_launch<float, uint32_t>(c, reinterpret_cast<const uint32_t*>(A), v, out, nrhs, s);
}

size_t coarse_project_scratch_elems(const CoarseGeom& c) { return (size_t)PROJ_PARTS * c.Nc * 9 * PROJ_NK * c.Nb; }

void launch_coarse_project(const CoarseGeom& c, const double2* b64, const double2* Y, int k0, int nk, double2* P,
                           double2* A64, hipStream_t s) {
    hipLaunchKernelGGL(coarse_project_kernel, dim3(c.Nc, (c.Nb + PROJ_ROWS - 1) / PROJ_ROWS, PROJ_PARTS), dim3(CWG), 0,
                       s, c, b64, Y, nk, P);
    hipLaunchKernelGGL(coarse_project_sum_kernel, dim3(grid_for((size_t)c.Nc * 9 * nk * c.Nb)), dim3(CWG), 0, s, c,
                       (const double2*)P, k0, nk, A64);
}

void launch_coarse_convert(const CoarseGeom& c, const double2* A64, hdcr_dtype dt, void* dst, hipStream_t s) {
    const size_t n = coarse_elems(c);
    hipLaunchKernelGGL(coarse_convert_kernel, dim3(grid_for(n)), dim3(CWG), 0, s, n, A64, (int)dt, dst);
}

void launch_coarse_export(const CoarseGeom& c, hdcr_dtype dt, const void* A, double2* out, hipStream_t s) {
    hipLaunchKernelGGL(coarse_export_kernel, dim3(grid_for(coarse_elems(c))), dim3(CWG), 0, s, c, (int)dt, A, out);
}

template void launch_restrict<double>(const CoarseGeom&, const double2*, const double2*, const double2*, double2*,
                                      hipStream_t);
template void launch_restrict<float>(const CoarseGeom&, const float2*, const float2*, const float2*, float2*,
                                     hipStream_t);
template void launch_prolong<double>(const CoarseGeom&, const double2*, const double2*, const double2*, double2*,
                                     hipStream_t);
template void launch_prolong<float>(const CoarseGeom&, const float2*, const float2*, const float2*, float2*,
                                    hipStream_t);
template void launch_coarse_apply<double>(const CoarseGeom&, const double2*, const double2*, double2*, int,
                                          hipStream_t);
template void launch_coarse_apply<float>(const CoarseGeom&, const float2*, const float2*, float2*, int, hipStream_t);

}  // namespace hdcr

// ---------------------------------------------------------------------------
// batched coarse apply on the matrix cores: out[r] = A v[r] for many right-hand
// sides with A in BF16C storage, v rounded to bf16, FP32 accumulation
// ---------------------------------------------------------------------------
namespace hdcr {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int MR = 16;  // right-hand sides per pass (the N of a 16x16x32 tile)

// bf16 pair (re, im) of a complex float, rounded to nearest even
__device__ __forceinline__ uint32_t pack_bf16c(float2 v) {
    return (uint32_t)__builtin_bit_cast(unsigned short, (__bf16)v.x) |
           ((uint32_t)__builtin_bit_cast(unsigned short, (__bf16)v.y) << 16);
}

// One workgroup per coarse site; NW wavefronts split the 2 Nb / 16 row tiles of
// the real form [[Ar, -Ai], [Ai, Ar]] (rows 2j + re/im, columns 2k + re/im) of
// each block A[a][d]; the right-hand sides are the 16 columns of a tile.  ALDS:
// the block is first staged in LDS with 16-byte loads (else each lane reads its
// 4 words from memory).  Every variant issues the same MFMA sequence per output.
// PRE (with ALDS): the 9 blocks of the site are loaded into registers up front
// (PRE 16-byte loads per work-item and block), so their latencies overlap
template <int NW, int TPW, bool ALDS, int PRE = 0>
__global__ void __launch_bounds__(64 * NW) coarse_mfma_kernel(CoarseGeom c, const uint32_t* __restrict__ A,
                                                              const float2* __restrict__ v, float2* __restrict__ out,
                                                              int nrhs) {
    extern __shared__ unsigned char smem_raw[];
    const int Nb = c.Nb;
    const int VST = Nb + 4;  // row stride of the staged vectors: the 16 columns of an operand load in distinct banks
    uint32_t* vb = reinterpret_cast<uint32_t*>(smem_raw);  // [9][MR][VST] bf16 pairs
    uint32_t* ab = vb + 9 * MR * VST;                       // [Nb][Nb] one block (ALDS)
    const int a = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // scalar: uniform row-tile tests
    const int kq = lane >> 4, col = lane & 15;
    // A-operand word of row 2j + (col & 1): (re, -im) for even rows, (im, re) for
    // odd rows; built branch-free (rotate by 0 or 16 bits, then flip a sign bit)
    const uint32_t rot = (col & 1) ? 16u : 0u;
    const uint32_t flip = (col & 1) ? 0u : 0x80000000u;
    for (int r0 = 0; r0 < nrhs; r0 += MR) {
        const int nr = min(MR, nrhs - r0);
        __syncthreads();  // the previous pass has finished reading vb
        for (int e = threadIdx.x; e < 9 * MR * Nb; e += 64 * NW) {
            const int d = e / (MR * Nb), rem = e - d * MR * Nb;
            const int r = rem / Nb, k = rem - r * Nb;
            const float2 x = (r < nr) ? v[((size_t)(r0 + r) * c.Nc + coarse_nbr(c, a, d)) * Nb + k] : make_float2(0, 0);
            vb[(d * MR + r) * VST + k] = pack_bf16c(x);
        }
        f32x4 acc[TPW];  // row tiles wave + NW t of this wavefront
#pragma unroll
        for (int t = 0; t < TPW; ++t) acc[t] = f32x4{0, 0, 0, 0};
        u32x4 pre[PRE > 0 ? 9 : 1][PRE > 0 ? PRE : 1];
        if constexpr (PRE > 0) {
            const uint32_t* Aa = A + (size_t)a * 9 * Nb * Nb;
#pragma unroll
            for (int d = 0; d < 9; ++d)
#pragma unroll
                for (int u = 0; u < PRE; ++u) {
                    const int e = 4 * (threadIdx.x + u * 64 * NW);
                    if (e < Nb * Nb) pre[d][u] = *reinterpret_cast<const u32x4*>(Aa + (size_t)d * Nb * Nb + e);
                }
        }
#pragma unroll
        for (int d = 0; d < 9; ++d) {
            const uint32_t* Ad = A + ((size_t)a * 9 + d) * Nb * Nb;
            if constexpr (ALDS) {
                __syncthreads();  // previous block consumed
                if constexpr (PRE > 0) {
#pragma unroll
                    for (int u = 0; u < PRE; ++u) {
                        const int e = 4 * (threadIdx.x + u * 64 * NW);
                        if (e < Nb * Nb) *reinterpret_cast<u32x4*>(ab + e) = pre[d][u];
                    }
                } else {
                    for (int e = 4 * threadIdx.x; e < Nb * Nb; e += 4 * 64 * NW)
                        *reinterpret_cast<u32x4*>(ab + e) = *reinterpret_cast<const u32x4*>(Ad + e);
                }
            }
            __syncthreads();
            const uint32_t* vd = vb + d * MR * VST;
            for (int ks = 0; ks < Nb / 16; ++ks) {
                const int k0 = 16 * ks + 4 * kq;
                const u32x4 bw = *reinterpret_cast<const u32x4*>(vd + col * VST + k0);
                const bf16x8 bop = __builtin_bit_cast(bf16x8, bw);
                // ntiles = NW * TPW exactly: every wavefront owns TPW row tiles, and
                // the accumulation chains carry no branch
#pragma unroll
                for (int t = 0; t < TPW; ++t) {
                    const int rt = wave + NW * t;
                    const int row = 16 * rt + col;
                    const int j = row >> 1;
                    u32x4 aw;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t w = ALDS ? ab[(k0 + q) * Nb + j] : Ad[(size_t)(k0 + q) * Nb + j];
                        aw[q] = __builtin_amdgcn_alignbit(w, w, rot) ^ flip;
                    }
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, aw), bop, acc[t], 0,
                                                                      0, 0);
                }
            }
        }
        // lane holds rows 16 rt + 4 kq + (0..3) = complex rows 8 rt + 2 kq + (0, 1) of column col
        if (col < nr) {
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int j0 = 8 * (wave + NW * t) + 2 * kq;
                float2* o = out + ((size_t)(r0 + col) * c.Nc + a) * Nb + j0;
                o[0] = make_float2(acc[t][0], acc[t][1]);
                o[1] = make_float2(acc[t][2], acc[t][3]);
            }
        }
    }
}

// Nb = 64, 8 wavefronts, one row tile each: the variant that keeps the memory
// system busy.  Every load is issued before the first of them is used: the
// first pass's neighbour vectors (16-byte pairs of complex entries, nine per
// work-item), then the 9 blocks of the site (two 16-byte words per work-item and
// block, held in registers across all passes of right-hand sides), so that the
// vectors are rounded to bf16 into LDS and block d is multiplied while the later
// blocks are still arriving.  The vector rows and the
// block copy in LDS have a row stride of Nb + 4 words, so the 16 columns of a
// B-operand load and the four k rows of an A-operand load fall in different banks.  The MFMA sequence per output is the
// other variants', so the results are the same bits.
constexpr int PF_NB = 64, PF_NW = 8, PF_AST = PF_NB + 4;
__global__ void __launch_bounds__(64 * PF_NW) coarse_mfma_pf_kernel(CoarseGeom c, const uint32_t* __restrict__ A,
                                                                    const float2* __restrict__ v,
                                                                    float2* __restrict__ out, int nrhs) {
    constexpr int NB = PF_NB, NT = 64 * PF_NW;
    constexpr int NV4 = 9 * MR * NB / 2 / NT;  // 16-byte vector loads per work-item and pass (9)
    constexpr int NA4 = NB * NB / 4 / NT;       // 16-byte block loads per work-item and block (2)
    extern __shared__ unsigned char smem_raw[];
    uint32_t* vb = reinterpret_cast<uint32_t*>(smem_raw);  // [9][MR][PF_AST] bf16 pairs
    uint32_t* ab = vb + 9 * MR * PF_AST;                    // [NB][PF_AST] one block
    const int a = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int kq = lane >> 4, col = lane & 15;
    const uint32_t rot = (col & 1) ? 16u : 0u;
    const uint32_t flip = (col & 1) ? 0u : 0x80000000u;
    const uint32_t* Aa = A + (size_t)a * 9 * NB * NB;
    int nbr[9];
#pragma unroll
    for (int d = 0; d < 9; ++d) nbr[d] = coarse_nbr(c, a, d);
    // the pass's neighbour vectors: 16-byte pairs [9][MR][NB / 2], zero beyond nrhs
    float4 vx[NV4];
    auto load_vectors = [&](int r0, int nr) {
#pragma unroll
        for (int u = 0; u < NV4; ++u) {
            const int e2 = threadIdx.x + u * NT;
            const int d = e2 / (MR * NB / 2), rem = e2 - d * (MR * NB / 2);
            const int r = rem / (NB / 2), kp = rem - r * (NB / 2);
            int nd = nbr[0];
#pragma unroll
            for (int q = 1; q < 9; ++q) nd = (d == q) ? nbr[q] : nd;
            vx[u] = (r < nr) ? *reinterpret_cast<const float4*>(v + ((size_t)(r0 + r) * c.Nc + nd) * NB + 2 * kp)
                             : make_float4(0, 0, 0, 0);
        }
    };
    // the first pass's vectors are requested before the blocks: loads complete in
    // order, so the vectors are usable while the blocks are still arriving, and
    // block d is consumed while blocks d + 1 .. 8 arrive
    load_vectors(0, min(MR, nrhs));
    __builtin_amdgcn_sched_barrier(0);
    u32x4 pre[9][NA4];
#pragma unroll
    for (int d = 0; d < 9; ++d)
#pragma unroll
        for (int u = 0; u < NA4; ++u)
            pre[d][u] = *reinterpret_cast<const u32x4*>(Aa + (size_t)d * NB * NB + 4 * (threadIdx.x + u * NT));
    __builtin_amdgcn_sched_barrier(0);
    for (int r0 = 0; r0 < nrhs; r0 += MR) {
        const int nr = min(MR, nrhs - r0);
        if (r0 > 0) load_vectors(r0, nr);
        __syncthreads();  // the previous pass has finished reading vb
#pragma unroll
        for (int u = 0; u < NV4; ++u) {
            const int e2 = threadIdx.x + u * NT;
            uint2 w;
            w.x = pack_bf16c(make_float2(vx[u].x, vx[u].y));
            w.y = pack_bf16c(make_float2(vx[u].z, vx[u].w));
            const int dr = e2 / (NB / 2), kp = e2 - dr * (NB / 2);  // (d, r) row and pair in the row
            *reinterpret_cast<uint2*>(vb + dr * PF_AST + 2 * kp) = w;
        }
        f32x4 acc = f32x4{0, 0, 0, 0};
        const int row = 16 * wave + col;
        const int j = row >> 1;
#pragma unroll
        for (int d = 0; d < 9; ++d) {
            __syncthreads();  // previous block consumed (and, for d = 0, vb written)
#pragma unroll
            for (int u = 0; u < NA4; ++u) {
                const int e = 4 * (threadIdx.x + u * NT);
                const int k = e / NB, jj = e - k * NB;
                *reinterpret_cast<u32x4*>(ab + k * PF_AST + jj) = pre[d][u];
            }
            __syncthreads();
            const uint32_t* vd = vb + d * MR * PF_AST;
#pragma unroll
            for (int ks = 0; ks < NB / 16; ++ks) {
                const int k0 = 16 * ks + 4 * kq;
                const bf16x8 bop = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(vd + col * PF_AST + k0));
                u32x4 aw;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t w = ab[(k0 + q) * PF_AST + j];
                    aw[q] = __builtin_amdgcn_alignbit(w, w, rot) ^ flip;
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, aw), bop, acc, 0, 0, 0);
            }
        }
        if (col < nr) {
            const int j0 = 8 * wave + 2 * kq;
            float2* o = out + ((size_t)(r0 + col) * c.Nc + a) * NB + j0;
            o[0] = make_float2(acc[0], acc[1]);
            o[1] = make_float2(acc[2], acc[3]);
        }
    }
}

// bf16 terms of a complex float: t = 1 is the rounding of v, t = 2 and 3 round
// what the earlier terms leave.  Each remainder is exact in FP32 (it holds the
// bits of v below the previous term's 8-bit significand), so three terms sum to
// v exactly and two to within 2^-16 of |v|.
template <int T>
__device__ __forceinline__ void split_bf16c(float2 x, uint32_t (&w)[T]) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const __bf16 hr = (__bf16)x.x, hi = (__bf16)x.y;
        w[t] = (uint32_t)__builtin_bit_cast(unsigned short, hr) | ((uint32_t)__builtin_bit_cast(unsigned short, hi) << 16);
        x.x -= (float)hr;
        x.y -= (float)hi;
    }
}

// Nb = NB, 2 NB / 16 wavefronts with one row tile each, the blocks of the site
// held for every right-hand side: the direction loop is outside the loop over
// passes of 16 right-hand sides, so each block goes through LDS and into the
// A-operand registers once per chunk of 16 NP right-hand sides (NP <= 4; one
// FP32 accumulator tile per pass), instead of once per pass; the blocks stay in
// registers across chunks.  With three or four passes per chunk the staging
// is double-buffered (the next step is written while the current one is read,
// one barrier per step) and the vectors are requested three (chunk, direction)
// steps ahead, across chunk boundaries; with fewer passes, where the stream of
// the blocks dominates, one buffer and one direction ahead.  Every load and
// store is a raw buffer access
// whose range ends at the chunk's last right-hand side, so the rows of a
// partial last pass read zero and their results are dropped, with no test in
// the kernel.  TERMS
// bf16 terms of each vector entry (split_bf16c) are multiplied in turn: with 1
// the products and their order per output are those of the other tile shapes
// (the same bits); with 3 the products are exact and only the FP32 sums round.
constexpr int RS_NB = 64;
template <int NB, int TERMS, int NP>
__global__ void __launch_bounds__(8 * NB) coarse_mfma_rs_kernel(CoarseGeom c, const uint32_t* __restrict__ A,
                                                                const float2* __restrict__ v,
                                                                float2* __restrict__ out, int nrhs) {
    constexpr int NT = 8 * NB, VST = NB + 4, RPC = 16 * NP;  // work-items, LDS row stride, rows per chunk
    constexpr int NA4 = NB * NB / 4 / NT;                     // 16-byte block loads per work-item and block
    constexpr int ABW = NB * VST, BUFW = ABW + TERMS * RPC * VST;  // words: one block; one staging buffer
    static_assert(NA4 * 4 * NT == NB * NB, "block loads must tile the block");
    // staging buffers [block NB x VST][TERMS][RPC][VST] (two at three or more
    // passes: step g (chunk, direction) is read from buffer g & 1 while step
    // g + 1 is written to the other)
    extern __shared__ unsigned char smem_raw[];
    uint32_t* const sbuf = reinterpret_cast<uint32_t*>(smem_raw);
    const int a = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int kq = lane >> 4, col = lane & 15;
    const uint32_t rot = (col & 1) ? 16u : 0u;
    const uint32_t flip = (col & 1) ? 0u : 0x80000000u;
    const int j = (16 * wave + col) >> 1;  // complex row of this lane's A-operand words
    int nbr[9];
#pragma unroll
    for (int d = 0; d < 9; ++d) nbr[d] = coarse_nbr(c, a, d);
    const __amdgpu_buffer_rsrc_t ra = make_rsrc(A + (size_t)a * 9 * NB * NB, 9u * NB * NB * 4u);
    // work-item's vector pair: row 16 p + vr of pass p, complex entries 2 kp, 2 kp + 1
    const int vr = threadIdx.x / (NB / 2), kp = threadIdx.x % (NB / 2);
    // DB (three or four passes per chunk): two staging buffers, one barrier per
    // step; the vectors of step g are requested AH = 3 steps (1 with B22) before
    // it is staged, across chunk boundaries, into a ring of AH register sets
    // (AH divides 9, so a direction always uses the same set).  Otherwise (the
    // stream of the blocks dominates): one buffer, staged and then read, the
    // vectors one direction ahead within the chunk.
    constexpr bool DB = NP >= 3;
    constexpr bool B22 = NP == 4 && TERMS > 1;  // 2 x 2 tile blocks per wave (products below)
    constexpr int AH = DB && !B22 ? 3 : 1;
    const int nch = (nrhs + RPC - 1) / RPC;
    auto vrsrc = [&](int ch) {
        const size_t chunk = (size_t)ch * RPC * c.Nc * NB;
        return make_rsrc(v + chunk, (uint32_t)((size_t)min(RPC, nrhs - ch * RPC) * c.Nc * NB * 8));
    };
    float4 vx[AH][NP];
    auto load_dir = [&](__amdgpu_buffer_rsrc_t rv, int slot, int nd) {
#pragma unroll
        for (int p = 0; p < NP; ++p)
            vx[slot][p] = __builtin_bit_cast(
                    float4, __builtin_amdgcn_raw_buffer_load_b128(
                                rv, (((uint32_t)(16 * p + vr) * c.Nc + nd) * NB + 2 * kp) * 8u, 0, 0));
    };
    u32x4 pre[9][NA4];
#pragma unroll
    for (int d = 0; d < 9; ++d)
#pragma unroll
        for (int u = 0; u < NA4; ++u)
            pre[d][u] = __builtin_amdgcn_raw_buffer_load_b128(ra, (d * NB * NB + 4 * (threadIdx.x + u * NT)) * 4u, 0, 0);
    // block d and the bf16 terms of ring set d % AH into staging buffer b
    auto stage = [&](int b, const u32x4 (&blk)[NA4], const float4 (&x)[NP]) {
        uint32_t* const ab = sbuf + b * BUFW;
        uint32_t* const vb = ab + ABW;
#pragma unroll
        for (int u = 0; u < NA4; ++u) {
            const int e = 4 * (threadIdx.x + u * NT);
            *reinterpret_cast<u32x4*>(ab + (e / NB) * VST + e % NB) = blk[u];
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            uint32_t w0[TERMS], w1[TERMS];
            split_bf16c<TERMS>(make_float2(x[p].x, x[p].y), w0);
            split_bf16c<TERMS>(make_float2(x[p].z, x[p].w), w1);
#pragma unroll
            for (int t = 0; t < TERMS; ++t)
                *reinterpret_cast<uint2*>(vb + (t * RPC + 16 * p + vr) * VST + 2 * kp) = make_uint2(w0[t], w1[t]);
        }
    };
    // products of one step from staging buffer b into acc.  B22 (four passes of
    // split vectors): each wave takes a 2 x 2 block of (row tile, pass) tiles,
    // rows 2 rp, 2 rp + 1 and passes 2 pp, 2 pp + 1 (acc[2 r + i]), so that it
    // reads half the staged vectors and two row slices of the block (a fifth
    // less LDS reading than one row tile by four passes; the vectors then go
    // one step ahead, for registers); otherwise row tile `wave` by every pass.
    // Either way each output takes the same products in the same order.
    auto products = [&](int b, f32x4 (&acc)[NP]) {
        const uint32_t* const ab = sbuf + b * BUFW;
        const uint32_t* const vb = ab + ABW;
        if constexpr (B22) {
            const int rp = wave & 3, pp = wave >> 2;
            // one k-slice at a time, so that only its operands are live
#pragma unroll
            for (int ks = 0; ks < NB / 16; ++ks) {
                u32x4 aw2[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int jr = (16 * (2 * rp + r) + col) >> 1;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t w = ab[(16 * ks + 4 * kq + q) * VST + jr];
                        aw2[r][q] = __builtin_amdgcn_alignbit(w, w, rot) ^ flip;
                    }
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int t = 0; t < TERMS; ++t) {
                        const u32x4 bw = *reinterpret_cast<const u32x4*>(
                                vb + (t * RPC + 16 * (2 * pp + i) + col) * VST + 16 * ks + 4 * kq);
#pragma unroll
                        for (int r = 0; r < 2; ++r)
                            acc[2 * r + i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                    __builtin_bit_cast(bf16x8, aw2[r]), __builtin_bit_cast(bf16x8, bw),
                                    acc[2 * r + i], 0, 0, 0);
                    }
                __builtin_amdgcn_sched_barrier(0);  // keeps the next slice's reads from being hoisted (spills)
            }
            return;
        }
        u32x4 aw[NB / 16];
#pragma unroll
        for (int ks = 0; ks < NB / 16; ++ks)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t w = ab[(16 * ks + 4 * kq + q) * VST + j];
                aw[ks][q] = __builtin_amdgcn_alignbit(w, w, rot) ^ flip;
            }
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int ks = 0; ks < NB / 16; ++ks)
#pragma unroll
                for (int t = 0; t < TERMS; ++t) {
                    const u32x4 bw =
                        *reinterpret_cast<const u32x4*>(vb + (t * RPC + 16 * p + col) * VST + 16 * ks + 4 * kq);
                    acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, aw[ks]),
                                                                     __builtin_bit_cast(bf16x8, bw), acc[p], 0, 0, 0);
                }
    };
    if constexpr (DB) {
        const __amdgpu_buffer_rsrc_t rv0 = vrsrc(0);
#pragma unroll
        for (int d = 0; d < AH; ++d) load_dir(rv0, d, nbr[d]);
        stage(0, pre[0], vx[0]);
        load_dir(rv0, 0, nbr[AH]);  // step AH, into the set just staged
        __syncthreads();
    }
    for (int ch = 0; ch < nch; ++ch) {
        const int r0 = ch * RPC;
        const size_t chunk = (size_t)r0 * c.Nc * NB;
        const __amdgpu_buffer_rsrc_t rv = vrsrc(ch);
        const bool more = ch + 1 < nch;
        const __amdgpu_buffer_rsrc_t rvn = more ? vrsrc(ch + 1) : rv;
        const __amdgpu_buffer_rsrc_t ro =
                make_rsrc(out + chunk, (uint32_t)((size_t)min(RPC, nrhs - r0) * c.Nc * NB * 8));
        f32x4 acc[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) acc[p] = f32x4{0, 0, 0, 0};
        if constexpr (!DB) load_dir(rv, 0, nbr[0]);
#pragma unroll
        for (int d = 0; d < 9; ++d) {
            if constexpr (DB) {
                const int cur = (ch + d) & 1;  // buffer of step 9 ch + d
                // stage step g + 1 into the other buffer, then request the
                // vectors of step g + 1 + AH into the ring set it used
                const int dn = d < 8 ? d + 1 : 0;  // direction of step g + 1
                const int dl = dn + AH;            // direction of step g + 1 + AH, counted from step g + 1's chunk
                if (d < 8) {
                    stage(cur ^ 1, pre[dn], vx[dn % AH]);
                    if (dl < 9)
                        load_dir(rv, dn % AH, nbr[dl < 9 ? dl : 0]);
                    else if (more)
                        load_dir(rvn, dn % AH, nbr[dl >= 9 ? dl - 9 : 0]);
                } else if (more) {
                    stage(cur ^ 1, pre[0], vx[0]);
                    load_dir(rvn, 0, nbr[AH]);  // step g + 1 + AH: direction AH of chunk ch + 1
                }
                products(cur, acc);
                __syncthreads();  // step g read; step g + 1 staged
            } else {
                __syncthreads();  // the previous direction's operands have been read
                stage(0, pre[d], vx[0]);
                if (d < 8) load_dir(rv, 0, nbr[d < 8 ? d + 1 : 0]);  // in flight during this direction's products
                __syncthreads();
                products(0, acc);
            }
        }
        // lane holds complex rows j0, j0 + 1 of right-hand side 16 p + col; rows
        // past the chunk's last right-hand side fall outside ro and are dropped
#pragma unroll
        for (int e = 0; e < NP; ++e) {
            const int rt = B22 ? 2 * (wave & 3) + e / 2 : wave;  // row tile
            const int p = B22 ? 2 * (wave >> 2) + e % 2 : e;      // pass
            const int j0 = 8 * rt + 2 * kq;
            store_b128<0>(__builtin_bit_cast(u32x4, acc[e]), ro, (((uint32_t)(16 * p + col) * c.Nc + a) * NB + j0) * 8u,
                          0u);
        }
    }
}

template <int TERMS, int NP>
void rs_launch(const CoarseGeom& c, const uint32_t* A, const float2* v, float2* out, int nrhs, hipStream_t s) {
    constexpr int NB = RS_NB;
    const size_t lds = (NP >= 3 ? 2 : 1) * ((size_t)NB * (NB + 4) * 4 + (size_t)TERMS * 16 * NP * (NB + 4) * 4);
    // per instantiation and device: raise the dynamic LDS limit once (setting
    // it twice from racing threads is harmless)
    static std::atomic<unsigned long long> attr_devices{0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (!((attr_devices.load(std::memory_order_relaxed) >> dev) & 1ull)) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(coarse_mfma_rs_kernel<NB, TERMS, NP>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr_devices.fetch_or(1ull << dev, std::memory_order_relaxed);
    }
    hipLaunchKernelGGL((coarse_mfma_rs_kernel<NB, TERMS, NP>), dim3(c.Nc), dim3(8 * NB), lds, s, c, A, v, out, nrhs);
}

template <int TERMS>
void rs_dispatch(const CoarseGeom& c, const uint32_t* A, const float2* v, float2* out, int nrhs, hipStream_t s) {
    // passes per chunk: all of them up to 4 (8 passes need more than the 256
    // registers of two waves per SIMD), else 3 or 4, whichever leaves fewer
    // empty passes in the last chunk (4 on a tie)
    const int passes = (nrhs + 15) / 16;
    const int np = passes <= 4 ? passes : ((passes + 2) / 3 * 3 - passes < (passes + 3) / 4 * 4 - passes ? 3 : 4);
    if (np == 1) rs_launch<TERMS, 1>(c, A, v, out, nrhs, s);
    else if (np == 2) rs_launch<TERMS, 2>(c, A, v, out, nrhs, s);
    else if (np == 3) rs_launch<TERMS, 3>(c, A, v, out, nrhs, s);
    else rs_launch<TERMS, 4>(c, A, v, out, nrhs, s);
}

template <int NW, bool ALDS>
void mfma_launch(const CoarseGeom& c, const uint32_t* A, const float2* v, float2* out, int nrhs, hipStream_t s) {
    const size_t lds = (size_t)9 * MR * (c.Nb + 4) * 4 + (ALDS ? (size_t)c.Nb * c.Nb * 4 : 0);
    const int tpw = (2 * c.Nb / 16) / NW;  // exact (coarse_mfma_eligible)
    if (tpw == 1) {
        hipLaunchKernelGGL((coarse_mfma_kernel<NW, 1, ALDS>), dim3(c.Nc), dim3(64 * NW), lds, s, c, A, v, out, nrhs);
    } else if (tpw == 2) {
        hipLaunchKernelGGL((coarse_mfma_kernel<NW, 2, ALDS>), dim3(c.Nc), dim3(64 * NW), lds, s, c, A, v, out, nrhs);
    } else if constexpr (NW <= 4) {
        if (tpw == 4) {
            hipLaunchKernelGGL((coarse_mfma_kernel<NW, 4, ALDS>), dim3(c.Nc), dim3(64 * NW), lds, s, c, A, v, out,
                               nrhs);
        } else if constexpr (NW <= 2) {
            hipLaunchKernelGGL((coarse_mfma_kernel<NW, 8, ALDS>), dim3(c.Nc), dim3(64 * NW), lds, s, c, A, v, out,
                               nrhs);
        }
    }
}

}  // namespace

// tile-shape variants of the batched apply: waves per coarse site x block staging
int coarse_mfma_variants() { return 9; }
const char* coarse_mfma_variant_name(int k) {
    static const char* names[9] = {"2 waves/site, A direct",  "4 waves/site, A direct",  "8 waves/site, A direct",
                                   "2 waves/site, A via LDS", "4 waves/site, A via LDS", "8 waves/site, A via LDS",
                                   "8 waves/site, A prefetched (Nb 64)",
                                   "8 waves/site, A held across passes, loads batched (Nb 64)",
                                   "8 waves/site, direction outside the passes, up to 64 rhs per chunk (Nb 64)"};
    return (k >= 1 && k <= 9) ? names[k - 1] : "";
}
// waves per coarse site of a variant
static int mfma_waves(int variant) { return variant == 1 || variant == 4 ? 2 : variant == 2 || variant == 5 ? 4 : 8; }
bool coarse_mfma_eligible(const CoarseGeom& c, int variant, int terms) {
    const int nb = c.Nb;
    if (nb != 16 && nb != 32 && nb != 64 && nb != 128) return false;
    if (terms < 1 || terms > 3 || (terms > 1 && variant != 9)) return false;  // split vectors: variant 9 only
    if (variant >= 7 && nb != RS_NB) return false;  // register prefetch sized for Nb = 64 blocks
    // variant 9 addresses a chunk of up to 64 right-hand sides with 32-bit byte offsets
    if (variant == 9 && (size_t)64 * c.Nc * nb * 8 > 0xffffffffu) return false;
    return mfma_waves(variant) <= 2 * nb / 16;
}
void launch_coarse_mfma(const CoarseGeom& c, int variant, int terms, const uint32_t* A, const float2* v, float2* out,
                        int nrhs, hipStream_t s) {
    switch (variant) {
        case 1: mfma_launch<2, false>(c, A, v, out, nrhs, s); break;
        case 2: mfma_launch<4, false>(c, A, v, out, nrhs, s); break;
        case 3: mfma_launch<8, false>(c, A, v, out, nrhs, s); break;
        case 4: mfma_launch<2, true>(c, A, v, out, nrhs, s); break;
        case 5: mfma_launch<4, true>(c, A, v, out, nrhs, s); break;
        case 6: mfma_launch<8, true>(c, A, v, out, nrhs, s); break;
        case 8: {
            const size_t lds = (size_t)9 * MR * PF_AST * 4 + (size_t)PF_NB * PF_AST * 4;
            hipLaunchKernelGGL(coarse_mfma_pf_kernel, dim3(c.Nc), dim3(64 * PF_NW), lds, s, c, A, v, out, nrhs);
            break;
        }
        case 9:
            if (terms == 1) rs_dispatch<1>(c, A, v, out, nrhs, s);
            else if (terms == 2) rs_dispatch<2>(c, A, v, out, nrhs, s);
            else rs_dispatch<3>(c, A, v, out, nrhs, s);
            break;
        default: {
            // 8 waves, Nb = 64: 16 KB blocks, 2 loads of 16 B per work-item and block
            const size_t lds = (size_t)9 * MR * (c.Nb + 4) * 4 + (size_t)c.Nb * c.Nb * 4;
            hipLaunchKernelGGL((coarse_mfma_kernel<8, 1, true, 2>), dim3(c.Nc), dim3(512), lds, s, c, A, v, out, nrhs);
            break;
        }
    }
}

}  // namespace hdcr
