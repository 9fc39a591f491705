// Coarse-space eigenvector deflation (Sec. 5 names it as the way to cut the
// cost of the coarse solve): the low eigenpairs of the little Dirac operator A
// by Chebyshev-filtered subspace iteration in A^2 with Rayleigh-Ritz steps, and
// the stand-alone coarse CR solve that uses them.
//
// The block of m coarse vectors lives in HBM as [m][Nc*Nb]; A^2 is applied to
// the whole block at once by the multi-right-hand-side coarse apply (A streams
// through once per application for all m vectors' work-groups), inner products
// accumulate in FP64 in a fixed order, and only the m x m Gram matrices travel
// to the host, where the small Hermitian eigenproblems are solved by Jacobi
// rotations.
#include <algorithm>
#include <cmath>
#include <complex>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "herm_eig.h"
#include "twolevel.h"

namespace hdcr {

namespace {

constexpr int DWG = 256;
constexpr int ROT_QC = 8;        // output vectors per work-item of the block rotation
constexpr int GRAM_I = 4, GRAM_J = 2;  // Gram tile per work-group
constexpr int GRAM_BLOCKS = 32;  // work-groups along the vector length

int dgrid(int64_t n) {
    int64_t b = (n + DWG - 1) / DWG;
    if (b > 4096) b = 4096;
    return (int)(b < 1 ? 1 : b);
}

// out = a X + b Y + c Z (real coefficients, FP64 arithmetic, one rounding to T);
// Z may be null (taken as 0) and out may alias Z
template <typename T>
__global__ void __launch_bounds__(DWG) lincomb_kernel(int64_t n, double a, const C2<T>* X, double b, const C2<T>* Y,
                                                      double c, const C2<T>* Z, C2<T>* out) {
    for (int64_t i = (int64_t)blockIdx.x * DWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * DWG) {
        const C2<T> x = X[i], y = Y[i];
        double re = a * x.x + b * y.x, im = a * x.y + b * y.y;
        if (Z) {
            const C2<T> z = Z[i];
            re += c * z.x;
            im += c * z.y;
        }
        out[i] = mk<T>((T)re, (T)im);
    }
}

// out[q] = sum_p Y[p][q] in[p] for q in [blockIdx.y * ROT_QC, +ROT_QC) and q < mo
// (Y: m x mo complex, row-major, device); in and out do not overlap
template <typename T>
__global__ void __launch_bounds__(DWG) block_rotate_kernel(int64_t n, int m, int mo, const C2<T>* __restrict__ in,
                                                           const double2* __restrict__ Y, C2<T>* __restrict__ out) {
    const int q0 = blockIdx.y * ROT_QC;
    const int nq = min(ROT_QC, mo - q0);
    for (int64_t i = (int64_t)blockIdx.x * DWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * DWG) {
        double2 acc[ROT_QC];
#pragma unroll
        for (int q = 0; q < ROT_QC; ++q) acc[q] = make_double2(0.0, 0.0);
        for (int p = 0; p < m; ++p) {
            const C2<T> v = in[(size_t)p * n + i];
            const double2 vd = make_double2(v.x, v.y);
#pragma unroll
            for (int q = 0; q < ROT_QC; ++q)
                if (q < nq) acc[q] = cfma<double>(Y[(size_t)p * mo + q0 + q], vd, acc[q]);
        }
#pragma unroll
        for (int q = 0; q < ROT_QC; ++q)
            if (q < nq) out[(size_t)(q0 + q) * n + i] = mk<T>((T)acc[q].x, (T)acc[q].y);
    }
}

// Partial sums of the Gram tile G[i][j] = <X_i, Y_j>, i in [GRAM_I ti, +GRAM_I),
// j in [GRAM_J tj, +GRAM_J), tile blockIdx.y = ti * ntj + tj:
// part[(blockIdx.y * 2 GRAM_I GRAM_J + q) * GRAM_BLOCKS + blockIdx.x]
template <typename T>
__global__ void __launch_bounds__(DWG) gram_kernel(int64_t n, int m, const C2<T>* __restrict__ X,
                                                   const C2<T>* __restrict__ Yv, double* __restrict__ part) {
    constexpr int NQ = 2 * GRAM_I * GRAM_J;
    const int ntj = (m + GRAM_J - 1) / GRAM_J;
    const int i0 = (blockIdx.y / ntj) * GRAM_I, j0 = (blockIdx.y % ntj) * GRAM_J;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * DWG + threadIdx.x; e < n; e += (int64_t)gridDim.x * DWG) {
        double2 x[GRAM_I], y[GRAM_J];
#pragma unroll
        for (int a = 0; a < GRAM_I; ++a) {
            x[a] = make_double2(0.0, 0.0);
            if (i0 + a < m) {
                const C2<T> t = X[(size_t)(i0 + a) * n + e];
                x[a] = make_double2(t.x, t.y);
            }
        }
#pragma unroll
        for (int b = 0; b < GRAM_J; ++b) {
            y[b] = make_double2(0.0, 0.0);
            if (j0 + b < m) {
                const C2<T> t = Yv[(size_t)(j0 + b) * n + e];
                y[b] = make_double2(t.x, t.y);
            }
        }
#pragma unroll
        for (int a = 0; a < GRAM_I; ++a)
#pragma unroll
            for (int b = 0; b < GRAM_J; ++b) {
                acc[2 * (a * GRAM_J + b)] += x[a].x * y[b].x + x[a].y * y[b].y;
                acc[2 * (a * GRAM_J + b) + 1] += x[a].x * y[b].y - x[a].y * y[b].x;
            }
    }
    block_reduce<NQ>(acc);
    if (threadIdx.x == 0) {
        for (int q = 0; q < NQ; ++q) part[((size_t)blockIdx.y * NQ + q) * GRAM_BLOCKS + blockIdx.x] = acc[q];
    }
}

// G[i * m + j] from the tile partials (fixed summation order)
__global__ void __launch_bounds__(DWG) gram_finalize_kernel(int m, const double* __restrict__ part,
                                                            double2* __restrict__ G) {
    constexpr int NQ = 2 * GRAM_I * GRAM_J;
    const int e = blockIdx.x * DWG + threadIdx.x;
    if (e >= m * m) return;
    const int i = e / m, j = e % m;
    const int ntj = (m + GRAM_J - 1) / GRAM_J;
    const int tile = (i / GRAM_I) * ntj + j / GRAM_J;
    const int q = 2 * ((i % GRAM_I) * GRAM_J + (j % GRAM_J));
    const double* pr = part + ((size_t)tile * NQ + q) * GRAM_BLOCKS;
    const double* pi = pr + GRAM_BLOCKS;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < GRAM_BLOCKS; ++b) {
        re += pr[b];
        im += pi[b];
    }
    G[e] = make_double2(re, im);
}

size_t gram_part_doubles(int m) {
    const size_t tiles = (size_t)((m + GRAM_I - 1) / GRAM_I) * ((m + GRAM_J - 1) / GRAM_J);
    return tiles * 2 * GRAM_I * GRAM_J * GRAM_BLOCKS;
}

template <typename T> struct DeflWork {
    C2<T>* B[4];     // blocks of m vectors
    double* part;    // reduction partials
    double* S;       // device scalars
    double2* G;      // m x m Gram matrix
    double2* Y;      // m x m rotation coefficients
};
constexpr int DS_COUNT = 512;
constexpr int DS_NORM = 256, DS_POW = 272;

template <typename T> DeflWork<T> defl_carve(Carver& w, const CoarseGeom& c, int m) {
    const size_t n = (size_t)c.Nc * c.Nb;
    DeflWork<T> k;
    for (int i = 0; i < 4; ++i) k.B[i] = w.take<C2<T>>((size_t)m * n);
    k.part = w.take<double>(std::max(gram_part_doubles(m), (size_t)(2 * MAXV + 1) * REDUCE_BLOCKS));
    k.S = w.take<double>(DS_COUNT);
    k.G = w.take<double2>((size_t)m * m);
    k.Y = w.take<double2>((size_t)m * m);
    return k;
}

template <typename T>
void coarse_apply_any(const CoarseGeom& c, hdcr_dtype dt, const void* A, const C2<T>* v, C2<T>* out, int nrhs,
                      hipStream_t s) {
    if constexpr (sizeof(T) == 8) {
        (void)dt;
        launch_coarse_apply<double>(c, static_cast<const double2*>(A), v, out, nrhs, s);
    } else if (dt == HDCR_C64) {
        launch_coarse_apply<float>(c, static_cast<const float2*>(A), v, out, nrhs, s);
    } else if (nrhs >= 8 && coarse_mfma_eligible(c, 9, 3)) {
        // a block of vectors on the matrix cores, each FP32 entry as three bf16
        // terms: the products are exact and only the FP32 sums round, as in the
        // vector-unit kernel
        launch_coarse_mfma(c, 9, 3, static_cast<const uint32_t*>(A), v, out, nrhs, s);
    } else {
        launch_coarse_apply_bf16(c, static_cast<const uint16_t*>(A), v, out, nrhs, s);
    }
}

typedef std::complex<double> cd;

template <typename T> class DeflBuilder {
  public:
    DeflBuilder(const CoarseGeom& c, hdcr_dtype dt, const void* A, int m, const DeflWork<T>& w, hipStream_t s)
        : c_(c), dt_(dt), A_(A), m_(m), n_((int64_t)c.Nc * c.Nb), w_(w), s_(s) {}

    void apply(const C2<T>* v, C2<T>* out, int nrhs) { coarse_apply_any<T>(c_, dt_, A_, v, out, nrhs, s_); }

    // Rayleigh quotient of A^2 after `iters` power steps from x (x, u, t: single vectors)
    int power(C2<T>* x, C2<T>* u, C2<T>* t, int iters, double* lam) {
        launch_norm2<T>(n_, x, w_.part, w_.S, DS_NORM, s_);
        launch_scale_inv_sqrt<T>(n_, x, w_.S, DS_NORM, s_);
        for (int it = 0; it < iters; ++it) {
            apply(x, u, 1);
            apply(u, t, 1);
            PtrListT<T> L{};
            L.p[0] = x;
            launch_multidot<T, T>(n_, L, 1, t, w_.part, w_.S + DS_POW, s_);
            launch_scale_inv_sqrt<T>(n_, t, w_.S, DS_POW + 2 * MAXV, s_);
            std::swap(x, t);
        }
        double h = 0.0;
        HDCR_HIP_CHECK(hipMemcpyAsync(&h, w_.S + DS_POW, sizeof(double), hipMemcpyDeviceToHost, s_));
        HDCR_HIP_CHECK(hipStreamSynchronize(s_));
        *lam = h;
        return HDCR_OK;
    }

    // T_degree((2 A^2 - hi - lo)/(hi - lo)) on the block in t0, by the recurrence scaled
    // so that the polynomial is 1 at A^2 = 0 (a point below [lo, hi]): the same
    // polynomial up to a constant factor, with no overflow in FP32.  Overwrites t0;
    // returns the buffer holding the result (t0 or t1).
    C2<T>* filter(C2<T>* t0, C2<T>* t1, C2<T>* u, C2<T>* y, int degree, double lo, double hi) {
        if (degree == 0) return t0;
        const int64_t nm = n_ * m_;
        const double e = 0.5 * (hi - lo), cc = 0.5 * (hi + lo);
        const double sigma1 = -e / cc;
        apply(t0, u, m_);
        apply(u, y, m_);
        // t1 = (sigma1 / e) (A^2 - cc) t0
        hipLaunchKernelGGL(lincomb_kernel<T>, dim3(dgrid(nm)), dim3(DWG), 0, s_, nm, sigma1 / e, y, -sigma1 * cc / e,
                           t0, 0.0, nullptr, t1);
        double sigma = sigma1;
        for (int j = 2; j <= degree; ++j) {
            const double sn = 1.0 / (2.0 / sigma1 - sigma);
            apply(t1, u, m_);
            apply(u, y, m_);
            // t0 <- (2 sn / e) (A^2 - cc) t1 - sigma sn t0
            hipLaunchKernelGGL(lincomb_kernel<T>, dim3(dgrid(nm)), dim3(DWG), 0, s_, nm, 2.0 * sn / e, y,
                               -2.0 * sn * cc / e, t1, -sigma * sn, t0, t0);
            std::swap(t0, t1);
            sigma = sn;
        }
        return t1;
    }

    // Gram-Schmidt in index order, applied twice per vector, then normalisation
    void orthonormalise(C2<T>* V) {
        for (int i = 0; i < m_; ++i) {
            C2<T>* yi = V + (size_t)i * n_;
            const int nq = (i + MAXV - 1) / MAXV;
            for (int pass = 0; pass < 2 && i > 0; ++pass) {
                for (int q = 0; q < nq; ++q) {
                    PtrListT<T> L{};
                    const int nv = std::min(MAXV, i - q * MAXV);
                    for (int j = 0; j < nv; ++j) L.p[j] = V + (size_t)(q * MAXV + j) * n_;
                    launch_multidot<T, T>(n_, L, nv, yi, w_.part, w_.S + q * (2 * MAXV + 1), s_);
                }
                for (int q = 0; q < nq; ++q) {
                    PtrListT<T> L{};
                    const int nv = std::min(MAXV, i - q * MAXV);
                    for (int j = 0; j < nv; ++j) L.p[j] = V + (size_t)(q * MAXV + j) * n_;
                    launch_multi_axpy<T>(n_, L, nv, w_.S + q * (2 * MAXV + 1), yi, s_);
                }
            }
            launch_norm2<T>(n_, yi, w_.part, w_.S, DS_NORM, s_);
            launch_scale_inv_sqrt<T>(n_, yi, w_.S, DS_NORM, s_);
        }
    }

    // host copy of G[i][j] = <X_i, Y_j> (m x m, row-major)
    int gram(const C2<T>* X, const C2<T>* Yv, std::vector<cd>& G) {
        const int tiles = ((m_ + GRAM_I - 1) / GRAM_I) * ((m_ + GRAM_J - 1) / GRAM_J);
        hipLaunchKernelGGL(gram_kernel<T>, dim3(GRAM_BLOCKS, tiles), dim3(DWG), 0, s_, n_, m_, X, Yv, w_.part);
        hipLaunchKernelGGL(gram_finalize_kernel, dim3((m_ * m_ + DWG - 1) / DWG), dim3(DWG), 0, s_, m_,
                           (const double*)w_.part, w_.G);
        G.assign((size_t)m_ * m_, cd(0.0, 0.0));
        HDCR_HIP_CHECK(hipMemcpyAsync(G.data(), w_.G, G.size() * sizeof(double2), hipMemcpyDeviceToHost, s_));
        HDCR_HIP_CHECK(hipStreamSynchronize(s_));
        return HDCR_OK;
    }

    // out[q] = sum_p Y[p][q] in[p], q < mo (Y host, m x mo row-major); synchronises
    // before returning so that the host coefficients may be reused
    int rotate(const C2<T>* in, const std::vector<cd>& Y, int mo, C2<T>* out) {
        HDCR_HIP_CHECK(hipMemcpyAsync(w_.Y, Y.data(), (size_t)m_ * mo * sizeof(double2), hipMemcpyHostToDevice, s_));
        hipLaunchKernelGGL(block_rotate_kernel<T>, dim3(dgrid(n_), (mo + ROT_QC - 1) / ROT_QC), dim3(DWG), 0, s_, n_,
                           m_, mo, in, (const double2*)w_.Y, out);
        HDCR_HIP_CHECK(hipGetLastError());
        HDCR_HIP_CHECK(hipStreamSynchronize(s_));
        return HDCR_OK;
    }

  private:
    const CoarseGeom& c_;
    hdcr_dtype dt_;
    const void* A_;
    int m_;
    int64_t n_;
    DeflWork<T> w_;
    hipStream_t s_;
};

// largest residual |A y - theta y| / |theta| of a kept eigenpair (|y| = 1)
constexpr double DEFL_RES_TOL = 1e-2;

template <typename T>
int build_deflation(const CoarseGeom& c, hdcr_dtype dt, const void* A, const hdcr_deflation_params* p,
                    const double2* v0, double* theta, C2<T>* Vout, C2<T>* Wout, double* theta_host, int32_t* k_found,
                    void* work, size_t work_bytes, hipStream_t s) {
    if (k_found) *k_found = 0;
    const int m = p->m, k = p->k;
    const int64_t n = (int64_t)c.Nc * c.Nb;
    Carver cw(work, work_bytes);
    DeflWork<T> w = defl_carve<T>(cw, c, m);
    if (!cw.ok()) return fail(HDCR_ENOMEM, "hdcr_build_deflation: workspace too small");
    DeflBuilder<T> db(c, dt, A, m, w, s);
    C2<T>* B[4] = {w.B[0], w.B[1], w.B[2], w.B[3]};
    launch_convert<double2, C2<T>>((int64_t)m * n, v0, B[0], s);
    launch_convert<C2<T>, C2<T>>(n, B[0], B[1], s);

    // top of the A^2 spectrum
    double lam = 0.0;
    int e = db.power(B[1], B[2], B[3], p->power_iters, &lam);
    if (e) return e;
    if (!(lam > 0.0) || !std::isfinite(lam))
        return fail(HDCR_ENAN, "hdcr_build_deflation: the power iteration found no positive spectrum of A^2");
    const double hi = 1.1 * lam;
    double lo = p->cut * hi;

    std::vector<cd> G, Y;
    std::vector<double> ev(m);
    C2<T>* V = B[0];
    for (int pass = 0; pass < p->iters; ++pass) {
        // the three other blocks serve the filter; V's block is overwritten
        C2<T>* o[3];
        int no = 0;
        for (int i = 0; i < 4; ++i)
            if (B[i] != V) o[no++] = B[i];
        C2<T>* R = db.filter(V, o[0], o[1], o[2], p->degree, lo, hi);
        db.orthonormalise(R);
        C2<T>* f[3];
        no = 0;
        for (int i = 0; i < 4; ++i)
            if (B[i] != R) f[no++] = B[i];
        db.apply(R, f[0], m);  // W = A V
        if ((e = db.gram(f[0], f[0], G))) return e;
        Y.assign((size_t)m * m, cd(0.0, 0.0));
        if (herm_eig(m, G.data(), ev.data(), Y.data()) < 0)
            return fail(HDCR_ENAN, "hdcr_build_deflation: Ritz problem of A^2 did not converge");
        if ((e = db.rotate(R, Y, m, f[1]))) return e;
        V = f[1];
        const double mu = ev[m - 1];
        if (!std::isfinite(mu)) return fail(HDCR_ENAN, "hdcr_build_deflation: non-finite Ritz value of A^2");
        lo = std::min(mu, 0.99 * hi);
    }
    // final Rayleigh-Ritz on A
    C2<T>* Wb = nullptr;
    for (int i = 0; i < 4; ++i)
        if (B[i] != V) {
            Wb = B[i];
            break;
        }
    db.apply(V, Wb, m);
    if ((e = db.gram(V, Wb, G))) return e;
    Y.assign((size_t)m * m, cd(0.0, 0.0));
    if (herm_eig(m, G.data(), ev.data(), Y.data()) < 0)
        return fail(HDCR_ENAN, "hdcr_build_deflation: Ritz problem of A did not converge");
    // residual of Ritz pair q, y = V Y_q (|y| = 1, A y = W Y_q):
    // |A y - theta y|^2 = Y_q^dag (W^dag W) Y_q - theta^2, since V^dag W Y_q = theta Y_q
    std::vector<cd> G2;
    if ((e = db.gram(Wb, Wb, G2))) return e;
    std::vector<double> res2(m);
    for (int q = 0; q < m; ++q) {
        cd acc(0.0, 0.0);
        for (int i = 0; i < m; ++i) {
            cd row(0.0, 0.0);
            for (int j = 0; j < m; ++j) row += G2[(size_t)i * m + j] * Y[(size_t)j * m + q];
            acc += std::conj(Y[(size_t)i * m + q]) * row;
        }
        res2[q] = acc.real() - ev[q] * ev[q];
    }
    // the found pairs (residual at most DEFL_RES_TOL |theta|) in ascending |theta|, at most k
    std::vector<int> order;
    for (int q = 0; q < m; ++q)
        if (std::isfinite(ev[q]) && ev[q] != 0.0 && std::isfinite(res2[q]) &&
            res2[q] <= DEFL_RES_TOL * DEFL_RES_TOL * ev[q] * ev[q])
            order.push_back(q);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return std::fabs(ev[a]) < std::fabs(ev[b]); });
    const int kf = std::min<int>(k, (int)order.size());
    if (kf == 0)
        return fail(HDCR_ENOTCONV, "hdcr_build_deflation: no Ritz pair of A reached a residual of " +
                                       std::to_string(DEFL_RES_TOL) + " |theta| (raise iters, degree or m)");
    std::vector<cd> Ysel((size_t)m * kf);
    std::vector<double> th(kf);
    for (int q = 0; q < kf; ++q) {
        th[q] = ev[order[q]];
        for (int pp = 0; pp < m; ++pp) Ysel[(size_t)pp * kf + q] = Y[(size_t)pp * m + order[q]];
    }
    if ((e = db.rotate(V, Ysel, kf, Vout))) return e;
    if ((e = db.rotate(Wb, Ysel, kf, Wout))) return e;
    HDCR_HIP_CHECK(hipMemcpyAsync(theta, th.data(), kf * sizeof(double), hipMemcpyHostToDevice, s));
    HDCR_HIP_CHECK(hipStreamSynchronize(s));
    if (theta_host)
        for (int q = 0; q < kf; ++q) theta_host[q] = th[q];
    if (k_found) *k_found = kf;
    return HDCR_OK;
}

int check_deflation_params(const CoarseGeom& c, const hdcr_deflation_params* p) {
    const int64_t n = (int64_t)c.Nc * c.Nb;
    if (p->m < 1 || p->m > DEFL_KMAX || p->m > n)
        return fail(HDCR_EINVAL, "hdcr_build_deflation: m must be in [1, " + std::to_string(DEFL_KMAX) +
                                     "] and at most Nc * Nb");
    if (p->k < 1 || p->k > p->m) return fail(HDCR_EINVAL, "hdcr_build_deflation: k must be in [1, m]");
    if (p->degree < 1 || p->degree > 1000) return fail(HDCR_EINVAL, "hdcr_build_deflation: degree must be in [1, 1000]");
    if (p->iters < 1 || p->iters > 100) return fail(HDCR_EINVAL, "hdcr_build_deflation: iters must be in [1, 100]");
    if (p->power_iters < 1 || p->power_iters > 10000)
        return fail(HDCR_EINVAL, "hdcr_build_deflation: power_iters must be in [1, 10000]");
    if (!(p->cut > 0.0 && p->cut < 1.0)) return fail(HDCR_EINVAL, "hdcr_build_deflation: cut must be in (0, 1)");
    return HDCR_OK;
}

bool coarse_dtype_ok(hdcr_dtype dt) { return dt == HDCR_C128 || dt == HDCR_C64 || dt == HDCR_BF16C; }

template <typename T>
int coarse_solve(const CoarseGeom& c, hdcr_dtype dt, const void* A, const hdcr_coarse_deflation* defl, const C2<T>* b,
                 C2<T>* x, int maxiter, double tol, int32_t* iters, void* work, size_t work_bytes, hipStream_t s) {
    Carver cw(work, work_bytes);
    CoarseCRWork<T> w = coarse_cr_carve<T>(cw, c);
    if (!cw.ok()) return fail(HDCR_ENOMEM, "hdcr_coarse_solve: workspace too small");
    launch_zero_i32(w.flags, CCR_FLAGS, s);  // the arrival counters must start at zero
    DeflView<T> dv{};
    if (defl) dv = DeflView<T>{defl->k, defl->theta, static_cast<const C2<T>*>(defl->V), static_cast<const C2<T>*>(defl->W)};
    int it = 0;
    int e = coarse_cr<T>(c, dt, A, b, x, maxiter, tol, w, 0, s, &it, defl ? &dv : nullptr);
    if (e) return e;
    int hf[5] = {0, 0, 0, 0, 0};
    HDCR_HIP_CHECK(hipMemcpyAsync(hf, w.flags, 5 * sizeof(int), hipMemcpyDeviceToHost, s));
    HDCR_HIP_CHECK(hipStreamSynchronize(s));
    if (iters) *iters = hf[1];
    if (hf[4] == 2) return HDCR_EBREAKDOWN;
    if (hf[4] == 3) return HDCR_ENAN;
    return HDCR_OK;
}

// Scratch of hdcr_coarse_solve_static: one array per GPU, in the library's own
// device memory (it lives until the process ends).  Host code never passes the
// array's name to a kernel (on the host it only names the symbol); it takes the
// device address from hipGetSymbolAddress once per device and uses that.
static __device__ __align__(256) unsigned char scratch[HDCR_COARSE_STATIC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch` (looked up on the
// first call on that device).
int static_scratch(void** out) {
    int dev = -1;
    HDCR_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(HDCR_EINVAL, "hdcr_coarse_solve_static: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HDCR_EHIP, std::string("hdcr_coarse_solve_static: hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HDCR_OK;
}

}  // namespace

size_t deflation_workspace_bytes(const CoarseGeom& c, hdcr_dtype dt, int m) {
    Carver w(nullptr, 0);
    if (dt == HDCR_C128)
        defl_carve<double>(w, c, m);
    else
        defl_carve<float>(w, c, m);
    return w.used();
}

}  // namespace hdcr

using namespace hdcr;

extern "C" {

size_t hdcr_deflation_workspace_bytes(const hdcr_coarse_desc* desc, hdcr_dtype A_dtype,
                                      const hdcr_deflation_params* params) {
    if (!desc || !params || check_coarse_desc(desc) || !coarse_dtype_ok(A_dtype)) return 0;
    const CoarseGeom c = make_coarse_geom(desc);
    if (check_deflation_params(c, params)) return 0;
    return deflation_workspace_bytes(c, A_dtype, params->m);
}

int hdcr_build_deflation(const hdcr_coarse_desc* desc, hdcr_dtype A_dtype, const void* A,
                         const hdcr_deflation_params* params, const void* v0, double* theta, void* V, void* W,
                         double* theta_host, int32_t* k_found, void* work, size_t work_bytes, hipStream_t stream) {
    if (k_found) *k_found = 0;
    if (!desc || !params) return fail(HDCR_EINVAL, "hdcr_build_deflation: null descriptor or params");
    int e = check_coarse_desc(desc);
    if (e) return e;
    if (!coarse_dtype_ok(A_dtype)) return fail(HDCR_EINVAL, "hdcr_build_deflation: A_dtype must be C128, C64 or BF16C");
    const CoarseGeom c = make_coarse_geom(desc);
    if ((e = check_deflation_params(c, params))) return e;
    const size_t vs = A_dtype == HDCR_C128 ? 16 : 8;
    if ((e = check_ptr(A, 4, "A")) || (e = check_ptr(v0, 16, "v0")) || (e = check_ptr(theta, 8, "theta")) ||
        (e = check_ptr(V, vs, "V")) || (e = check_ptr(W, vs, "W")) || (e = check_ptr(work, 256, "work")))
        return e;
    const size_t n = (size_t)c.Nc * c.Nb;
    const size_t vb = (size_t)params->k * n * vs;
    if (overlap(V, vb, W, vb) || overlap(theta, params->k * sizeof(double), V, vb) ||
        overlap(theta, params->k * sizeof(double), W, vb))
        return fail(HDCR_EINVAL, "hdcr_build_deflation: theta, V and W overlap");
    if (work_bytes < deflation_workspace_bytes(c, A_dtype, params->m))
        return fail(HDCR_ENOMEM, "hdcr_build_deflation: workspace too small");
    if (A_dtype == HDCR_C128)
        return build_deflation<double>(c, A_dtype, A, params, (const double2*)v0, theta, (double2*)V, (double2*)W,
                                       theta_host, k_found, work, work_bytes, stream);
    return build_deflation<float>(c, A_dtype, A, params, (const double2*)v0, theta, (float2*)V, (float2*)W, theta_host,
                                  k_found, work, work_bytes, stream);
}

int hdcr_coarse_solve(const hdcr_coarse_desc* desc, hdcr_dtype A_dtype, const void* A,
                      const hdcr_coarse_deflation* defl, const void* b, void* x, int32_t maxiter, double tol,
                      int32_t* iters, void* work, size_t work_bytes, hipStream_t stream) {
    int e = check_coarse_desc(desc);
    if (e) return e;
    if (!coarse_dtype_ok(A_dtype)) return fail(HDCR_EINVAL, "hdcr_coarse_solve: A_dtype must be C128, C64 or BF16C");
    if (maxiter < 0) return fail(HDCR_EINVAL, "hdcr_coarse_solve: maxiter must be >= 0");
    if (!std::isfinite(tol)) return fail(HDCR_EINVAL, "hdcr_coarse_solve: tol must be finite");
    const hdcr_dtype vdt = A_dtype == HDCR_C128 ? HDCR_C128 : HDCR_C64;
    const size_t vs = vdt == HDCR_C128 ? 16 : 8;
    if ((e = check_ptr(A, 4, "A")) || (e = check_ptr(b, vs, "b")) || (e = check_ptr(x, vs, "x")) ||
        (e = check_ptr(work, 256, "work")))
        return e;
    const CoarseGeom c = make_coarse_geom(desc);
    const size_t nb = (size_t)c.Nc * c.Nb * vs;
    if (overlap(b, nb, x, nb)) return fail(HDCR_EINVAL, "hdcr_coarse_solve: b and x overlap");
    if (defl && (e = check_deflation(c, defl, vdt, "hdcr_coarse_solve"))) return e;
    const size_t need = vdt == HDCR_C128 ? coarse_cr_bytes<double>(c) : coarse_cr_bytes<float>(c);
    if (work_bytes < need) return fail(HDCR_ENOMEM, "hdcr_coarse_solve: workspace too small");
    if (vdt == HDCR_C128)
        return coarse_solve<double>(c, A_dtype, A, defl, (const double2*)b, (double2*)x, maxiter, tol, iters, work,
                                    work_bytes, stream);
    return coarse_solve<float>(c, A_dtype, A, defl, (const float2*)b, (float2*)x, maxiter, tol, iters, work,
                               work_bytes, stream);
}

int hdcr_coarse_solve_static(const hdcr_coarse_desc* desc, hdcr_dtype A_dtype, const void* A,
                             const hdcr_coarse_deflation* defl, const void* b, void* x, int32_t maxiter, double tol,
                             int32_t* iters, hipStream_t stream) {
    int e = check_coarse_desc(desc);
    if (e) return e;
    if (!coarse_dtype_ok(A_dtype))
        return fail(HDCR_EINVAL, "hdcr_coarse_solve_static: A_dtype must be C128, C64 or BF16C");
    const CoarseGeom c = make_coarse_geom(desc);
    const size_t need = A_dtype == HDCR_C128 ? coarse_cr_bytes<double>(c) : coarse_cr_bytes<float>(c);
    if (need > (size_t)HDCR_COARSE_STATIC_BYTES)
        return fail(HDCR_ENOMEM, "hdcr_coarse_solve_static: the coarse solve needs " + std::to_string(need) +
                                     " bytes of scratch, more than the static " +
                                     std::to_string((size_t)HDCR_COARSE_STATIC_BYTES) +
                                     " (use hdcr_coarse_solve with a workspace)");
    void* ws = nullptr;
    if ((e = static_scratch(&ws))) return e;
    return hdcr_coarse_solve(desc, A_dtype, A, defl, b, x, maxiter, tol, iters, ws, (size_t)HDCR_COARSE_STATIC_BYTES,
                             stream);
}

}  // extern "C"
