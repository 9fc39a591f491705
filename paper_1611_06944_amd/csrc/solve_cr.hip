// Plain conjugate residual on the Hermitian indefinite H = Gamma5 D_dwf (Sec. 3), FP64.
//
//   r = b - H x;  p = r;  Ar = H r;  Ap = Ar
//   repeat:  alpha = Re<r,Ar>/|Ap|^2;  x += alpha p;  r -= alpha Ap
//            Ar = H r;  beta = Re<r',Ar'>/Re<r,Ar>;  p = r + beta p;  Ap = Ar + beta Ap
//
// The scalars live in device memory and are consumed by the update kernels
// directly; the host reads back |r|^2, <r,Ar> and |Ar|^2 once per iteration
// (one synchronisation) to test convergence and breakdown.  On convergence of
// the updated residual the true residual b - H x is recomputed; if it does not
// meet the tolerance the iteration restarts from it.
#include <chrono>
#include <cmath>

#include "solver.h"

namespace hdcr {

namespace {

enum { S_RAR = 0, S_RAR_NEW = 1, S_APAP = 2, S_RR = 3, S_ARAR = 4, S_BB = 5, S_COUNT = 8 };

__global__ void __launch_bounds__(REDUCE_THREADS) cr_update_xr_kernel(int64_t n, double2* __restrict__ x,
                                                                      double2* __restrict__ r,
                                                                      const double2* __restrict__ p,
                                                                      const double2* __restrict__ Ap,
                                                                      const double* __restrict__ S,
                                                                      double* __restrict__ partials) {
    const double alpha = S[S_RAR] / S[S_APAP];
    double v[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double2 xi = x[i], ri = r[i];
        const double2 pi = p[i], api = Ap[i];
        xi.x = fma(alpha, pi.x, xi.x);
        xi.y = fma(alpha, pi.y, xi.y);
        ri.x = fma(-alpha, api.x, ri.x);
        ri.y = fma(-alpha, api.y, ri.y);
        x[i] = xi;
        r[i] = ri;
        v[0] += ri.x * ri.x + ri.y * ri.y;
    }
    block_reduce<1>(v);
    if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

// p = r + beta p;  Ap = Ar + beta Ap;  partial |Ap|^2   (beta = S[RAR_NEW]/S[RAR]);
// with init = true: p = r, Ap = Ar (beta = 0)
__global__ void __launch_bounds__(REDUCE_THREADS) cr_update_p_kernel(int64_t n, const double2* __restrict__ r,
                                                                     double2* __restrict__ p,
                                                                     const double2* __restrict__ Ar,
                                                                     double2* __restrict__ Ap,
                                                                     const double* __restrict__ S, int init,
                                                                     double* __restrict__ partials) {
    const double beta = init ? 0.0 : S[S_RAR_NEW] / S[S_RAR];
    double v[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double2 ri = r[i], ari = Ar[i];
        double2 pi, api;
        if (init) {
            pi = ri;
            api = ari;
        } else {
            pi = p[i];
            api = Ap[i];
            pi.x = fma(beta, pi.x, ri.x);
            pi.y = fma(beta, pi.y, ri.y);
            api.x = fma(beta, api.x, ari.x);
            api.y = fma(beta, api.y, ari.y);
        }
        p[i] = pi;
        Ap[i] = api;
        v[0] += api.x * api.x + api.y * api.y;
    }
    block_reduce<1>(v);
    if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

// partials of (Re<r,Ar>, |Ar|^2)
__global__ void __launch_bounds__(REDUCE_THREADS) cr_dots_kernel(int64_t n, const double2* __restrict__ r,
                                                                 const double2* __restrict__ Ar,
                                                                 double* __restrict__ partials) {
    double v[2] = {0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double2 a = r[i], b = Ar[i];
        v[0] += a.x * b.x + a.y * b.y;
        v[1] += b.x * b.x + b.y * b.y;
    }
    block_reduce<2>(v);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = v[0];
        partials[REDUCE_BLOCKS + blockIdx.x] = v[1];
    }
}

// r = b - Hx; partial |r|^2
__global__ void __launch_bounds__(REDUCE_THREADS) residual_kernel(int64_t n, const double2* __restrict__ b,
                                                                  const double2* __restrict__ Hx,
                                                                  double2* __restrict__ r,
                                                                  double* __restrict__ partials) {
    double v[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double2 bi = b[i], hi = Hx[i];
        const double2 ri = make_double2(bi.x - hi.x, bi.y - hi.y);
        r[i] = ri;
        v[0] += ri.x * ri.x + ri.y * ri.y;
    }
    block_reduce<1>(v);
    if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

}  // namespace

size_t cr_workspace_bytes(const FineGeom& g) {
    Carver c(nullptr, 0);
    const int64_t n = 12LL * g.N5;
    for (int k = 0; k < 4; ++k) c.take<double2>(n);
    c.take<double>(2 * REDUCE_BLOCKS);
    c.take<double>(S_COUNT);
    return c.used();
}

int cr_solve(const FineGeom& g, const hdcr_solve_params* prm, const double2* U, const double2* b, double2* x,
             hdcr_solve_stats* st, double* history, int hcap, void* work, size_t work_bytes, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = 12LL * g.N5;
    Carver c(work, work_bytes);
    double2* r = c.take<double2>(n);
    double2* p = c.take<double2>(n);
    double2* Ar = c.take<double2>(n);
    double2* Ap = c.take<double2>(n);
    double* part = c.take<double>(2 * REDUCE_BLOCKS);
    double* S = c.take<double>(S_COUNT);
    if (!c.ok()) return fail(HDCR_ENOMEM, "hdcr_solve: workspace too small for CR");

    const dim3 rg(REDUCE_BLOCKS), rt(REDUCE_THREADS);
    double hS[S_COUNT];
    auto readS = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(hS, S, sizeof(hS), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);
    };

    int64_t napply = 0;
    // |b|^2
    hipLaunchKernelGGL(cr_dots_kernel, rg, rt, 0, s, n, b, b, part);
    launch_finalize_real(part, 1, S, S_BB, -1, -1, -1, s);
    // r = b - H x
    launch_dslash<double>(g, U, x, Ar, s);
    ++napply;
    hipLaunchKernelGGL(residual_kernel, rg, rt, 0, s, n, b, Ar, r, part);
    launch_finalize_real(part, 1, S, S_RR, -1, -1, -1, s);
    HDCR_HIP_CHECK(readS());
    const double bb = hS[S_BB];
    const double tol2 = prm->tol * prm->tol * bb;
    int status = HDCR_ENOTCONV;
    int it = 0;
    int hl = 0;
    double rr = hS[S_RR];
    if (bb == 0.0) {
        HDCR_HIP_CHECK(hipMemsetAsync(x, 0, n * sizeof(double2), s));
        HDCR_HIP_CHECK(hipStreamSynchronize(s));
        status = HDCR_OK;
        rr = 0.0;
    } else if (!std::isfinite(rr) || !std::isfinite(bb)) {
        status = HDCR_ENAN;
    } else if (rr <= tol2) {
        status = HDCR_OK;
    }
    bool need_init = true;
    while (status == HDCR_ENOTCONV && it < prm->maxiter) {
        if (need_init) {
            // p = r, Ar = H r, Ap = Ar, <r,Ar>, |Ar|^2, |Ap|^2
            launch_dslash<double>(g, U, r, Ar, s);
            ++napply;
            hipLaunchKernelGGL(cr_dots_kernel, rg, rt, 0, s, n, r, Ar, part);
            launch_finalize_real(part, 2, S, S_RAR, S_ARAR, -1, -1, s);
            hipLaunchKernelGGL(cr_update_p_kernel, rg, rt, 0, s, n, r, p, Ar, Ap, S, 1, part);
            launch_finalize_real(part, 1, S, S_APAP, -1, -1, -1, s);
            HDCR_HIP_CHECK(readS());
            need_init = false;
            const double rAr = hS[S_RAR];
            if (!(std::fabs(rAr) >= 1e-13 * std::sqrt(rr) * std::sqrt(hS[S_ARAR]))) {
                status = std::isfinite(rAr) ? HDCR_EBREAKDOWN : HDCR_ENAN;
                break;
            }
        }
        // x += alpha p; r -= alpha Ap; |r|^2; then speculatively Ar = H r, <r,Ar>, |Ar|^2
        hipLaunchKernelGGL(cr_update_xr_kernel, rg, rt, 0, s, n, x, r, p, Ap, S, part);
        launch_finalize_real(part, 1, S, S_RR, -1, -1, -1, s);
        launch_dslash<double>(g, U, r, Ar, s);
        ++napply;
        hipLaunchKernelGGL(cr_dots_kernel, rg, rt, 0, s, n, r, Ar, part);
        launch_finalize_real(part, 2, S, S_RAR_NEW, S_ARAR, -1, -1, s);
        HDCR_HIP_CHECK(readS());
        ++it;
        rr = hS[S_RR];
        if (history && hl < hcap) history[hl++] = std::sqrt(rr / bb);
        if (!std::isfinite(rr)) {
            status = HDCR_ENAN;
            break;
        }
        if (rr <= tol2) {
            // true residual
            launch_dslash<double>(g, U, x, Ar, s);
            ++napply;
            hipLaunchKernelGGL(residual_kernel, rg, rt, 0, s, n, b, Ar, r, part);
            launch_finalize_real(part, 1, S, S_RR, -1, -1, -1, s);
            HDCR_HIP_CHECK(readS());
            rr = hS[S_RR];
            if (rr <= tol2) {
                status = HDCR_OK;
                break;
            }
            need_init = true;
            continue;
        }
        const double rAr_new = hS[S_RAR_NEW];
        const double ArAr = hS[S_ARAR];
        if (!(std::fabs(rAr_new) >= 1e-13 * std::sqrt(rr) * std::sqrt(ArAr))) {
            status = std::isfinite(rAr_new) ? HDCR_EBREAKDOWN : HDCR_ENAN;
            break;
        }
        // p = r + beta p; Ap = Ar + beta Ap; |Ap|^2; then <r,Ar> becomes the old value
        hipLaunchKernelGGL(cr_update_p_kernel, rg, rt, 0, s, n, r, p, Ar, Ap, S, 0, part);
        launch_finalize_real(part, 1, S, S_APAP, -1, S_RAR_NEW, S_RAR, s);
    }
    // final true residual (also when not converged)
    launch_dslash<double>(g, U, x, Ar, s);
    ++napply;
    hipLaunchKernelGGL(residual_kernel, rg, rt, 0, s, n, b, Ar, r, part);
    launch_finalize_real(part, 1, S, S_RR, -1, -1, -1, s);
    HDCR_HIP_CHECK(readS());
    HDCR_HIP_CHECK(hipGetLastError());
    const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st) {
        st->status = status;
        st->outer_iters = it;
        st->coarse_iters = 0;
        st->fine_applies_f64 = napply;
        st->fine_applies_inner = 0;
        st->coarse_applies = 0;
        st->true_rel_residual = bb > 0 ? std::sqrt(hS[S_RR] / bb) : 0.0;
        st->seconds_total = t;
        st->seconds_fine = 0;
        st->seconds_coarse = 0;
        st->seconds_outer = t;
        st->history_len = hl;
    }
    return status;
}

}  // namespace hdcr
