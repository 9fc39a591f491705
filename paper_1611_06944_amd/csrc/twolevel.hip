// Two-level HDCR solve (Sec. 4) on gfx950: coarse conjugate residual, the
// Chebyshev smoother, the symmetric two-level cycle, flexible GCR in FP64,
// the Chebyshev low-pass subspace filter and a power-iteration estimate of the
// top of the H^2 spectrum.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>

#include <initializer_list>
#include <utility>

#include "twolevel.h"

namespace hdcr {

// ---------------------------------------------------------------------------
// phase timer (HIP events on the solve's stream)
// ---------------------------------------------------------------------------
hipEvent_t PhaseTimer::get() {
    hipEvent_t e = nullptr;
    if (!pool.empty()) {
        e = pool.back();
        pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}
void PhaseTimer::begin(int phase) {
    if (!on) return;
    if (open_phase == phase) return;
    end();
    open_ev = get();
    if (open_ev) (void)hipEventRecord(open_ev, s);
    open_phase = phase;
}
void PhaseTimer::end() {
    if (!on || open_phase < 0) return;
    hipEvent_t b = get();
    if (b && open_ev) {
        (void)hipEventRecord(b, s);
        recs.push_back({open_ev, b, open_phase});
    }
    open_phase = -1;
    open_ev = nullptr;
}
void PhaseTimer::totals(double out[3]) {
    out[0] = out[1] = out[2] = 0.0;
    for (auto& r : recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) out[r.phase] += ms * 1e-3;
    }
}
PhaseTimer::~PhaseTimer() {
    for (auto& r : recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
    if (open_ev) (void)hipEventDestroy(open_ev);
}

// ---------------------------------------------------------------------------
// coarse CR driver
// ---------------------------------------------------------------------------
template <typename T> CoarseCRWork<T> coarse_cr_carve(Carver& w, const CoarseGeom& c) {
    const size_t n = (size_t)c.Nc * c.Nb;
    CoarseCRWork<T> k;
    k.r = w.take<C2<T>>(n);
    k.p = w.take<C2<T>>(n);
    k.Ar = w.take<C2<T>>(n);
    k.Ap = w.take<C2<T>>(n);
    k.part = w.take<double>(3 * (size_t)c.Nc + 2 * (size_t)std::max(CCR_BLOCKS, DEFL_INIT_BLOCKS) +
                            4 * (size_t)CCR_UPDATE_MAX);
    k.cs = w.take<double>(8);
    k.flags = w.take<int>(CCR_FLAGS);
    k.dpart = w.take<double>((size_t)2 * DEFL_KMAX * DEFL_BLOCKS);
    k.dcoef = w.take<double>((size_t)2 * DEFL_KMAX);
    return k;
}
template <typename T> size_t coarse_cr_bytes(const CoarseGeom& c) {
    Carver w(nullptr, 0);
    coarse_cr_carve<T>(w, c);
    return w.used();
}

template <typename T>
int coarse_cr(const CoarseGeom& c, hdcr_dtype A_dtype, const void* A, const C2<T>* b, C2<T>* x, int maxiter,
              double tol, const CoarseCRWork<T>& w, int hint, hipStream_t s, int* iters, const DeflView<T>* defl,
              int* reason) {
    if (reason) *reason = 0;
    if (defl)
        launch_ccr_init_defl<T>(c, b, x, w, *defl, maxiter, tol, s);
    else
        launch_ccr_init<T>(c, b, x, w, maxiter, tol, s);
    launch_ccr_step<T>(c, A_dtype, A, x, w, 0, s);
    if (tol <= 0) {
        for (int i = 1; i <= maxiter; ++i) launch_ccr_step<T>(c, A_dtype, A, x, w, i, s);
        if (iters) *iters = maxiter;
        HDCR_HIP_CHECK(hipGetLastError());
        return HDCR_OK;
    }
    // enqueue a batch sized by the previous solve, then check the device flag
    int enq = 0;
    int batch = std::max(4, std::min(hint > 0 ? hint + 2 : 16, maxiter));
    int hf[5] = {0, 0, 0, 0, 0};
    while (enq < maxiter) {
        const int nb = std::min(batch, maxiter - enq);
        for (int i = 1; i <= nb; ++i) launch_ccr_step<T>(c, A_dtype, A, x, w, enq + i, s);
        enq += nb;
        HDCR_HIP_CHECK(hipMemcpyAsync(hf, w.flags, 5 * sizeof(int), hipMemcpyDeviceToHost, s));
        HDCR_HIP_CHECK(hipStreamSynchronize(s));
        if (hf[0]) break;
        batch = 8;
    }
    if (iters) *iters = hf[1];
    if (reason) *reason = hf[4];
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}

template CoarseCRWork<double> coarse_cr_carve<double>(Carver&, const CoarseGeom&);
template CoarseCRWork<float> coarse_cr_carve<float>(Carver&, const CoarseGeom&);
template size_t coarse_cr_bytes<double>(const CoarseGeom&);
template size_t coarse_cr_bytes<float>(const CoarseGeom&);
template int coarse_cr<double>(const CoarseGeom&, hdcr_dtype, const void*, const double2*, double2*, int, double,
                               const CoarseCRWork<double>&, int, hipStream_t, int*, const DeflView<double>*, int*);
template int coarse_cr<float>(const CoarseGeom&, hdcr_dtype, const void*, const float2*, float2*, int, double,
                              const CoarseCRWork<float>&, int, hipStream_t, int*, const DeflView<float>*, int*);

// ---------------------------------------------------------------------------
// Chebyshev smoother
// ---------------------------------------------------------------------------
void cheby_coeffs(int n, double lo, double hi, double* c) {
    // interpolant of 1/y at the n Chebyshev points of [lo, hi]:
    // p(y) = sum_j c_j T_j(yhat) - c_0/2,  yhat = (2y - hi - lo)/(hi - lo)
    const double pi = 3.14159265358979323846;
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) {
            const double th = pi * (k + 0.5) / n;
            const double y = 0.5 * (hi + lo) + 0.5 * (hi - lo) * std::cos(th);
            s += std::cos(j * th) / y;
        }
        c[j] = 2.0 * s / n;
    }
}

// Stencil operations of the smoother on fields of precision T.
template <typename T> struct SmootherOps {
    const FineGeom& g;
    const C2<T>* U;
    hipStream_t s;
    void apply(const C2<T>* a, C2<T>* b) const { launch_dslash<T>(g, U, a, b, s); }
    void epi(const C2<T>* a, C2<T>* b, const Epi<T>& e) const { launch_dslash_epi<T>(g, U, a, b, e, s); }
    void scale_u(const C2<T>* u, double c0, C2<T>* out, bool accumulate) const {
        const int64_t n = 12LL * g.N5;
        if (accumulate)
            launch_axpby<T>(n, (T)c0, u, (T)1, out, s);
        else
            launch_scale<T>(n, (T)c0, u, out, s);
    }
};
// The same on FP16-stored fields (the float2 pointers address (fp16 re, fp16 im)
// entries; FP32 links and arithmetic): the combination of a fused epilogue is
// a separate element-wise pass over tmp, the stencil's output.  Needs at least
// two Chebyshev terms.
struct SmootherOpsH16 {
    const FineGeom& g;
    const float2* U;
    void* tmp;
    hipStream_t s;
    void apply(const float2* a, float2* b) const { launch_dslash_h16(g, U, a, b, s); }
    // the combination fused into the stencil's epilogue; variant 6: a plain
    // pass into tmp, then an element-wise combination (one more FP16 write
    // and read of the field, one more rounding)
    void epi(const float2* a, float2* b, const Epi<float>& e) const {
        if (g.variant != 6) {
            launch_dslash_h16_epi(g, U, a, b, e, s);
            return;
        }
        launch_dslash_h16(g, U, a, tmp, s);
        const void* z[4] = {e.y[0], e.y[1], e.y[2], e.y[3]};
        launch_h16_combine(12LL * g.N5, e.beta, tmp, z, e.g, e.ny, b, s);
    }
    void scale_u(const float2*, double, float2*, bool) const {}
};

// out = p(H^2) H in   (accumulate: out += p(H^2) H in), with
// p(y) = sum_{j<n} c'_j T_j(yhat), c'_0 = c_0 / 2, c'_j = c_j, yhat = a1 y + b1,
// evaluated by Clenshaw's recurrence on u = H in:
//   b_{n-1} = c'_{n-1} u,  b_k = c'_k u + 2 yhat b_{k+1} - b_{k+2},
//   result = c'_0 u + yhat b_1 - b_2,
// where yhat b = a1 H (H b) + b1 b.  Each step's second stencil application
// carries the combination in its epilogue, so a step costs two stencil passes
// and no separate vector pass.  tmp: four fields (u, V, and two b_k); `in` is
// read only by the first stencil pass.
template <typename T, typename Ops>
void clenshaw(const Ops& ops, const C2<T>* in, C2<T>* out, bool accumulate, C2<T>* const tmp[4], int order,
              double lo, double hi) {
    const int nc = order;
    std::vector<double> c(nc);
    cheby_coeffs(nc, lo, hi, c.data());
    c[0] *= 0.5;
    const double a1 = 2.0 / (hi - lo), b1 = -(hi + lo) / (hi - lo);
    C2<T>* u = tmp[0];
    C2<T>* V = tmp[1];
    C2<T>* bk1 = tmp[2];  // b_{k+1}
    C2<T>* bk2 = tmp[3];  // b_{k+2}, overwritten in place by b_k
    ops.apply(in, u);
    if (nc == 1) {
        ops.scale_u(u, c[0], out, accumulate);
        return;
    }
    auto epi = [&](const C2<T>* src, C2<T>* dst, double beta, std::initializer_list<std::pair<const C2<T>*, double>> ys,
                   bool acc_out) {
        Epi<T> e{{nullptr, nullptr, nullptr, nullptr}, {0, 0, 0, 0}, (T)beta, 0};
        for (const auto& y : ys) {
            e.y[e.ny] = y.first;
            e.g[e.ny] = (T)y.second;
            ++e.ny;
        }
        if (acc_out) {
            e.y[e.ny] = out;
            e.g[e.ny] = (T)1;
            ++e.ny;
        }
        ops.epi(src, dst, e);
    };
    ops.apply(u, V);
    if (nc == 2) {
        // result = c'_0 u + yhat (c'_1 u) = (c'_0 + b1 c'_1) u + a1 c'_1 H H u
        epi(V, out, a1 * c[1], {{u, c[0] + b1 * c[1]}}, accumulate);
        return;
    }
    // b_{n-2} = (c'_{n-2} + 2 b1 c'_{n-1}) u + 2 a1 c'_{n-1} H H u
    epi(V, bk1, 2 * a1 * c[nc - 1], {{u, c[nc - 2] + 2 * b1 * c[nc - 1]}}, false);
    bool implicit2 = true;  // b_{k+2} = b_{n-1} = c'_{n-1} u is not stored
    for (int k = nc - 3; k >= 1; --k) {
        ops.apply(bk1, V);
        if (implicit2)
            epi(V, bk2, 2 * a1, {{u, c[k] - c[nc - 1]}, {bk1, 2 * b1}}, false);
        else
            epi(V, bk2, 2 * a1, {{u, c[k]}, {bk1, 2 * b1}, {bk2, -1.0}}, false);
        implicit2 = false;
        std::swap(bk1, bk2);
    }
    ops.apply(bk1, V);
    if (implicit2)
        epi(V, out, a1, {{u, c[0] - c[nc - 1]}, {bk1, b1}}, accumulate);
    else
        epi(V, out, a1, {{u, c[0]}, {bk1, b1}, {bk2, -1.0}}, accumulate);
}

template <typename T>
void cheb_smoother(const FineGeom& g, const C2<T>* U, const C2<T>* in, C2<T>* out, bool accumulate,
                   C2<T>* const tmp[4], int order, double lo, double hi, hipStream_t s) {
    clenshaw<T>(SmootherOps<T>{g, U, s}, in, out, accumulate, tmp, order, lo, hi);
}

void cheb_smoother_h16(const FineGeom& g, const float2* U, const float2* in, float2* out, bool accumulate,
                       void* const h[6], double* part, double* S, int order, double lo, double hi, hipStream_t s) {
    const int64_t n = 12LL * g.N5;
    float2* hb[5];
    for (int i = 0; i < 5; ++i) hb[i] = static_cast<float2*>(h[i]);
    launch_norm2<float>(n, in, part, S, 0, s);
    launch_to_h16_scaled(n, in, S, 0, hb[0], s);
    float2* const tmp[4] = {hb[1], hb[2], hb[3], hb[4]};
    // hb[0] holds the scaled input for the first pass and then the result
    clenshaw<float>(SmootherOpsH16{g, U, h[5], s}, hb[0], hb[0], false, tmp, order, lo, hi);
    launch_from_h16_scaled(n, hb[0], S, 0, out, accumulate, s);
}

// ---------------------------------------------------------------------------
// two-level cycle
// ---------------------------------------------------------------------------
template <typename T> struct CycleWork {
    C2<T>* t;
    C2<T>* d;
    C2<T>* sm[4];
    C2<T>* vc;
    C2<T>* cx;
    CoarseCRWork<T> ccr;
    void* h16[6];   // FP16 smoother fields (inside sm[0..2], FP32 cycle only)
    double* hpart;  // reduction scratch of the FP16 smoother
    double* hS;
};
template <typename T> CycleWork<T> cycle_carve(Carver& w, const CoarseGeom& c) {
    const size_t n = (size_t)12 * c.f.N5;
    CycleWork<T> k;
    k.t = w.take<C2<T>>(n);
    k.d = w.take<C2<T>>(n);
    for (int i = 0; i < 4; ++i) k.sm[i] = w.take<C2<T>>(n);
    k.vc = w.take<C2<T>>((size_t)c.Nc * c.Nb);
    k.cx = w.take<C2<T>>((size_t)c.Nc * c.Nb);
    k.ccr = coarse_cr_carve<T>(w, c);
    for (int j = 0; j < 6; ++j)
        k.h16[j] = k.sm[j / 2] ? static_cast<void*>(reinterpret_cast<char*>(k.sm[j / 2]) + (j % 2) * n * 4) : nullptr;
    k.hpart = w.take<double>(REDUCE_BLOCKS);
    k.hS = w.take<double>(8);
    return k;
}

struct CycleCounts {
    int64_t fine = 0, coarse_iters = 0, coarse_applies = 0;
    int last_coarse = 0;
    int coarse_stops = 0;  // coarse solves ended by near-breakdown or a non-finite value
};

// e = B r:  e1 = S r;  e2 = e1 + Q (r - H e1);  e = e2 + S (r - H e2),  Q = P A^-1 P^dag
// bh: FP16 copy of the basis used for restriction and prolongation instead of
// `basis` (FP32 cycle only), or null
template <typename T>
int vcycle(const CoarseGeom& c, const hdcr_solve_params* prm, const C2<T>* U, const C2<T>* basis, const uint32_t* bh,
           const void* A, const DeflView<T>* defl, const C2<T>* r, C2<T>* e, const CycleWork<T>& w, PhaseTimer& tm,
           CycleCounts& cnt, hipStream_t s) {
    const FineGeom& g = c.f;
    const int order = prm->cheb_order;
    tm.begin(PhaseTimer::FINE);
    const bool h16 = sizeof(T) == 4 && prm->inner_dtype == HDCR_F16C;
    auto smooth = [&](const C2<T>* in, C2<T>* out, bool acc) {
        if constexpr (sizeof(T) == 4) {
            if (h16) {
                cheb_smoother_h16(g, U, in, out, acc, w.h16, w.hpart, w.hS, order, prm->cheb_lo, prm->cheb_hi, s);
                return;
            }
        }
        cheb_smoother<T>(g, U, in, out, acc, w.sm, order, prm->cheb_lo, prm->cheb_hi, s);
    };
    smooth(r, e, false);
    // t = r - H e1 (fused into the stencil's epilogue; the same single rounding
    // as subtracting H e1 inside the restriction), then P^dag t
    launch_dslash_epi<T>(g, U, e, w.t, Epi<T>{{r, nullptr, nullptr, nullptr}, {(T)1, 0, 0, 0}, (T)-1, 1}, s);
    tm.begin(PhaseTimer::COARSE);
    if constexpr (sizeof(T) == 4) {
        if (bh)
            launch_restrict_h(c, bh, w.t, nullptr, w.vc, s);
        else
            launch_restrict<T>(c, basis, w.t, nullptr, w.vc, s);
    } else {
        launch_restrict<T>(c, basis, w.t, nullptr, w.vc, s);
    }
    int it = 0, reason = 0;
    int st = coarse_cr<T>(c, (hdcr_dtype)prm->coarse_dtype, A, w.vc, w.cx, prm->coarse_maxiter, prm->coarse_tol, w.ccr,
                          cnt.last_coarse, s, &it, defl, &reason);
    if (st) return st;
    if (reason) ++cnt.coarse_stops;
    cnt.last_coarse = it;
    cnt.coarse_iters += it;
    cnt.coarse_applies += it + 1;
    if constexpr (sizeof(T) == 4) {
        if (bh)
            launch_prolong_h(c, bh, w.cx, e, e, s);
        else
            launch_prolong<T>(c, basis, w.cx, e, e, s);
    } else {
        launch_prolong<T>(c, basis, w.cx, e, e, s);
    }
    tm.begin(PhaseTimer::FINE);
    // d = r - H e2 (fused), e = e2 + S d
    launch_dslash_epi<T>(g, U, e, w.d, Epi<T>{{r, nullptr, nullptr, nullptr}, {(T)1, 0, 0, 0}, (T)-1, 1}, s);
    smooth(w.d, e, true);
    cnt.fine += 2 * (2 * order - 1) + 2;
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}

// ---------------------------------------------------------------------------
// flexible GCR (FP64 outer iteration) preconditioned with the two-level cycle
// ---------------------------------------------------------------------------
// Search directions Z_i (cycle outputs) and W_i = H Z_i are stored in the inner
// precision T and W_i is computed by the stencil in T; x, r, every inner
// product and the true residual at each restart are FP64.
template <typename T> struct FgcrWork {
    C2<T>* Z[MAXV];
    C2<T>* W[MAXV];
    double2* r;
    double2* tmp;
    double* part;
    double* S;        // device scalars: D1 [0,17), D2 [17,34), D3 [34,51), rr 51, bb 52, 1/|W_j|^2 [53,61)
    C2<T>* U_in;      // inner-precision links (FP32 copy, or null for FP64)
    C2<T>* r_in;      // r in the inner precision (FP32 cycle only)
    CycleWork<T> cyc;
};
constexpr int SD1 = 0, SD2 = 2 * MAXV + 1, SD3 = 2 * (2 * MAXV + 1), SRR = 3 * (2 * MAXV + 1), SBB = SRR + 1,
              SINV = SBB + 1, SCOUNT = SINV + MAXV;

template <typename T> FgcrWork<T> fgcr_carve(Carver& w, const CoarseGeom& c, int m) {
    const size_t n = (size_t)12 * c.f.N5;
    FgcrWork<T> k;
    for (int i = 0; i < MAXV; ++i) {
        k.Z[i] = (i < m) ? w.take<C2<T>>(n) : nullptr;
        k.W[i] = (i < m) ? w.take<C2<T>>(n) : nullptr;
    }
    k.r = w.take<double2>(n);
    k.tmp = w.take<double2>(n);
    k.part = w.take<double>((size_t)(2 * MAXV + 1) * REDUCE_BLOCKS);
    k.S = w.take<double>(SCOUNT);
    if (sizeof(T) == 4) {
        k.U_in = w.take<C2<T>>((size_t)36 * c.f.V4);
        k.r_in = w.take<C2<T>>(n);
    } else {
        k.U_in = nullptr;
        k.r_in = nullptr;
    }
    k.cyc = cycle_carve<T>(w, c);
    return k;
}

template <typename T> size_t fgcr_bytes(const CoarseGeom& c, int m) {
    Carver w(nullptr, 0);
    fgcr_carve<T>(w, c, m);
    return w.used();
}

template <typename T>
int fgcr_solve(const CoarseGeom& c, const hdcr_solve_params* prm, const double2* U, const void* basis, const void* A,
               const DeflView<T>* defl, const double2* b, double2* x, hdcr_solve_stats* st, double* history, int hcap,
               void* work, size_t work_bytes, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const FineGeom& g = c.f;
    const int64_t n = 12LL * g.N5;
    const int m = prm->restart;
    Carver cw(work, work_bytes);
    FgcrWork<T> w = fgcr_carve<T>(cw, c, m);
    if (!cw.ok()) return fail(HDCR_ENOMEM, "hdcr_solve: workspace too small for the two-level solve");
    PhaseTimer tm;
    tm.s = s;
    tm.on = true;
    CycleCounts cnt;
    int64_t n64 = 0;  // FP64 fine applications

    const C2<T>* Uin;
    const C2<T>* bas;
    const uint32_t* bh = nullptr;
    if constexpr (sizeof(T) == 4) {
        launch_convert<double2, float2>(36LL * g.V4, U, w.U_in, s);
        Uin = w.U_in;
        bas = basis32(c, basis);
        if (prm->basis_dtype == HDCR_F16C) bh = basis16(c, basis);
    } else {
        Uin = U;
        bas = basis64(basis);
    }
    HDCR_HIP_CHECK(hipMemsetAsync(w.cyc.ccr.flags, 0, CCR_FLAGS * sizeof(int), s));

    double hS[SCOUNT];
    auto readS = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(hS, w.S, sizeof(hS), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);
    };
    // |b|^2 and r = b - H x
    tm.begin(PhaseTimer::OUTER);
    launch_norm2<double>(n, b, w.part, w.S, SBB, s);
    launch_dslash<double>(g, U, x, w.tmp, s);
    ++n64;
    launch_sub<double>(n, b, w.tmp, w.r, s);
    launch_norm2<double>(n, w.r, w.part, w.S, SRR, s);
    tm.end();
    HDCR_HIP_CHECK(readS());
    const double bb = hS[SBB];
    double rr = hS[SRR];
    const double tol2 = prm->tol * prm->tol * bb;
    int status = HDCR_ENOTCONV;
    int it = 0, hl = 0;
    if (bb == 0.0) {
        HDCR_HIP_CHECK(hipMemsetAsync(x, 0, n * sizeof(double2), s));
        status = HDCR_OK;
        rr = 0.0;
    } else if (!std::isfinite(bb) || !std::isfinite(rr)) {
        status = HDCR_ENAN;
    } else if (rr <= tol2) {
        status = HDCR_OK;
    }
    typedef std::complex<double> cd;
    bool true_res = true;  // r is the true residual of x
    bool rin_ok = false;   // r_in holds r rounded to FP32 (written by the last r update)
    while (status == HDCR_ENOTCONV && it < prm->maxiter) {
        true_res = false;
        // coefficient of the normalised directions zhat_i over the raw Z_j
        std::vector<std::vector<cd>> coef;
        std::vector<cd> alpha;
        std::vector<double> wnorm;  // |W_j| of the stored, unnormalised W_j
        int i = 0;
        bool stop = false;
        for (; i < m && it < prm->maxiter; ++i) {
            // z_i = B r
            int e;
            if constexpr (sizeof(T) == 4) {
                tm.begin(PhaseTimer::OUTER);
                if (!rin_ok) launch_convert<double2, float2>(n, w.r, w.r_in, s);
                e = vcycle<T>(c, prm, Uin, bas, bh, A, defl, w.r_in, w.Z[i], w.cyc, tm, cnt, s);
            } else {
                e = vcycle<T>(c, prm, Uin, bas, bh, A, defl, w.r, w.Z[i], w.cyc, tm, cnt, s);
            }
            if (e) return e;
            tm.begin(PhaseTimer::OUTER);
            // w_i = H z_i, orthogonalised twice against the previous w_j.  The W_j are
            // kept unnormalised: the projections take the coefficients <W_j, w>
            // times 1 / |W_j|^2 (S[SINV + j]), and the host divides the same inner
            // products by |W_j| for the normalised directions of its bookkeeping.
            launch_dslash<T>(g, Uin, w.Z[i], w.W[i], s);
            if (sizeof(T) == 8)
                ++n64;
            else
                ++cnt.fine;
            PtrListT<T> Wl{};
            for (int j = 0; j < i; ++j) Wl.p[j] = w.W[j];
            if (i > 0) {  // the second pass's inner products ride on the first pass's update
                launch_multidot<T, T>(n, Wl, i, w.W[i], w.part, w.S + SD1, s);
                launch_multi_axpy_dot<T>(n, Wl, i, w.S + SD1, w.W[i], w.part, w.S + SD2, s, w.S + SINV);
                launch_multi_axpy<T>(n, Wl, i, w.S + SD2, w.W[i], s, w.S + SINV);
            }
            // <r, w>, |w|^2; r -= (<w, r>/|w|^2) w; 1 / |w|^2 for the later projections
            PtrList Rl{};
            Rl.p[0] = w.r;
            launch_multidot<double, T>(n, Rl, 1, w.W[i], w.part, w.S + SD3, s);
            if constexpr (sizeof(T) == 4) {
                launch_r_update<T>(n, w.S, SD3, SD3 + 2 * MAXV, w.W[i], w.r, w.part, s, w.r_in);
                rin_ok = true;  // the next cycle's input, rounded as the conversion would
            } else {
                launch_r_update<T>(n, w.S, SD3, SD3 + 2 * MAXV, w.W[i], w.r, w.part, s);
            }
            launch_finalize_real(w.part, 1, w.S, SRR, -1, -1, -1, s);
            launch_inv_copy(w.S, SD3 + 2 * MAXV, SINV + i, s);
            tm.end();
            HDCR_HIP_CHECK(readS());
            ++it;
            rr = hS[SRR];
            const double ww = hS[SD3 + 2 * MAXV];
            if (!std::isfinite(rr) || !std::isfinite(ww)) {
                status = HDCR_ENAN;
                stop = true;
                ++i;
                break;
            }
            if (!(ww > 0.0)) {
                status = HDCR_EBREAKDOWN;
                stop = true;
                break;
            }
            const double nw = std::sqrt(ww);
            // zhat_i = (Z_i - sum_j beta_ij zhat_j) / |w_i|
            std::vector<cd> ci(m, cd(0, 0));
            ci[i] = cd(1, 0);
            for (int j = 0; j < i; ++j) {
                // <what_j, w> over both passes, what_j = W_j / |W_j|
                const cd beta =
                        (cd(hS[SD1 + 2 * j], hS[SD1 + 2 * j + 1]) + cd(hS[SD2 + 2 * j], hS[SD2 + 2 * j + 1])) / wnorm[j];
                for (int q = 0; q < m; ++q) ci[q] -= beta * coef[j][q];
            }
            for (auto& v : ci) v /= nw;
            coef.push_back(ci);
            wnorm.push_back(nw);
            // step along zhat_i: <what_i, r> = conj(<r, w_i>) / |w_i|
            alpha.push_back(std::conj(cd(hS[SD3], hS[SD3 + 1])) / nw);
            if (history && hl < hcap) history[hl++] = std::sqrt(rr / bb);
            if (rr <= tol2) {
                ++i;
                break;
            }
        }
        // x += sum_i alpha_i zhat_i = sum_q gamma_q Z_q
        const int nz = (int)coef.size();
        if (nz > 0) {
            std::vector<double2> gam(m, make_double2(0, 0));
            for (int q = 0; q < m; ++q) {
                cd gq(0, 0);
                for (int k = 0; k < nz; ++k) gq += alpha[k] * coef[k][q];
                gam[q] = make_double2(gq.real(), gq.imag());
            }
            PtrListT<T> Zl{};
            for (int q = 0; q < m && q < MAXV; ++q) Zl.p[q] = w.Z[q];
            tm.begin(PhaseTimer::OUTER);
            launch_multi_update<T>(n, Zl, std::min(m, MAXV), gam.data(), x, s);
        }
        if (stop) break;
        // true residual at every restart (r then holds b - H x for the current x)
        rin_ok = false;
        tm.begin(PhaseTimer::OUTER);
        launch_dslash<double>(g, U, x, w.tmp, s);
        ++n64;
        launch_sub<double>(n, b, w.tmp, w.r, s);
        launch_norm2<double>(n, w.r, w.part, w.S, SRR, s);
        tm.end();
        HDCR_HIP_CHECK(readS());
        rr = hS[SRR];
        if (!std::isfinite(rr)) {
            status = HDCR_ENAN;
            break;
        }
        if (rr <= tol2) status = HDCR_OK;
        true_res = true;
    }
    // final true residual (unless the restart just computed it for this x)
    if (!true_res) {
        tm.begin(PhaseTimer::OUTER);
        launch_dslash<double>(g, U, x, w.tmp, s);
        ++n64;
        launch_sub<double>(n, b, w.tmp, w.r, s);
        launch_norm2<double>(n, w.r, w.part, w.S, SRR, s);
        tm.end();
        HDCR_HIP_CHECK(readS());
    }
    HDCR_HIP_CHECK(hipGetLastError());
    const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st) {
        double ph[3];
        tm.totals(ph);
        st->status = status;
        st->outer_iters = it;
        st->coarse_iters = cnt.coarse_iters;
        st->fine_applies_f64 = n64;
        st->fine_applies_inner = cnt.fine;
        st->coarse_applies = cnt.coarse_applies;
        st->true_rel_residual = bb > 0 ? std::sqrt(hS[SRR] / bb) : 0.0;
        st->seconds_total = t;
        st->seconds_fine = ph[PhaseTimer::FINE];
        st->seconds_coarse = ph[PhaseTimer::COARSE];
        st->seconds_outer = ph[PhaseTimer::OUTER];
        st->history_len = hl;
        st->coarse_breakdowns = cnt.coarse_stops;
    }
    return status;
}

int check_two_level_params(const hdcr_solve_params* p) {
    if (p->restart < 1 || p->restart > MAXV)
        return fail(HDCR_EINVAL, "restart must be in [1, " + std::to_string(MAXV) + "]");
    if (p->cheb_order < 1 || p->cheb_order > 1000) return fail(HDCR_EINVAL, "cheb_order must be in [1, 1000]");
    if (!(p->cheb_lo > 0) || !(p->cheb_hi > p->cheb_lo)) return fail(HDCR_EINVAL, "need 0 < cheb_lo < cheb_hi");
    if (p->coarse_maxiter < 0) return fail(HDCR_EINVAL, "coarse_maxiter must be >= 0");
    if (p->inner_dtype == HDCR_C128) {
        if (p->coarse_dtype != HDCR_C128) return fail(HDCR_EINVAL, "inner C128 needs coarse_dtype C128");
    } else if (p->inner_dtype == HDCR_C64 || p->inner_dtype == HDCR_F16C) {
        if (p->coarse_dtype != HDCR_C64 && p->coarse_dtype != HDCR_BF16C)
            return fail(HDCR_EINVAL, "inner C64 / F16C needs coarse_dtype C64 or BF16C");
        if (p->inner_dtype == HDCR_F16C && p->cheb_order < 2)
            return fail(HDCR_EINVAL, "inner F16C needs cheb_order >= 2");
    } else {
        return fail(HDCR_EINVAL, "inner_dtype must be C128, C64 or F16C");
    }
    if (p->basis_dtype == HDCR_F16C && p->inner_dtype == HDCR_C128)
        return fail(HDCR_EINVAL, "basis_dtype F16C needs an FP32 cycle (inner_dtype C64 or F16C)");
    if (p->basis_dtype != HDCR_F16C && p->basis_dtype != HDCR_C64 && p->basis_dtype != HDCR_C128)
        return fail(HDCR_EINVAL, "basis_dtype must be C128, C64 or F16C");
    return HDCR_OK;
}

size_t two_level_workspace_bytes(const CoarseGeom& c, const hdcr_solve_params* p) {
    if (p->inner_dtype != HDCR_C128) return fgcr_bytes<float>(c, p->restart);
    return fgcr_bytes<double>(c, p->restart);
}

int check_deflation(const CoarseGeom& c, const hdcr_coarse_deflation* d, hdcr_dtype dtype, const char* where) {
    (void)c;
    const std::string w(where);
    if (d->k < 1 || d->k > DEFL_KMAX)
        return fail(HDCR_EINVAL, w + ": deflation k must be in [1, " + std::to_string(DEFL_KMAX) + "]");
    if (d->dtype != dtype)
        return fail(HDCR_EINVAL, w + ": deflation vectors must be C128 with an FP64 coarse solve, C64 with FP32");
    if (!d->theta || !d->V || !d->W || (reinterpret_cast<uintptr_t>(d->theta) & 7) ||
        (reinterpret_cast<uintptr_t>(d->V) & 7) || (reinterpret_cast<uintptr_t>(d->W) & 7))
        return fail(HDCR_EINVAL, w + ": deflation theta, V and W must be non-null and 8-byte aligned");
    return HDCR_OK;
}

template <typename T> DeflView<T> defl_view(const hdcr_coarse_deflation* d) {
    return DeflView<T>{d->k, d->theta, static_cast<const C2<T>*>(d->V), static_cast<const C2<T>*>(d->W)};
}

int two_level_solve(const CoarseGeom& c, const hdcr_solve_params* p, const double2* U, const void* basis,
                    const void* A, const hdcr_coarse_deflation* defl, const double2* b, double2* x,
                    hdcr_solve_stats* st, double* history, int hcap, void* work, size_t work_bytes, hipStream_t s) {
    if (p->inner_dtype != HDCR_C128) {
        const DeflView<float> dv = defl ? defl_view<float>(defl) : DeflView<float>{};
        return fgcr_solve<float>(c, p, U, basis, A, defl ? &dv : nullptr, b, x, st, history, hcap, work, work_bytes,
                                 s);
    }
    const DeflView<double> dv = defl ? defl_view<double>(defl) : DeflView<double>{};
    return fgcr_solve<double>(c, p, U, basis, A, defl ? &dv : nullptr, b, x, st, history, hcap, work, work_bytes, s);
}

// one application of the two-level cycle on a C128 vector (inner precision from p)
size_t vcycle_workspace_bytes(const CoarseGeom& c, const hdcr_solve_params* p) {
    Carver w(nullptr, 0);
    const size_t n = (size_t)12 * c.f.N5;
    if (p->inner_dtype != HDCR_C128) {
        w.take<float2>((size_t)36 * c.f.V4);
        w.take<float2>(n);
        w.take<float2>(n);
        cycle_carve<float>(w, c);
    } else {
        cycle_carve<double>(w, c);
    }
    return w.used();
}

int vcycle_apply(const CoarseGeom& c, const hdcr_solve_params* p, const double2* U, const void* basis, const void* A,
                 const hdcr_coarse_deflation* defl, const double2* r, double2* e, void* work, size_t work_bytes,
                 hipStream_t s) {
    Carver w(work, work_bytes);
    PhaseTimer tm;
    CycleCounts cnt;
    const int64_t n = 12LL * c.f.N5;
    if (p->inner_dtype != HDCR_C128) {
        float2* U32 = w.take<float2>((size_t)36 * c.f.V4);
        float2* r32 = w.take<float2>(n);
        float2* e32 = w.take<float2>(n);
        CycleWork<float> cw = cycle_carve<float>(w, c);
        if (!w.ok()) return fail(HDCR_ENOMEM, "hdcr_vcycle: workspace too small");
        HDCR_HIP_CHECK(hipMemsetAsync(cw.ccr.flags, 0, CCR_FLAGS * sizeof(int), s));
        launch_convert<double2, float2>(36LL * c.f.V4, U, U32, s);
        launch_convert<double2, float2>(n, r, r32, s);
        const DeflView<float> dv = defl ? defl_view<float>(defl) : DeflView<float>{};
        int st = vcycle<float>(c, p, U32, basis32(c, basis), p->basis_dtype == HDCR_F16C ? basis16(c, basis) : nullptr,
                               A, defl ? &dv : nullptr, r32, e32, cw, tm, cnt, s);
        if (st) return st;
        launch_convert<float2, double2>(n, e32, e, s);
    } else {
        CycleWork<double> cw = cycle_carve<double>(w, c);
        if (!w.ok()) return fail(HDCR_ENOMEM, "hdcr_vcycle: workspace too small");
        HDCR_HIP_CHECK(hipMemsetAsync(cw.ccr.flags, 0, CCR_FLAGS * sizeof(int), s));
        const DeflView<double> dv = defl ? defl_view<double>(defl) : DeflView<double>{};
        int st = vcycle<double>(c, p, U, basis64(basis), nullptr, A, defl ? &dv : nullptr, r, e, cw, tm, cnt, s);
        if (st) return st;
    }
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}

// ---------------------------------------------------------------------------
// subspace generation: Chebyshev low-pass filter of Gaussian noise (Sec. 4)
// ---------------------------------------------------------------------------
// T_d(yhat) eta with yhat = (2 H^2 - hi - lo)/(hi - lo) for d = degree; emit(buf, j)
// is called with the buffer holding T_j eta (times a positive constant) for
// every j <= degree, after step j.  The pair (t0, t1) is rescaled every 16
// steps (the recurrence is linear) so FP32 cannot overflow.  Returns the buffer
// (one of t0, t1) that holds the result.
template <typename T, typename Emit>
C2<T>* cheb_filter(const FineGeom& g, const C2<T>* U, int degree, double lo, double hi, C2<T>* t0, C2<T>* t1,
                   C2<T>* v, C2<T>* wv, double* part, double* S, hipStream_t s, Emit emit) {
    const int64_t n = 12LL * g.N5;
    emit(t0, 0);
    if (degree == 0) return t0;
    const double a1 = 2.0 / (hi - lo), b1 = -(hi + lo) / (hi - lo);
    // the combinations ride in the epilogue of the second stencil pass
    launch_dslash<T>(g, U, t0, v, s);
    launch_dslash_epi<T>(g, U, v, wv, Epi<T>{{t0, nullptr, nullptr, nullptr}, {(T)b1, 0, 0, 0}, (T)a1, 1}, s);
    std::swap(t1, wv);                              // t1 = T_1 = yhat t0
    emit(t1, 1);
    const double a2 = 4.0 / (hi - lo), b2 = -2.0 * (hi + lo) / (hi - lo);
    for (int j = 2; j <= degree; ++j) {
        // t0 <- 2 yhat t1 - t0 = a2 H (H t1) + b2 t1 - t0 (in place)
        launch_dslash<T>(g, U, t1, v, s);
        launch_dslash_epi<T>(g, U, v, t0, Epi<T>{{t1, t0, nullptr, nullptr}, {(T)b2, (T)-1, 0, 0}, (T)a2, 2}, s);
        std::swap(t0, t1);
        if (j % 16 == 0) {
            launch_norm2<T>(n, t1, part, S, 0, s);
            launch_scale_inv_sqrt<T>(n, t0, S, 0, s);
            launch_scale_inv_sqrt<T>(n, t1, S, 0, s);
        }
        emit(t1, j);
    }
    return t1;
}

// Filters nnoise noise fields and writes the normalised T_d eta for each degree
// d in degrees (ascending) to out[k * ndeg + q] (FP64); the arithmetic of the
// recurrence is T's.
template <typename T>
int make_subspace_degrees(const FineGeom& g, const double2* U, const double2* noise, int nnoise, const int* degrees,
                          int ndeg, double lo, double hi, double2* out, void* work, size_t work_bytes, hipStream_t s) {
    const int64_t n = 12LL * g.N5;
    Carver w(work, work_bytes);
    const C2<T>* Uin;
    if constexpr (sizeof(T) == 4) {
        float2* U32 = w.take<float2>((size_t)36 * g.V4);
        launch_convert<double2, float2>(36LL * g.V4, U, U32, s);
        Uin = U32;
    } else {
        Uin = U;
    }
    C2<T>* b[4];
    for (int i = 0; i < 4; ++i) b[i] = w.take<C2<T>>(n);
    double* part = w.take<double>(REDUCE_BLOCKS * (2 * MAXV + 1));
    double* S = w.take<double>(64);
    if (!w.ok()) return fail(HDCR_ENOMEM, "hdcr_make_subspace: workspace too small");
    for (int k = 0; k < nnoise; ++k) {
        launch_convert<double2, C2<T>>(n, noise + k * n, b[0], s);
        int q = 0;
        double2* dst = out + (size_t)k * ndeg * n;
        cheb_filter<T>(g, Uin, degrees[ndeg - 1], lo, hi, b[0], b[1], b[2], b[3], part, S, s,
                       [&](const C2<T>* t, int j) {
                           if (q < ndeg && degrees[q] == j) {
                               // a normalised FP64 copy; the recurrence keeps its own scale
                               launch_convert<C2<T>, double2>(n, t, dst + (size_t)q * n, s);
                               launch_norm2<double>(n, dst + (size_t)q * n, part, S, 1, s);
                               launch_scale_inv_sqrt<double>(n, dst + (size_t)q * n, S, 1, s);
                               ++q;
                           }
                       });
    }
    return HDCR_OK;
}

// The same with FP16 storage of the recurrence's fields (Ls = 16, even extents):
// the noise is scaled to unit RMS per entry before rounding, and the pair (t0,
// t1) is brought back to unit RMS every 16 steps (the recurrence is linear and
// the outputs are normalised), so the FP16 range holds the growth of the low
// modes.  Each step: two FP16 stencil passes and one element-wise combination.
int make_subspace_degrees_h16(const FineGeom& g, const double2* U, const double2* noise, int nnoise,
                              const int* degrees, int ndeg, double lo, double hi, double2* out, void* work,
                              size_t work_bytes, hipStream_t s) {
    const int64_t n = 12LL * g.N5;
    Carver w(work, work_bytes);
    float2* U32 = w.take<float2>((size_t)36 * g.V4);
    float2* f32 = w.take<float2>(n);
    void* h[4];
    for (int i = 0; i < 4; ++i) h[i] = w.take<uint32_t>(n);
    double* part = w.take<double>(REDUCE_BLOCKS * (2 * MAXV + 1));
    double* S = w.take<double>(64);
    if (!w.ok()) return fail(HDCR_ENOMEM, "hdcr_make_subspace: workspace too small");
    launch_convert<double2, float2>(36LL * g.V4, U, U32, s);
    const double a1 = 2.0 / (hi - lo), b1 = -(hi + lo) / (hi - lo);
    const double a2 = 4.0 / (hi - lo), b2 = -2.0 * (hi + lo) / (hi - lo);
    const int degree = degrees[ndeg - 1];
    for (int k = 0; k < nnoise; ++k) {
        launch_convert<double2, float2>(n, noise + k * n, f32, s);
        launch_norm2<float>(n, f32, part, S, 0, s);
        void *t0 = h[0], *t1 = h[1], *v = h[2], *wv = h[3];
        launch_to_h16_scaled(n, f32, S, 0, t0, s);
        int q = 0;
        double2* dst = out + (size_t)k * ndeg * n;
        auto emit = [&](const void* t, int j) {
            if (q < ndeg && degrees[q] == j) {
                launch_h16_to_c128(n, t, dst + (size_t)q * n, s);
                launch_norm2<double>(n, dst + (size_t)q * n, part, S, 1, s);
                launch_scale_inv_sqrt<double>(n, dst + (size_t)q * n, S, 1, s);
                ++q;
            }
        };
        emit(t0, 0);
        if (degree == 0) continue;
        // the second pass of each step carries the combination in its epilogue
        // (variant 6: a plain pass, then an element-wise combination)
        auto second = [&](const void* src, void* dst, float beta, int ny, const void* y0, float g0, const void* y1,
                          float g1) {
            if (g.variant != 6) {
                const Epi<float> e{{static_cast<const float2*>(y0), static_cast<const float2*>(y1), nullptr, nullptr},
                                   {g0, g1, 0.0f, 0.0f}, beta, ny};
                launch_dslash_h16_epi(g, U32, src, dst, e, s);
                return;
            }
            launch_dslash_h16(g, U32, src, wv, s);
            const void* z[4] = {y0, y1, nullptr, nullptr};
            const float gz[4] = {g0, g1, 0, 0};
            launch_h16_combine(n, beta, wv, z, gz, ny, dst, s);
        };
        // t1 = yhat t0 = a1 H (H t0) + b1 t0
        launch_dslash_h16(g, U32, t0, v, s);
        second(v, t1, (float)a1, 1, t0, (float)b1, nullptr, 0.0f);
        emit(t1, 1);
        for (int j = 2; j <= degree; ++j) {
            // t0 <- 2 yhat t1 - t0 = a2 H (H t1) + b2 t1 - t0 (in place)
            launch_dslash_h16(g, U32, t1, v, s);
            second(v, t0, (float)a2, 2, t1, (float)b2, t0, -1.0f);
            std::swap(t0, t1);
            if (j % 16 == 0) {
                launch_h16_norm2(n, t1, part, S, 0, s);
                launch_h16_scale_rms(n, t0, S, 0, s);
                launch_h16_scale_rms(n, t1, S, 0, s);
            }
            emit(t1, j);
        }
    }
    return HDCR_OK;
}

}  // namespace hdcr

using namespace hdcr;

extern "C" {

int hdcr_smooth(const hdcr_fine_desc* desc, hdcr_dtype dtype, const void* U, int32_t order, double lo, double hi,
                const void* in, void* out, void* work, size_t work_bytes, hipStream_t stream) {
    int e = check_fine_desc(desc);
    if (e) return e;
    if (dtype != HDCR_C128 && dtype != HDCR_C64 && dtype != HDCR_F16C)
        return fail(HDCR_EINVAL, "hdcr_smooth: dtype C128, C64 or F16C");
    if (order < 1 || order > 1000 || !(lo > 0) || !(hi > lo)) return fail(HDCR_EINVAL, "hdcr_smooth: bad polynomial");
    const size_t cs = dtype == HDCR_C128 ? 16 : 8;  // F16C: U, in and out are C64
    if ((e = check_ptr(U, cs, "U")) || (e = check_ptr(in, cs, "in")) || (e = check_ptr(out, cs, "out")) ||
        (e = check_ptr(work, 256, "work")))
        return e;
    const FineGeom g = make_geom(desc);
    const size_t n = (size_t)12 * g.N5;
    if (work_bytes < 4 * n * cs + 4 * 256) return fail(HDCR_ENOMEM, "hdcr_smooth: workspace too small");
    Carver w(work, work_bytes);
    if (dtype == HDCR_F16C) {
        if (!dslash_h16_ok(g)) return fail(HDCR_EINVAL, "hdcr_smooth: F16C needs Ls = 16 and even extents");
        if (order < 2) return fail(HDCR_EINVAL, "hdcr_smooth: F16C needs order >= 2");
        if (overlap(in, n * cs, out, n * cs)) return fail(HDCR_EINVAL, "hdcr_smooth: in and out overlap");
        void* h[6];
        for (int i = 0; i < 6; ++i) h[i] = w.take<uint32_t>(n);
        double* part = w.take<double>(REDUCE_BLOCKS);
        double* S = w.take<double>(8);
        if (!w.ok()) return fail(HDCR_ENOMEM, "hdcr_smooth: workspace too small");
        cheb_smoother_h16(g, (const float2*)U, (const float2*)in, (float2*)out, false, h, part, S, order, lo, hi,
                          stream);
    } else if (dtype == HDCR_C128) {
        double2* tmp[4];
        for (int i = 0; i < 4; ++i) tmp[i] = w.take<double2>(n);
        cheb_smoother<double>(g, (const double2*)U, (const double2*)in, (double2*)out, false, tmp, order, lo, hi, stream);
    } else {
        float2* tmp[4];
        for (int i = 0; i < 4; ++i) tmp[i] = w.take<float2>(n);
        cheb_smoother<float>(g, (const float2*)U, (const float2*)in, (float2*)out, false, tmp, order, lo, hi, stream);
    }
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}

int hdcr_vcycle(const hdcr_coarse_desc* desc, const hdcr_solve_params* params, const void* U, const void* basis,
                const void* A, const hdcr_coarse_deflation* defl, const void* r, void* e, void* work,
                size_t work_bytes, hipStream_t stream) {
    int st = check_coarse_desc(desc);
    if (st) return st;
    if (!params) return fail(HDCR_EINVAL, "hdcr_vcycle: null params");
    if ((st = check_two_level_params(params))) return st;
    if ((st = check_ptr(U, 16, "U")) || (st = check_ptr(basis, 16, "basis")) || (st = check_ptr(A, 4, "A")) ||
        (st = check_ptr(r, 16, "r")) || (st = check_ptr(e, 16, "e")) || (st = check_ptr(work, 256, "work")))
        return st;
    const CoarseGeom c = make_coarse_geom(desc);
    if (params->inner_dtype == HDCR_F16C && !dslash_h16_ok(c.f))
        return fail(HDCR_EINVAL, "hdcr_vcycle: inner F16C needs Ls = 16 and even extents");
    if (defl && (st = check_deflation(c, defl, params->inner_dtype == HDCR_C128 ? HDCR_C128 : HDCR_C64,
                                      "hdcr_vcycle")))
        return st;
    if (work_bytes < vcycle_workspace_bytes(c, params)) return fail(HDCR_ENOMEM, "hdcr_vcycle: workspace too small");
    return vcycle_apply(c, params, (const double2*)U, basis, A, defl, (const double2*)r, (double2*)e, work,
                        work_bytes, stream);
}

size_t hdcr_subspace_workspace_bytes(const hdcr_fine_desc* desc, hdcr_dtype dtype) {
    if (check_fine_desc(desc)) return 0;
    const FineGeom g = make_geom(desc);
    Carver w(nullptr, 0);
    const size_t n = (size_t)12 * g.N5;
    if (dtype == HDCR_C64) {
        w.take<float2>((size_t)36 * g.V4);
        for (int i = 0; i < 4; ++i) w.take<float2>(n);
    } else if (dtype == HDCR_F16C) {
        w.take<float2>((size_t)36 * g.V4);
        w.take<float2>(n);
        for (int i = 0; i < 4; ++i) w.take<uint32_t>(n);
    } else {
        for (int i = 0; i < 4; ++i) w.take<double2>(n);
    }
    w.take<double>(REDUCE_BLOCKS * (2 * MAXV + 1));
    w.take<double>(64);
    return w.used();
}

int hdcr_make_subspace(const hdcr_fine_desc* desc, hdcr_dtype dtype, int32_t nvec, int32_t degree, double lo,
                       double hi, const void* U, const void* noise, void* vecs, void* work, size_t work_bytes,
                       hipStream_t stream) {
    int e = check_fine_desc(desc);
    if (e) return e;
    if (dtype != HDCR_C128 && dtype != HDCR_C64 && dtype != HDCR_F16C)
        return fail(HDCR_EINVAL, "hdcr_make_subspace: dtype C128, C64 or F16C");
    if (nvec < 1 || degree < 0 || degree > 100000 || !(hi > lo)) return fail(HDCR_EINVAL, "hdcr_make_subspace: bad args");
    if ((e = check_ptr(U, 16, "U")) || (e = check_ptr(noise, 16, "noise")) || (e = check_ptr(vecs, 16, "vecs")) ||
        (e = check_ptr(work, 256, "work")))
        return e;
    const FineGeom g = make_geom(desc);
    if (work_bytes < hdcr_subspace_workspace_bytes(desc, dtype))
        return fail(HDCR_ENOMEM, "hdcr_make_subspace: workspace too small");
    const int64_t n = 12LL * g.N5;
    Carver w(work, work_bytes);
    const double2* nz = static_cast<const double2*>(noise);
    double2* out = static_cast<double2*>(vecs);
    if (dtype == HDCR_F16C) {
        if (!dslash_h16_ok(g)) return fail(HDCR_EINVAL, "hdcr_make_subspace: F16C needs Ls = 16 and even extents");
        if ((e = make_subspace_degrees_h16(g, (const double2*)U, nz, nvec, &degree, 1, lo, hi, out, work, work_bytes,
                                           stream)))
            return e;
    } else if (dtype == HDCR_C64) {
        float2* U32 = w.take<float2>((size_t)36 * g.V4);
        float2* b[4];
        for (int i = 0; i < 4; ++i) b[i] = w.take<float2>(n);
        double* part = w.take<double>(REDUCE_BLOCKS * (2 * MAXV + 1));
        double* S = w.take<double>(64);
        launch_convert<double2, float2>(36LL * g.V4, (const double2*)U, U32, stream);
        for (int k = 0; k < nvec; ++k) {
            launch_convert<double2, float2>(n, nz + k * n, b[0], stream);
            float2* res = cheb_filter<float>(g, U32, degree, lo, hi, b[0], b[1], b[2], b[3], part, S, stream,
                                             [](const float2*, int) {});
            launch_norm2<float>(n, res, part, S, 1, stream);
            launch_scale_inv_sqrt<float>(n, res, S, 1, stream);
            launch_convert<float2, double2>(n, res, out + k * n, stream);
        }
    } else {
        double2* b[4];
        for (int i = 0; i < 4; ++i) b[i] = w.take<double2>(n);
        double* part = w.take<double>(REDUCE_BLOCKS * (2 * MAXV + 1));
        double* S = w.take<double>(64);
        for (int k = 0; k < nvec; ++k) {
            launch_convert<double2, double2>(n, nz + k * n, b[0], stream);
            double2* res = cheb_filter<double>(g, (const double2*)U, degree, lo, hi, b[0], b[1], b[2], b[3], part, S,
                                               stream, [](const double2*, int) {});
            launch_norm2<double>(n, res, part, S, 1, stream);
            launch_scale_inv_sqrt<double>(n, res, S, 1, stream);
            launch_convert<double2, double2>(n, res, out + k * n, stream);
        }
    }
    HDCR_HIP_CHECK(hipGetLastError());
    HDCR_HIP_CHECK(hipStreamSynchronize(stream));
    return HDCR_OK;
}

int hdcr_make_subspace_degrees(const hdcr_fine_desc* desc, hdcr_dtype dtype, int32_t nnoise, int32_t ndeg,
                               const int32_t* degrees, double lo, double hi, const void* U, const void* noise, void* vecs,
                               void* work, size_t work_bytes, hipStream_t stream) {
    int e = check_fine_desc(desc);
    if (e) return e;
    if (dtype != HDCR_C128 && dtype != HDCR_C64 && dtype != HDCR_F16C)
        return fail(HDCR_EINVAL, "hdcr_make_subspace_degrees: dtype C128, C64 or F16C");
    if (nnoise < 1 || ndeg < 1 || !degrees || !(hi > lo))
        return fail(HDCR_EINVAL, "hdcr_make_subspace_degrees: bad args");
    for (int q = 0; q < ndeg; ++q)
        if (degrees[q] < 0 || degrees[q] > 100000 || (q > 0 && degrees[q] <= degrees[q - 1]))
            return fail(HDCR_EINVAL, "hdcr_make_subspace_degrees: degrees must be ascending, in [0, 100000]");
    if ((e = check_ptr(U, 16, "U")) || (e = check_ptr(noise, 16, "noise")) || (e = check_ptr(vecs, 16, "vecs")) ||
        (e = check_ptr(work, 256, "work")))
        return e;
    const FineGeom g = make_geom(desc);
    const size_t fbytes = (size_t)12 * g.N5 * 16;
    if (overlap(noise, fbytes * nnoise, vecs, fbytes * nnoise * ndeg))
        return fail(HDCR_EINVAL, "hdcr_make_subspace_degrees: noise and vecs overlap");
    if (work_bytes < hdcr_subspace_workspace_bytes(desc, dtype))
        return fail(HDCR_ENOMEM, "hdcr_make_subspace_degrees: workspace too small");
    if (dtype == HDCR_F16C && !dslash_h16_ok(g))
        return fail(HDCR_EINVAL, "hdcr_make_subspace_degrees: F16C needs Ls = 16 and even extents");
    const std::vector<int> deg(degrees, degrees + ndeg);
    if (dtype == HDCR_F16C)
        e = make_subspace_degrees_h16(g, (const double2*)U, (const double2*)noise, nnoise, deg.data(), ndeg, lo, hi,
                                      (double2*)vecs, work, work_bytes, stream);
    else if (dtype == HDCR_C64)
        e = make_subspace_degrees<float>(g, (const double2*)U, (const double2*)noise, nnoise, deg.data(), ndeg, lo, hi,
                                         (double2*)vecs, work, work_bytes, stream);
    else
        e = make_subspace_degrees<double>(g, (const double2*)U, (const double2*)noise, nnoise, deg.data(), ndeg, lo,
                                          hi, (double2*)vecs, work, work_bytes, stream);
    if (e) return e;
    HDCR_HIP_CHECK(hipGetLastError());
    HDCR_HIP_CHECK(hipStreamSynchronize(stream));
    return HDCR_OK;
}

int hdcr_power_max(const hdcr_fine_desc* desc, const void* U, const void* v0, int32_t iters, double* lam, void* work,
                   size_t work_bytes, hipStream_t stream) {
    int e = check_fine_desc(desc);
    if (e) return e;
    if (iters < 1 || !lam) return fail(HDCR_EINVAL, "hdcr_power_max: iters >= 1 and lam required");
    if ((e = check_ptr(U, 16, "U")) || (e = check_ptr(v0, 16, "v0")) || (e = check_ptr(work, 256, "work"))) return e;
    const FineGeom g = make_geom(desc);
    const int64_t n = 12LL * g.N5;
    if (work_bytes < hdcr_subspace_workspace_bytes(desc, HDCR_C128))
        return fail(HDCR_ENOMEM, "hdcr_power_max: workspace too small");
    Carver w(work, work_bytes);
    double2* v = w.take<double2>(n);
    double2* t = w.take<double2>(n);
    double2* u = w.take<double2>(n);
    w.take<double2>(n);
    double* part = w.take<double>(REDUCE_BLOCKS * (2 * MAXV + 1));
    double* S = w.take<double>(64);
    const double2* Ud = static_cast<const double2*>(U);
    // v = v0/|v0|; repeat: u = H^2 v, lambda = <v, u>, v = u/|u|
    launch_convert<double2, double2>(n, static_cast<const double2*>(v0), v, stream);
    launch_norm2<double>(n, v, part, S, 0, stream);
    launch_scale_inv_sqrt<double>(n, v, S, 0, stream);
    PtrList Vl{};
    for (int i = 0; i < iters; ++i) {
        launch_dslash<double>(g, Ud, v, t, stream);
        launch_dslash<double>(g, Ud, t, u, stream);
        Vl.p[0] = v;
        launch_multidot<double, double>(n, Vl, 1, u, part, S + 8, stream);  // S[8] = Re<v,u>, S[8+2*MAXV] = |u|^2
        launch_scale_inv_sqrt<double>(n, u, S, 8 + 2 * MAXV, stream);
        std::swap(v, u);
    }
    double h = 0.0;
    HDCR_HIP_CHECK(hipMemcpyAsync(&h, S + 8, sizeof(double), hipMemcpyDeviceToHost, stream));
    HDCR_HIP_CHECK(hipStreamSynchronize(stream));
    *lam = h;
    return HDCR_OK;
}

}  // extern "C"
