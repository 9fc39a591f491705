// Fine operator H = Gamma5 D_dwf (Sec. 3) for gfx950.
//
// One work-item per 5d site (x, s), s fastest, so a 64-wide wavefront covers
// 64/Ls consecutive 4d sites times all of Ls: every component load of the
// site-major SoA field psi[c][site4][s] is one contiguous run, the SU(3) link
// of a 4d site is shared (and cached) by the Ls lanes that use it, and the
// fifth-dimension neighbours come from the same cache lines as the site itself.
//
// All loads and stores go through buffer descriptors: the per-lane part of an
// address is one 32-bit byte offset per neighbouring site, and the component
// (or link element) offset is a uniform scalar, so the ~100 loads of a site
// cost one vector register of addressing per neighbour.
//
// The 4d hops use the chiral-basis spin projection: with psi = (u, d) (upper and
// lower spin pairs) and g_mu = [[0, w_mu], [w_mu^dag, 0]] (w_k = -i sigma_k,
// w_t = 1),
//   (1 - g_mu) psi = (h, -w_mu^dag h),  h = u - w_mu d,
//   (1 + g_mu) psi = (h, +w_mu^dag h),  h = u + w_mu d,
// so each hop multiplies a half spinor (2 spins x 3 colours) by the link.
// The output is written at (x, Ls-1-s) with the lower spins negated:
// H = gamma5 R5 D.
#include "internal.h"

namespace hdcr {

namespace {

struct FieldRefs {
    __amdgpu_buffer_rsrc_t in, U, out;
    uint32_t cstride;  // bytes between field components (N5 complex)
    uint32_t lstride;  // bytes between link elements (V4 complex)
};

// H[r] = sum_c U[r][c] h[c]  (DAG = false)   or   sum_c conj(U[c][r]) h[c]  (DAG = true)
// for the link of direction MU at 4d site `lsite`
template <typename T, int MU, bool DAG>
__device__ __forceinline__ void su3_mul(const FieldRefs& f, uint32_t loff, const C2<T> (&h)[3], C2<T> (&o)[3]) {
    C2<T> u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = Buf<T>::ld(f.U, loff, (uint32_t)(MU * 9 + e) * f.lstride);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        C2<T> acc = mk<T>(0, 0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (DAG)
                acc = cjfma<T>(u[c * 3 + r], h[c], acc);
            else
                acc = cfma<T>(u[r * 3 + c], h[c], acc);
        }
        o[r] = acc;
    }
}

// One hop in direction MU (0..3 = x, y, z, t), forward (FWD) or backward:
// psi at the neighbouring 5d site (byte offset noff), link at byte offset
// loff, scaled by coef (= -1/2 times the boundary sign), added into acc.
template <typename T, int MU, bool FWD>
__device__ __forceinline__ void hop(const FieldRefs& f, uint32_t noff, uint32_t loff, T coef, C2<T> (&acc)[12]) {
    C2<T> h0[3], h1[3];
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        const C2<T> u0 = Buf<T>::ld(f.in, noff, (uint32_t)(0 * 3 + col) * f.cstride);
        const C2<T> u1 = Buf<T>::ld(f.in, noff, (uint32_t)(1 * 3 + col) * f.cstride);
        const C2<T> d0 = Buf<T>::ld(f.in, noff, (uint32_t)(2 * 3 + col) * f.cstride);
        const C2<T> d1 = Buf<T>::ld(f.in, noff, (uint32_t)(3 * 3 + col) * f.cstride);
        // h = u -+ w_mu d  (minus for the forward hop (1 - g), plus for backward (1 + g))
        if (MU == 0) {        // w_x d = (-i d1, -i d0)
            h0[col] = FWD ? cadd<T>(u0, cmuli<T>(d1)) : csub<T>(u0, cmuli<T>(d1));
            h1[col] = FWD ? cadd<T>(u1, cmuli<T>(d0)) : csub<T>(u1, cmuli<T>(d0));
        } else if (MU == 1) { // w_y d = (-d1, d0)
            h0[col] = FWD ? cadd<T>(u0, d1) : csub<T>(u0, d1);
            h1[col] = FWD ? csub<T>(u1, d0) : cadd<T>(u1, d0);
        } else if (MU == 2) { // w_z d = (-i d0, i d1)
            h0[col] = FWD ? cadd<T>(u0, cmuli<T>(d0)) : csub<T>(u0, cmuli<T>(d0));
            h1[col] = FWD ? csub<T>(u1, cmuli<T>(d1)) : cadd<T>(u1, cmuli<T>(d1));
        } else {              // w_t d = (d0, d1)
            h0[col] = FWD ? csub<T>(u0, d0) : cadd<T>(u0, d0);
            h1[col] = FWD ? csub<T>(u1, d1) : cadd<T>(u1, d1);
        }
        h0[col] = cscale<T>(coef, h0[col]);
        h1[col] = cscale<T>(coef, h1[col]);
    }
    C2<T> H0[3], H1[3];
    su3_mul<T, MU, !FWD>(f, loff, h0, H0);
    su3_mul<T, MU, !FWD>(f, loff, h1, H1);
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        acc[0 * 3 + col] = cadd<T>(acc[0 * 3 + col], H0[col]);
        acc[1 * 3 + col] = cadd<T>(acc[1 * 3 + col], H1[col]);
        // lower spins: -w^dag H (forward) or +w^dag H (backward)
        C2<T> l0, l1;
        if (MU == 0) {        // w_x^dag H = (i H1, i H0)
            l0 = cmuli<T>(H1[col]);
            l1 = cmuli<T>(H0[col]);
        } else if (MU == 1) { // w_y^dag H = (H1, -H0)
            l0 = H1[col];
            l1 = cneg<T>(H0[col]);
        } else if (MU == 2) { // w_z^dag H = (i H0, -i H1)
            l0 = cmuli<T>(H0[col]);
            l1 = cmulmi<T>(H1[col]);
        } else {              // w_t^dag H = (H0, H1)
            l0 = H0[col];
            l1 = H1[col];
        }
        if (FWD) {
            acc[2 * 3 + col] = csub<T>(acc[2 * 3 + col], l0);
            acc[3 * 3 + col] = csub<T>(acc[3 * 3 + col], l1);
        } else {
            acc[2 * 3 + col] = cadd<T>(acc[2 * 3 + col], l0);
            acc[3 * 3 + col] = cadd<T>(acc[3 * 3 + col], l1);
        }
    }
}

template <typename T, int MU>
__device__ __forceinline__ void hop_pair(const FineGeom& g, const FieldRefs& f, int site, int s, int xmu,
                                         C2<T> (&acc)[12]) {
    constexpr uint32_t CB = sizeof(C2<T>);
    // branch-free neighbour indices: the wrap-around is a select between uniform steps
    const bool wrap_f = (xmu == g.L[MU] - 1);
    const bool wrap_b = (xmu == 0);
    const int sf = site + (wrap_f ? -g.wrap[MU] : g.stride[MU]);
    const int sb = site + (wrap_b ? g.wrap[MU] : -g.stride[MU]);
    const T half = (T)(-0.5);
    const T cf = wrap_f ? half * (T)g.bc[MU] : half;
    const T cb = wrap_b ? half * (T)g.bc[MU] : half;
    // forward: -1/2 (1 - g_mu) U_mu(x) psi(x + mu)
    hop<T, MU, true>(f, (uint32_t)(sf * g.Ls + s) * CB, (uint32_t)site * CB, cf, acc);
    // backward: -1/2 (1 + g_mu) U_mu(x - mu)^dag psi(x - mu)
    hop<T, MU, false>(f, (uint32_t)(sb * g.Ls + s) * CB, (uint32_t)sb * CB, cb, acc);
}

template <typename T>
__global__ void __launch_bounds__(256) dslash_dwf_kernel(FineGeom g, const C2<T>* U, const C2<T>* in, C2<T>* out) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= g.N5) return;
    constexpr uint32_t CB = sizeof(C2<T>);
    FieldRefs f;
    f.cstride = (uint32_t)g.N5 * CB;
    f.lstride = (uint32_t)g.V4 * CB;
    f.in = make_rsrc(in, 12u * f.cstride);
    f.out = make_rsrc(out, 12u * f.cstride);
    f.U = make_rsrc(U, 36u * f.lstride);

    const int Ls = g.Ls;
    const int s = gid % Ls;
    const int site = gid / Ls;
    int rem = site;
    const int x0 = rem % g.L[0];
    rem /= g.L[0];
    const int x1 = rem % g.L[1];
    rem /= g.L[1];
    const int x2 = rem % g.L[2];
    const int x3 = rem / g.L[2];

    C2<T> acc[12];
    // diagonal (5 - M5) and the fifth-dimension hops: -P+ psi(s-1) on the upper
    // spins, -P- psi(s+1) on the lower spins, +mf on the walls
    {
        const T diag = (T)g.diag;
        const T mf = (T)g.mf;
        const int sm = (s == 0) ? Ls - 1 : s - 1;
        const int sp = (s == Ls - 1) ? 0 : s + 1;
        const T cm = (s == 0) ? mf : (T)(-1);
        const T cp = (s == Ls - 1) ? mf : (T)(-1);
        const uint32_t o0 = (uint32_t)(site * Ls + s) * CB;
        const uint32_t om = (uint32_t)(site * Ls + sm) * CB;
        const uint32_t op = (uint32_t)(site * Ls + sp) * CB;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const C2<T> v = Buf<T>::ld(f.in, o0, (uint32_t)c * f.cstride);
            const C2<T> w = Buf<T>::ld(f.in, (c < 6) ? om : op, (uint32_t)c * f.cstride);
            const T cw = (c < 6) ? cm : cp;
            acc[c] = mk<T>(diag * v.x + cw * w.x, diag * v.y + cw * w.y);
        }
    }
    hop_pair<T, 0>(g, f, site, s, x0, acc);
    hop_pair<T, 1>(g, f, site, s, x1, acc);
    hop_pair<T, 2>(g, f, site, s, x2, acc);
    hop_pair<T, 3>(g, f, site, s, x3, acc);

    const uint32_t oo = (uint32_t)(site * Ls + (Ls - 1 - s)) * CB;
#pragma unroll
    for (int c = 0; c < 12; ++c) Buf<T>::st((c < 6) ? acc[c] : cneg<T>(acc[c]), f.out, oo, (uint32_t)c * f.cstride);
}

}  // namespace

template <typename T>
void launch_dslash(const FineGeom& g, const C2<T>* U, const C2<T>* in, C2<T>* out, hipStream_t s) {
    const int threads = 256;
    const int blocks = (g.N5 + threads - 1) / threads;
    hipLaunchKernelGGL(dslash_dwf_kernel<T>, dim3(blocks), dim3(threads), 0, s, g, U, in, out);
}

template void launch_dslash<double>(const FineGeom&, const double2*, const double2*, double2*, hipStream_t);
template void launch_dslash<float>(const FineGeom&, const float2*, const float2*, float2*, hipStream_t);

}  // namespace hdcr
