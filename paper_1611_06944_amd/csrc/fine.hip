// Fine operator H = Gamma5 D_dwf (Sec. 3) for gfx950.
//
// Work-items own SPT consecutive fifth-dimension coordinates of one 4d site,
// s fastest, so a 64-wide wavefront covers a few consecutive 4d sites times
// all of Ls: every component load of the site-major SoA field psi[c][site4][s]
// is one contiguous run (SPT = 2 turns the FP32 loads into 16-byte ones), and
// the fifth-dimension neighbours come from the same cache lines as the site.
//
// The SU(3) links of the sites a workgroup touches (forward links at the site,
// backward links at the site minus mu) are staged once into LDS, so the Ls
// work-items sharing a link read it from LDS instead of issuing their own
// vector-memory loads.
//
// Field loads and stores go through buffer descriptors: the per-lane part of an
// address is one 32-bit byte offset per neighbouring site, the component offset
// is a uniform scalar.
//
// Workgroups are remapped so that each XCD sweeps one contiguous range of a
// traversal order (x, y-part, t-in-slab, z, y-split, t-slab) in which the z and
// t neighbours of a site are a few rows apart: they are re-read from the XCD's
// own L2 instead of another XCD's.
//
// The 4d hops use the chiral-basis spin projection: with psi = (u, d) (upper and
// lower spin pairs) and g_mu = [[0, w_mu], [w_mu^dag, 0]] (w_k = -i sigma_k,
// w_t = 1),
//   (1 - g_mu) psi = (h, -w_mu^dag h),  h = u - w_mu d,
//   (1 + g_mu) psi = (h, +w_mu^dag h),  h = u + w_mu d,
// so each hop multiplies a half spinor (2 spins x 3 colours) by the link.
// The output is written at (x, Ls-1-s) with the lower spins negated:
// H = gamma5 R5 D.
#include "coarse.h"

namespace hdcr {

namespace {

constexpr int WG = 256;
constexpr int MIN_SLOTS = 8;                 // work-items per site required by the LDS-link variant
constexpr int MAX_WG_SITES = WG / MIN_SLOTS + 1;
constexpr int LINK_STRIDE = 8 * 9 + 1;       // complex entries per staged site (padded against bank conflicts)

// Hop-class selection used by the little-Dirac-operator build: cls = -1 keeps
// every term; cls = 0 keeps the diagonal, the fifth-dimension hops and the 4d
// hops that stay inside a block of extent B; cls = 1+mu (5+mu) keeps only the
// forward (backward) mu hops that cross the block face.
struct ClassSel {
    int B[4];
    int cls;
};

struct FieldRefs {
    __amdgpu_buffer_rsrc_t in, U, out;
    uint32_t cstride;  // bytes between field components (N5 complex)
    uint32_t lstride;  // bytes between link elements (V4 complex)
};

// SPT consecutive complex entries of one component
template <typename T, int SPT> struct Vec;
template <typename T> struct Vec<T, 1> {
    static __device__ __forceinline__ void ld(const __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, C2<T> (&o)[1]) {
        o[0] = Buf<T>::ld(r, v, s);
    }
    static __device__ __forceinline__ void st(const C2<T> (&a)[1], __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
        Buf<T>::st(a[0], r, v, s);
    }
};
template <> struct Vec<float, 2> {
    typedef __attribute__((ext_vector_type(4))) unsigned u4;
    static __device__ __forceinline__ void ld(const __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, float2 (&o)[2]) {
        const float4 q = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, v, s, 0));
        o[0] = make_float2(q.x, q.y);
        o[1] = make_float2(q.z, q.w);
    }
    static __device__ __forceinline__ void st(const float2 (&a)[2], __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
        const float4 q = make_float4(a[0].x, a[0].y, a[1].x, a[1].y);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, q), r, v, s, 0);
    }
};
template <> struct Vec<double, 2> {
    static __device__ __forceinline__ void ld(const __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, double2 (&o)[2]) {
        o[0] = Buf<double>::ld(r, v, s);
        o[1] = Buf<double>::ld(r, v + 16, s);
    }
    static __device__ __forceinline__ void st(const double2 (&a)[2], __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
        Buf<double>::st(a[0], r, v, s);
        Buf<double>::st(a[1], r, v + 16, s);
    }
};

// H[r] = sum_c U[r][c] h[c]  (DAG = false)   or   sum_c conj(U[c][r]) h[c]  (DAG = true)
template <typename T, bool DAG>
__device__ __forceinline__ void su3_mul(const C2<T> (&u)[9], const C2<T> (&h)[3], C2<T> (&o)[3]) {
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

// One hop in direction MU (0..3 = x, y, z, t), forward (FWD) or backward, for
// the SPT fifth-dimension slots of a work-item: psi at the neighbouring site
// (byte offset noff of its first slot), link u, scaled by coef (-1/2 times the
// boundary sign), added into acc.
template <typename T, int SPT, int MU, bool FWD>
__device__ __forceinline__ void hop(const FieldRefs& f, uint32_t noff, const C2<T> (&u)[9], T coef,
                                    C2<T> (&acc)[SPT][12]) {
    C2<T> h0[SPT][3], h1[SPT][3];
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        C2<T> u0[SPT], u1[SPT], d0[SPT], d1[SPT];
        Vec<T, SPT>::ld(f.in, noff, (uint32_t)(0 * 3 + col) * f.cstride, u0);
        Vec<T, SPT>::ld(f.in, noff, (uint32_t)(1 * 3 + col) * f.cstride, u1);
        Vec<T, SPT>::ld(f.in, noff, (uint32_t)(2 * 3 + col) * f.cstride, d0);
        Vec<T, SPT>::ld(f.in, noff, (uint32_t)(3 * 3 + col) * f.cstride, d1);
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            // h = u -+ w_mu d  (minus for the forward hop (1 - g), plus for backward (1 + g))
            C2<T> a, b;
            if (MU == 0) {        // w_x d = (-i d1, -i d0)
                a = FWD ? cadd<T>(u0[k], cmuli<T>(d1[k])) : csub<T>(u0[k], cmuli<T>(d1[k]));
                b = FWD ? cadd<T>(u1[k], cmuli<T>(d0[k])) : csub<T>(u1[k], cmuli<T>(d0[k]));
            } else if (MU == 1) { // w_y d = (-d1, d0)
                a = FWD ? cadd<T>(u0[k], d1[k]) : csub<T>(u0[k], d1[k]);
                b = FWD ? csub<T>(u1[k], d0[k]) : cadd<T>(u1[k], d0[k]);
            } else if (MU == 2) { // w_z d = (-i d0, i d1)
                a = FWD ? cadd<T>(u0[k], cmuli<T>(d0[k])) : csub<T>(u0[k], cmuli<T>(d0[k]));
                b = FWD ? csub<T>(u1[k], cmuli<T>(d1[k])) : cadd<T>(u1[k], cmuli<T>(d1[k]));
            } else {              // w_t d = (d0, d1)
                a = FWD ? csub<T>(u0[k], d0[k]) : cadd<T>(u0[k], d0[k]);
                b = FWD ? csub<T>(u1[k], d1[k]) : cadd<T>(u1[k], d1[k]);
            }
            h0[k][col] = cscale<T>(coef, a);
            h1[k][col] = cscale<T>(coef, b);
        }
    }
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
        C2<T> H0[3], H1[3];
        su3_mul<T, !FWD>(u, h0[k], H0);
        su3_mul<T, !FWD>(u, h1[k], H1);
#pragma unroll
        for (int col = 0; col < 3; ++col) {
            acc[k][0 * 3 + col] = cadd<T>(acc[k][0 * 3 + col], H0[col]);
            acc[k][1 * 3 + col] = cadd<T>(acc[k][1 * 3 + col], H1[col]);
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
                acc[k][2 * 3 + col] = csub<T>(acc[k][2 * 3 + col], l0);
                acc[k][3 * 3 + col] = csub<T>(acc[k][3 * 3 + col], l1);
            } else {
                acc[k][2 * 3 + col] = cadd<T>(acc[k][2 * 3 + col], l0);
                acc[k][3 * 3 + col] = cadd<T>(acc[k][3 * 3 + col], l1);
            }
        }
    }
}

// Workgroup -> sites.  Hardware dispatch sends workgroup w to XCD w % 8; the
// remap gives each XCD one contiguous range of logical workgroups.
__device__ __forceinline__ int logical_block(int w, int nwg) {
    const int per = nwg / NUM_XCD, rem = nwg % NUM_XCD;
    const int xcd = w % NUM_XCD, local = w / NUM_XCD;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

struct Site {
    int site;  // lexicographic 4d site index
    int x[4];
};

// logical site l -> coordinates, traversal order x, y-part, t-in-slab, z, y-split, t-slab
__device__ __forceinline__ Site traverse(const FineGeom& g, int l) {
    Site tr;
    const int yq = g.L[1] / g.ysplit;
    tr.x[0] = l % g.L[0];
    l /= g.L[0];
    const int yi = l % yq;
    l /= yq;
    const int ti = l % g.tslab;
    l /= g.tslab;
    tr.x[2] = l % g.L[2];
    l /= g.L[2];
    const int yo = l % g.ysplit;
    l /= g.ysplit;
    tr.x[1] = yo * yq + yi;
    tr.x[3] = l * g.tslab + ti;
    tr.site = ((tr.x[3] * g.L[2] + tr.x[2]) * g.L[1] + tr.x[1]) * g.L[0] + tr.x[0];
    return tr;
}

template <typename T, int SPT, bool LDSL, bool CLS, int MU>
__device__ __forceinline__ void hop_pair(const FineGeom& g, const FieldRefs& f, const Site& st, int s0,
                                         const C2<T>* lnk, const ClassSel& cs, C2<T> (&acc)[SPT][12]) {
    constexpr uint32_t CB = sizeof(C2<T>);
    const int site = st.site;
    const int xmu = st.x[MU];
    // branch-free neighbour indices: the wrap-around is a select between uniform steps
    const bool wrap_f = (xmu == g.L[MU] - 1);
    const bool wrap_b = (xmu == 0);
    const int sf = site + (wrap_f ? -g.wrap[MU] : g.stride[MU]);
    const int sb = site + (wrap_b ? g.wrap[MU] : -g.stride[MU]);
    const T half = (T)(-0.5);
    T cf = wrap_f ? half * (T)g.bc[MU] : half;
    T cb = wrap_b ? half * (T)g.bc[MU] : half;
    if constexpr (CLS) {
        // keep a hop only if its class is the selected one
        const int lx = xmu % cs.B[MU];
        const bool cross_f = (lx == cs.B[MU] - 1), cross_b = (lx == 0);
        const bool keep_f = cross_f ? (cs.cls == 1 + MU) : (cs.cls == 0);
        const bool keep_b = cross_b ? (cs.cls == 5 + MU) : (cs.cls == 0);
        cf = keep_f ? cf : (T)0;
        cb = keep_b ? cb : (T)0;
    }
    C2<T> u[9];
    // forward: -1/2 (1 - g_mu) U_mu(x) psi(x + mu)
    if constexpr (LDSL) {
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = lnk[MU * 9 + e];
    } else {
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = Buf<T>::ld(f.U, (uint32_t)site * CB, (uint32_t)(MU * 9 + e) * f.lstride);
    }
    hop<T, SPT, MU, true>(f, (uint32_t)(sf * g.Ls + s0) * CB, u, cf, acc);
    // backward: -1/2 (1 + g_mu) U_mu(x - mu)^dag psi(x - mu)
    if constexpr (LDSL) {
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = lnk[(4 + MU) * 9 + e];
    } else {
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = Buf<T>::ld(f.U, (uint32_t)sb * CB, (uint32_t)(MU * 9 + e) * f.lstride);
    }
    hop<T, SPT, MU, false>(f, (uint32_t)(sb * g.Ls + s0) * CB, u, cb, acc);
}

// SPT: fifth-dimension slots per work-item; LDSL: links staged in LDS
// (requires Ls / SPT >= MIN_SLOTS).
template <typename T, int SPT, bool LDSL, bool CLS>
__global__ void __launch_bounds__(WG) dslash_dwf_kernel(FineGeom g, const C2<T>* U, const C2<T>* in, C2<T>* out,
                                                        ClassSel cs) {
    constexpr uint32_t CB = sizeof(C2<T>);
    const int lb = logical_block(blockIdx.x, gridDim.x);
    const int slots = g.Ls / SPT;  // work-items per 4d site
    const int gid = lb * WG + threadIdx.x;
    const bool active = gid < g.V4 * slots;
    FieldRefs f;
    f.cstride = (uint32_t)g.N5 * CB;
    f.lstride = (uint32_t)g.V4 * CB;
    f.in = make_rsrc(in, 12u * f.cstride);
    f.out = make_rsrc(out, 12u * f.cstride);
    f.U = make_rsrc(U, 36u * f.lstride);

    const int lsite = gid / slots;
    const int s0 = (gid % slots) * SPT;

    __shared__ C2<T> lds_links[LDSL ? MAX_WG_SITES * LINK_STRIDE : 1];
    const C2<T>* lnk = nullptr;
    if (LDSL) {
        // stage the forward links U_mu(x) and backward links U_mu(x - mu) of every site of the workgroup
        const int first = (lb * WG) / slots;
        const int last = min((lb * WG + WG - 1) / slots, g.V4 - 1);
        const int ns = last - first + 1;
        for (int e = threadIdx.x; e < ns * 72; e += WG) {
            const int sl = e / 72, r = e - sl * 72;
            const int d = r / 9, el = r - d * 9;
            const int mu = d & 3;
            const Site t = traverse(g, first + sl);
            const int src = (d < 4) ? t.site : ((t.x[mu] == 0) ? t.site + g.wrap[mu] : t.site - g.stride[mu]);
            lds_links[sl * LINK_STRIDE + r] = Buf<T>::ld(f.U, (uint32_t)src * CB, (uint32_t)(mu * 9 + el) * f.lstride);
        }
        __syncthreads();
        lnk = lds_links + (lsite - first) * LINK_STRIDE;
    }
    if (!active) return;
    const Site st = traverse(g, lsite);
    const int site = st.site;
    const int Ls = g.Ls;

    C2<T> acc[SPT][12];
    // diagonal (5 - M5) and the fifth-dimension hops: -P+ psi(s-1) on the upper
    // spins, -P- psi(s+1) on the lower spins, +mf on the walls
    {
        // the diagonal and fifth-dimension terms belong to hop class 0
        const T keep = (!CLS || cs.cls == 0) ? (T)1 : (T)0;
        const T diag = keep * (T)g.diag;
        const T mf = keep * (T)g.mf;
        const int sm = (s0 == 0) ? Ls - 1 : s0 - 1;           // below the first slot
        const int sp = (s0 + SPT == Ls) ? 0 : s0 + SPT;        // above the last slot
        const T cm = (s0 == 0) ? mf : -keep;
        const T cp = (s0 + SPT == Ls) ? mf : -keep;
        const uint32_t o0 = (uint32_t)(site * Ls + s0) * CB;
        const uint32_t om = (uint32_t)(site * Ls + sm) * CB;
        const uint32_t op = (uint32_t)(site * Ls + sp) * CB;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            C2<T> v[SPT];
            Vec<T, SPT>::ld(f.in, o0, (uint32_t)c * f.cstride, v);
            const C2<T> w = Buf<T>::ld(f.in, (c < 6) ? om : op, (uint32_t)c * f.cstride);
#pragma unroll
            for (int k = 0; k < SPT; ++k) {
                // neighbour in s: upper spins take s-1, lower spins s+1
                C2<T> nb;
                T cw;
                if (c < 6) {
                    nb = (k == 0) ? w : v[k > 0 ? k - 1 : 0];
                    cw = (k == 0) ? cm : -keep;
                } else {
                    nb = (k == SPT - 1) ? w : v[k + 1 < SPT ? k + 1 : k];
                    cw = (k == SPT - 1) ? cp : -keep;
                }
                acc[k][c] = mk<T>(diag * v[k].x + cw * nb.x, diag * v[k].y + cw * nb.y);
            }
        }
    }
    hop_pair<T, SPT, LDSL, CLS, 0>(g, f, st, s0, lnk, cs, acc);
    hop_pair<T, SPT, LDSL, CLS, 1>(g, f, st, s0, lnk, cs, acc);
    hop_pair<T, SPT, LDSL, CLS, 2>(g, f, st, s0, lnk, cs, acc);
    hop_pair<T, SPT, LDSL, CLS, 3>(g, f, st, s0, lnk, cs, acc);

    // slot k (s = s0 + k) goes to s' = Ls - 1 - s0 - k: the SPT outputs are
    // consecutive, in reverse order, starting at Ls - s0 - SPT
    const uint32_t oo = (uint32_t)(site * Ls + (Ls - s0 - SPT)) * CB;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        C2<T> o[SPT];
#pragma unroll
        for (int k = 0; k < SPT; ++k) o[SPT - 1 - k] = (c < 6) ? acc[k][c] : cneg<T>(acc[k][c]);
        Vec<T, SPT>::st(o, f.out, oo, (uint32_t)c * f.cstride);
    }
}

template <typename T, int SPT, bool LDSL, bool CLS = false>
void launch_variant(const FineGeom& g, const C2<T>* U, const C2<T>* in, C2<T>* out, hipStream_t s,
                    ClassSel cs = ClassSel{{1, 1, 1, 1}, -1}) {
    const int items = g.V4 * (g.Ls / SPT);
    const int blocks = (items + WG - 1) / WG;
    hipLaunchKernelGGL((dslash_dwf_kernel<T, SPT, LDSL, CLS>), dim3(blocks), dim3(WG), 0, s, g, U, in, out, cs);
}

}  // namespace

template <typename T>
void launch_dslash(const FineGeom& g, const C2<T>* U, const C2<T>* in, C2<T>* out, hipStream_t s) {
    // variant 0 (default) and 2: one slot per work-item, links from global
    // memory (measured fastest at 24^4 x 16).  variant 1: links staged in LDS
    // (one slot; FP32 with Ls/2 >= MIN_SLOTS takes two slots).  The LDS
    // variants need Ls / SPT >= MIN_SLOTS and fall back otherwise.
    if (g.variant == 1 && g.Ls >= MIN_SLOTS) {
        if (sizeof(T) == 4 && g.Ls % 2 == 0 && g.Ls / 2 >= MIN_SLOTS)
            launch_variant<T, 2, true>(g, U, in, out, s);
        else
            launch_variant<T, 1, true>(g, U, in, out, s);
    } else {
        launch_variant<T, 1, false>(g, U, in, out, s);
    }
}

void launch_dslash_class(const CoarseGeom& c, const double2* U, const double2* in, double2* out, int cls,
                         hipStream_t s) {
    ClassSel cs;
    for (int mu = 0; mu < 4; ++mu) cs.B[mu] = c.B[mu];
    cs.cls = cls;
    launch_variant<double, 1, false, true>(c.f, U, in, out, s, cs);
}

template void launch_dslash<double>(const FineGeom&, const double2*, const double2*, double2*, hipStream_t);
template void launch_dslash<float>(const FineGeom&, const float2*, const float2*, float2*, hipStream_t);

}  // namespace hdcr
