// Fine operator H = Gamma5 D_dwf (Sec. 3) for gfx950.
//
// One work-item per 5d site (x, s), s fastest, so a 64-wide wavefront covers
// 64/Ls whole 4d sites (Ls dividing 64): every component load of the
// site-major SoA field psi[c][site4][s] is one contiguous run.
//
// Data-return traffic of the vector memory path is what limits a gather
// stencil on this chip, so the tile kernel keeps it to the spinor gathers:
//  * the 8 SU(3) links a 4d site needs (forward links at the site, backward
//    links at the site minus mu) are loaded once per site by its Ls
//    work-items into LDS, instead of once per work-item;
//  * for Ls = 8 and 16 the fifth-dimension neighbours psi(s -+ 1) are taken
//    from the neighbouring lanes with DPP moves instead of memory loads.
// The generic kernel (other Ls, and the hop-class split used by the coarse
// build) loads links and fifth-dimension neighbours directly.
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
// so each hop multiplies a half spinor (2 spins x 3 colours) by the link; the
// hop coefficient (-1/2, times bc[mu] across the boundary) is applied in the
// accumulating FMAs.  The output is written at (x, Ls-1-s) with the lower
// spins negated: H = gamma5 R5 D.
#include "coarse.h"

namespace hdcr {

namespace {

constexpr int WG = 256;
constexpr int LPAD = 10;  // complex entries per staged link matrix (9 used; keeps FP32 matrices 16-byte aligned)

// Blocks of the little-Dirac-operator build: a mu hop from a site with local
// coordinate B[mu] - 1 (forward) or 0 (backward) crosses the block face.
struct ClassSel {
    int B[4];  // block extents
};

struct FieldRefs {
    __amdgpu_buffer_rsrc_t in, U, out;
    uint32_t cstride;  // bytes between field components (N5 complex)
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

// y += a x  and  y += a (i x)
template <typename T> __device__ __forceinline__ void axpy(T a, C2<T> x, C2<T>& y) {
    y.x = fma(a, x.x, y.x);
    y.y = fma(a, x.y, y.y);
}
template <typename T> __device__ __forceinline__ void axpy_i(T a, C2<T> x, C2<T>& y) {
    y.x = fma(-a, x.y, y.x);
    y.y = fma(a, x.x, y.y);
}

// Arithmetic of one hop in direction MU (0..3 = x, y, z, t), forward (FWD) or
// backward: the 12 components v of psi at the neighbouring 5d site, link u
// (U_mu(x) forward, U_mu(x - mu) backward), hop coefficient coef, accumulated
// into acc.
template <typename T, int MU, bool FWD>
__device__ __forceinline__ void hop_core(const C2<T> (&v)[12], const C2<T> (&u)[9], T coef, C2<T> (&acc)[12]) {
    C2<T> h0[3], h1[3];
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        const C2<T> u0 = v[0 * 3 + col], u1 = v[1 * 3 + col], d0 = v[2 * 3 + col], d1 = v[3 * 3 + col];
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
    }
    C2<T> H0[3], H1[3];
    su3_mul<T, !FWD>(u, h0, H0);
    su3_mul<T, !FWD>(u, h1, H1);
    // upper spins += coef H; lower spins -+= coef w^dag H (minus forward, plus backward)
    const T sl = FWD ? -coef : coef;
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        axpy<T>(coef, H0[col], acc[0 * 3 + col]);
        axpy<T>(coef, H1[col], acc[1 * 3 + col]);
        if (MU == 0) {        // w_x^dag H = (i H1, i H0)
            axpy_i<T>(sl, H1[col], acc[2 * 3 + col]);
            axpy_i<T>(sl, H0[col], acc[3 * 3 + col]);
        } else if (MU == 1) { // w_y^dag H = (H1, -H0)
            axpy<T>(sl, H1[col], acc[2 * 3 + col]);
            axpy<T>(-sl, H0[col], acc[3 * 3 + col]);
        } else if (MU == 2) { // w_z^dag H = (i H0, -i H1)
            axpy_i<T>(sl, H0[col], acc[2 * 3 + col]);
            axpy_i<T>(-sl, H1[col], acc[3 * 3 + col]);
        } else {              // w_t^dag H = (H0, H1)
            axpy<T>(sl, H0[col], acc[2 * 3 + col]);
            axpy<T>(sl, H1[col], acc[3 * 3 + col]);
        }
    }
}

// The same hop with the direction given at run time: sg = +1 forward, -1
// backward, and m the matrix already oriented for it (U_mu(x) forward,
// U_mu(x - mu)^dag backward), so every hop multiplies by m.  The forward and
// backward forms of hop_core compute the same floating-point operations.
template <typename T, int MU>
__device__ __forceinline__ void hop_core_rt(const C2<T> (&v)[12], const C2<T> (&m)[9], T sg, T coef,
                                            C2<T> (&acc)[12]) {
    C2<T> h0[3], h1[3];
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        const C2<T> u0 = v[0 * 3 + col], u1 = v[1 * 3 + col], d0 = v[2 * 3 + col], d1 = v[3 * 3 + col];
        // h = u - sg w_mu d
        if (MU == 0) {        // w_x d = (-i d1, -i d0):  h = u + sg i (d1, d0)
            h0[col] = mk<T>(fma(-sg, d1.y, u0.x), fma(sg, d1.x, u0.y));
            h1[col] = mk<T>(fma(-sg, d0.y, u1.x), fma(sg, d0.x, u1.y));
        } else if (MU == 1) { // w_y d = (-d1, d0):  h = (u0 + sg d1, u1 - sg d0)
            h0[col] = mk<T>(fma(sg, d1.x, u0.x), fma(sg, d1.y, u0.y));
            h1[col] = mk<T>(fma(-sg, d0.x, u1.x), fma(-sg, d0.y, u1.y));
        } else if (MU == 2) { // w_z d = (-i d0, i d1):  h = (u0 + sg i d0, u1 - sg i d1)
            h0[col] = mk<T>(fma(-sg, d0.y, u0.x), fma(sg, d0.x, u0.y));
            h1[col] = mk<T>(fma(sg, d1.y, u1.x), fma(-sg, d1.x, u1.y));
        } else {              // w_t d = (d0, d1):  h = u - sg d
            h0[col] = mk<T>(fma(-sg, d0.x, u0.x), fma(-sg, d0.y, u0.y));
            h1[col] = mk<T>(fma(-sg, d1.x, u1.x), fma(-sg, d1.y, u1.y));
        }
    }
    C2<T> H0[3], H1[3];
    su3_mul<T, false>(m, h0, H0);
    su3_mul<T, false>(m, h1, H1);
    const T sl = -sg * coef;
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        axpy<T>(coef, H0[col], acc[0 * 3 + col]);
        axpy<T>(coef, H1[col], acc[1 * 3 + col]);
        if (MU == 0) {
            axpy_i<T>(sl, H1[col], acc[2 * 3 + col]);
            axpy_i<T>(sl, H0[col], acc[3 * 3 + col]);
        } else if (MU == 1) {
            axpy<T>(sl, H1[col], acc[2 * 3 + col]);
            axpy<T>(-sl, H0[col], acc[3 * 3 + col]);
        } else if (MU == 2) {
            axpy_i<T>(sl, H0[col], acc[2 * 3 + col]);
            axpy_i<T>(-sl, H1[col], acc[3 * 3 + col]);
        } else {
            axpy<T>(sl, H0[col], acc[2 * 3 + col]);
            axpy<T>(sl, H1[col], acc[3 * 3 + col]);
        }
    }
}

// One hop in direction MU, forward (FWD) or backward: psi at the neighbouring 5d
// site (byte offset noff) loaded from the field, link u (U_mu(x) forward,
// U_mu(x - mu) backward), hop coefficient coef, accumulated into acc.
template <typename T, int MU, bool FWD>
__device__ __forceinline__ void hop(const FieldRefs& f, uint32_t noff, const C2<T> (&u)[9], T coef,
                                    C2<T> (&acc)[12]) {
    C2<T> v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = Buf<T>::ld(f.in, noff, (uint32_t)c * f.cstride);
    hop_core<T, MU, FWD>(v, u, coef, acc);
}

// Neighbouring 4d sites of a work-item's site and the hop coefficients
// (-b/2, times bc[mu] for a hop across the lattice boundary).  The wrap-around
// is a select between uniform steps, so no branch depends on the lane.
template <typename T> struct Nbrs {
    int f[4], b[4];
    T cf[4], cb[4];
};
template <typename T> __device__ __forceinline__ Nbrs<T> neighbours(const FineGeom& g, const Site& st) {
    Nbrs<T> n;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const bool wf = (st.x[mu] == g.L[mu] - 1), wb = (st.x[mu] == 0);
        n.f[mu] = st.site + (wf ? -g.wrap[mu] : g.stride[mu]);
        n.b[mu] = st.site + (wb ? g.wrap[mu] : -g.stride[mu]);
        const T half = (T)g.hop;
        n.cf[mu] = wf ? half * (T)g.bc[mu] : half;
        n.cb[mu] = wb ? half * (T)g.bc[mu] : half;
    }
    return n;
}

// DPP lane moves inside a row of 16 lanes (dpp_ctrl row_shl:n = 0x100 + n,
// row_shr:n = 0x110 + n, row_ror:n = 0x120 + n).
template <int CTRL> __device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_f(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL, typename T> __device__ __forceinline__ C2<T> dpp_c(C2<T> v) {
    return mk<T>(dpp_f<CTRL>(v.x), dpp_f<CTRL>(v.y));
}
// value held by the lane of fifth coordinate s - 1 (DOWN) or s + 1, cyclic in
// groups of LS lanes (LS = 8 or 16, so a group never straddles a DPP row)
template <typename T, int LS, bool DOWN> __device__ __forceinline__ C2<T> s_neighbour(C2<T> v, int s) {
    if constexpr (LS == 16) {
        return DOWN ? dpp_c<0x121, T>(v) : dpp_c<0x12F, T>(v);
    } else {
        static_assert(LS == 8, "DPP fifth-dimension exchange needs LS = 8 or 16");
        if (DOWN) {
            const C2<T> a = dpp_c<0x111, T>(v), w = dpp_c<0x100 + LS - 1, T>(v);
            return (s == 0) ? w : a;
        } else {
            const C2<T> a = dpp_c<0x101, T>(v), w = dpp_c<0x110 + LS - 1, T>(v);
            return (s == LS - 1) ? w : a;
        }
    }
}

template <typename T, int MU>
__device__ __forceinline__ void hop_pair_lds(const FieldRefs& f, const Nbrs<T>& n, int Ls, int s, const C2<T>* lnk,
                                             C2<T> (&acc)[12]) {
    constexpr uint32_t CB = sizeof(C2<T>);
    C2<T> u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = lnk[MU * LPAD + e];
    hop<T, MU, true>(f, (uint32_t)(n.f[MU] * Ls + s) * CB, u, n.cf[MU], acc);
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = lnk[(4 + MU) * LPAD + e];
    hop<T, MU, false>(f, (uint32_t)(n.b[MU] * Ls + s) * CB, u, n.cb[MU], acc);
}

// Writes the 12 components of a work-item's output element (byte offset oo):
// H = gamma5 R5 D negates the lower spins; with NY > 0 the result is
// beta (H in) + sum_i g[i] y[i].  NT: non-temporal stores.
template <typename T, int NY, bool NT, bool BATCH = false>
__device__ __forceinline__ void store_out(const FieldRefs& f, uint32_t oo, const Epi<T>& ep, const C2<T> (&acc)[12]) {
    // BATCH: the epilogue fields of a chunk of components are all requested
    // before the first of them is combined (otherwise the compiler serialises
    // one round trip per component); chunks of about 48 registers of loaded
    // data.  Only where the registers do not lower the occupancy.
    constexpr int PER = NY > 0 ? NY * (int)sizeof(C2<T>) / 4 : 1;  // registers per component
    constexpr int CH =
        (NY == 0 || !BATCH) ? 1 : (48 / PER >= 12 ? 12 : (48 / PER >= 6 ? 6 : (48 / PER >= 4 ? 4 : 3)));
    __amdgpu_buffer_rsrc_t yr[NY > 0 ? NY : 1];
#pragma unroll
    for (int i = 0; i < NY; ++i) yr[i] = make_rsrc(ep.y[i], 12u * f.cstride);
#pragma unroll
    for (int c0 = 0; c0 < 12; c0 += CH) {
        C2<T> yv[NY > 0 ? NY : 1][CH];
        if constexpr (NY > 0 && BATCH) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = 0; c < CH; ++c)
#pragma unroll
                for (int i = 0; i < NY; ++i) yv[i][c] = Buf<T>::ld(yr[i], oo, (uint32_t)(c0 + c) * f.cstride);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int cc = c0 + c;
            C2<T> o = (cc < 6) ? acc[cc] : cneg<T>(acc[cc]);
            if constexpr (NY > 0) {
                o = cscale<T>(ep.beta, o);
#pragma unroll
                for (int i = 0; i < NY; ++i)
                    axpy<T>(ep.g[i], BATCH ? yv[i][c] : Buf<T>::ld(yr[i], oo, (uint32_t)cc * f.cstride), o);
            }
            if constexpr (NT)
                Buf<T>::st_nt(o, f.out, oo, (uint32_t)cc * f.cstride);
            else
                Buf<T>::st(o, f.out, oo, (uint32_t)cc * f.cstride);
        }
    }
}

// Tile kernel: Ls = LS divides WG; a workgroup holds WG / LS whole 4d sites.
// NT: stores with the non-temporal hint (streamed past the L2); NY: epilogue terms.
template <typename T, int LS, bool NT, int NY>
__global__ void __launch_bounds__(WG) dslash_tile_kernel(FineGeom g, const C2<T>* U, const C2<T>* in, C2<T>* out,
                                                         Epi<T> ep) {
    constexpr uint32_t CB = sizeof(C2<T>);
    constexpr int SITES = WG / LS;
    constexpr bool DPP = (LS == 8 || LS == 16);
    __shared__ C2<T> lds[SITES * 8 * LPAD];

    const int lb = logical_block(blockIdx.x, gridDim.x);
    const int gid = lb * WG + threadIdx.x;
    const int lsite = gid / LS;
    const int s = gid % LS;
    const int j = threadIdx.x / LS;  // site slot inside the workgroup
    const bool active = lsite < g.V4;
    FieldRefs f;
    f.cstride = (uint32_t)g.N5 * CB;
    f.in = make_rsrc(in, 12u * f.cstride);
    f.out = make_rsrc(out, 12u * f.cstride);
    f.U = make_rsrc(U, (uint32_t)g.V4 * 36u * CB);

    const Site st = traverse(g, active ? lsite : 0);
    const Nbrs<T> n = neighbours<T>(g, st);

    // stage the 8 link matrices of the site: matrix d < 4 is U_d(x), d >= 4 is
    // U_{d-4}(x - (d-4)); the LS work-items of the site load 9 entries each pass
    if (active) {
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const int src = (d < 4) ? st.site : n.b[d - 4];
#pragma unroll
            for (int e0 = 0; e0 < 9; e0 += LS) {
                const int e = e0 + s;
                if (e < 9)
                    lds[(j * 8 + d) * LPAD + e] =
                        Buf<T>::ld(f.U, (uint32_t)(src * 36 + (d & 3) * 9 + e) * CB, 0u);
            }
        }
    }
    __syncthreads();
    if (!active) return;
    const C2<T>* lnk = lds + j * 8 * LPAD;

    // diagonal (5 - M5) and the fifth-dimension hops: -P+ psi(s-1) on the upper
    // spins, -P- psi(s+1) on the lower spins, +mf across the walls
    C2<T> acc[12];
    {
        const T diag = (T)g.diag, mf = (T)g.mf;
        const T cm = (s == 0) ? mf : (T)-1;
        const T cp = (s == LS - 1) ? mf : (T)-1;
        const uint32_t o0 = (uint32_t)(st.site * LS + s) * CB;
        const uint32_t om = (uint32_t)(st.site * LS + (s == 0 ? LS - 1 : s - 1)) * CB;
        const uint32_t op = (uint32_t)(st.site * LS + (s == LS - 1 ? 0 : s + 1)) * CB;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const C2<T> v = Buf<T>::ld(f.in, o0, (uint32_t)c * f.cstride);
            C2<T> w;
            if constexpr (DPP)
                w = (c < 6) ? s_neighbour<T, LS, true>(v, s) : s_neighbour<T, LS, false>(v, s);
            else
                w = Buf<T>::ld(f.in, (c < 6) ? om : op, (uint32_t)c * f.cstride);
            const T cw = (c < 6) ? cm : cp;
            acc[c] = mk<T>(fma(diag, v.x, cw * w.x), fma(diag, v.y, cw * w.y));
        }
    }
    hop_pair_lds<T, 0>(f, n, LS, s, lnk, acc);
    hop_pair_lds<T, 1>(f, n, LS, s, lnk, acc);
    hop_pair_lds<T, 2>(f, n, LS, s, lnk, acc);
    hop_pair_lds<T, 3>(f, n, LS, s, lnk, acc);

    store_out<T, NY, NT>(f, (uint32_t)(st.site * LS + (LS - 1 - s)) * CB, ep, acc);
}

// Parity-tile kernel (FP32, Ls = 16, every extent even).  The lattice is cut
// into 2^4 tiles and a workgroup (256 work-items) holds one tile: work-item
// (p, s) with p the parity pattern of its site inside the tile (bit mu = the
// site's position along mu).  The tile's spinors are staged in LDS once; in
// every direction one of the two hops stays in the tile (forward if bit mu is
// 0, backward if it is 1) and reads the partner site's spinor from LDS, so
// only four of the eight hops gather through the vector-memory path.  The
// link matrices are staged already oriented for each hop (U_mu(x) forward,
// U_mu(x - mu)^dag backward), so the direction is a run-time sign and the code
// has no branch.
struct TileGeom {
    FineGeom t;  // the lattice of tiles (extents L / 2), traversal order of the tiles
};

template <typename T, int NY>
__global__ void __launch_bounds__(WG) dslash_par_kernel(FineGeom g, TileGeom tg, const C2<T>* U, const C2<T>* in,
                                                        C2<T>* out, Epi<T> ep) {
    constexpr int LS = 16;
    constexpr uint32_t CB = sizeof(C2<T>);
    __shared__ C2<T> spin[12 * 16 * LS];   // [c][pattern][s]
    __shared__ C2<T> lds[16 * 8 * LPAD];   // [pattern][matrix][entry]
    const int p = threadIdx.x >> 4, s = threadIdx.x & 15;
    const int tile = logical_block(blockIdx.x, gridDim.x);
    const Site tt = traverse(tg.t, tile);
    Site st;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) st.x[mu] = 2 * tt.x[mu] + ((p >> mu) & 1);
    st.site = ((st.x[3] * g.L[2] + st.x[2]) * g.L[1] + st.x[1]) * g.L[0] + st.x[0];
    const Nbrs<T> n = neighbours<T>(g, st);
    FieldRefs f;
    f.cstride = (uint32_t)g.N5 * CB;
    f.in = make_rsrc(in, 12u * f.cstride);
    f.out = make_rsrc(out, 12u * f.cstride);
    f.U = make_rsrc(U, (uint32_t)g.V4 * 36u * CB);
    // LDS matrix 2 mu: the hop of direction mu inside the tile, 2 mu + 1: the one
    // leaving it (backward matrices stored conjugate-transposed)
    if (s < 9) {
        const int r = s / 3, cc = s - 3 * (s / 3);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const bool up = (p >> mu) & 1;  // the forward hop stays in the tile for up = 0
            const C2<T> uf = Buf<T>::ld(f.U, (uint32_t)(st.site * 36 + mu * 9 + s) * CB, 0u);
            const C2<T> ub = Buf<T>::ld(f.U, (uint32_t)(n.b[mu] * 36 + mu * 9 + s) * CB, 0u);
            lds[(p * 8 + 2 * mu + (up ? 1 : 0)) * LPAD + s] = uf;
            lds[(p * 8 + 2 * mu + (up ? 0 : 1)) * LPAD + cc * 3 + r] = mk<T>(ub.x, -ub.y);
        }
    }
    C2<T> v[12];
    {
        const uint32_t o0 = (uint32_t)(st.site * LS + s) * CB;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            v[c] = Buf<T>::ld(f.in, o0, (uint32_t)c * f.cstride);
            spin[(c * 16 + p) * LS + s] = v[c];
        }
    }
    __syncthreads();
    const C2<T>* lnk = lds + p * 8 * LPAD;

    C2<T> acc[12];
    {
        const T diag = (T)g.diag, mf = (T)g.mf;
        const T cm = (s == 0) ? mf : (T)-1;
        const T cp = (s == LS - 1) ? mf : (T)-1;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const C2<T> w = (c < 6) ? s_neighbour<T, LS, true>(v[c], s) : s_neighbour<T, LS, false>(v[c], s);
            const T cw = (c < 6) ? cm : cp;
            acc[c] = mk<T>(fma(diag, v[c].x, cw * w.x), fma(diag, v[c].y, cw * w.y));
        }
    }
    // direction MU: the hop inside the tile reads the partner's spinor from
    // LDS, the hop leaving the tile gathers from the field
#define HDCR_PAR_HOPS(MU)                                                                                    \
    {                                                                                                        \
        const bool up = (p >> MU) & 1;                                                                       \
        const T sg_in = up ? (T)-1 : (T)1;                                                                   \
        const int q = p ^ (1 << MU);                                                                         \
        C2<T> m[9];                                                                                          \
        _Pragma("unroll") for (int e = 0; e < 9; ++e) m[e] = lnk[(2 * MU) * LPAD + e];                       \
        _Pragma("unroll") for (int c = 0; c < 12; ++c) v[c] = spin[(c * 16 + q) * LS + s];                   \
        hop_core_rt<T, MU>(v, m, sg_in, up ? n.cb[MU] : n.cf[MU], acc);                                      \
        _Pragma("unroll") for (int e = 0; e < 9; ++e) m[e] = lnk[(2 * MU + 1) * LPAD + e];                   \
        const uint32_t noff = (uint32_t)((up ? n.f[MU] : n.b[MU]) * LS + s) * CB;                            \
        _Pragma("unroll") for (int c = 0; c < 12; ++c) v[c] = Buf<T>::ld(f.in, noff, (uint32_t)c * f.cstride); \
        hop_core_rt<T, MU>(v, m, -sg_in, up ? n.cf[MU] : n.cb[MU], acc);                                     \
    }
    HDCR_PAR_HOPS(0)
    HDCR_PAR_HOPS(1)
    HDCR_PAR_HOPS(2)
    HDCR_PAR_HOPS(3)
#undef HDCR_PAR_HOPS
    store_out<T, NY, true, (sizeof(T) == 8)>(f, (uint32_t)(st.site * LS + (LS - 1 - s)) * CB, ep, acc);
}

// Paired parity-tile kernel (FP32, Ls = 16): the tile scheme above with each
// work-item holding two adjacent fifth-dimension slices (s0 = 2k, s0 + 1), so
// that every field access is one 16-byte load or store of two FP32 complex
// numbers.  The vector-memory data path returns a fixed number of lanes per
// clock whatever the access width, so 16-byte accesses move twice the bytes
// per cycle of the 8-byte ones.  A workgroup of 128 work-items holds one
// tile: work-item (p, k), p the parity pattern of its site, k the slice pair.
// The fifth-dimension neighbours of a pair are the partner slice in the same
// work-item and one slice of the neighbouring pair, read from the staged tile
// in LDS; the output pair lands at slices Ls-2-s0, Ls-1-s0 in reverse order.
constexpr int PAR2_WG = 128;

__device__ __forceinline__ float4 ld_pair(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
__device__ __forceinline__ void st_pair_nt(float4 v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    store_b128<CPOL_NT>(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), r, voff, soff);
}

// FP16 field storage (H16): a complex entry is (fp16 re, fp16 im) in 4 bytes,
// a slice pair one 8-byte access; conversion to FP32 on load, round to nearest
// on store.  The staged tile, the links and the arithmetic stay FP32.
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef unsigned uint2_t __attribute__((ext_vector_type(2)));
template <bool H16>
__device__ __forceinline__ float4 ld_pair_s(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (H16) {
        const half4_t h = __builtin_bit_cast(half4_t, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
        return make_float4((float)h.x, (float)h.y, (float)h.z, (float)h.w);
    } else {
        return ld_pair(r, voff, soff);
    }
}
template <bool H16>
__device__ __forceinline__ void st_pair_s_nt(float4 v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (H16) {
        const half4_t h = {(_Float16)v.x, (_Float16)v.y, (_Float16)v.z, (_Float16)v.w};
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(uint2_t, h), r, voff + soff, 0, CPOL_NT);
    } else {
        st_pair_nt(v, r, voff, soff);
    }
}

template <int NY, bool H16>
__global__ void __launch_bounds__(PAR2_WG) __attribute__((amdgpu_waves_per_eu(2))) dslash_par2_kernel(FineGeom g, TileGeom tg, const float2* U,
                                                               const float2* in, float2* out, Epi<float> ep) {
    typedef float T;
    constexpr int LS = 16, NK = LS / 2;
    constexpr uint32_t CB = H16 ? 4u : (uint32_t)sizeof(float2);  // bytes per complex entry of a field
    constexpr uint32_t UB = sizeof(float2);                         // bytes per complex entry of a link
    __shared__ float4 spin[12 * 16 * NK];   // [c][pattern][k]: slices 2k, 2k+1
    __shared__ float2 lds[16 * 8 * LPAD];   // [pattern][matrix][entry]
    const int p = threadIdx.x >> 3, k = threadIdx.x & 7;
    const int s0 = 2 * k;
    const int tile = logical_block(blockIdx.x, gridDim.x);
    const Site tt = traverse(tg.t, tile);
    Site st;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) st.x[mu] = 2 * tt.x[mu] + ((p >> mu) & 1);
    st.site = ((st.x[3] * g.L[2] + st.x[2]) * g.L[1] + st.x[1]) * g.L[0] + st.x[0];
    const Nbrs<T> n = neighbours<T>(g, st);
    FieldRefs f;
    f.cstride = (uint32_t)g.N5 * CB;
    f.in = make_rsrc(in, 12u * f.cstride);
    f.out = make_rsrc(out, 12u * f.cstride);
    f.U = make_rsrc(U, (uint32_t)g.V4 * 36u * (uint32_t)sizeof(float2));
    // LDS matrix 2 mu: the hop of direction mu inside the tile, 2 mu + 1: the
    // one leaving it (backward matrices stored conjugate-transposed)
    for (int e = k; e < 9; e += NK) {
        const int r = e / 3, cc = e - 3 * (e / 3);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const bool up = (p >> mu) & 1;
            const C2<T> uf = Buf<T>::ld(f.U, (uint32_t)(st.site * 36 + mu * 9 + e) * UB, 0u);
            const C2<T> ub = Buf<T>::ld(f.U, (uint32_t)(n.b[mu] * 36 + mu * 9 + e) * UB, 0u);
            lds[(p * 8 + 2 * mu + (up ? 1 : 0)) * LPAD + e] = uf;
            lds[(p * 8 + 2 * mu + (up ? 0 : 1)) * LPAD + cc * 3 + r] = mk<T>(ub.x, -ub.y);
        }
    }
    C2<T> v0[12], v1[12];
    {
        const uint32_t o0 = (uint32_t)(st.site * LS + s0) * CB;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const float4 q = ld_pair_s<H16>(f.in, o0, (uint32_t)c * f.cstride);
            v0[c] = mk<T>(q.x, q.y);
            v1[c] = mk<T>(q.z, q.w);
            spin[(c * 16 + p) * NK + k] = q;
        }
    }
    // out-of-tile partners, two directions in flight: directions 0 and 1 are
    // requested before the barrier, direction mu + 2 once direction mu's
    // partners have been used
#define HDCR_PAR2_GATHER(MU, DST)                                                                             \
    {                                                                                                         \
        const uint32_t noff = (uint32_t)((((p >> MU) & 1) ? n.f[MU] : n.b[MU]) * LS + s0) * CB;              \
        _Pragma("unroll") for (int c = 0; c < 12; ++c) DST[c] = ld_pair_s<H16>(f.in, noff, (uint32_t)c * f.cstride); \
    }
    float4 nx0[12], nx1[12];
    HDCR_PAR2_GATHER(0, nx0)
    HDCR_PAR2_GATHER(1, nx1)
    __syncthreads();
    const C2<T>* lnk = lds + p * 8 * LPAD;

    // diagonal and fifth-dimension terms: upper spins take slice s - 1, lower
    // spins slice s + 1 (wall coefficient mf at s = 0 and s = Ls - 1); the
    // slices of the neighbouring pairs come from the staged tile in LDS
    C2<T> a0[12], a1[12];
    {
        const T diag = (T)g.diag, mf = (T)g.mf;
        const T cm = (k == 0) ? mf : (T)-1;
        const T cp = (k == NK - 1) ? mf : (T)-1;
        const int kd = (k + NK - 1) & (NK - 1), ku = (k + 1) & (NK - 1);
        const float2* sp = reinterpret_cast<const float2*>(spin);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            if (c < 6) {
                const C2<T> w = sp[((c * 16 + p) * NK + kd) * 2 + 1];  // slice s0 - 1
                a0[c] = mk<T>(fma(diag, v0[c].x, cm * w.x), fma(diag, v0[c].y, cm * w.y));
                a1[c] = mk<T>(fma(diag, v1[c].x, -v0[c].x), fma(diag, v1[c].y, -v0[c].y));
            } else {
                const C2<T> w = sp[((c * 16 + p) * NK + ku) * 2];  // slice s0 + 2
                a0[c] = mk<T>(fma(diag, v0[c].x, -v1[c].x), fma(diag, v0[c].y, -v1[c].y));
                a1[c] = mk<T>(fma(diag, v1[c].x, cp * w.x), fma(diag, v1[c].y, cp * w.y));
            }
        }
    }
#define HDCR_PAR2_HOPS(MU, NX)                                                                                \
    {                                                                                                         \
        const bool up = (p >> MU) & 1;                                                                        \
        const T sg_in = up ? (T)-1 : (T)1;                                                                    \
        const int q = p ^ (1 << MU);                                                                          \
        C2<T> m[9];                                                                                           \
        _Pragma("unroll") for (int e = 0; e < 9; ++e) m[e] = lnk[(2 * MU) * LPAD + e];                        \
        _Pragma("unroll") for (int c = 0; c < 12; ++c) {                                                      \
            const float4 w = spin[(c * 16 + q) * NK + k];                                                     \
            v0[c] = mk<T>(w.x, w.y);                                                                          \
            v1[c] = mk<T>(w.z, w.w);                                                                          \
        }                                                                                                     \
        hop_core_rt<T, MU>(v0, m, sg_in, up ? n.cb[MU] : n.cf[MU], a0);                                       \
        hop_core_rt<T, MU>(v1, m, sg_in, up ? n.cb[MU] : n.cf[MU], a1);                                       \
        _Pragma("unroll") for (int e = 0; e < 9; ++e) m[e] = lnk[(2 * MU + 1) * LPAD + e];                    \
        _Pragma("unroll") for (int c = 0; c < 12; ++c) {                                                      \
            v0[c] = mk<T>(NX[c].x, NX[c].y);                                                                  \
            v1[c] = mk<T>(NX[c].z, NX[c].w);                                                                  \
        }                                                                                                     \
        hop_core_rt<T, MU>(v0, m, -sg_in, up ? n.cf[MU] : n.cb[MU], a0);                                      \
        hop_core_rt<T, MU>(v1, m, -sg_in, up ? n.cf[MU] : n.cb[MU], a1);                                      \
    }
    HDCR_PAR2_HOPS(0, nx0)
    __builtin_amdgcn_sched_barrier(0);
    HDCR_PAR2_GATHER(2, nx0)
    __builtin_amdgcn_sched_barrier(0);
    HDCR_PAR2_HOPS(1, nx1)
    __builtin_amdgcn_sched_barrier(0);
    HDCR_PAR2_GATHER(3, nx1)
    __builtin_amdgcn_sched_barrier(0);
    HDCR_PAR2_HOPS(2, nx0)
    HDCR_PAR2_HOPS(3, nx1)
#undef HDCR_PAR2_HOPS
#undef HDCR_PAR2_GATHER
    // slice s0 goes to Ls-1-s0, slice s0+1 to Ls-2-s0: one pair at Ls-2-s0,
    // lower spins negated (H = gamma5 R5 D)
    const uint32_t oo = (uint32_t)(st.site * LS + (LS - 2 - s0)) * CB;
    if constexpr (NY == 0) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const C2<T> lo = (c < 6) ? a1[c] : cneg<T>(a1[c]);
            const C2<T> hi = (c < 6) ? a0[c] : cneg<T>(a0[c]);
            st_pair_s_nt<H16>(make_float4(lo.x, lo.y, hi.x, hi.y), f.out, oo, (uint32_t)c * f.cstride);
        }
    } else {
        // every epilogue load is issued before the first combination: left to
        // itself the compiler loads one component's fields, stores it and only
        // then loads the next, twelve dependent round trips at the end of the
        // workgroup.  The hop temporaries are dead here, so the NY x 12 loaded
        // pairs fit the register budget (in two halves of 6 components for
        // four FP32 fields).
        constexpr int CH = (!H16 && NY >= 4) ? 6 : 12;
        __amdgpu_buffer_rsrc_t yr[NY];
#pragma unroll
        for (int i = 0; i < NY; ++i) yr[i] = make_rsrc(ep.y[i], 12u * f.cstride);
#pragma unroll
        for (int c0 = 0; c0 < 12; c0 += CH) {
            float4 yv[NY][CH];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = 0; c < CH; ++c)
#pragma unroll
                for (int i = 0; i < NY; ++i) yv[i][c] = ld_pair_s<H16>(yr[i], oo, (uint32_t)(c0 + c) * f.cstride);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int cc = c0 + c;
                C2<T> lo = (cc < 6) ? a1[cc] : cneg<T>(a1[cc]);
                C2<T> hi = (cc < 6) ? a0[cc] : cneg<T>(a0[cc]);
                lo = cscale<T>(ep.beta, lo);
                hi = cscale<T>(ep.beta, hi);
#pragma unroll
                for (int i = 0; i < NY; ++i) {
                    axpy<T>(ep.g[i], mk<T>(yv[i][c].x, yv[i][c].y), lo);
                    axpy<T>(ep.g[i], mk<T>(yv[i][c].z, yv[i][c].w), hi);
                }
                st_pair_s_nt<H16>(make_float4(lo.x, lo.y, hi.x, hi.y), f.out, oo, (uint32_t)cc * f.cstride);
            }
        }
    }
}

// FP16-storage kernel with four fifth-dimension slices per work-item (Ls = 16,
// even extents): every field access is one 16-byte run of four (fp16 re, fp16
// im) entries, and the tile is staged in LDS in its FP16 form (12 KB), so a
// workgroup of 64 work-items holds one 2^4 tile: work-item (p, k), p the parity
// pattern of its site, slices 4k .. 4k + 3.  Per slice this issues half the
// vector-memory instructions of the paired kernel on FP16 fields.  Links,
// arithmetic and the order of the operations per output are the paired
// kernel's.  The output quad lands at slices Ls-4-4k .. Ls-1-4k in reverse order.
constexpr int QUAD_WG = 64;
typedef _Float16 half2v_t __attribute__((ext_vector_type(2)));
typedef unsigned uint4_t __attribute__((ext_vector_type(4)));

// slice i (0 .. 3) of a quad word as an FP32 complex entry.  The element goes
// through a named scalar: this clang reads element 0 whatever the index when
// __builtin_bit_cast is applied to the subscript of a vector directly.
__device__ __forceinline__ C2<float> quad_slice(uint4_t w, int i) {
    const unsigned e = w[i];
    const half2v_t h = __builtin_bit_cast(half2v_t, e);
    return mk<float>((float)h.x, (float)h.y);
}

template <int NY>
__global__ void __launch_bounds__(QUAD_WG) __attribute__((amdgpu_waves_per_eu(2)))
dslash_quad_h16_kernel(FineGeom g, TileGeom tg, const float2* U, const uint4_t* in, uint4_t* out, Epi<float> ep) {
    typedef float T;
    constexpr int LS = 16, NQ = LS / 4;
    constexpr uint32_t CB = 4;  // bytes per complex entry of a field
    constexpr uint32_t UB = sizeof(float2);
    __shared__ uint4_t spin[12 * 16 * NQ];  // [c][pattern][k]: slices 4k .. 4k+3, FP16
    __shared__ float2 lds[16 * 8 * LPAD];   // [pattern][matrix][entry]
    const int p = threadIdx.x >> 2, k = threadIdx.x & 3;
    const int s0 = 4 * k;
    const int tile = logical_block(blockIdx.x, gridDim.x);
    const Site tt = traverse(tg.t, tile);
    Site st;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) st.x[mu] = 2 * tt.x[mu] + ((p >> mu) & 1);
    st.site = ((st.x[3] * g.L[2] + st.x[2]) * g.L[1] + st.x[1]) * g.L[0] + st.x[0];
    const Nbrs<T> n = neighbours<T>(g, st);
    FieldRefs f;
    f.cstride = (uint32_t)g.N5 * CB;
    f.in = make_rsrc(in, 12u * f.cstride);
    f.out = make_rsrc(out, 12u * f.cstride);
    f.U = make_rsrc(U, (uint32_t)g.V4 * 36u * UB);
    // LDS matrix 2 mu: the hop of direction mu inside the tile, 2 mu + 1: the
    // one leaving it (backward matrices stored conjugate-transposed)
    for (int e = k; e < 9; e += NQ) {
        const int r = e / 3, cc = e - 3 * (e / 3);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const bool up = (p >> mu) & 1;
            const C2<T> uf = Buf<T>::ld(f.U, (uint32_t)(st.site * 36 + mu * 9 + e) * UB, 0u);
            const C2<T> ub = Buf<T>::ld(f.U, (uint32_t)(n.b[mu] * 36 + mu * 9 + e) * UB, 0u);
            lds[(p * 8 + 2 * mu + (up ? 1 : 0)) * LPAD + e] = uf;
            lds[(p * 8 + 2 * mu + (up ? 0 : 1)) * LPAD + cc * 3 + r] = mk<T>(ub.x, -ub.y);
        }
    }
    uint4_t w[12];  // the four slices of all 12 components, as stored
    {
        const uint32_t o0 = (uint32_t)(st.site * LS + s0) * CB;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            w[c] = __builtin_amdgcn_raw_buffer_load_b128(f.in, o0, (uint32_t)c * f.cstride, 0);
            spin[(c * 16 + p) * NQ + k] = w[c];
        }
    }
    __syncthreads();
    const C2<T>* lnk = lds + p * 8 * LPAD;

    // diagonal and fifth-dimension terms: upper spins take slice s - 1, lower
    // spins slice s + 1 (wall coefficient mf at s = 0 and s = Ls - 1); the
    // slices of the neighbouring quads come from the staged tile in LDS
    C2<T> a[4][12];
    {
        const T diag = (T)g.diag, mf = (T)g.mf;
        const T cm = (k == 0) ? mf : (T)-1;
        const T cp = (k == NQ - 1) ? mf : (T)-1;
        const int kd = (k + NQ - 1) & (NQ - 1), ku = (k + 1) & (NQ - 1);
        const unsigned* sp = reinterpret_cast<const unsigned*>(spin);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            C2<T> x[6];  // slices s0 - 1 .. s0 + 4
            x[1] = quad_slice(w[c], 0);
            x[2] = quad_slice(w[c], 1);
            x[3] = quad_slice(w[c], 2);
            x[4] = quad_slice(w[c], 3);
            if (c < 6) {
                const half2v_t hw = __builtin_bit_cast(half2v_t, sp[((c * 16 + p) * NQ + kd) * 4 + 3]);
                x[0] = mk<T>(cm * (float)hw.x, cm * (float)hw.y);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const T cl = (i == 0) ? (T)1 : (T)-1;  // the wall coefficient is folded into x[0]
                    a[i][c] = mk<T>(fma(diag, x[i + 1].x, cl * x[i].x), fma(diag, x[i + 1].y, cl * x[i].y));
                }
            } else {
                const half2v_t hw = __builtin_bit_cast(half2v_t, sp[((c * 16 + p) * NQ + ku) * 4]);
                x[5] = mk<T>(cp * (float)hw.x, cp * (float)hw.y);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const T cl = (i == 3) ? (T)1 : (T)-1;
                    a[i][c] = mk<T>(fma(diag, x[i + 1].x, cl * x[i + 2].x), fma(diag, x[i + 1].y, cl * x[i + 2].y));
                }
            }
        }
    }
#define HDCR_QUAD_HOPS(MU)                                                                                    \
    {                                                                                                         \
        const bool up = (p >> MU) & 1;                                                                        \
        const T sg_in = up ? (T)-1 : (T)1;                                                                    \
        const int q = p ^ (1 << MU);                                                                          \
        C2<T> m[9], v[12];                                                                                    \
        _Pragma("unroll") for (int e = 0; e < 9; ++e) m[e] = lnk[(2 * MU) * LPAD + e];                        \
        _Pragma("unroll") for (int c = 0; c < 12; ++c) w[c] = spin[(c * 16 + q) * NQ + k];                    \
        _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                                       \
            _Pragma("unroll") for (int c = 0; c < 12; ++c) v[c] = quad_slice(w[c], i);                        \
            hop_core_rt<T, MU>(v, m, sg_in, up ? n.cb[MU] : n.cf[MU], a[i]);                                  \
        }                                                                                                     \
        _Pragma("unroll") for (int e = 0; e < 9; ++e) m[e] = lnk[(2 * MU + 1) * LPAD + e];                    \
        const uint32_t noff = (uint32_t)((up ? n.f[MU] : n.b[MU]) * LS + s0) * CB;                            \
        _Pragma("unroll") for (int c = 0; c < 12; ++c)                                                        \
            w[c] = __builtin_amdgcn_raw_buffer_load_b128(f.in, noff, (uint32_t)c * f.cstride, 0);             \
        _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                                       \
            _Pragma("unroll") for (int c = 0; c < 12; ++c) v[c] = quad_slice(w[c], i);                        \
            hop_core_rt<T, MU>(v, m, -sg_in, up ? n.cf[MU] : n.cb[MU], a[i]);                                 \
        }                                                                                                     \
    }
    // the scheduling barriers keep each direction's loads from being hoisted
    // above the previous direction's arithmetic (that hoisting spills)
    HDCR_QUAD_HOPS(0)
    __builtin_amdgcn_sched_barrier(0);
    HDCR_QUAD_HOPS(1)
    __builtin_amdgcn_sched_barrier(0);
    HDCR_QUAD_HOPS(2)
    __builtin_amdgcn_sched_barrier(0);
    HDCR_QUAD_HOPS(3)
#undef HDCR_QUAD_HOPS
    // slice s0 + i goes to Ls-1-s0-i: one quad at Ls-4-s0 holding slices
    // s0+3, s0+2, s0+1, s0; lower spins negated (H = gamma5 R5 D); epilogue
    // out = beta H in + sum_i g_i y_i on the FP16-stored y_i
    const uint32_t oo = (uint32_t)(st.site * LS + (LS - 4 - s0)) * CB;
    // epilogue loads issued a chunk of components at a time before any of
    // them is combined (as in the paired kernel); chunks sized so the loaded
    // quads and the 4 x 12 accumulators fit the register budget
    constexpr int CH = NY <= 1 ? 12 : (NY == 2 ? 6 : (NY == 3 ? 4 : 3));
    __amdgpu_buffer_rsrc_t yr[NY > 0 ? NY : 1];
#pragma unroll
    for (int i = 0; i < NY; ++i) yr[i] = make_rsrc(ep.y[i], 12u * f.cstride);
#pragma unroll
    for (int c0 = 0; c0 < 12; c0 += CH) {
        uint4_t yv[NY > 0 ? NY : 1][CH];
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (NY > 0) {
#pragma unroll
            for (int c = 0; c < CH; ++c)
#pragma unroll
                for (int q = 0; q < NY; ++q)
                    yv[q][c] = __builtin_amdgcn_raw_buffer_load_b128(yr[q], oo, (uint32_t)(c0 + c) * f.cstride, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int cc = c0 + c;
            C2<T> o[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) o[i] = (cc < 6) ? a[3 - i][cc] : cneg<T>(a[3 - i][cc]);
            if constexpr (NY > 0) {
#pragma unroll
                for (int i = 0; i < 4; ++i) o[i] = cscale<T>(ep.beta, o[i]);
#pragma unroll
                for (int q = 0; q < NY; ++q)
#pragma unroll
                    for (int i = 0; i < 4; ++i) axpy<T>(ep.g[q], quad_slice(yv[q][c], i), o[i]);
            }
            const half4_t h0 = {(_Float16)o[0].x, (_Float16)o[0].y, (_Float16)o[1].x, (_Float16)o[1].y};
            const half4_t h1 = {(_Float16)o[2].x, (_Float16)o[2].y, (_Float16)o[3].x, (_Float16)o[3].y};
            const uint2_t w0 = __builtin_bit_cast(uint2_t, h0), w1 = __builtin_bit_cast(uint2_t, h1);
            store_b128<CPOL_NT>(uint4_t{w0.x, w0.y, w1.x, w1.y}, f.out, oo, (uint32_t)cc * f.cstride);
        }
    }
}

// Generic kernel: any Ls, links and fifth-dimension neighbours loaded
// directly.
template <typename T, int NY>
__global__ void __launch_bounds__(WG) dslash_dwf_kernel(FineGeom g, const C2<T>* U, const C2<T>* in, C2<T>* out,
                                                        Epi<T> ep) {
    constexpr uint32_t CB = sizeof(C2<T>);
    const int lb = logical_block(blockIdx.x, gridDim.x);
    const int Ls = g.Ls;
    const int gid = lb * WG + threadIdx.x;
    if (gid >= g.N5) return;
    FieldRefs f;
    f.cstride = (uint32_t)g.N5 * CB;
    f.in = make_rsrc(in, 12u * f.cstride);
    f.out = make_rsrc(out, 12u * f.cstride);
    f.U = make_rsrc(U, (uint32_t)g.V4 * 36u * CB);
    const int lsite = gid / Ls;
    const int s = gid - lsite * Ls;
    const Site st = traverse(g, lsite);
    const Nbrs<T> n = neighbours<T>(g, st);
    C2<T> acc[12];
    {
        const T diag = (T)g.diag, mf = (T)g.mf;
        const T cm = (s == 0) ? mf : (T)-1;
        const T cp = (s == Ls - 1) ? mf : (T)-1;
        const uint32_t o0 = (uint32_t)(st.site * Ls + s) * CB;
        const uint32_t om = (uint32_t)(st.site * Ls + (s == 0 ? Ls - 1 : s - 1)) * CB;
        const uint32_t op = (uint32_t)(st.site * Ls + (s == Ls - 1 ? 0 : s + 1)) * CB;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const C2<T> v = Buf<T>::ld(f.in, o0, (uint32_t)c * f.cstride);
            const C2<T> w = Buf<T>::ld(f.in, (c < 6) ? om : op, (uint32_t)c * f.cstride);
            const T cw = (c < 6) ? cm : cp;
            acc[c] = mk<T>(fma(diag, v.x, cw * w.x), fma(diag, v.y, cw * w.y));
        }
    }
#define HDCR_GENERIC_HOPS(MU)                                                                              \
    {                                                                                                      \
        C2<T> u[9];                                                                                        \
        for (int e = 0; e < 9; ++e) u[e] = Buf<T>::ld(f.U, (uint32_t)st.site * (36u * CB), (uint32_t)(MU * 9 + e) * CB); \
        hop<T, MU, true>(f, (uint32_t)(n.f[MU] * Ls + s) * CB, u, n.cf[MU], acc);                          \
        for (int e = 0; e < 9; ++e) u[e] = Buf<T>::ld(f.U, (uint32_t)n.b[MU] * (36u * CB), (uint32_t)(MU * 9 + e) * CB); \
        hop<T, MU, false>(f, (uint32_t)(n.b[MU] * Ls + s) * CB, u, n.cb[MU], acc);                         \
    }
    HDCR_GENERIC_HOPS(0)
    HDCR_GENERIC_HOPS(1)
    HDCR_GENERIC_HOPS(2)
    HDCR_GENERIC_HOPS(3)
#undef HDCR_GENERIC_HOPS
    store_out<T, NY, false>(f, (uint32_t)(st.site * Ls + (Ls - 1 - s)) * CB, ep, acc);
}

template <typename T, int LS, bool NT, int NY>
void launch_tile(const FineGeom& g, const C2<T>* U, const C2<T>* in, C2<T>* out, const Epi<T>& ep, hipStream_t s) {
    const int blocks = (g.N5 + WG - 1) / WG;
    hipLaunchKernelGGL((dslash_tile_kernel<T, LS, NT, NY>), dim3(blocks), dim3(WG), 0, s, g, U, in, out, ep);
}

template <typename T, int NY>
void launch_generic(const FineGeom& g, const C2<T>* U, const C2<T>* in, C2<T>* out, const Epi<T>& ep, hipStream_t s) {
    const int blocks = (g.N5 + WG - 1) / WG;
    hipLaunchKernelGGL((dslash_dwf_kernel<T, NY>), dim3(blocks), dim3(WG), 0, s, g, U, in, out, ep);
}

// All nine hop classes of the coarse build in one FP64 pass: class field d is
// out + d * fstride.  d = 0 gets the diagonal, fifth-dimension and block-interior
// hop terms at every site; d = 1 + mu (5 + mu) gets the forward (backward) mu hop
// that crosses the face of the site's block, written only at the sites on that
// face, where the projection reads it (elsewhere the class field is not
// written).  Each output is H's output element: lower spins negated, at s ->
// Ls - 1 - s.
__global__ void __launch_bounds__(WG) dslash_classes_kernel(FineGeom g, ClassSel cs, const double2* U,
                                                            const double2* in, double2* out, size_t fstride) {
    typedef double T;
    constexpr uint32_t CB = sizeof(double2);
    const int lb = logical_block(blockIdx.x, gridDim.x);
    const int Ls = g.Ls;
    const int gid = lb * WG + threadIdx.x;
    if (gid >= g.N5) return;
    FieldRefs f;
    f.cstride = (uint32_t)g.N5 * CB;
    f.in = make_rsrc(in, 12u * f.cstride);
    f.U = make_rsrc(U, (uint32_t)g.V4 * 36u * CB);
    const int lsite = gid / Ls;
    const int s = gid - lsite * Ls;
    const Site st = traverse(g, lsite);
    const Nbrs<T> n = neighbours<T>(g, st);
    const uint32_t oo = (uint32_t)(st.site * Ls + (Ls - 1 - s)) * CB;
    const Epi<T> none{{nullptr, nullptr, nullptr, nullptr}, {0, 0, 0, 0}, 1.0, 0};
    C2<T> acc[12];
    {
        const T diag = (T)g.diag, mf = (T)g.mf;
        const T cm = (s == 0) ? mf : (T)-1;
        const T cp = (s == Ls - 1) ? mf : (T)-1;
        const uint32_t o0 = (uint32_t)(st.site * Ls + s) * CB;
        const uint32_t om = (uint32_t)(st.site * Ls + (s == 0 ? Ls - 1 : s - 1)) * CB;
        const uint32_t op = (uint32_t)(st.site * Ls + (s == Ls - 1 ? 0 : s + 1)) * CB;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const C2<T> v = Buf<T>::ld(f.in, o0, (uint32_t)c * f.cstride);
            const C2<T> w = Buf<T>::ld(f.in, (c < 6) ? om : op, (uint32_t)c * f.cstride);
            const T cw = (c < 6) ? cm : cp;
            acc[c] = mk<T>(fma(diag, v.x, cw * w.x), fma(diag, v.y, cw * w.y));
        }
    }
    // a hop term into tmp, then either into class 0 or out to its face class
    auto route = [&](const C2<T> (&tmp)[12], bool face, int cls) {
        if (face) {
            f.out = make_rsrc(out + (size_t)cls * fstride, 12u * f.cstride);
            store_out<T, 0, false>(f, oo, none, tmp);
        } else {
#pragma unroll
            for (int c = 0; c < 12; ++c) acc[c] = cadd<T>(acc[c], tmp[c]);
        }
    };
#define HDCR_CLASS_HOPS(MU)                                                                                \
    {                                                                                                      \
        const int lx = st.x[MU] % cs.B[MU];                                                                \
        C2<T> u[9], tmp[12];                                                                               \
        for (int e = 0; e < 9; ++e) u[e] = Buf<T>::ld(f.U, (uint32_t)st.site * (36u * CB), (uint32_t)(MU * 9 + e) * CB); \
        _Pragma("unroll") for (int c = 0; c < 12; ++c) tmp[c] = mk<T>(0, 0);                               \
        hop<T, MU, true>(f, (uint32_t)(n.f[MU] * Ls + s) * CB, u, n.cf[MU], tmp);                          \
        route(tmp, lx == cs.B[MU] - 1, 1 + MU);                                                            \
        for (int e = 0; e < 9; ++e) u[e] = Buf<T>::ld(f.U, (uint32_t)n.b[MU] * (36u * CB), (uint32_t)(MU * 9 + e) * CB); \
        _Pragma("unroll") for (int c = 0; c < 12; ++c) tmp[c] = mk<T>(0, 0);                               \
        hop<T, MU, false>(f, (uint32_t)(n.b[MU] * Ls + s) * CB, u, n.cb[MU], tmp);                         \
        route(tmp, lx == 0, 5 + MU);                                                                       \
    }
    HDCR_CLASS_HOPS(0)
    HDCR_CLASS_HOPS(1)
    HDCR_CLASS_HOPS(2)
    HDCR_CLASS_HOPS(3)
#undef HDCR_CLASS_HOPS
    f.out = make_rsrc(out, 12u * f.cstride);
    store_out<T, 0, false>(f, oo, none, acc);
}

template <typename T, bool NT, int NY>
bool launch_tile_ls(const FineGeom& g, const C2<T>* U, const C2<T>* in, C2<T>* out, const Epi<T>& ep,
                    hipStream_t s) {
    switch (g.Ls) {
        case 8: launch_tile<T, 8, NT, NY>(g, U, in, out, ep, s); return true;
        case 16: launch_tile<T, 16, NT, NY>(g, U, in, out, ep, s); return true;
        case 32: launch_tile<T, 32, NT, NY>(g, U, in, out, ep, s); return true;
        case 64: launch_tile<T, 64, NT, NY>(g, U, in, out, ep, s); return true;
        default: return false;
    }
}

// tile kernel for Ls = 8, 16, 32, 64 with non-temporal output stores (the
// output is not re-read by this launch; streaming it keeps the L2 for the
// neighbour re-reads); generic kernel otherwise.  Tuning switch: variant 1
// uses cached stores for the plain apply, variant 2 the generic kernel.
// the lattice of 2^4 tiles for the parity-tile kernel (traversal order chosen
// as for a lattice of those extents)
TileGeom tile_geom(const FineGeom& g) {
    TileGeom t;
    t.t = g;
    t.t.V4 = 1;
    for (int mu = 0; mu < 4; ++mu) {
        t.t.L[mu] = g.L[mu] / 2;
        t.t.V4 *= t.t.L[mu];
    }
    // t slabs of about a quarter of the tile extent, x and y parts of about 3
    // tiles: each block is swept along z with a cross-section of some 27
    // tiles, so the z and t neighbours of a tile are still in the XCD's L2
    // when it is processed (measured best for 12^4 tiles, the 24^4 lattice,
    // among cross-sections of 8 to 216 tiles)
    int ts = t.t.L[3] >= 4 ? t.t.L[3] / 4 : t.t.L[3];
    while (ts > 1 && t.t.L[3] % ts != 0) --ts;
    int ys = t.t.L[1] / 3 > 0 ? t.t.L[1] / 3 : 1;
    while (ys > 1 && t.t.L[1] % ys != 0) --ys;
    int xs = t.t.L[0] / 3 > 0 ? t.t.L[0] / 3 : 1;
    while (xs > 1 && t.t.L[0] % xs != 0) --xs;
    choose_traversal(t.t, ts, ys, xs);  // the caller's choices in g.tune, if any, replace these
    return t;
}

// Dynamic LDS that caps the resident workgroups of a parity-tile kernel at
// g.tune.wg_per_cu per compute unit (160 KB of LDS each): fewer tiles in flight
// per XCD keep more of the L2 for the neighbours a tile re-reads.  0: no cap.
constexpr int LDS_PER_CU = 160 * 1024;
template <typename K> int lds_pad(const FineGeom& g, K kernel) {
    const int cap = g.tune.wg_per_cu;
    if (cap <= 0) return 0;
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(kernel)) != hipSuccess) return 0;
    const int want = LDS_PER_CU / (cap + 1) + 1 - (int)a.sharedSizeBytes;  // one byte over the share of cap + 1
    if (want <= 0) return 0;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              want);
    return want;
}

bool par_ok(const FineGeom& g) {
    return g.Ls == 16 && g.L[0] % 2 == 0 && g.L[1] % 2 == 0 && g.L[2] % 2 == 0 && g.L[3] % 2 == 0;
}

template <typename T, int NY>
void launch_ny(const FineGeom& g, const C2<T>* U, const C2<T>* in, C2<T>* out, const Epi<T>& ep, hipStream_t s) {
    // parity-tile kernels at Ls = 16 with even extents: FP32 with paired slices
    // by default (variant 4: one slice per work-item), FP64 with one slice per
    // work-item (variants 0 and 4); variants 1 to 3 select the tile and generic
    // kernels
    if ((g.variant == 0 || g.variant == 4) && par_ok(g)) {
        const TileGeom tg = tile_geom(g);
        if constexpr (sizeof(T) == 4) {
            if (g.variant == 0) {
                const int pad = lds_pad(g, dslash_par2_kernel<NY, false>);
                hipLaunchKernelGGL((dslash_par2_kernel<NY, false>), dim3(tg.t.V4), dim3(PAR2_WG), pad, s, g, tg, U,
                                   in, out, ep);
                return;
            }
        }
        const int pad = lds_pad(g, dslash_par_kernel<T, NY>);
        hipLaunchKernelGGL((dslash_par_kernel<T, NY>), dim3(tg.t.V4), dim3(WG), pad, s, g, tg, U, in, out, ep);
        return;
    }
    if (g.variant != 2) {
        if (NY == 0 && g.variant == 1) {
            if (launch_tile_ls<T, false, NY>(g, U, in, out, ep, s)) return;
        } else if (launch_tile_ls<T, true, NY>(g, U, in, out, ep, s)) {
            return;
        }
    }
    launch_generic<T, NY>(g, U, in, out, ep, s);
}

}  // namespace

template <typename T>
void launch_dslash(const FineGeom& g, const C2<T>* U, const C2<T>* in, C2<T>* out, hipStream_t s) {
    launch_ny<T, 0>(g, U, in, out, Epi<T>{{nullptr, nullptr, nullptr, nullptr}, {0, 0, 0, 0}, (T)1, 0}, s);
}

template <typename T>
void launch_dslash_epi(const FineGeom& g, const C2<T>* U, const C2<T>* in, C2<T>* out, const Epi<T>& e,
                       hipStream_t s) {
    switch (e.ny) {
        case 1: launch_ny<T, 1>(g, U, in, out, e, s); break;
        case 2: launch_ny<T, 2>(g, U, in, out, e, s); break;
        case 3: launch_ny<T, 3>(g, U, in, out, e, s); break;
        case 4: launch_ny<T, 4>(g, U, in, out, e, s); break;
        default: launch_ny<T, 0>(g, U, in, out, e, s); break;
    }
}

bool launch_dslash_h16(const FineGeom& g, const float2* U, const void* in, void* out, hipStream_t s) {
    if (!par_ok(g)) return false;
    const TileGeom tg = tile_geom(g);
    if (g.variant == 5) {  // the paired kernel on FP16 fields (two slices per work-item)
        hipLaunchKernelGGL((dslash_par2_kernel<0, true>), dim3(tg.t.V4), dim3(PAR2_WG), 0, s, g, tg, U,
                           static_cast<const float2*>(in), static_cast<float2*>(out),
                           Epi<float>{{nullptr, nullptr, nullptr, nullptr}, {0, 0, 0, 0}, 1.0f, 0});
        return true;
    }
    hipLaunchKernelGGL(dslash_quad_h16_kernel<0>, dim3(tg.t.V4), dim3(QUAD_WG), lds_pad(g, dslash_quad_h16_kernel<0>),
                       s, g, tg, U, static_cast<const uint4_t*>(in), static_cast<uint4_t*>(out),
                       Epi<float>{{nullptr, nullptr, nullptr, nullptr}, {0, 0, 0, 0}, 1.0f, 0});
    return true;
}

bool launch_dslash_h16_epi(const FineGeom& g, const float2* U, const void* in, void* out, const Epi<float>& e,
                           hipStream_t s) {
    if (!par_ok(g) || e.ny < 0 || e.ny > 4) return false;
    const TileGeom tg = tile_geom(g);
    if (g.variant == 5) {  // the paired kernel (two slices per work-item, 8-byte accesses)
        const float2* ip = static_cast<const float2*>(in);
        float2* op = static_cast<float2*>(out);
        const dim3 grid(tg.t.V4), block(PAR2_WG);
        switch (e.ny) {
            case 0: hipLaunchKernelGGL((dslash_par2_kernel<0, true>), grid, block, 0, s, g, tg, U, ip, op, e); break;
            case 1: hipLaunchKernelGGL((dslash_par2_kernel<1, true>), grid, block, 0, s, g, tg, U, ip, op, e); break;
            case 2: hipLaunchKernelGGL((dslash_par2_kernel<2, true>), grid, block, 0, s, g, tg, U, ip, op, e); break;
            case 3: hipLaunchKernelGGL((dslash_par2_kernel<3, true>), grid, block, 0, s, g, tg, U, ip, op, e); break;
            default: hipLaunchKernelGGL((dslash_par2_kernel<4, true>), grid, block, 0, s, g, tg, U, ip, op, e); break;
        }
        return true;
    }
    const uint4_t* ip = static_cast<const uint4_t*>(in);
    uint4_t* op = static_cast<uint4_t*>(out);
    const dim3 grid(tg.t.V4), block(QUAD_WG);
    switch (e.ny) {
        case 0: hipLaunchKernelGGL(dslash_quad_h16_kernel<0>, grid, block, 0, s, g, tg, U, ip, op, e); break;
        case 1: hipLaunchKernelGGL(dslash_quad_h16_kernel<1>, grid, block, 0, s, g, tg, U, ip, op, e); break;
        case 2: hipLaunchKernelGGL(dslash_quad_h16_kernel<2>, grid, block, 0, s, g, tg, U, ip, op, e); break;
        case 3: hipLaunchKernelGGL(dslash_quad_h16_kernel<3>, grid, block, 0, s, g, tg, U, ip, op, e); break;
        default: hipLaunchKernelGGL(dslash_quad_h16_kernel<4>, grid, block, 0, s, g, tg, U, ip, op, e); break;
    }
    return true;
}

bool dslash_h16_ok(const FineGeom& g) { return par_ok(g); }

void launch_dslash_classes(const CoarseGeom& c, const double2* U, const double2* in, double2* out, size_t fstride,
                           hipStream_t s) {
    ClassSel cs;
    for (int mu = 0; mu < 4; ++mu) cs.B[mu] = c.B[mu];
    const int blocks = (c.f.N5 + WG - 1) / WG;
    hipLaunchKernelGGL(dslash_classes_kernel, dim3(blocks), dim3(WG), 0, s, c.f, cs, U, in, out, fstride);
}

namespace {

// Continued-fraction operator (Sec. 3): one work-item per 5d site (4d site j of
// the workgroup, slice s), s fastest, k.sites whole 4d sites per workgroup.
// The 8 link matrices of each site (U_mu(x), then U_mu(x - mu)) and the
// workgroup's own spinors are staged in LDS: the slice couplings read their
// partners psi(s -+ 1) from there, so only the 4d hops gather through the
// vector-memory path.  Each output is written once, at its own slice.
constexpr int CF_WG = 256;
constexpr int CF_SITES_MAX = 16;

template <typename T>
__global__ void __launch_bounds__(CF_WG) cf_kernel(FineGeom g, CfCoef k, const C2<T>* U, const C2<T>* in, C2<T>* out) {
    constexpr uint32_t CB = sizeof(C2<T>);
    __shared__ C2<T> lds[CF_SITES_MAX * 8 * LPAD];
    __shared__ C2<T> spin[12 * CF_WG];  // [c][work-item]
    const int Ls = g.Ls, m = Ls - 1;
    const int lb = logical_block(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x;
    const int j = tid / Ls, s = tid - (tid / Ls) * Ls;
    const int lsite = lb * k.sites + j;
    const bool active = (j < k.sites) && (lsite < g.V4);
    FieldRefs f;
    f.cstride = (uint32_t)g.N5 * CB;
    f.in = make_rsrc(in, 12u * f.cstride);
    f.out = make_rsrc(out, 12u * f.cstride);
    f.U = make_rsrc(U, (uint32_t)g.V4 * 36u * CB);
    const Site st = traverse(g, active ? lsite : 0);
    const Nbrs<T> n = neighbours<T>(g, st);
    const uint32_t o0 = (uint32_t)(st.site * Ls + s) * CB;
    C2<T> v[12];
    if (active) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            v[c] = Buf<T>::ld(f.in, o0, (uint32_t)c * f.cstride);
            spin[c * CF_WG + tid] = v[c];
        }
        // matrix d < 4: U_d(x); d >= 4: U_(d-4)(x - (d-4)); the site's Ls work-items share the loads
        for (int q = s; q < 72; q += Ls) {
            const int d = q / 9, e = q - 9 * (q / 9);
            // a select, not n.b[d - 4]: a run-time index would put the neighbour table in scratch
            const int src = (d < 4) ? st.site : (d == 4 ? n.b[0] : d == 5 ? n.b[1] : d == 6 ? n.b[2] : n.b[3]);
            lds[(j * 8 + d) * LPAD + e] = Buf<T>::ld(f.U, (uint32_t)(src * 36 + (d & 3) * 9 + e) * CB, 0u);
        }
    }
    __syncthreads();
    if (!active) return;
    // D_W(-M5) psi_s: diagonal 4 - M5, then the eight 4d hops
    C2<T> acc[12];
    const T wd = (T)k.wdiag;
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = cscale<T>(wd, v[c]);
    const C2<T>* lnk = lds + j * 8 * LPAD;
    hop_pair_lds<T, 0>(f, n, Ls, s, lnk, acc);
    hop_pair_lds<T, 1>(f, n, Ls, s, lnk, acc);
    hop_pair_lds<T, 2>(f, n, Ls, s, lnk, acc);
    hop_pair_lds<T, 3>(f, n, Ls, s, lnk, acc);
    // sigma_s gamma5 D_W psi_s + [s = m] R gamma5 psi_s + couplings to the neighbouring slices
    const T sg = (T)k.sigma[s];
    const T rr = (s == m) ? (T)k.R : (T)0;
    const T cd = (T)k.cdn[s], cu = (T)k.cup[s];
    const int td = (s > 0) ? tid - 1 : tid, tu = (s < m) ? tid + 1 : tid;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const T g5 = (c < 6) ? (T)1 : (T)-1;
        C2<T> o = cscale<T>(g5 * sg, acc[c]);
        axpy<T>(g5 * rr, v[c], o);
        axpy<T>(cd, spin[c * CF_WG + td], o);
        axpy<T>(cu, spin[c * CF_WG + tu], o);
        Buf<T>::st_nt(o, f.out, o0, (uint32_t)c * f.cstride);
    }
}

// Continued-fraction operator on 2^4 parity tiles (even extents, Ls <= 16): the
// tile scheme of the domain wall kernels.  A workgroup holds one tile, 16 sites
// x Ls slices; work-item (p, kk) handles the site whose position in the tile is
// the bit pattern p and slice kk (W = 1), or slices 2 kk, 2 kk + 1 with every
// field access one 16-byte load or store of two FP32 complex numbers (W = 2,
// FP32, even Ls).  The tile's spinors are staged in LDS; in each direction one
// of the two hops stays in the tile and reads its partner there, the other is
// gathered from the field, two directions ahead.  The links are staged already
// oriented (U_mu(x) forward, U_mu(x - mu)^dag backward), so the hop direction is
// a run-time sign.  The slice couplings read psi(s -+ 1) of the same site from
// the staged tile.  The output lands at its own slice.
constexpr int CFT_LS = 16;

template <typename T, int W> struct CfWord;
template <typename T> struct CfWord<T, 1> {
    typedef C2<T> type;
    static __device__ __forceinline__ type ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        return Buf<T>::ld(r, voff, soff);
    }
    static __device__ __forceinline__ C2<T> slice(type w, int) { return w; }
};
template <> struct CfWord<float, 2> {
    typedef float4 type;
    static __device__ __forceinline__ type ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        return ld_pair(r, voff, soff);
    }
    static __device__ __forceinline__ C2<float> slice(type w, int i) {
        return i == 0 ? mk<float>(w.x, w.y) : mk<float>(w.z, w.w);
    }
};

template <typename T, int W>
__global__ void __launch_bounds__(16 * CFT_LS / W) __attribute__((amdgpu_waves_per_eu(2))) cf_tile_kernel(FineGeom g, TileGeom tg, CfCoef k,
                                                                  const C2<T>* U, const C2<T>* in, C2<T>* out) {
    static_assert(W == 1 || sizeof(T) == 4, "paired slices are FP32 only");
    typedef CfWord<T, W> Wd;
    typedef typename Wd::type Word;
    constexpr int NKMAX = CFT_LS / W;
    constexpr uint32_t CB = sizeof(C2<T>);
    __shared__ Word spin[12 * 16 * NKMAX];  // [c][pattern][kk]
    __shared__ C2<T> lds[16 * 8 * LPAD];     // [pattern][matrix][entry]
    const int Ls = g.Ls, m = Ls - 1, NK = Ls / W;
    const int p = threadIdx.x / NK, kk = threadIdx.x - (threadIdx.x / NK) * NK;
    const int s0 = W * kk;
    const int tile = logical_block(blockIdx.x, gridDim.x);
    const Site tt = traverse(tg.t, tile);
    Site st;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) st.x[mu] = 2 * tt.x[mu] + ((p >> mu) & 1);
    st.site = ((st.x[3] * g.L[2] + st.x[2]) * g.L[1] + st.x[1]) * g.L[0] + st.x[0];
    const Nbrs<T> n = neighbours<T>(g, st);
    FieldRefs f;
    f.cstride = (uint32_t)g.N5 * CB;
    f.in = make_rsrc(in, 12u * f.cstride);
    f.out = make_rsrc(out, 12u * f.cstride);
    f.U = make_rsrc(U, (uint32_t)g.V4 * 36u * CB);
    for (int e = kk; e < 9; e += NK) {
        const int r = e / 3, cc = e - 3 * (e / 3);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const bool up = (p >> mu) & 1;
            const C2<T> uf = Buf<T>::ld(f.U, (uint32_t)(st.site * 36 + mu * 9 + e) * CB, 0u);
            const C2<T> ub = Buf<T>::ld(f.U, (uint32_t)(n.b[mu] * 36 + mu * 9 + e) * CB, 0u);
            lds[(p * 8 + 2 * mu + (up ? 1 : 0)) * LPAD + e] = uf;
            lds[(p * 8 + 2 * mu + (up ? 0 : 1)) * LPAD + cc * 3 + r] = mk<T>(ub.x, -ub.y);
        }
    }
    C2<T> acc[W][12];
    {
        // D_W(-M5) psi starts with the diagonal 4 - M5; the own spinor is read
        // back from the staged tile for the slice terms at the end
        const uint32_t o0 = (uint32_t)(st.site * Ls + s0) * CB;
        const T wd = (T)k.wdiag;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const Word w = Wd::ld(f.in, o0, (uint32_t)c * f.cstride);
            spin[(c * 16 + p) * NKMAX + kk] = w;
#pragma unroll
            for (int i = 0; i < W; ++i) acc[i][c] = cscale<T>(wd, Wd::slice(w, i));
        }
    }
#define HDCR_CFT_GATHER(MU, DST)                                                                              \
    {                                                                                                         \
        const uint32_t noff = (uint32_t)((((p >> MU) & 1) ? n.f[MU] : n.b[MU]) * Ls + s0) * CB;              \
        _Pragma("unroll") for (int c = 0; c < 12; ++c) DST[c] = Wd::ld(f.in, noff, (uint32_t)c * f.cstride);  \
    }
    Word nx0[12], nx1[12];
    HDCR_CFT_GATHER(0, nx0)
    HDCR_CFT_GATHER(1, nx1)
    __syncthreads();
    const C2<T>* lnk = lds + p * 8 * LPAD;
    // the eight 4d hops
#define HDCR_CFT_HOPS(MU, NX)                                                                                 \
    {                                                                                                         \
        const bool up = (p >> MU) & 1;                                                                        \
        const T sg_in = up ? (T)-1 : (T)1;                                                                    \
        const int q = p ^ (1 << MU);                                                                          \
        C2<T> mm[9], v[12];                                                                                   \
        _Pragma("unroll") for (int e = 0; e < 9; ++e) mm[e] = lnk[(2 * MU) * LPAD + e];                       \
        _Pragma("unroll") for (int i = 0; i < W; ++i) {                                                       \
            _Pragma("unroll") for (int c = 0; c < 12; ++c) v[c] = Wd::slice(spin[(c * 16 + q) * NKMAX + kk], i); \
            hop_core_rt<T, MU>(v, mm, sg_in, up ? n.cb[MU] : n.cf[MU], acc[i]);                              \
        }                                                                                                     \
        _Pragma("unroll") for (int e = 0; e < 9; ++e) mm[e] = lnk[(2 * MU + 1) * LPAD + e];                   \
        _Pragma("unroll") for (int i = 0; i < W; ++i) {                                                       \
            _Pragma("unroll") for (int c = 0; c < 12; ++c) v[c] = Wd::slice(NX[c], i);                        \
            hop_core_rt<T, MU>(v, mm, -sg_in, up ? n.cf[MU] : n.cb[MU], acc[i]);                             \
        }                                                                                                     \
    }
    HDCR_CFT_HOPS(0, nx0)
    __builtin_amdgcn_sched_barrier(0);
    HDCR_CFT_GATHER(2, nx0)
    __builtin_amdgcn_sched_barrier(0);
    HDCR_CFT_HOPS(1, nx1)
    __builtin_amdgcn_sched_barrier(0);
    HDCR_CFT_GATHER(3, nx1)
    __builtin_amdgcn_sched_barrier(0);
    HDCR_CFT_HOPS(2, nx0)
    HDCR_CFT_HOPS(3, nx1)
#undef HDCR_CFT_HOPS
#undef HDCR_CFT_GATHER
    // sigma_s gamma5 D_W psi_s + [s = m] R gamma5 psi_s + couplings to slices s -+ 1
    // of the same site, from the staged tile (a coupling of 0 at s = 0 and s = m)
    const int kd = kk > 0 ? kk - 1 : kk, ku = kk < NK - 1 ? kk + 1 : kk;
    const uint32_t oo = (uint32_t)(st.site * Ls + s0) * CB;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        const T g5 = (c < 6) ? (T)1 : (T)-1;
        const Word wown = spin[(c * 16 + p) * NKMAX + kk];
        const Word wdn = spin[(c * 16 + p) * NKMAX + kd], wup = spin[(c * 16 + p) * NKMAX + ku];
        C2<T> o[W];
#pragma unroll
        for (int i = 0; i < W; ++i) {
            const int si = s0 + i;
            // slice si - 1: the other half of this word, else the last slice of the word below
            const C2<T> dn = (i > 0) ? Wd::slice(wown, i - 1) : Wd::slice(wdn, W - 1);
            const C2<T> upn = (i < W - 1) ? Wd::slice(wown, i + 1) : Wd::slice(wup, 0);
            o[i] = cscale<T>(g5 * (T)k.sigma[si], acc[i][c]);
            axpy<T>(g5 * ((si == m) ? (T)k.R : (T)0), Wd::slice(wown, i), o[i]);
            axpy<T>((T)k.cdn[si], dn, o[i]);
            axpy<T>((T)k.cup[si], upn, o[i]);
        }
        if constexpr (W == 2)
            st_pair_nt(make_float4(o[0].x, o[0].y, o[1].x, o[1].y), f.out, oo, (uint32_t)c * f.cstride);
        else
            Buf<T>::st_nt(o[0], f.out, oo, (uint32_t)c * f.cstride);
    }
}

}  // namespace

template <typename T>
void launch_cf(const FineGeom& g, const CfCoef& k, const C2<T>* U, const C2<T>* in, C2<T>* out, hipStream_t s) {
    // parity tiles for even extents and Ls <= 16 (paired slices in FP32 with even
    // Ls; tune.dslash_variant 4: one slice per work-item), else one work-item
    // per 5d site (tune.dslash_variant 2 forces it)
    const bool tiles = g.variant != 2 && g.Ls <= CFT_LS && g.L[0] % 2 == 0 && g.L[1] % 2 == 0 && g.L[2] % 2 == 0 &&
                       g.L[3] % 2 == 0;
    if (tiles) {
        const TileGeom tg = tile_geom(g);
        if constexpr (sizeof(T) == 4) {
            if (g.Ls % 2 == 0 && g.variant != 4) {
                hipLaunchKernelGGL((cf_tile_kernel<float, 2>), dim3(tg.t.V4), dim3(16 * g.Ls / 2), 0, s, g, tg, k, U,
                                   in, out);
                return;
            }
        }
        hipLaunchKernelGGL((cf_tile_kernel<T, 1>), dim3(tg.t.V4), dim3(16 * g.Ls), 0, s, g, tg, k, U, in, out);
        return;
    }
    const int blocks = (g.V4 + k.sites - 1) / k.sites;
    hipLaunchKernelGGL((cf_kernel<T>), dim3(blocks), dim3(k.sites * g.Ls), 0, s, g, k, U, in, out);
}

template void launch_cf<double>(const FineGeom&, const CfCoef&, const double2*, const double2*, double2*, hipStream_t);
template void launch_cf<float>(const FineGeom&, const CfCoef&, const float2*, const float2*, float2*, hipStream_t);

template void launch_dslash<double>(const FineGeom&, const double2*, const double2*, double2*, hipStream_t);
template void launch_dslash<float>(const FineGeom&, const float2*, const float2*, float2*, hipStream_t);
template void launch_dslash_epi<double>(const FineGeom&, const double2*, const double2*, double2*, const Epi<double>&,
                                        hipStream_t);
template void launch_dslash_epi<float>(const FineGeom&, const float2*, const float2*, float2*, const Epi<float>&,
                                       hipStream_t);

}  // namespace hdcr
