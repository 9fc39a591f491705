// Gauge-link gradient and su(3) force of L = Re <chi, H psi>, H = Gamma5 D_dwf
// (Sec. 3), for gfx950.  This is the HMC fermion force that the abstract,
// Sec. 1 and Sec. 5 name as the setting the solver is meant for.
//
// U_mu(x) enters H only through the forward mu hop at x and the backward mu
// hop at x + mu.  With chi~(x,s) = chi(x, Ls-1-s) (the R5 reflection of
// Gamma5 = gamma5 R5, whose gamma5 is absorbed below) the gradient
//   W_mu(x) = dL/dRe U_mu(x) + i dL/dIm U_mu(x)
// is -1/2 b_mu(x) times the sum over s of two colour outer products traced
// over spin, b_mu(x) = bc[mu] on the link that crosses the lattice boundary.
// In the chiral basis, with v = (v_u, v_d) (upper and lower spin pairs),
// g_mu = [[0, w_mu], [w_mu^dag, 0]] and the half spinors P+-_mu v = v_u +- w_mu v_d,
// both products take one form, local (x) neighbour^*:
//   first  term  sum_j [P+_mu chi~(x,s)]_j  (x)  [P-_mu psi(x+mu,s)]_j^*
//   second term  sum_j [P+_mu psi(x,s)]_j   (x)  [P-_mu chi~(x+mu,s)]_j^*
// so one code path computes either term with the roles of chi and psi
// swapped.  The force is T_mu(x) = P_TA(U_mu(x) W_mu(x)^dag) (traceless
// anti-Hermitian part): under U -> exp(eps X) U, dL/deps = Re tr(X T).
//
// Work split: a workgroup owns SITES = 64/R consecutive 4d sites and runs
// 2*MS wavefronts over them.  Wave w computes term (w & 1) for the MU group
// (w >> 1) of 4/MS directions; each of its lanes is one (site, s-lane) pair and
// walks s = s-lane, s-lane + R, ... < Ls.  The R lanes of a site sum their
// partial outer products with DPP moves inside a 16-lane row, the two terms
// meet in LDS, and the whole workgroup then forms W and T per (site, mu).
#include "internal.h"

namespace hdcr {

namespace {

// h = v_u + SG w_mu v_d for the 12 components v (c = spin*3 + colour); h holds
// the two resulting spins, h[j*3 + colour].  w_x = -i sigma_x, w_y = -i sigma_y,
// w_z = -i sigma_z, w_t = 1.
template <typename T, int SG, int MU>
__device__ __forceinline__ void half_spinor(const C2<T> (&v)[12], C2<T> (&h)[6]) {
    const T sg = (T)SG;
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        const C2<T> u0 = v[col], u1 = v[3 + col], d0 = v[6 + col], d1 = v[9 + col];
        if constexpr (MU == 0) {         // w_x d = (-i d1, -i d0)
            h[col] = mk<T>(fma(sg, d1.y, u0.x), fma(-sg, d1.x, u0.y));
            h[3 + col] = mk<T>(fma(sg, d0.y, u1.x), fma(-sg, d0.x, u1.y));
        } else if constexpr (MU == 1) {  // w_y d = (-d1, d0)
            h[col] = mk<T>(fma(-sg, d1.x, u0.x), fma(-sg, d1.y, u0.y));
            h[3 + col] = mk<T>(fma(sg, d0.x, u1.x), fma(sg, d0.y, u1.y));
        } else if constexpr (MU == 2) {  // w_z d = (-i d0, i d1)
            h[col] = mk<T>(fma(sg, d0.y, u0.x), fma(-sg, d0.x, u0.y));
            h[3 + col] = mk<T>(fma(-sg, d1.y, u1.x), fma(sg, d1.x, u1.y));
        } else {                         // w_t d = (d0, d1)
            h[col] = mk<T>(fma(sg, d0.x, u0.x), fma(sg, d0.y, u0.y));
            h[3 + col] = mk<T>(fma(sg, d1.x, u1.x), fma(sg, d1.y, u1.y));
        }
    }
}

// w[c][d] += sum_j a_j[c] conj(b_j[d])
template <typename T>
__device__ __forceinline__ void outer_acc(const C2<T> (&a)[6], const C2<T> (&b)[6], C2<T> (&w)[9]) {
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const C2<T> x = a[j * 3 + c], y = b[j * 3 + d];
                C2<T>& o = w[c * 3 + d];
                o.x = fma(x.x, y.x, o.x);
                o.x = fma(x.y, y.y, o.x);
                o.y = fma(x.y, y.x, o.y);
                o.y = fma(-x.x, y.y, o.y);
            }
}

// DPP lane moves inside a row of 16 lanes: quad_perm [1,0,3,2] (0xB1),
// quad_perm [2,3,0,1] (0x4E), row_half_mirror (0x141), row_mirror (0x140).
template <int CTRL> __device__ __forceinline__ float lane_mov(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ __forceinline__ double lane_mov(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Sum over the R aligned consecutive lanes of a group (R a power of two <= 16):
// after step k every lane of an aligned group of 2^k lanes holds the group's
// sum, and each move pairs a lane with one in the other half of the next
// larger group.  The summation order is fixed.
template <int R, typename T> __device__ __forceinline__ T group_sum(T v) {
    static_assert(R == 1 || R == 2 || R == 4 || R == 8 || R == 16, "R");
    if constexpr (R >= 2) v += lane_mov<0xB1>(v);
    if constexpr (R >= 4) v += lane_mov<0x4E>(v);
    if constexpr (R >= 8) v += lane_mov<0x141>(v);
    if constexpr (R >= 16) v += lane_mov<0x140>(v);
    return v;
}

// One direction of one term at one s: neighbour components at byte offset on,
// local components v, accumulated into w.
template <typename T, int MU>
__device__ __forceinline__ void link_term(__amdgpu_buffer_rsrc_t rn, uint32_t cstride, uint32_t on,
                                          const C2<T> (&v)[12], C2<T> (&w)[9]) {
    C2<T> n[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) n[c] = Buf<T>::ld(rn, on, (uint32_t)c * cstride);
    C2<T> a[6], b[6];
    half_spinor<T, 1, MU>(v, a);
    half_spinor<T, -1, MU>(n, b);
    outer_acc<T>(a, b, w);
}

template <typename T, int K, int MU, int NM>
__device__ __forceinline__ void dir_step(__amdgpu_buffer_rsrc_t rn, uint32_t cstride, const int (&nb)[4], int Ls,
                                         int sn, const C2<T> (&v)[12], C2<T> (&w)[NM][9]) {
    link_term<T, MU>(rn, cstride, (uint32_t)(nb[MU] * Ls + sn) * (uint32_t)sizeof(C2<T>), v, w[K]);
}

// Workgroup-index remap: hardware dispatch sends workgroup b to XCD b % 8; the
// remap gives each XCD one contiguous range of sites.
__device__ __forceinline__ int xcd_block(int b, int nwg) {
    const int per = nwg / NUM_XCD, rem = nwg % NUM_XCD;
    const int xcd = b % NUM_XCD, local = b / NUM_XCD;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

template <typename T, int R, int MS>
__global__ void __launch_bounds__(128 * MS) link_force_kernel(FineGeom g, const C2<T>* U, const C2<T>* chi,
                                                                const C2<T>* psi, C2<T>* Wout, C2<T>* Tout) {
    constexpr int SITES = 64 / R;
    constexpr int NM = 4 / MS;
    constexpr int NT = 128 * MS;
    constexpr uint32_t CB = sizeof(C2<T>);
    __shared__ C2<T> red[SITES * 4 * 9];

    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int term = wave & 1;  // 0: chi~ local, psi neighbour;  1: psi local, chi~ neighbour
    const int mg = wave >> 1;   // directions mg*NM .. mg*NM + NM-1
    const int lane = threadIdx.x & 63;
    const int site0 = xcd_block(blockIdx.x, gridDim.x) * SITES;
    // past the last site a group repeats the last site and stores nothing
    const int site = min(site0 + lane / R, g.V4 - 1);
    const int sl = lane % R;

    int nb[4];
    {
        int r = site;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const int xm = r % g.L[mu];
            r /= g.L[mu];
            nb[mu] = site + (xm == g.L[mu] - 1 ? -g.wrap[mu] : g.stride[mu]);
        }
    }

    const uint32_t cstride = (uint32_t)g.N5 * CB;
    const uint32_t fbytes = 12u * cstride;
    const __amdgpu_buffer_rsrc_t rl = make_rsrc(term ? psi : chi, fbytes);
    const __amdgpu_buffer_rsrc_t rn = make_rsrc(term ? chi : psi, fbytes);

    C2<T> w[NM][9];
#pragma unroll
    for (int k = 0; k < NM; ++k)
#pragma unroll
        for (int e = 0; e < 9; ++e) w[k][e] = mk<T>(0, 0);

    for (int s = sl; s < g.Ls; s += R) {
        const int sr = g.Ls - 1 - s;
        const int sloc = term ? s : sr, sn = term ? sr : s;
        C2<T> v[12];
        const uint32_t ol = (uint32_t)(site * g.Ls + sloc) * CB;
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = Buf<T>::ld(rl, ol, (uint32_t)c * cstride);
        if constexpr (MS == 1) {
            dir_step<T, 0, 0, NM>(rn, cstride, nb, g.Ls, sn, v, w);
            dir_step<T, 1, 1, NM>(rn, cstride, nb, g.Ls, sn, v, w);
            dir_step<T, 2, 2, NM>(rn, cstride, nb, g.Ls, sn, v, w);
            dir_step<T, 3, 3, NM>(rn, cstride, nb, g.Ls, sn, v, w);
        } else if constexpr (MS == 2) {
            if (mg == 0) {
                dir_step<T, 0, 0, NM>(rn, cstride, nb, g.Ls, sn, v, w);
                dir_step<T, 1, 1, NM>(rn, cstride, nb, g.Ls, sn, v, w);
            } else {
                dir_step<T, 0, 2, NM>(rn, cstride, nb, g.Ls, sn, v, w);
                dir_step<T, 1, 3, NM>(rn, cstride, nb, g.Ls, sn, v, w);
            }
        } else {
            if (mg == 0)
                dir_step<T, 0, 0, NM>(rn, cstride, nb, g.Ls, sn, v, w);
            else if (mg == 1)
                dir_step<T, 0, 1, NM>(rn, cstride, nb, g.Ls, sn, v, w);
            else if (mg == 2)
                dir_step<T, 0, 2, NM>(rn, cstride, nb, g.Ls, sn, v, w);
            else
                dir_step<T, 0, 3, NM>(rn, cstride, nb, g.Ls, sn, v, w);
        }
    }

#pragma unroll
    for (int k = 0; k < NM; ++k)
#pragma unroll
        for (int e = 0; e < 9; ++e) w[k][e] = mk<T>(group_sum<R>(w[k][e].x), group_sum<R>(w[k][e].y));

    // the two terms meet in LDS: term 0 stores, then term 1 adds
    const int slot = (lane / R) * 4 + mg * NM;
    if (term == 0 && sl == 0) {
#pragma unroll
        for (int k = 0; k < NM; ++k)
#pragma unroll
            for (int e = 0; e < 9; ++e) red[(slot + k) * 9 + e] = w[k][e];
    }
    __syncthreads();
    if (term == 1 && sl == 0) {
#pragma unroll
        for (int k = 0; k < NM; ++k)
#pragma unroll
            for (int e = 0; e < 9; ++e) red[(slot + k) * 9 + e] = cadd<T>(red[(slot + k) * 9 + e], w[k][e]);
    }
    __syncthreads();

    // W = -1/2 b (sum), T = P_TA(U W^dag), one (site, mu) per work-item
    for (int p = threadIdx.x; p < SITES * 4; p += NT) {
        const int st = site0 + (p >> 2), mu = p & 3;
        if (st >= g.V4) break;
        const int stride = mu == 0 ? g.stride[0] : mu == 1 ? g.stride[1] : mu == 2 ? g.stride[2] : g.stride[3];
        const int ext = mu == 0 ? g.L[0] : mu == 1 ? g.L[1] : mu == 2 ? g.L[2] : g.L[3];
        const int bc = mu == 0 ? g.bc[0] : mu == 1 ? g.bc[1] : mu == 2 ? g.bc[2] : g.bc[3];
        const bool cross = (st / stride) % ext == ext - 1;
        const T f = cross ? (T)(-0.5) * (T)bc : (T)(-0.5);
        const size_t base = ((size_t)st * 4 + mu) * 9;
        C2<T> W[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) W[e] = cscale<T>(f, red[p * 9 + e]);
        if (Wout) {
#pragma unroll
            for (int e = 0; e < 9; ++e) Wout[base + e] = W[e];
        }
        if (Tout) {
            C2<T> u[9], M[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) u[e] = U[base + e];
            // M[r][c] = sum_k U[r][k] conj(W[c][k])
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    C2<T> acc = mk<T>(0, 0);
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const C2<T> a = u[r * 3 + k], b = W[c * 3 + k];
                        acc.x = fma(a.x, b.x, acc.x);
                        acc.x = fma(a.y, b.y, acc.x);
                        acc.y = fma(a.y, b.x, acc.y);
                        acc.y = fma(-a.x, b.y, acc.y);
                    }
                    M[r * 3 + c] = acc;
                }
            // A = (M - M^dag)/2, T = A - tr(A)/3
            C2<T> A[9];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const C2<T> m = M[r * 3 + c], n = M[c * 3 + r];
                    A[r * 3 + c] = mk<T>((T)0.5 * (m.x - n.x), (T)0.5 * (m.y + n.y));
                }
            const T tri = (A[0].y + A[4].y + A[8].y) / (T)3;
#pragma unroll
            for (int e = 0; e < 9; ++e) {
                C2<T> t = A[e];
                if (e == 0 || e == 4 || e == 8) t = mk<T>((T)0, t.y - tri);
                Tout[base + e] = t;
            }
        }
    }
}

template <typename T, int R, int MS>
void launch_r(const FineGeom& g, const C2<T>* U, const C2<T>* chi, const C2<T>* psi, C2<T>* W, C2<T>* T_,
              hipStream_t s) {
    constexpr int SITES = 64 / R;
    const int nwg = (g.V4 + SITES - 1) / SITES;
    hipLaunchKernelGGL((link_force_kernel<T, R, MS>), dim3(nwg), dim3(128 * MS), 0, s, g, U, chi, psi, W, T_);
}

template <typename T, int R>
void launch_ms(const FineGeom& g, int ms, const C2<T>* U, const C2<T>* chi, const C2<T>* psi, C2<T>* W,
               C2<T>* T_, hipStream_t s) {
    if (ms == 1)
        launch_r<T, R, 1>(g, U, chi, psi, W, T_, s);
    else if (ms == 2)
        launch_r<T, R, 2>(g, U, chi, psi, W, T_, s);
    else
        launch_r<T, R, 4>(g, U, chi, psi, W, T_, s);
}

}  // namespace

ForceShape choose_force_shape(const FineGeom& g, int dtype_bytes, int r, int ms) {
    ForceShape f;
    // lanes per site: a power of two <= min(Ls, 4); at Ls = 16 each lane takes
    // four fifth-dimension slices, so the cross-lane sums are few per product
    if (r <= 0) {
        r = 1;
        while (r * 2 <= g.Ls && r * 2 <= 4) r *= 2;
    }
    // directions per wave: all four need the most registers
    if (ms <= 0) ms = (dtype_bytes == 16) ? 4 : 2;
    f.r = r;
    f.ms = ms;
    return f;
}

bool force_shape_ok(const FineGeom& g, const ForceShape& f) {
    const bool r_ok = (f.r == 1 || f.r == 2 || f.r == 4 || f.r == 8 || f.r == 16) && f.r <= g.Ls;
    const bool ms_ok = (f.ms == 1 || f.ms == 2 || f.ms == 4);
    return r_ok && ms_ok;
}

template <typename T>
void launch_link_force(const FineGeom& g, const ForceShape& f, const C2<T>* U, const C2<T>* chi, const C2<T>* psi,
                       C2<T>* W, C2<T>* T_, hipStream_t s) {
    switch (f.r) {
        case 1: launch_ms<T, 1>(g, f.ms, U, chi, psi, W, T_, s); break;
        case 2: launch_ms<T, 2>(g, f.ms, U, chi, psi, W, T_, s); break;
        case 4: launch_ms<T, 4>(g, f.ms, U, chi, psi, W, T_, s); break;
        case 8: launch_ms<T, 8>(g, f.ms, U, chi, psi, W, T_, s); break;
        default: launch_ms<T, 16>(g, f.ms, U, chi, psi, W, T_, s); break;
    }
}

template void launch_link_force<double>(const FineGeom&, const ForceShape&, const double2*, const double2*,
                                        const double2*, double2*, double2*, hipStream_t);
template void launch_link_force<float>(const FineGeom&, const ForceShape&, const float2*, const float2*,
                                       const float2*, float2*, float2*, hipStream_t);

}  // namespace hdcr
