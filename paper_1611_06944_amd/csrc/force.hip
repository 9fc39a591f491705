// Gauge-link gradient and su(3) force of L = Re <chi, H psi>, H = Gamma5 D_dwf
// (Sec. 3), for gfx950.  This is the HMC fermion force that the abstract,
// Sec. 1 and Sec. 5 name as the setting the solver is meant for.
//
// U_mu(x) enters H only through the forward mu hop at x and the backward mu
// hop at x + mu.  With chi~(x,s) = chi(x, Ls-1-s) (the R5 reflection of
// Gamma5 = gamma5 R5, whose gamma5 is absorbed below) the gradient
//   W_mu(x) = dL/dRe U_mu(x) + i dL/dIm U_mu(x)
// is -b/2 b_mu(x) times the sum over s of two colour outer products traced
// over spin (b the Cayley scale of the 4d part), b_mu(x) = bc[mu] on the link
// that crosses the lattice boundary.
// In the chiral basis, with v = (v_u, v_d) (upper and lower spin pairs),
// g_mu = [[0, w_mu], [w_mu^dag, 0]] and the half spinors P+-_mu v = v_u +- w_mu v_d,
// both products take one form, local (x) neighbour^*:
//   first  term  sum_j [P+_mu chi~(x,s)]_j  (x)  [P-_mu psi(x+mu,s)]_j^*
//   second term  sum_j [P+_mu psi(x,s)]_j   (x)  [P-_mu chi~(x+mu,s)]_j^*
// so one code path computes either term with the roles of chi and psi
// swapped.  The force is T_mu(x) = P_TA(U_mu(x) W_mu(x)^dag) (traceless
// anti-Hermitian part): under U -> exp(eps X) U, dL/deps = Re tr(X T).
//
// Work split: a workgroup owns SITES = 64/R consecutive 4d sites of the fine
// stencil's traversal order (t slabs inside z, so the z and t neighbours of a
// site are re-read from the XCD's L2) and runs 2*MS wavefronts over them.
// Wave w computes term (w & 1) for the direction group (w >> 1) of 4/MS
// directions; each lane is one (site, s-lane) pair and owns load units of P
// adjacent fifth-dimension slices (P = 2: two FP32 complex numbers per 16-byte
// load).  Per direction the R lanes of a site sum their partial outer
// products, with DPP adds inside a 16-lane row (FP32) or through a transpose
// in LDS (FP64, where a DPP move of a double costs two moves plus the add);
// the two terms meet in LDS and the whole workgroup then forms W and T per
// (site, mu).
#include <type_traits>

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

// Load unit: P consecutive fifth-dimension slices of the 12 components at one
// 4d site, one buffer load per component (P = 2: two FP32 complex numbers in
// one 16-byte load).
template <typename T, int P>
__device__ __forceinline__ void load_unit(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t cstride,
                                          C2<T> (&v)[P][12]) {
    if constexpr (P == 1) {
#pragma unroll
        for (int c = 0; c < 12; ++c) v[0][c] = Buf<T>::ld(r, off, (uint32_t)c * cstride);
    } else {
        static_assert(P == 2 && sizeof(T) == 4, "paired slices are loaded for FP32 only");
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const float4 q = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, c * cstride, 0));
            v[0][c] = mk<float>(q.x, q.y);
            v[1][c] = mk<float>(q.z, q.w);
        }
    }
}

// Outer products of one unit in direction MU.  The unit at s0 = P*k pairs the
// local slices with the neighbour's in reverse order: one of the two fields is
// read at the reflected slices Ls-P-s0 .. Ls-1-s0 (chi~), so local slice p
// meets neighbour slice P-1-p in both terms.
template <typename T, int P, int MU>
__device__ __forceinline__ void unit_products(const C2<T> (&v)[P][12], const C2<T> (&n)[P][12], C2<T> (&w)[9]) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
        C2<T> a[6], b[6];
        half_spinor<T, 1, MU>(v[p], a);
        half_spinor<T, -1, MU>(n[P - 1 - p], b);
        outer_acc<T>(a, b, w);
    }
}

template <int N> using IC = std::integral_constant<int, N>;

template <typename T, int R, int MS, int P, bool LDSRED>
__global__ void __launch_bounds__(128 * MS) link_force_kernel(FineGeom g, const C2<T>* U, const C2<T>* chi,
                                                                const C2<T>* psi, C2<T>* Wout, C2<T>* Tout) {
    static_assert(R >= 2 && R <= 16, "2 <= R <= 16 lanes per site");
    constexpr int SITES = 64 / R;
    constexpr int NT = 128 * MS;
    constexpr uint32_t CB = sizeof(C2<T>);
    // RSTRIDE: row stride of the per-wave transpose buffer (one complex of
    // padding keeps the nine rows on distinct LDS banks)
    constexpr int RSTRIDE = 65;
    __shared__ C2<T> red[2][SITES * 4 * 9];
    __shared__ C2<T> tbuf[LDSRED ? 2 * MS : 1][LDSRED ? 9 * RSTRIDE : 1];

    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int term = wave & 1;  // 0: chi~ local, psi neighbour;  1: psi local, chi~ neighbour
    const int mg = wave >> 1;   // direction group: directions mg*(4/MS) .. (mg+1)*(4/MS) - 1
    const int lane = threadIdx.x & 63;
    // logical sites l0 .. l0 + SITES-1 in the stencil's traversal order
    const int l0 = logical_block(blockIdx.x, gridDim.x) * SITES;
    const int lsite = lane / R;
    // past the last site a group repeats the last site and stores nothing
    const Site st = traverse(g, min(l0 + lsite, g.V4 - 1));
    const int site = st.site;
    const int sl = lane % R;

    int nb[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) nb[mu] = site + (st.x[mu] == g.L[mu] - 1 ? -g.wrap[mu] : g.stride[mu]);

    const uint32_t cstride = (uint32_t)g.N5 * CB;
    const uint32_t fbytes = 12u * cstride;
    const __amdgpu_buffer_rsrc_t rl = make_rsrc(term ? psi : chi, fbytes);
    const __amdgpu_buffer_rsrc_t rn = make_rsrc(term ? chi : psi, fbytes);
    // units of P slices per lane group of R lanes
    const int nunits = (g.Ls / P + R - 1) / R;
    // slice offsets of unit k: the local field and the neighbour's
    auto s_local = [&](int s0) { return term ? s0 : g.Ls - P - s0; };
    auto s_nbr = [&](int s0) { return term ? g.Ls - P - s0 : s0; };

    // sum of the R lanes' partial products of one direction, into red[term]
    auto finish = [&](int mu, C2<T> (&w)[9]) {
        C2<T>* dst = &red[term][(lsite * 4 + mu) * 9];
        if constexpr (LDSRED) {
            // transpose through LDS: each lane writes its nine entries, then
            // lane sl of a group adds entry sl (and sl + R, ...) over the
            // group's lanes in lane order
            C2<T>* tb = tbuf[wave];
#pragma unroll
            for (int e = 0; e < 9; ++e) tb[e * RSTRIDE + lane] = w[e];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            const int g0 = lane - sl;
            for (int e = sl; e < 9; e += R) {
                C2<T> acc = tb[e * RSTRIDE + g0];
#pragma unroll
                for (int k = 1; k < R; ++k) acc = cadd<T>(acc, tb[e * RSTRIDE + g0 + k]);
                dst[e] = acc;
            }
            // the next direction overwrites the buffer only after every lane has read it
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        } else {
#pragma unroll
            for (int e = 0; e < 9; ++e) w[e] = mk<T>(group_sum<R>(w[e].x), group_sum<R>(w[e].y));
            if (sl == 0) {
#pragma unroll
                for (int e = 0; e < 9; ++e) dst[e] = w[e];
            }
        }
    };
    auto for_dirs = [&](auto&& body) {
        if constexpr (MS == 1) {
            body(IC<0>{});
            body(IC<1>{});
            body(IC<2>{});
            body(IC<3>{});
        } else if constexpr (MS == 2) {
            if (mg == 0) {
                body(IC<0>{});
                body(IC<1>{});
            } else {
                body(IC<2>{});
                body(IC<3>{});
            }
        } else {
            if (mg == 0)
                body(IC<0>{});
            else if (mg == 1)
                body(IC<1>{});
            else if (mg == 2)
                body(IC<2>{});
            else
                body(IC<3>{});
        }
    };

    if (nunits == 1) {
        // one unit per lane: the local slices stay in registers across directions
        const int s0 = sl * P;
        const bool on = s0 < g.Ls;
        C2<T> v[P][12];
        if (on) load_unit<T, P>(rl, (uint32_t)(site * g.Ls + s_local(s0)) * CB, cstride, v);
        for_dirs([&](auto MUc) {
            constexpr int MU = decltype(MUc)::value;
            C2<T> w[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) w[e] = mk<T>(0, 0);
            if (on) {
                C2<T> n[P][12];
                load_unit<T, P>(rn, (uint32_t)(nb[MU] * g.Ls + s_nbr(s0)) * CB, cstride, n);
                unit_products<T, P, MU>(v, n, w);
            }
            finish(MU, w);
        });
    } else {
        for_dirs([&](auto MUc) {
            constexpr int MU = decltype(MUc)::value;
            C2<T> w[9];
#pragma unroll
            for (int e = 0; e < 9; ++e) w[e] = mk<T>(0, 0);
            for (int k = 0; k < nunits; ++k) {
                const int s0 = (sl + R * k) * P;
                if (s0 < g.Ls) {
                    C2<T> v[P][12], n[P][12];
                    load_unit<T, P>(rl, (uint32_t)(site * g.Ls + s_local(s0)) * CB, cstride, v);
                    load_unit<T, P>(rn, (uint32_t)(nb[MU] * g.Ls + s_nbr(s0)) * CB, cstride, n);
                    unit_products<T, P, MU>(v, n, w);
                }
            }
            finish(MU, w);
        });
    }
    __syncthreads();

    // W = -b/2 b_mu (sum of both terms), T = P_TA(U W^dag), one (site, mu) per work-item
    for (int p = threadIdx.x; p < SITES * 4; p += NT) {
        const int l = l0 + (p >> 2), mu = p & 3;
        if (l >= g.V4) break;
        const Site sp = traverse(g, l);
        const int xm = mu == 0 ? sp.x[0] : mu == 1 ? sp.x[1] : mu == 2 ? sp.x[2] : sp.x[3];
        const int ext = mu == 0 ? g.L[0] : mu == 1 ? g.L[1] : mu == 2 ? g.L[2] : g.L[3];
        const int bc = mu == 0 ? g.bc[0] : mu == 1 ? g.bc[1] : mu == 2 ? g.bc[2] : g.bc[3];
        const T f = (xm == ext - 1) ? (T)g.hop * (T)bc : (T)g.hop;
        const size_t base = ((size_t)sp.site * 4 + mu) * 9;
        C2<T> W[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) W[e] = cscale<T>(f, cadd<T>(red[0][p * 9 + e], red[1][p * 9 + e]));
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

template <typename T, int R, int MS, int P, bool LDSRED>
void launch_r(const FineGeom& g, const C2<T>* U, const C2<T>* chi, const C2<T>* psi, C2<T>* W, C2<T>* T_,
              hipStream_t s) {
    constexpr int SITES = 64 / R;
    const int nwg = (g.V4 + SITES - 1) / SITES;
    hipLaunchKernelGGL((link_force_kernel<T, R, MS, P, LDSRED>), dim3(nwg), dim3(128 * MS), 0, s, g, U, chi, psi, W,
                       T_);
}

template <typename T, int R, int P>
void launch_ms(const FineGeom& g, const ForceShape& f, const C2<T>* U, const C2<T>* chi, const C2<T>* psi, C2<T>* W,
               C2<T>* T_, hipStream_t s) {
    if (f.ms == 1) {
        if (f.lds_sum)
            launch_r<T, R, 1, P, true>(g, U, chi, psi, W, T_, s);
        else
            launch_r<T, R, 1, P, false>(g, U, chi, psi, W, T_, s);
    } else {
        if (f.lds_sum)
            launch_r<T, R, 2, P, true>(g, U, chi, psi, W, T_, s);
        else
            launch_r<T, R, 2, P, false>(g, U, chi, psi, W, T_, s);
    }
}

template <typename T, int P>
void launch_p(const FineGeom& g, const ForceShape& f, const C2<T>* U, const C2<T>* chi, const C2<T>* psi, C2<T>* W,
              C2<T>* T_, hipStream_t s) {
    switch (f.r) {
        case 2: launch_ms<T, 2, P>(g, f, U, chi, psi, W, T_, s); break;
        case 4: launch_ms<T, 4, P>(g, f, U, chi, psi, W, T_, s); break;
        case 8: launch_ms<T, 8, P>(g, f, U, chi, psi, W, T_, s); break;
        default: launch_ms<T, 16, P>(g, f, U, chi, psi, W, T_, s); break;
    }
}

}  // namespace

ForceShape choose_force_shape(const FineGeom& g, int dtype_bytes, int r, int ms, int p, int lds_sum) {
    ForceShape f;
    // slices per load: two FP32 complex numbers per 16-byte load when Ls is even
    if (p <= 0) p = (dtype_bytes == 8 && g.Ls % 2 == 0) ? 2 : 1;
    // lanes per site: one load unit per lane where Ls allows (a power of two
    // between 2 and 16)
    if (r <= 0) {
        const int units = g.Ls / p;
        r = 2;
        while (r * 2 <= units && r * 2 <= 16) r *= 2;
    }
    // directions per wave: two wave groups with paired FP32 loads (measured
    // best at 16^4 x 16), one otherwise
    if (ms <= 0) ms = (p == 2) ? 2 : 1;
    // cross-lane sums: through LDS for FP64 (a DPP move of a double takes two
    // moves and the add its own instruction), DPP adds for FP32
    if (lds_sum < 0) lds_sum = (dtype_bytes == 16) ? 1 : 0;
    f.r = r;
    f.ms = ms;
    f.p = p;
    f.lds_sum = lds_sum != 0;
    return f;
}

bool force_shape_ok(const FineGeom& g, int dtype_bytes, const ForceShape& f) {
    const bool r_ok = (f.r == 2 || f.r == 4 || f.r == 8 || f.r == 16);
    const bool ms_ok = (f.ms == 1 || f.ms == 2);
    const bool p_ok = f.p == 1 || (f.p == 2 && dtype_bytes == 8 && g.Ls % 2 == 0);
    return r_ok && ms_ok && p_ok;
}

template <typename T>
void launch_link_force(const FineGeom& g, const ForceShape& f, const C2<T>* U, const C2<T>* chi, const C2<T>* psi,
                       C2<T>* W, C2<T>* T_, hipStream_t s) {
    if constexpr (std::is_same<T, float>::value) {
        if (f.p == 2) {
            launch_p<float, 2>(g, f, U, chi, psi, W, T_, s);
            return;
        }
    }
    launch_p<T, 1>(g, f, U, chi, psi, W, T_, s);
}

template void launch_link_force<double>(const FineGeom&, const ForceShape&, const double2*, const double2*,
                                        const double2*, double2*, double2*, hipStream_t);
template void launch_link_force<float>(const FineGeom&, const ForceShape&, const float2*, const float2*,
                                       const float2*, float2*, float2*, hipStream_t);

}  // namespace hdcr
