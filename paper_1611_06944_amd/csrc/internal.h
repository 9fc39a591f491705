// Internal declarations shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/hdcr.h"

namespace hdcr {

// ---------------------------------------------------------------------------
// complex helpers on HIP vector types (re = .x, im = .y)
// ---------------------------------------------------------------------------
template <typename T> struct C2t;
template <> struct C2t<double> { typedef double2 type; };
template <> struct C2t<float> { typedef float2 type; };
template <typename T> using C2 = typename C2t<T>::type;

template <typename T> __host__ __device__ __forceinline__ C2<T> mk(T re, T im) {
    C2<T> r;
    r.x = re;
    r.y = im;
    return r;
}
template <typename T> __device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ C2<T> cscale(T s, C2<T> a) { return mk<T>(s * a.x, s * a.y); }
// a * b
template <typename T> __device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename T> __device__ __forceinline__ C2<T> cjmul(C2<T> a, C2<T> b) {
    return mk<T>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// acc + a * b
template <typename T> __device__ __forceinline__ C2<T> cfma(C2<T> a, C2<T> b, C2<T> acc) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc + conj(a) * b
template <typename T> __device__ __forceinline__ C2<T> cjfma(C2<T> a, C2<T> b, C2<T> acc) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
// i * a, -i * a
template <typename T> __device__ __forceinline__ C2<T> cmuli(C2<T> a) { return mk<T>(-a.y, a.x); }
template <typename T> __device__ __forceinline__ C2<T> cmulmi(C2<T> a) { return mk<T>(a.y, -a.x); }
template <typename T> __device__ __forceinline__ C2<T> cneg(C2<T> a) { return mk<T>(-a.x, -a.y); }

// ---------------------------------------------------------------------------
// buffer addressing: a scalar resource descriptor plus a 32-bit per-lane byte
// offset and a uniform (scalar) byte offset.  Every field kernel addresses its
// arrays this way so that the many component loads of a site share one vector
// address register.  Loads past the descriptor's byte range return zero.
// ---------------------------------------------------------------------------
constexpr int BUF_FLAGS = 0x00020000;  // gfx9 raw-buffer descriptor word 3
constexpr int CPOL_NT = 2;             // cache-policy operand of buffer stores: non-temporal

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, BUF_FLAGS);
}

// 16-byte buffer stores.  A store wider than 8 bytes reads its data registers
// after issue, and a vector instruction that overwrites the first of them right
// behind the store can change what is written (observed on gfx950 as a wrong
// first dword, at random).  The compiler separates the two only for stores
// whose scalar offset is an inline constant, so these helpers fold the scalar
// offset into the per-lane offset and pass 0.
template <int CPOL>
__device__ __forceinline__ void store_b128(__attribute__((ext_vector_type(4))) unsigned v, __amdgpu_buffer_rsrc_t r,
                                           uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b128(v, r, voff + soff, 0, CPOL);
}

template <typename T> struct Buf;
template <> struct Buf<double> {
    static __device__ __forceinline__ double2 ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    }
    static __device__ __forceinline__ void st(double2 v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        store_b128<0>(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), r, voff, soff);
    }
    // store with the non-temporal hint (cache policy bit NT)
    static __device__ __forceinline__ void st_nt(double2 v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        store_b128<CPOL_NT>(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), r, voff, soff);
    }
};
template <> struct Buf<float> {
    static __device__ __forceinline__ float2 ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    }
    static __device__ __forceinline__ void st(float2 v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                              voff, soff, 0);
    }
    static __device__ __forceinline__ void st_nt(float2 v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                              voff, soff, CPOL_NT);
    }
};

// ---------------------------------------------------------------------------
// geometry passed to kernels by value
// ---------------------------------------------------------------------------
struct FineGeom {
    int L[4];
    int Ls;
    int V4;
    int N5;       // V4 * Ls
    int bc[4];
    int stride[4];  // 4d site-index stride of direction mu
    int wrap[4];    // (L[mu] - 1) * stride[mu]
    double diag;    // b (4 - M5) + 1 (5 - M5 for the Shamir kernel b = 1)
    double hop;     // -b/2, the coefficient of a 4d hop
    double mf;
    // traversal order of the stencil kernels:
    // t is cut into slabs of tslab slices, x into xsplit and y into ysplit
    // parts; inside a block the order is x-part, y-part, t, z, so a block is
    // swept along z with a cross-section of (Lx/xsplit)(Ly/ysplit) tslab
    // sites, and its t and z neighbours are a few rows apart; workgroups are
    // remapped so each XCD sweeps one contiguous range of that order.
    int tslab;
    int xsplit;
    int ysplit;
    int variant;  // fine-stencil kernel variant (0 = default choice)
    hdcr_tuning tune;  // the caller's kernel-shape choices (0 = the library's)
};

// number of XCDs (separate L2 caches) that hardware workgroup dispatch
// round-robins over on gfx950
constexpr int NUM_XCD = 8;

// Device side of the stencil traversal (the fine operator and the force
// kernel visit sites in this order).
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

// logical site l -> coordinates, traversal order x-part, y-part, t-in-slab, z,
// x-split, y-split, t-slab
__device__ __forceinline__ Site traverse(const FineGeom& g, int l) {
    Site tr;
    const int xq = g.L[0] / g.xsplit, yq = g.L[1] / g.ysplit;
    const int xi = l % xq;
    l /= xq;
    const int yi = l % yq;
    l /= yq;
    const int ti = l % g.tslab;
    l /= g.tslab;
    tr.x[2] = l % g.L[2];
    l /= g.L[2];
    const int xo = l % g.xsplit;
    l /= g.xsplit;
    const int yo = l % g.ysplit;
    l /= g.ysplit;
    tr.x[0] = xo * xq + xi;
    tr.x[1] = yo * yq + yi;
    tr.x[3] = l * g.tslab + ti;
    tr.site = ((tr.x[3] * g.L[2] + tr.x[2]) * g.L[1] + tr.x[1]) * g.L[0] + tr.x[0];
    return tr;
}

// choose the traversal parameters for a lattice (host)
void choose_traversal(FineGeom& g, int tslab, int ysplit, int xsplit = 1);

FineGeom make_geom(const hdcr_fine_desc* d);

// ---------------------------------------------------------------------------
// error handling
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
const char* last_error_cstr();
int fail(int code, const std::string& msg);

#define HDCR_HIP_CHECK(expr)                                                              \
    do {                                                                                  \
        hipError_t _e = (expr);                                                           \
        if (_e != hipSuccess)                                                             \
            return ::hdcr::fail(HDCR_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

int check_fine_desc(const hdcr_fine_desc* d);
int check_ptr(const void* p, size_t align, const char* name);

// ---------------------------------------------------------------------------
// kernels launched from host code (implemented in the .hip files)
// ---------------------------------------------------------------------------
// out = H in  (fine operator), precision T
template <typename T>
void launch_dslash(const FineGeom& g, const C2<T>* U, const C2<T>* in, C2<T>* out, hipStream_t s);

// Fused epilogue of a stencil launch: out = beta (H in) + sum_{i < ny} g[i] y[i]
// (0 <= ny <= 4).  y[i] is read at the element the work-item writes, before the
// write, so y[i] may be the output buffer itself; it must not be `in`.
template <typename T> struct Epi {
    const C2<T>* y[4];
    T g[4];
    T beta;
    int ny;
};
template <typename T>
void launch_dslash_epi(const FineGeom& g, const C2<T>* U, const C2<T>* in, C2<T>* out, const Epi<T>& e,
                       hipStream_t s);
// out = H in with FP16 field storage: in and out hold (fp16 re, fp16 im) per
// complex entry; links FP32, FP32 arithmetic.  Only Ls = 16 with even extents
// (dslash_h16_ok); returns false otherwise.
bool dslash_h16_ok(const FineGeom& g);
bool launch_dslash_h16(const FineGeom& g, const float2* U, const void* in, void* out, hipStream_t s);
// out = beta H in + sum_i g_i y_i with every field FP16-stored (e.y point at
// FP16 fields; ny 0 to 4), one rounding per output component; out may be one
// of the y_i.  Same conditions as launch_dslash_h16.
bool launch_dslash_h16_epi(const FineGeom& g, const float2* U, const void* in, void* out, const Epi<float>& e,
                           hipStream_t s);

// Continued-fraction form of the overlap operator (Sec. 3) on Ls = m + 1 slices:
//   out_s = sigma_s H_W psi_s + [s = m] R gamma5 psi_s + cdn_s psi_(s-1) + cup_s psi_(s+1),
// H_W = gamma5 D_W(-M5) with D_W's diagonal wdiag = 4 - M5 and the 4d hops of
// FineGeom (coefficient g.hop = -1/2, boundary factors bc).  sites: 4d sites per
// workgroup (sites * Ls <= 256 work-items).
constexpr int CF_MAX_LS = 64;
struct CfCoef {
    double sigma[CF_MAX_LS];
    double cdn[CF_MAX_LS];  // coupling to slice s - 1 (0 at s = 0)
    double cup[CF_MAX_LS];  // coupling to slice s + 1 (0 at s = m)
    double R;
    double wdiag;
    int sites;
};
template <typename T>
void launch_cf(const FineGeom& g, const CfCoef& k, const C2<T>* U, const C2<T>* in, C2<T>* out, hipStream_t s);

// Gauge-link gradient W and su(3) force T of L = Re <chi, H psi> (W or T may be
// null).  Shape: r lanes per 4d site (2, 4, 8 or 16), ms wave groups splitting
// the four directions (1 or 2), p fifth-dimension slices per load (2: FP32
// with even Ls only), lds_sum: cross-lane sums through LDS instead of DPP.
struct ForceShape {
    int r;
    int ms;
    int p;
    bool lds_sum;
};
// r, ms, p <= 0 and lds_sum < 0 select the defaults
ForceShape choose_force_shape(const FineGeom& g, int dtype_bytes, int r, int ms, int p, int lds_sum);
bool force_shape_ok(const FineGeom& g, int dtype_bytes, const ForceShape& f);
template <typename T>
void launch_link_force(const FineGeom& g, const ForceShape& f, const C2<T>* U, const C2<T>* chi, const C2<T>* psi,
                       C2<T>* W, C2<T>* T_, hipStream_t s);

// Reductions: every reduction writes REDUCE_BLOCKS partial sums (as double2)
// into `partials` and a finalize step sums them in fixed order into `result`.
constexpr int REDUCE_BLOCKS = 1024;
constexpr int REDUCE_THREADS = 256;
static_assert((REDUCE_BLOCKS + 1) * 16 <= HDCR_DOT_WORK_BYTES, "dot scratch");

// Workgroup tree reduction of NQ double values per thread; thread 0 of the
// workgroup returns the sums.  Uses LDS, REDUCE_THREADS threads.
template <int NQ>
__device__ __forceinline__ void block_reduce(double (&v)[NQ]) {
    __shared__ double sh[NQ][REDUCE_THREADS];
    const int t = threadIdx.x;
    __syncthreads();  // a previous reduction in the same kernel may still be reading sh
#pragma unroll
    for (int q = 0; q < NQ; ++q) sh[q][t] = v[q];
    __syncthreads();
    for (int w = REDUCE_THREADS / 2; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) sh[q][t] += sh[q][t + w];
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = sh[q][0];
}

template <typename T>
void launch_dot(int64_t n, const C2<T>* x, const C2<T>* y, double2* partials, double2* result, hipStream_t s);
// dst = src, bytes a multiple of 16 (the bandwidth-calibration copy)
void launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
void launch_finalize(const double2* partials, int np, double2* result, hipStream_t s);

}  // namespace hdcr
