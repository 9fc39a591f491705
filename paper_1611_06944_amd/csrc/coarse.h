// Coarse-space geometry and the kernels of the block-projected subspace.
#pragma once

#include "internal.h"

namespace hdcr {

// Blocks of B[mu] 4d sites spanning all of Ls (Sec. 4).  The basis of a block
// is chirally split: phi^{a,+}_k and phi^{a,-}_k lie in the +1 and -1
// eigenspaces of Gamma5 = gamma5 R5, which is block-local.  Such a vector is
// fixed by its values on s < Ls/2:  phi(x, Ls-1-s, spin) = sigma g(spin) phi(x, s, spin)
// with sigma = +-1 the chirality and g = gamma5's diagonal (+1 upper, -1 lower
// spins).  The library stores sqrt(2) * phi on s < Ls/2 only ("compressed"),
// which makes the compressed vectors orthonormal in C^{nhalf} and halves the
// basis memory and traffic.
//
// Compressed index inside a block: i = (comp * bvol + sl) * Lh + s, comp =
// spin*3 + colour, sl = lexicographic site inside the block, s < Lh = Ls/2.
// Basis buffer: [FP64 part][FP32 part], each [a][h][k][i] (h = 0: +, 1: -).
struct CoarseGeom {
    FineGeom f;
    int B[4];    // block extents
    int C[4];    // coarse extents
    int Nc;      // coarse sites
    int bvol;    // 4d sites per block
    int nvec;    // vectors per chirality
    int Nb;      // 2 * nvec
    int Lh;      // Ls / 2
    int nhalf;   // bvol * Lh * 12
    int cstride[4];  // coarse site-index strides
};

CoarseGeom make_coarse_geom(const hdcr_coarse_desc* d);
int check_coarse_desc(const hdcr_coarse_desc* d);
size_t build_workspace_bytes(const CoarseGeom& c);

inline size_t basis_elems(const CoarseGeom& c) { return (size_t)c.Nc * 2 * c.nvec * c.nhalf; }
// FP64 region, FP32 region, then an FP16 copy for the FP32 inner cycle that
// holds HBASIS_SCALE * phi as (fp16 re, fp16 im) words (the scale keeps the
// O(1/sqrt(block dof)) entries in the normal FP16 range)
inline size_t basis_bytes(const CoarseGeom& c) { return basis_elems(c) * (16 + 8 + 4); }
constexpr float HBASIS_SCALE = 256.0f;
inline const double2* basis64(const void* b) { return static_cast<const double2*>(b); }
inline double2* basis64(void* b) { return static_cast<double2*>(b); }
inline const float2* basis32(const CoarseGeom& c, const void* b) {
    return reinterpret_cast<const float2*>(static_cast<const char*>(b) + basis_elems(c) * 16);
}
inline float2* basis32(const CoarseGeom& c, void* b) {
    return reinterpret_cast<float2*>(static_cast<char*>(b) + basis_elems(c) * 16);
}
inline const uint32_t* basis16(const CoarseGeom& c, const void* b) {
    return reinterpret_cast<const uint32_t*>(static_cast<const char*>(b) + basis_elems(c) * 24);
}
inline uint32_t* basis16(const CoarseGeom& c, void* b) {
    return reinterpret_cast<uint32_t*>(static_cast<char*>(b) + basis_elems(c) * 24);
}

// little Dirac operator storage (opaque): [a][d][k][j], column-major Nb x Nb
// blocks (a wavefront lane owns a row j); BF16C packs (bf16 re, bf16 im) in 32 bits
__host__ __device__ inline size_t coarse_elems(const CoarseGeom& c) { return (size_t)c.Nc * 9 * c.Nb * c.Nb; }
size_t coarse_bytes(const CoarseGeom& c, hdcr_dtype dt);

// --- kernels (coarse.hip) ---
// raw chiral folds of the subspace vectors into the FP64 basis region
void launch_basis_fold(const CoarseGeom& c, const double2* vecs, double2* b64, hipStream_t s);
// per block and chirality: classical Gram-Schmidt applied twice, in index
// order; rank_flag[0] is set to 1 if a vector is dependent (|w| <= 1e-12 |w0|)
void launch_block_orth(const CoarseGeom& c, double2* b64, int* rank_flag, hipStream_t s);
// Cholesky QR form of the same orthonormalisation (nvec <= 32): one pass of
// Gram matrices and factors (flag[1]: a first-pass pivot out of reach, use
// launch_block_orth on the unchanged vectors; flag[2]: a second-pass failure),
// then V <- V R^-1 with launch_chq_apply.  scratch: chq_scratch_elems entries.
bool chq_ok(const CoarseGeom& c);
size_t chq_scratch_elems(const CoarseGeom& c);
void launch_chq_pass(const CoarseGeom& c, double2* b64, double2* scratch, int pass, int* flag, hipStream_t s);
void launch_chq_apply(const CoarseGeom& c, double2* b64, const double2* scratch, hipStream_t s);
void launch_basis_to_f32(const CoarseGeom& c, const double2* b64, float2* b32, hipStream_t s);
void launch_basis_to_f16(const CoarseGeom& c, const double2* b64, uint32_t* b16, hipStream_t s);
// full fine fields of basis vectors k0 .. k0+nk-1 (k < nvec: + half, else - half), FP64
void launch_basis_expand(const CoarseGeom& c, const double2* b64, int k0, int nk, double2* fields, hipStream_t s);

// v[a][j] = <phi^a_j, psi - psi2>   (psi2 may be null)
template <typename T>
void launch_restrict(const CoarseGeom& c, const C2<T>* basis, const C2<T>* psi, const C2<T>* psi2, C2<T>* v,
                     hipStream_t s);
// psi = y + P v   (y may be null: psi = P v)
template <typename T>
void launch_prolong(const CoarseGeom& c, const C2<T>* basis, const C2<T>* v, const C2<T>* y, C2<T>* psi,
                    hipStream_t s);
// the same two with the FP16 copy of the basis (FP32 vectors)
void launch_restrict_h(const CoarseGeom& c, const uint32_t* basis, const float2* psi, const float2* psi2, float2* v,
                       hipStream_t s);
void launch_prolong_h(const CoarseGeom& c, const uint32_t* basis, const float2* v, const float2* y, float2* psi,
                      hipStream_t s);

// batched BF16 contraction on the matrix cores (variant 1..coarse_mfma_variants())
int coarse_mfma_variants();
const char* coarse_mfma_variant_name(int k);
// Nb in {16, 32, 64, 128}, no more waves than 16-row tiles (2 Nb / 16); terms:
// bf16 terms per vector entry, 1 for every variant, 2 or 3 for variant 9 only
bool coarse_mfma_eligible(const CoarseGeom& c, int variant, int terms);
void launch_coarse_mfma(const CoarseGeom& c, int variant, int terms, const uint32_t* A, const float2* v, float2* out,
                        int nrhs, hipStream_t s);

// out[r][a] = sum_d A[a][d] v[r][a+d]  (C128 / C64 storage, column-major blocks)
template <typename T>
void launch_coarse_apply(const CoarseGeom& c, const C2<T>* A, const C2<T>* v, C2<T>* out, int nrhs, hipStream_t s);
// BF16 storage with FP32 accumulation
void launch_coarse_apply_bf16(const CoarseGeom& c, const uint16_t* A, const float2* v, float2* out, int nrhs,
                              hipStream_t s);

// Coarse conjugate residual (the subspace inverse by a Krylov method, Sec. 4)
// with device-resident scalars: every kernel reads a done flag and returns at
// once when it is set, so a batch of iterations can be enqueued without
// synchronising; reductions finish in the last-arriving workgroup in a fixed
// order (reproducible).
template <typename T> struct CoarseCRWork {
    C2<T>* r;
    C2<T>* p;
    C2<T>* Ar;
    C2<T>* Ap;
    double* part;   // partial sums: [3][Nc] of the apply, [2][work-groups] of the start kernels,
                    // then two halves of [2][CCR_UPDATE_MAX] of the update kernel (even / odd steps)
    double* cs;     // scalars: 3 |r|^2 of the start, 4 |b|^2, 5 tol^2, 6 / 7 <r,Ar> of the even / odd steps
    int* flags;     // 0 done, 1 iterations, 2 (unused), 3 maxiter,
                    // 4 stop reason (0 none, 2 near-breakdown, 3 not finite);
                    // CCR_COUNTERS.. arrival counters (CCR_FLAGS ints)
    double* dpart;  // partial sums of the deflated start: [2 * DEFL_KMAX][DEFL_BLOCKS]
    double* dcoef;  // its coefficients <V_j, b> / theta_j: [2 * DEFL_KMAX] (re, im)
};
// Deflation space of the coarse solve: k orthonormal approximate eigenvectors V_i
// of A, W_i = A V_i and the Ritz values theta_i (device arrays; V, W [k][Nc*Nb]).
constexpr int DEFL_KMAX = 64;
constexpr int DEFL_BLOCKS = 256;       // work-groups per chunk of 8 dot products
constexpr int DEFL_INIT_BLOCKS = 512;  // work-groups of the start kernel
template <typename T> struct DeflView {
    int k;
    const double* theta;
    const C2<T>* V;
    const C2<T>* W;
};
constexpr int CCR_BLOCKS = 64;        // work-groups of the start kernel
constexpr int CCR_UPDATE_MAX = 512;   // most work-groups of the update kernel (one element per work-item below it)
constexpr int ARRIVE_GROUPS = 16;   // group counters of the last-arrival test
constexpr int ARRIVE_STRIDE = 64;   // ints between counters (each counter on its own 256-byte line)
constexpr int CCR_COUNTERS = 64;    // first arrival counter in flags
constexpr int CCR_FLAGS = CCR_COUNTERS + (1 + ARRIVE_GROUPS) * ARRIVE_STRIDE;  // ints of the flags array
// p[0 .. n) = 0 with a fill kernel (no memset node in the stream)
void launch_zero_i32(int* p, int n, hipStream_t s);
// r = b, x = 0, |b|^2; resets the iteration state
template <typename T>
void launch_ccr_init(const CoarseGeom& c, const C2<T>* b, C2<T>* x, const CoarseCRWork<T>& w, int maxiter, double tol,
                     hipStream_t s);
// the Galerkin start from the deflation space: x = sum_i (<V_i, b> / theta_i) V_i,
// r = b - sum_i (<V_i, b> / theta_i) W_i (so V^dag r = 0 when W = A V and the V_i
// are eigenvectors); |b|^2, |r|^2 and the iteration state as launch_ccr_init
template <typename T>
void launch_ccr_init_defl(const CoarseGeom& c, const C2<T>* b, C2<T>* x, const CoarseCRWork<T>& w,
                          const DeflView<T>& d, int maxiter, double tol, hipStream_t s);
// CR step `step` (1, 2, ...: the p, x and r updates of step `step`, then
// Ar = A r for the next one); step 0 issues the first apply Ar = A r instead
template <typename T>
void launch_ccr_step(const CoarseGeom& c, hdcr_dtype A_dtype, const void* A, C2<T>* x, const CoarseCRWork<T>& w,
                     int step, hipStream_t s);

// little Dirac operator build: A64[a][d][k][j] for basis vectors in [k0, k0+nk),
// nk <= 4, given the class-split fine fields Y[(kk*9 + d)] = H^(d) Phi_{k0+kk}
// (read only on the sites of class d); P: coarse_project_scratch_elems() of
// partial sums
size_t coarse_project_scratch_elems(const CoarseGeom& c);
void launch_coarse_project(const CoarseGeom& c, const double2* b64, const double2* Y, int k0, int nk, double2* P,
                           double2* A64, hipStream_t s);
// The nine hop classes of H in: out + d * fstride = H^(d) in, d = 0: diagonal,
// fifth dimension and hops inside a block, at every site; d = 1+mu / 5+mu: the
// forward / backward mu hop that crosses the block face, written only at the
// sites on that face (the other entries of those fields are left as they were)
void launch_dslash_classes(const CoarseGeom& c, const double2* U, const double2* in, double2* out, size_t fstride,
                           hipStream_t s);
// A64 (column-major) -> other storage
void launch_coarse_convert(const CoarseGeom& c, const double2* A64, hdcr_dtype dt, void* dst, hipStream_t s);
// any storage -> logical A[a][d][j][k] complex double
void launch_coarse_export(const CoarseGeom& c, hdcr_dtype dt, const void* A, double2* out, hipStream_t s);

}  // namespace hdcr
