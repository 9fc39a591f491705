/*
 * hdcr.h -- C ABI of the MI355X (gfx950) hot path of the Hierarchically
 * Deflated Conjugate Residual solver (Yamaguchi & Boyle, Lattice 2016).
 *
 * The library solves H x = b for the Hermitian indefinite 5d domain wall
 * operator H = Gamma5 D_dwf = gamma5 R5 D_dwf (Sec. 3), either by plain
 * conjugate residual (Sec. 3) or by flexible GCR preconditioned with a
 * two-level cycle built on a chirally split, block-local coarse space whose
 * little Dirac operator is a 9-point nearest-neighbour stencil of dense
 * Nb x Nb blocks (Sec. 4).  To solve D_dwf psi = eta, pass b = Gamma5 eta.
 *
 * Conventions (fixed; the paper leaves them open):
 *   D_dwf (Cayley form with c = 0, scale b of the 4d part; Sec. 3 names this
 *   Mobius case under the same H; b = 1 is the Shamir kernel):
 *     (D psi)(x,s) = (b (4 - M5) + 1) psi(x,s)
 *        - b/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu,s) + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu,s)]
 *        - P- psi(x,s+1) - P+ psi(x,s-1),
 *     walls: -P- psi(x,Ls) -> +mf P- psi(x,0), -P+ psi(x,-1) -> +mf P+ psi(x,Ls-1);
 *     a 4d hop that crosses the lattice boundary in direction mu picks up bc[mu].
 *   (H psi)(x,s) = g5 (D psi)(x, Ls-1-s).
 *   Gamma matrices: chiral basis, g_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = x, y, z),
 *     g_t = [[0, 1], [1, 0]], g5 = diag(1, 1, -1, -1), P+- = (1 +- g5)/2.
 *   Sites: site4 = ((t*Lz + z)*Ly + y)*Lx + x.
 *
 * Memory layouts of caller buffers (device memory unless stated):
 *   fine field  psi[c][site4][s], c = spin*3 + colour (12), complex interleaved (re, im);
 *               C128 = 2 x double, C64 = 2 x float per complex entry.
 *   gauge field U[site4][mu][row][col] (the 36 entries of a site contiguous), complex
 *               interleaved, same precision as the field.
 *   coarse vector v[rhs][site_c][k], k < Nb = 2*nvec, site_c ordered like site4 over the
 *               coarse lattice (extent L[mu]/block[mu]); C128 or C64.
 *   basis, A:   opaque device buffers of hdcr_basis_bytes() / hdcr_coarse_bytes() bytes;
 *               read them through hdcr_export_basis() / hdcr_export_coarse().
 *
 * Ownership: the caller owns every buffer.  The library never allocates or
 * frees device memory; scratch space comes in through (work, work_bytes),
 * sized by hdcr_workspace_bytes(), except for hdcr_coarse_solve_static, whose
 * scratch is a fixed array in the library's own device memory.  Every call
 * except hdcr_solve, hdcr_coarse_solve, hdcr_coarse_solve_static,
 * hdcr_build_deflation, hdcr_make_subspace, hdcr_make_subspace_degrees,
 * hdcr_power_max and hdcr_vec_dot is stream-ordered and returns before the
 * work is done; those eight return after it has completed.
 * In and out buffers of one call must not overlap.
 *
 * Errors: 0 = success.  Negative codes are caller errors found before any
 * launch (HDCR_EINVAL), runtime failures (HDCR_EHIP) or a workspace that is
 * too small (HDCR_ENOMEM).  Positive codes are numerical outcomes of a solve.
 * hdcr_last_error() returns a thread-local description of the last failure.
 */
#ifndef HDCR_H
#define HDCR_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HDCR_API __attribute__((visibility("default")))

#define HDCR_OK 0
#define HDCR_EINVAL (-1)
#define HDCR_EHIP (-2)
#define HDCR_ENOMEM (-3)
#define HDCR_ENOTCONV 1    /* maxiter reached; x holds the last iterate */
#define HDCR_EBREAKDOWN 2  /* |<r,Hr>| or |w| fell to rounding level */
#define HDCR_ENAN 3        /* a NaN or Inf appeared in a residual */
#define HDCR_ERANK 4       /* block basis numerically rank deficient */

typedef enum {
    HDCR_C128 = 0,  /* complex double */
    HDCR_C64 = 1,   /* complex float */
    HDCR_BF16C = 2, /* (bf16 re, bf16 im): little Dirac operator storage only */
    HDCR_F16C = 3   /* (fp16 re, fp16 im): FP16 copy of the block basis used with FP32 vectors */
} hdcr_dtype;

/* Kernel-shape choices of one call, for tests and tuning sweeps.  Every field 0
 * selects the library's own choice; the results of every choice agree (bit for
 * bit for the traversal and the FP16 kernels, to rounding for the others).
 *   dslash_variant  fine-apply kernel: 1 tile kernel with cached stores, 2 generic
 *                   kernel, 3 tile kernel with non-temporal stores, 4 parity-tile
 *                   kernel with one fifth-dimension slice per work-item (FP32),
 *                   5 paired-slice kernel on FP16 fields, 6 FP16 smoother and filter
 *                   steps as a plain pass plus a separate combination; for
 *                   hdcr_apply_cf: 2 one work-item per 5d site, 4 parity tiles with
 *                   one slice per work-item (else paired slices in FP32 with even Ls)
 *   tslab, ysplit, xsplit  traversal blocking of the stencil's tiles (or sites):
 *                   t slabs of tslab tiles, y and x cut into ysplit and xsplit parts
 *                   (a value that does not divide the extent selects no cut)
 *   force_r, force_ms, force_p, force_sum  work split of hdcr_fermion_force: lanes
 *                   per 4d site (2, 4, 8, 16), wave groups over the directions (1, 2),
 *                   fifth-dimension slices per load (1, 2: FP32, even Ls), cross-lane
 *                   sums by DPP (1) or through LDS (2); an unsupported split is
 *                   rejected with HDCR_EINVAL
 *   restrict_w, restrict_rkg  restriction: s slots per work-item (1, 2, 4, 8; 0: 8
 *                   with the FP16 basis copy, else 4), vectors per workgroup (16, 32)
 *   prolong_ni      prolongation with the FP16 basis: indices per work-item (2, 4)
 *   prolong_split   prolongation: workgroups per coarse site (1 .. 16; 0: about
 *                   7800 workgroups in all, each part at least one sweep long)
 *   wg_per_cu       at most this many workgroups of the parity-tile stencil kernels
 *                   resident per compute unit (enforced through their LDS size; 0 or a
 *                   value above what fits: no cap) */
typedef struct hdcr_tuning {
    int32_t dslash_variant;
    int32_t tslab, ysplit, xsplit;
    int32_t force_r, force_ms, force_p, force_sum;
    int32_t restrict_w, restrict_rkg, prolong_ni;
    int32_t wg_per_cu;
    int32_t prolong_split;
} hdcr_tuning;

/* Fine lattice: L = (Lx, Ly, Lz, Lt), Ls, bc per direction (+1 periodic, -1
 * antiperiodic), domain wall height M5, quark mass mf, and cayley_b, the scale b
 * of the 4d part (0 is read as 1, the Shamir kernel, so a zero-initialised
 * descriptor describes the Shamir operator with the library's kernel choices). */
typedef struct hdcr_fine_desc {
    int32_t L[4];
    int32_t Ls;
    int32_t bc[4];
    int32_t reserved;
    double M5;
    double mf;
    double cayley_b;
    hdcr_tuning tune;
} hdcr_fine_desc;

/* Coarse space: blocks of block[mu] sites in 4d covering the whole fifth
 * dimension (Sec. 4), nvec subspace vectors, Nb = 2*nvec after the chiral
 * split.  Requires L[mu] % block[mu] == 0 and Ls even. */
typedef struct hdcr_coarse_desc {
    hdcr_fine_desc fine;
    int32_t block[4];
    int32_t nvec;
    int32_t reserved;
} hdcr_coarse_desc;

typedef enum { HDCR_PRECOND_NONE = 0, HDCR_PRECOND_TWO_LEVEL = 1 } hdcr_precond;

/* Solver parameters.  precond NONE: plain conjugate residual in FP64 (Sec. 3).
 * TWO_LEVEL: FP64 flexible GCR(restart) whose preconditioner is the symmetric
 * two-level cycle (Sec. 4, M_outer) in inner_dtype: Chebyshev smoother of
 * cheb_order terms approximating 1/y on [cheb_lo, cheb_hi] applied as
 * p(H^2) H, and a coarse CR solve on A (coarse_dtype storage) to relative
 * tolerance coarse_tol or coarse_maxiter iterations. */
typedef struct hdcr_solve_params {
    double tol;             /* relative true residual |b - Hx|/|b| */
    int32_t maxiter;        /* outer iterations */
    int32_t restart;        /* FGCR window (TWO_LEVEL) */
    int32_t precond;        /* hdcr_precond */
    int32_t cheb_order;     /* number of Chebyshev terms, 10 in the paper */
    double cheb_lo;         /* 1.0 in the paper */
    double cheb_hi;         /* 64.0 in the paper */
    double coarse_tol;
    int32_t coarse_maxiter;
    int32_t inner_dtype;    /* HDCR_C64 or HDCR_C128: smoother, restriction, prolongation */
    int32_t coarse_dtype;   /* storage of A passed to hdcr_solve: C128, C64 or BF16C */
    int32_t basis_dtype;    /* HDCR_F16C: the C64 inner cycle restricts and prolongs with the FP16
                               basis copy; any other value: the basis in the inner precision */
    int32_t verbose;
} hdcr_solve_params;

/* Statistics of one solve (the columns of the paper's Table 1 and more). */
typedef struct hdcr_solve_stats {
    int32_t status;
    int32_t outer_iters;
    int64_t coarse_iters;       /* total coarse CR iterations */
    int64_t fine_applies_f64;   /* H applications in FP64 */
    int64_t fine_applies_inner; /* H applications in the inner precision */
    int64_t coarse_applies;
    double true_rel_residual;
    double seconds_total;
    double seconds_fine;        /* smoother + inner residuals (event-timed) */
    double seconds_coarse;      /* restriction + coarse solve + prolongation */
    double seconds_outer;       /* FP64 apply + orthogonalisation + updates */
    int32_t history_len;        /* entries written to the caller's history array */
    int32_t coarse_breakdowns;  /* coarse solves that stopped early on near-breakdown
                                   (|<r,Ar>| < eps |r||Ar|, see hdcr_coarse_solve) */
} hdcr_solve_stats;

/* Coarse-space eigenvector deflation (Sec. 5 names it as the way to cut the
 * coarse-solve cost): k orthonormal approximate eigenvectors V_i of the little
 * Dirac operator A with the smallest |theta_i|, W_i = A V_i and the Ritz values
 * theta_i.  The coarse CR then starts from the Galerkin projection
 * x0 = sum_i (<V_i, b> / theta_i) V_i with r0 = b - sum_i (<V_i, b> / theta_i) W_i,
 * which removes the deflated modes from the residual.  theta, V, W are device
 * buffers owned by the caller (V, W: [k][site_c][Nb], the coarse vector
 * layout); dtype C128 for an FP64 coarse solve (C128 storage of A), C64 for an
 * FP32 one (C64 or BF16C storage). */
#define HDCR_DEFL_MAX 64
typedef struct hdcr_coarse_deflation {
    int32_t k;            /* 1 <= k <= HDCR_DEFL_MAX */
    int32_t dtype;        /* C128 or C64 */
    const double* theta;  /* k Ritz values (device) */
    const void* V;
    const void* W;
} hdcr_coarse_deflation;

/* Set-up parameters of hdcr_build_deflation. */
typedef struct hdcr_deflation_params {
    int32_t k;            /* eigenpairs kept, 1 <= k <= m */
    int32_t m;            /* block size (start vectors), k <= m <= HDCR_DEFL_MAX, m <= Nc * Nb */
    int32_t degree;       /* Chebyshev filter degree in A^2 per pass, 1 .. 1000 */
    int32_t iters;        /* filtered passes, 1 .. 100 */
    int32_t power_iters;  /* power iterations for the top of the A^2 spectrum, 1 .. 10000 */
    int32_t reserved;
    double cut;           /* lower filter edge of the first pass as a fraction of the top, 0 < cut < 1 */
} hdcr_deflation_params;

/* Text of a status code, and a thread-local description of the last failure
 * (library plumbing, not a step of the method). */
HDCR_API const char* hdcr_strerror(int code);
HDCR_API const char* hdcr_last_error(void);

/* out = H psi with H = Gamma5 D_dwf (Sec. 3).  dtype C128 or C64; U, psi and
 * out in that precision.  One kernel launch on `stream`. */
HDCR_API int hdcr_apply_fine(const hdcr_fine_desc* desc, hdcr_dtype dtype, const void* U, const void* psi, void* out,
                    hipStream_t stream);

/* The continued-fraction form of the overlap operator (Sec. 3, the
 * continued-fraction matrix: a 5d operator that is already Hermitian indefinite
 * and nearest-neighbour) on a field of Ls = m + 1 slices, m >= 1 pole slices:
 *   out_i = sigma_i H_W psi_i + [i = m] R g5 psi_m + c_(i-1) psi_(i-1) + c_i psi_(i+1),
 *   H_W = g5 D_W(-M5), D_W psi(x) = (4 - M5) psi(x) - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu)
 *         + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)] (bc[mu] on boundary-crossing hops),
 *   sigma_i = (-1)^i for i < m, sigma_m = beta[0];
 *   c_i = 1/sqrt(beta[i] beta[i+1]) for i < m - 1, c_(m-1) = 1/sqrt(beta[m-1]),
 *   and no coupling beyond the first and last slices (c_(-1) = c_m = 0).
 * The paper prints this matrix for four pole slices and gives neither the
 * beta_i nor R; they are the caller's (beta: host array of the m = Ls - 1 values,
 * each finite and > 0; R finite), e.g. from a Zolotarev approximation of the
 * sign function.  desc: Ls = m + 1 in [2, 64], M5 the Wilson mass, bc; mf unused;
 * cayley_b 0 or 1.  Fields in the fine-field layout with s = the slice i; U, psi,
 * out in dtype (C128 or C64); psi and out must not overlap.  One kernel launch
 * on `stream`. */
HDCR_API int hdcr_apply_cf(const hdcr_fine_desc* desc, hdcr_dtype dtype, const double* beta, double R, const void* U,
                           const void* psi, void* out, hipStream_t stream);

/* Gauge-link gradient and su(3) force of L = Re <chi, H psi> (the HMC
 * fermion force of the setting named in the abstract, Sec. 1 and Sec. 5; H as
 * in Sec. 3 and the conventions above):
 *   W[site4][mu][a][b] = dL/dRe U_mu(x)[a][b] + i dL/dIm U_mu(x)[a][b]
 *                      = -b/2 b_mu(x) sum_s [ ((1 - g_mu) chi'(x,s)) (x) psi(x+mu,s)^dag
 *                                          + psi(x,s) (x) ((1 + g_mu) chi'(x+mu,s))^dag ]_ab,
 *   chi'(x,s) = g5 chi(x, Ls-1-s), (x) the colour outer product summed over
 *   spin, b_mu(x) = bc[mu] on the link that crosses the lattice boundary;
 *   T[site4][mu] = P_TA(U_mu(x) W_mu(x)^dag), P_TA(M) = (M - M^dag)/2 - tr(M - M^dag)/6,
 *   so that under U_mu(x) -> exp(eps X) U_mu(x) (X traceless anti-Hermitian)
 *   dL/deps = Re tr(X T_mu(x)).
 * W and T use the gauge-field layout; either may be NULL (not both).  The
 * gradient with respect to psi is H chi (H is Hermitian): hdcr_apply_fine.
 * dtype C128 or C64 for every buffer.  One kernel launch on `stream`;
 * outputs must not overlap the inputs or each other. */
HDCR_API int hdcr_fermion_force(const hdcr_fine_desc* desc, hdcr_dtype dtype, const void* U, const void* chi,
                       const void* psi, void* W, void* T, hipStream_t stream);

/* <x, y> = sum conj(x_i) y_i over n complex entries (C128 or C64 data, FP64
 * accumulation, fixed reduction order), written to out[0] (re), out[1] (im) on
 * the host: the inner product of the conjugate residual iterations (Sec. 3) and
 * of the GCR orthogonalisation (Sec. 4).  work: device scratch of at least HDCR_DOT_WORK_BYTES bytes.
 * Synchronises `stream`. */
#define HDCR_DOT_WORK_BYTES 32768
HDCR_API int hdcr_vec_dot(hdcr_dtype dtype, int64_t n, const void* x, const void* y, double* out, void* work,
                 size_t work_bytes, hipStream_t stream);

/* dst = src for `bytes` bytes (a multiple of 16; 16-byte aligned, not
 * overlapping) with a plain streaming kernel: not a step of the method but the
 * device's measured copy rate, the practical ceiling beside the datasheet HBM
 * bandwidth, and the reference the memory-traffic counters are scaled by.
 * Stream-ordered. */
HDCR_API int hdcr_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t stream);

/* Scratch bytes needed by the calls below: which = HDCR_WS_SOLVE (hdcr_solve
 * with the given params), HDCR_WS_BUILD (hdcr_build_coarse), HDCR_WS_SUBSPACE
 * (hdcr_make_subspace / hdcr_power_max), HDCR_WS_SMOOTH (hdcr_smooth),
 * HDCR_WS_VCYCLE (hdcr_vcycle with the given params), HDCR_WS_COARSE
 * (hdcr_coarse_solve with A in params->coarse_dtype). */
#define HDCR_WS_SOLVE 0
#define HDCR_WS_BUILD 1
#define HDCR_WS_SUBSPACE 2
#define HDCR_WS_SMOOTH 3
#define HDCR_WS_VCYCLE 4
#define HDCR_WS_COARSE 5
HDCR_API size_t hdcr_workspace_bytes(int which, const hdcr_coarse_desc* desc, const hdcr_solve_params* params);

/* Bytes of the opaque basis buffer (FP64, FP32 and FP16 copies of the chirally
 * compressed block basis phi^b_k of Sec. 4; it always holds all three, so its size
 * does not depend on the precision the caller's cycles run in) and of the little
 * Dirac operator A of Sec. 4 in `dtype` storage. */
HDCR_API size_t hdcr_basis_bytes(const hdcr_coarse_desc* desc);
HDCR_API size_t hdcr_coarse_bytes(const hdcr_coarse_desc* desc, hdcr_dtype dtype);

/* Coarse space (Sec. 4).  vecs: nvec fine fields (C128, [k][12][V4][Ls]), the
 * subspace vectors phi_k.  Each is split into its two Gamma5 = gamma5 R5
 * chiralities, restricted to the blocks (block[mu] sites x all of Ls) and, per
 * block and chirality, orthonormalised in index order (Q of a thin QR with a
 * positive real R diagonal): basis vector j < nvec of block a is phi^{a,+}_j,
 * j >= nvec is phi^{a,-}_{j-nvec}.  Then the little Dirac operator
 *   A[a][d][j][k] = <phi^a_j | H^(d) | phi^{a+d}_k>,  d in D9 = (0,+x,+y,+z,+t,-x,-y,-z,-t),
 * where H^(d), d != 0, holds the hops from block a+d into block a across the
 * face d and H^(0) everything else (diagonal, fifth dimension, hops inside a);
 * summing the nine blocks over equal a+d gives <phi^a_j|H|phi^b_k>.  Built in
 * FP64 and stored in A_dtype.  U in C128.  work: hdcr_workspace_bytes(
 * HDCR_WS_BUILD).  Synchronous; returns HDCR_ERANK if a block's vectors are
 * dependent (remaining norm below 1e-12 of the chiral projection's). */
HDCR_API int hdcr_build_coarse(const hdcr_coarse_desc* desc, const void* U, const void* vecs, void* basis, void* A,
                      hdcr_dtype A_dtype, void* work, size_t work_bytes, hipStream_t stream);

/* The little Dirac operator A of Sec. 4 in C128 storage -> A in C64 or BF16C
 * storage (round to nearest; the paper leaves the storage precision open). */
HDCR_API int hdcr_convert_coarse(const hdcr_coarse_desc* desc, const void* A128, hdcr_dtype dtype, void* A_dst,
                        hipStream_t stream);

/* Batched coarse apply on the matrix cores (Sec. 4, the little Dirac operator
 * applied to many right-hand sides at once): out[r] = A v[r], r < nrhs, with A
 * in BF16C storage and a BF16 x BF16 contraction with FP32 accumulation.
 * rhs_terms says how each FP32 component of v enters it: 1, rounded to bf16
 * (round to nearest even; relative error up to 2^-9 per entry); 2 or 3, as the
 * sum of that many bf16 terms, each rounding what the earlier ones leave, so
 * that two terms carry it to within 2^-16 and three exactly (every product is
 * then exact and only the FP32 sums round: the complex64 apply of the stored A).
 * v, out: C64 [nrhs][site_c][k], not overlapping.  Needs Nb in {16, 32, 64, 128}.
 * variant 0: the tile shape hdcr_tune_coarse_batched chose for this shape and
 * rhs_terms (if it has not been tuned: 9 for Nb = 64, else 2, or 1 for Nb =
 * 16); 1..HDCR_MFMA_VARIANTS: an explicit tile shape (2,
 * 4, 8 wavefronts per coarse site, blocks read directly or staged in LDS; 7: 8
 * wavefronts with all 9 blocks prefetched; 8: as 7 with the blocks held in
 * registers across passes of 16 right-hand sides and every load of a pass
 * issued before its first use; 9: the direction loop outside the passes, each
 * block staged once per chunk of up to 64 right-hand sides).  Variants 7 to 9
 * need Nb = 64, rhs_terms 2 and 3 need variant 9, and a variant with more
 * wavefronts than Nb / 8 is rejected (HDCR_EINVAL).  For one rhs_terms, all
 * variants perform the same operations per output element in the same order,
 * so they give identical results.  Stream-ordered. */
#define HDCR_MFMA_VARIANTS 9
HDCR_API int hdcr_apply_coarse_batched(const hdcr_coarse_desc* desc, const void* A, const void* v, void* out,
                                       int32_t nrhs, int32_t variant, int32_t rhs_terms, hipStream_t stream);
/* Autotuner of the batched apply of A (Sec. 4): times every tile shape that
 * takes rhs_terms on the caller's buffers (out is overwritten), records the
 * fastest for (Nc, Nb, nrhs, rhs_terms, device) in a process-wide table used by
 * variant 0, and reports the winner (best) and the median time of each variant
 * in ms[HDCR_MFMA_VARIANTS] (-1 for a variant that does not apply; either
 * pointer may be null).  Returns after the timing runs have completed. */
HDCR_API int hdcr_tune_coarse_batched(const hdcr_coarse_desc* desc, const void* A, const void* v, void* out,
                                      int32_t nrhs, int32_t rhs_terms, int32_t* best, double* ms, hipStream_t stream);

/* Read back the opaque buffers: the little Dirac operator of Sec. 4 (any
 * storage) as logical A[a][d][j][k] complex double; the block basis phi^b_k of
 * Sec. 4 as Nb full fine fields (C128, [j][12][V4][Ls]), field j holding phi^a_j
 * on every block a. */
HDCR_API int hdcr_export_coarse(const hdcr_coarse_desc* desc, hdcr_dtype dtype, const void* A, void* A_c128,
                       hipStream_t stream);
HDCR_API int hdcr_export_basis(const hdcr_coarse_desc* desc, const void* basis, void* fields_c128, hipStream_t stream);

/* Restriction v[a][j] = <phi^a_j, psi> (P^dag) and prolongation
 * psi(x) = sum_j phi^{b(x)}_j(x) v[b(x)][j] (P) (Sec. 4), in C128 or C64 (the
 * basis copy of that precision is used), or F16C: FP32 vectors with the FP16
 * basis copy (entries rounded to 11 significant bits). */
HDCR_API int hdcr_restrict(const hdcr_coarse_desc* desc, hdcr_dtype dtype, const void* basis, const void* psi, void* v,
                  hipStream_t stream);
HDCR_API int hdcr_prolong(const hdcr_coarse_desc* desc, hdcr_dtype dtype, const void* basis, const void* v, void* psi,
                 hipStream_t stream);

/* The little Dirac operator of Sec. 4 (the coarse matrix A = P^dag H P, whose
 * nearest-neighbour block structure Sec. 3 and Sec. 4 point out) applied as a
 * 9-point stencil: out[r][a] = sum_d A[a][d] v[r][a+d] (coarse-periodic; the fine
 * antiperiodic sign is inside A) for nrhs right-hand sides.  dtype is
 * A's storage; vectors are C128 for C128 storage, C64 otherwise (BF16C storage
 * accumulates in FP32). */
HDCR_API int hdcr_apply_coarse(const hdcr_coarse_desc* desc, hdcr_dtype dtype, const void* A, const void* v, void* out,
                      int32_t nrhs, hipStream_t stream);

/* Chebyshev smoother (Sec. 4): out = p(H^2) H in, p the Chebyshev interpolant of
 * 1/y on [lo, hi] with `order` terms (the paper: order 10 on [1, 64]), so that
 * out ~ H^-1 in on the modes with lo <= lambda^2 <= hi.  dtype C128 or C64 (U, in
 * and out in that precision).  work: hdcr_workspace_bytes(HDCR_WS_SMOOTH)
 * (4 fields).  2*order - 1 applications of H. */
HDCR_API int hdcr_smooth(const hdcr_fine_desc* desc, hdcr_dtype dtype, const void* U, int32_t order, double lo, double hi,
                const void* in, void* out, void* work, size_t work_bytes, hipStream_t stream);

/* One application of the symmetric two-level cycle (Sec. 4, M_outer):
 *   e1 = S r;  e2 = e1 + Q (r - H e1);  e = e2 + S (r - H e2),  Q = P CR_A(P^dag .)
 * with the smoother and coarse solve of params (coarse CR from 0, or from the
 * Galerkin start of defl when it is not NULL, to coarse_tol, or exactly
 * coarse_maxiter iterations when coarse_tol <= 0).
 * r, e, U: C128; computed in params->inner_dtype.  work:
 * hdcr_workspace_bytes(HDCR_WS_VCYCLE). */
HDCR_API int hdcr_vcycle(const hdcr_coarse_desc* desc, const hdcr_solve_params* params, const void* U, const void* basis,
                const void* A, const hdcr_coarse_deflation* defl, const void* r, void* e, void* work,
                size_t work_bytes, hipStream_t stream);

/* Coarse solve A x = b by conjugate residual (Sec. 4: the subspace inverse by
 * a Krylov method), the solve inside the two-level cycle: from x = 0, or from
 * the Galerkin start of the deflation space defl (host struct, may be NULL;
 * dtype as for the solve).  tol <= 0 runs exactly maxiter iterations, else CR
 * stops when the updated |r| <= tol |b| or after maxiter.  Either way it stops
 * early, keeping the current iterate, at a near-breakdown |<r,Ar>| < eps |r| |Ar|
 * (eps = 1e-13 with C128 vectors, 1e-6 with C64 vectors) and returns
 * HDCR_EBREAKDOWN, or HDCR_ENAN if <r,Ar> or |Ar| is not finite.  b, x: C128 for
 * C128 storage of A, C64 for C64 / BF16C; not overlapping.  *iters (may be
 * NULL) gets the iteration count.  work: hdcr_workspace_bytes(HDCR_WS_COARSE)
 * with params->coarse_dtype = A_dtype.  Synchronous. */
HDCR_API int hdcr_coarse_solve(const hdcr_coarse_desc* desc, hdcr_dtype A_dtype, const void* A,
                               const hdcr_coarse_deflation* defl, const void* b, void* x, int32_t maxiter, double tol,
                               int32_t* iters, void* work, size_t work_bytes, hipStream_t stream);

/* hdcr_coarse_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results, with the scratch taken from a static device array
 * of the library instead of a workspace argument.  That array holds
 * HDCR_COARSE_STATIC_BYTES (8 MiB) per GPU for as long as the process runs; a
 * coarse space whose solve needs more (hdcr_workspace_bytes(HDCR_WS_COARSE)) is
 * rejected with HDCR_ENOMEM before any launch (8 MiB covers, e.g., 6^4 coarse
 * sites with Nb = 64 in FP64).  The caller passes A, defl, b and x as for
 * hdcr_coarse_solve.  Every call on one GPU uses that GPU's single array, so
 * calls that overlap on one GPU (other host threads, other streams) race and
 * must be serialised by the caller; each call clears the counters it needs.
 * The call itself allocates nothing.  Synchronous. */
#define HDCR_COARSE_STATIC_BYTES (8u << 20)
HDCR_API int hdcr_coarse_solve_static(const hdcr_coarse_desc* desc, hdcr_dtype A_dtype, const void* A,
                                      const hdcr_coarse_deflation* defl, const void* b, void* x, int32_t maxiter,
                                      double tol, int32_t* iters, hipStream_t stream);

/* Deflation set-up (Sec. 5, coarse-space eigenvector deflation): the k
 * eigenpairs of A of smallest |lambda| by Chebyshev-filtered subspace
 * iteration in A^2 (positive definite, so its Ritz values bound its spectrum
 * from above, unlike those of the indefinite A) on the m start vectors v0:
 * hi = 1.1 x the power-iteration estimate of the top of A^2 from v0[0]; each
 * pass filters the block with T_degree((2 A^2 - hi - lo)/(hi - lo)), makes it
 * orthonormal (Gram-Schmidt in index order, twice) and rotates it to the Ritz
 * vectors of A^2; lo = cut * hi in the first pass and the largest Ritz value
 * of A^2 in the block (at most 0.99 hi) afterwards.  A final Rayleigh-Ritz on A
 * gives the pairs (theta, y), |y| = 1.  A pair is found when its residual
 * |A y - theta y| is at most 1e-2 |theta|: a block that is not yet an
 * invariant subspace of A can mix eigenvectors of opposite sign into a Ritz
 * vector whose theta lies anywhere between them, near zero included.  The
 * found pairs of smallest |theta|, at most k of them, are written to theta
 * (device doubles), V and W = A V (device, [.][site_c][Nb] in C128 for C128
 * storage of A, C64 otherwise: the vector precision of the coarse solve that
 * uses them), and to theta_host (may be NULL) in ascending |theta|; *k_found
 * (may be NULL) gets their number, and only that many entries are written
 * (buffers sized for k).  Computed in that vector precision with FP64 inner
 * products; the small dense eigenproblems are solved on the host.  v0: m C128
 * coarse vectors.  work: hdcr_deflation_workspace_bytes().  Synchronous;
 * HDCR_ENOTCONV if no pair was found (raise iters, degree or m), HDCR_ENAN if
 * the spectrum estimate or a Ritz problem is not finite. */
HDCR_API size_t hdcr_deflation_workspace_bytes(const hdcr_coarse_desc* desc, hdcr_dtype A_dtype,
                                               const hdcr_deflation_params* params);
HDCR_API int hdcr_build_deflation(const hdcr_coarse_desc* desc, hdcr_dtype A_dtype, const void* A,
                                  const hdcr_deflation_params* params, const void* v0, double* theta, void* V, void* W,
                                  double* theta_host, int32_t* k_found, void* work, size_t work_bytes,
                                  hipStream_t stream);

/* Subspace generation (Sec. 4, Fig. 1): vecs[k] = T_degree(yhat) noise[k] / |.|
 * with yhat = (2 H^2 - hi - lo)/(hi - lo): the Chebyshev low-pass filter that
 * leaves the modes with lo <= lambda^2 <= hi bounded by 1 and amplifies those
 * below lo.  noise, vecs: nvec C128 fields; U: C128; computed in dtype: C128, C64,
 * or F16C (FP32 links and arithmetic, the recurrence's fields stored as (fp16 re,
 * fp16 im), brought to unit RMS per entry at the start and every 16 steps;
 * Ls = 16 and even extents).  work: hdcr_subspace_workspace_bytes().
 * Synchronous. */
HDCR_API size_t hdcr_subspace_workspace_bytes(const hdcr_fine_desc* desc, hdcr_dtype dtype);
HDCR_API int hdcr_make_subspace(const hdcr_fine_desc* desc, hdcr_dtype dtype, int32_t nvec, int32_t degree, double lo,
                       double hi, const void* U, const void* noise, void* vecs, void* work, size_t work_bytes,
                       hipStream_t stream);

/* Several filter degrees from one recurrence per noise field (Sec. 5 notes that
 * the Chebyshev recurrence yields every lower order along the way at no extra
 * cost): vecs[k * ndeg + q] = T_{degrees[q]}(yhat) noise[k] / |.| for k < nnoise,
 * q < ndeg, with yhat as for hdcr_make_subspace; degrees (host, ndeg entries)
 * strictly ascending in [0, 100000].  Each output equals hdcr_make_subspace's at
 * that degree up to rounding.  noise: nnoise C128 fields, vecs: nnoise * ndeg
 * C128 fields (not overlapping noise); U: C128; computed in dtype (C128, C64 or
 * F16C, as for hdcr_make_subspace).  work: hdcr_subspace_workspace_bytes().
 * Synchronous. */
HDCR_API int hdcr_make_subspace_degrees(const hdcr_fine_desc* desc, hdcr_dtype dtype, int32_t nnoise, int32_t ndeg,
                                        const int32_t* degrees, double lo, double hi, const void* U, const void* noise,
                                        void* vecs, void* work, size_t work_bytes, hipStream_t stream);

/* Power-iteration estimate of the largest eigenvalue of H^2 (Rayleigh quotient
 * after `iters` steps from v0), the upper edge lambda_max of the Chebyshev
 * filter interval (Sec. 4, Fig. 1 caption); C128.  work: hdcr_subspace_workspace_bytes(desc,
 * HDCR_C128).  Synchronous. */
HDCR_API int hdcr_power_max(const hdcr_fine_desc* desc, const void* U, const void* v0, int32_t iters, double* lam,
                   void* work, size_t work_bytes, hipStream_t stream);

/* Solve H x = b to |b - H x| <= tol |b| (x: initial guess in, solution out;
 * C128 fields; U in C128): plain conjugate residual on the Hermitian indefinite
 * H (Sec. 3) with precond NONE, or variable-preconditioned GCR whose
 * preconditioner is the two-level cycle M_outer (Sec. 4) with TWO_LEVEL.
 * precond NONE ignores basis and A (may be NULL).
 * TWO_LEVEL needs the basis and A of hdcr_build_coarse (A in
 * params->coarse_dtype); defl (host struct, may be NULL) deflates every coarse
 * solve (vectors in params->inner_dtype).  history (host, may be NULL) receives up to
 * history_cap relative residual norms, one per outer iteration.  Returns 0 or
 * a positive status (stats->status holds the same).  Synchronous. */
HDCR_API int hdcr_solve(const hdcr_coarse_desc* desc, const hdcr_solve_params* params, const void* U, const void* basis,
               const void* A, const hdcr_coarse_deflation* defl, const void* b, void* x, hdcr_solve_stats* stats,
               double* history, int32_t history_cap, void* work, size_t work_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HDCR_H */
