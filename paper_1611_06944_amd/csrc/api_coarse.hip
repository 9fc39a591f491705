// C-ABI entry points of the coarse space: basis and little Dirac operator
// build, restriction, prolongation, coarse apply, export.
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "coarse.h"
#include "solver.h"

namespace hdcr {

int check_coarse_desc(const hdcr_coarse_desc* d) {
    if (!d) return fail(HDCR_EINVAL, "null coarse descriptor");
    int e = check_fine_desc(&d->fine);
    if (e) return e;
    if (d->fine.Ls % 2 != 0) return fail(HDCR_EINVAL, "the coarse space needs an even Ls (chiral halves of Gamma5)");
    if (d->fine.Ls > 512) return fail(HDCR_EINVAL, "the coarse space supports Ls <= 512");
    int64_t bvol = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (d->block[mu] < 1 || d->fine.L[mu] % d->block[mu] != 0)
            return fail(HDCR_EINVAL, "block[" + std::to_string(mu) + "] must divide L[" + std::to_string(mu) + "]");
        bvol *= d->block[mu];
    }
    const int64_t nhalf = bvol * (d->fine.Ls / 2) * 12;
    if (d->nvec < 1 || d->nvec > nhalf)
        return fail(HDCR_EINVAL, "nvec must be in [1, block dof / 2] (the dimension of one chirality half)");
    if (2 * d->nvec > 128) return fail(HDCR_EINVAL, "Nb = 2*nvec must be <= 128");
    return HDCR_OK;
}

CoarseGeom make_coarse_geom(const hdcr_coarse_desc* d) {
    CoarseGeom c;
    c.f = make_geom(&d->fine);
    c.bvol = 1;
    c.Nc = 1;
    int st = 1;
    for (int mu = 0; mu < 4; ++mu) {
        c.B[mu] = d->block[mu];
        c.C[mu] = d->fine.L[mu] / d->block[mu];
        c.bvol *= c.B[mu];
        c.Nc *= c.C[mu];
        c.cstride[mu] = st;
        st *= c.C[mu];
    }
    c.nvec = d->nvec;
    c.Nb = 2 * d->nvec;
    c.Lh = d->fine.Ls / 2;
    c.nhalf = c.bvol * c.Lh * 12;
    return c;
}

// columns of A built per pass of the class-split stencil
// columns per projection launch: at most 4 (one per wavefront of the projection work-group)
static int build_chunk(const CoarseGeom& c) { return c.Nb < 4 ? c.Nb : 4; }

size_t build_workspace_bytes(const CoarseGeom& c) {
    Carver w(nullptr, 0);
    const size_t fsz = (size_t)12 * c.f.N5;
    const int kc = build_chunk(c);
    w.take<double2>(fsz * kc);          // expanded basis fields
    w.take<double2>(fsz * kc * 9);      // class-split images
    w.take<double2>(coarse_elems(c));   // A in FP64
    w.take<double2>(coarse_project_scratch_elems(c));  // projection partial sums
    w.take<int>(64);                    // flags of the orthonormalisation
    w.take<double2>(chq_scratch_elems(c));  // Gram matrices and R^-1 of the Cholesky QR
    return w.used();
}

// bytes of one vector entry: FP32 vectors go with the C64 and F16C (FP16 basis) forms
static size_t csize(hdcr_dtype dt) { return dt == HDCR_C128 ? 16 : (dt == HDCR_C64 || dt == HDCR_F16C) ? 8 : 4; }

}  // namespace hdcr

namespace hdcr {
// tile shape chosen by the autotuner per (Nc, Nb, nrhs, terms, device)
static std::mutex tune_mutex;
static std::map<std::tuple<int, int, int, int, int>, int> tune_table;

static int tuned_variant(const CoarseGeom& c, int nrhs, int terms) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    std::lock_guard<std::mutex> lk(tune_mutex);
    auto it = tune_table.find(std::make_tuple(c.Nc, c.Nb, nrhs, terms, dev));
    if (it != tune_table.end()) return it->second;
    // untuned: for Nb = 64 the direction-outside variant (fastest measured at 12
    // to 192 right-hand sides; the only one for split vectors), else four
    // wavefronts per site where Nb allows them
    if (terms > 1 || coarse_mfma_eligible(c, 9, 1)) return 9;
    return coarse_mfma_eligible(c, 2, 1) ? 2 : 1;
}

static int check_batched(const hdcr_coarse_desc* desc, const void* A, const void* v, void* out, int nrhs,
                         const char* who) {
    int e = check_coarse_desc(desc);
    if (e) return e;
    if (nrhs < 1) return fail(HDCR_EINVAL, std::string(who) + ": nrhs must be >= 1");
    const int nb = 2 * desc->nvec;
    if (nb != 16 && nb != 32 && nb != 64 && nb != 128)
        return fail(HDCR_EINVAL, std::string(who) + ": needs Nb = 2 nvec in {16, 32, 64, 128}");
    if ((e = check_ptr(A, 16, "A")) || (e = check_ptr(v, 8, "v")) || (e = check_ptr(out, 8, "out"))) return e;
    const CoarseGeom c = make_coarse_geom(desc);
    const size_t bytes = (size_t)nrhs * c.Nc * c.Nb * 8;
    const char* pv = static_cast<const char*>(v);
    const char* po = static_cast<const char*>(out);
    if (pv < po + bytes && po < pv + bytes) return fail(HDCR_EINVAL, std::string(who) + ": v and out overlap");
    return HDCR_OK;
}
}  // namespace hdcr

using namespace hdcr;

extern "C" {

size_t hdcr_basis_bytes(const hdcr_coarse_desc* desc) {
    if (check_coarse_desc(desc)) return 0;
    return basis_bytes(make_coarse_geom(desc));
}

size_t hdcr_coarse_bytes(const hdcr_coarse_desc* desc, hdcr_dtype dtype) {
    if (check_coarse_desc(desc)) return 0;
    if (dtype != HDCR_C128 && dtype != HDCR_C64 && dtype != HDCR_BF16C) return 0;
    return coarse_bytes(make_coarse_geom(desc), dtype);
}

int hdcr_build_coarse(const hdcr_coarse_desc* desc, const void* U, const void* vecs, void* basis, void* A,
                      hdcr_dtype A_dtype, void* work, size_t work_bytes, hipStream_t stream) {
    int e = check_coarse_desc(desc);
    if (e) return e;
    if (A_dtype != HDCR_C128 && A_dtype != HDCR_C64 && A_dtype != HDCR_BF16C)
        return fail(HDCR_EINVAL, "hdcr_build_coarse: bad A dtype");
    if ((e = check_ptr(U, 16, "U")) || (e = check_ptr(vecs, 16, "vecs")) || (e = check_ptr(basis, 16, "basis")) ||
        (e = check_ptr(A, 16, "A")) || (e = check_ptr(work, 256, "work")))
        return e;
    const CoarseGeom c = make_coarse_geom(desc);
    if (work_bytes < build_workspace_bytes(c)) return fail(HDCR_ENOMEM, "hdcr_build_coarse: workspace too small");
    const size_t fsz = (size_t)12 * c.f.N5;
    const int kc = build_chunk(c);
    Carver w(work, work_bytes);
    double2* X = w.take<double2>(fsz * kc);
    double2* Y = w.take<double2>(fsz * kc * 9);
    double2* A64 = w.take<double2>(coarse_elems(c));
    double2* Pp = w.take<double2>(coarse_project_scratch_elems(c));
    int* flag = w.take<int>(64);
    double2* chq = w.take<double2>(chq_scratch_elems(c));
    double2* b64 = basis64(basis);
    // chiral split and block orthonormalisation: Cholesky QR twice where its
    // first pass's pivots are in reach (flag[1] clear), else Gram-Schmidt with
    // its rank test (flag[0])
    HDCR_HIP_CHECK(hipMemsetAsync(flag, 0, 3 * sizeof(int), stream));
    launch_basis_fold(c, static_cast<const double2*>(vecs), b64, stream);
    bool gs = !chq_ok(c);
    if (!gs) {
        launch_chq_pass(c, b64, chq, 0, flag, stream);
        int hf[2] = {0, 0};
        HDCR_HIP_CHECK(hipMemcpyAsync(hf, flag + 1, 2 * sizeof(int), hipMemcpyDeviceToHost, stream));
        HDCR_HIP_CHECK(hipStreamSynchronize(stream));
        gs = hf[0] != 0;
        if (!gs) {
            launch_chq_apply(c, b64, chq, stream);
            launch_chq_pass(c, b64, chq, 1, flag, stream);
            launch_chq_apply(c, b64, chq, stream);
        }
    }
    if (gs) launch_block_orth(c, b64, flag, stream);
    launch_basis_to_f32(c, b64, basis32(c, basis), stream);
    launch_basis_to_f16(c, b64, basis16(c, basis), stream);
    HDCR_HIP_CHECK(hipGetLastError());
    // A = P^dag H P, kc columns at a time
    double2* Adst = (A_dtype == HDCR_C128) ? static_cast<double2*>(A) : A64;
    const double2* U64 = static_cast<const double2*>(U);
    for (int k0 = 0; k0 < c.Nb; k0 += kc) {
        const int nk = (c.Nb - k0 < kc) ? c.Nb - k0 : kc;
        launch_basis_expand(c, b64, k0, nk, X, stream);
        for (int kk = 0; kk < nk; ++kk)
            launch_dslash_classes(c, U64, X + kk * fsz, Y + kk * 9 * fsz, fsz, stream);
        launch_coarse_project(c, b64, Y, k0, nk, Pp, Adst, stream);
        HDCR_HIP_CHECK(hipGetLastError());
    }
    if (A_dtype != HDCR_C128) launch_coarse_convert(c, A64, A_dtype, A, stream);
    HDCR_HIP_CHECK(hipGetLastError());
    int hflag[3] = {0, 0, 0};
    HDCR_HIP_CHECK(hipMemcpyAsync(hflag, flag, 3 * sizeof(int), hipMemcpyDeviceToHost, stream));
    HDCR_HIP_CHECK(hipStreamSynchronize(stream));
    if (hflag[0]) return fail(HDCR_ERANK, "hdcr_build_coarse: a block's subspace vectors are numerically dependent");
    if (hflag[2])
        return fail(HDCR_ERANK, "hdcr_build_coarse: the second Cholesky QR pass lost positive definiteness");
    return HDCR_OK;
}

int hdcr_convert_coarse(const hdcr_coarse_desc* desc, const void* A128, hdcr_dtype dtype, void* Adst,
                        hipStream_t stream) {
    int e = check_coarse_desc(desc);
    if (e) return e;
    if (dtype != HDCR_C64 && dtype != HDCR_BF16C) return fail(HDCR_EINVAL, "hdcr_convert_coarse: dtype C64 or BF16C");
    if ((e = check_ptr(A128, 16, "A128")) || (e = check_ptr(Adst, 4, "Adst"))) return e;
    const CoarseGeom c = make_coarse_geom(desc);
    launch_coarse_convert(c, static_cast<const double2*>(A128), dtype, Adst, stream);
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}

int hdcr_export_coarse(const hdcr_coarse_desc* desc, hdcr_dtype dtype, const void* A, void* out, hipStream_t stream) {
    int e = check_coarse_desc(desc);
    if (e) return e;
    if (dtype != HDCR_C128 && dtype != HDCR_C64 && dtype != HDCR_BF16C)
        return fail(HDCR_EINVAL, "hdcr_export_coarse: bad dtype");
    if ((e = check_ptr(A, 4, "A")) || (e = check_ptr(out, 16, "out"))) return e;
    const CoarseGeom c = make_coarse_geom(desc);
    launch_coarse_export(c, dtype, A, static_cast<double2*>(out), stream);
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}

int hdcr_export_basis(const hdcr_coarse_desc* desc, const void* basis, void* fields, hipStream_t stream) {
    int e = check_coarse_desc(desc);
    if (e) return e;
    if ((e = check_ptr(basis, 16, "basis")) || (e = check_ptr(fields, 16, "fields"))) return e;
    const CoarseGeom c = make_coarse_geom(desc);
    launch_basis_expand(c, basis64(basis), 0, c.Nb, static_cast<double2*>(fields), stream);
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}

int hdcr_restrict(const hdcr_coarse_desc* desc, hdcr_dtype dtype, const void* basis, const void* psi, void* v,
                  hipStream_t stream) {
    int e = check_coarse_desc(desc);
    if (e) return e;
    if (dtype != HDCR_C128 && dtype != HDCR_C64 && dtype != HDCR_F16C)
        return fail(HDCR_EINVAL, "hdcr_restrict: dtype C128, C64 or F16C");
    if ((e = check_ptr(basis, 16, "basis")) || (e = check_ptr(psi, csize(dtype), "psi")) ||
        (e = check_ptr(v, csize(dtype), "v")))
        return e;
    const CoarseGeom c = make_coarse_geom(desc);
    if (dtype == HDCR_C128)
        launch_restrict<double>(c, basis64(basis), static_cast<const double2*>(psi), nullptr, static_cast<double2*>(v),
                                stream);
    else if (dtype == HDCR_F16C)
        launch_restrict_h(c, basis16(c, basis), static_cast<const float2*>(psi), nullptr, static_cast<float2*>(v),
                          stream);
    else
        launch_restrict<float>(c, basis32(c, basis), static_cast<const float2*>(psi), nullptr, static_cast<float2*>(v),
                               stream);
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}

int hdcr_prolong(const hdcr_coarse_desc* desc, hdcr_dtype dtype, const void* basis, const void* v, void* psi,
                 hipStream_t stream) {
    int e = check_coarse_desc(desc);
    if (e) return e;
    if (dtype != HDCR_C128 && dtype != HDCR_C64 && dtype != HDCR_F16C)
        return fail(HDCR_EINVAL, "hdcr_prolong: dtype C128, C64 or F16C");
    if ((e = check_ptr(basis, 16, "basis")) || (e = check_ptr(psi, csize(dtype), "psi")) ||
        (e = check_ptr(v, csize(dtype), "v")))
        return e;
    const CoarseGeom c = make_coarse_geom(desc);
    if (dtype == HDCR_C128)
        launch_prolong<double>(c, basis64(basis), static_cast<const double2*>(v), nullptr, static_cast<double2*>(psi),
                               stream);
    else if (dtype == HDCR_F16C)
        launch_prolong_h(c, basis16(c, basis), static_cast<const float2*>(v), nullptr, static_cast<float2*>(psi),
                         stream);
    else
        launch_prolong<float>(c, basis32(c, basis), static_cast<const float2*>(v), nullptr, static_cast<float2*>(psi),
                              stream);
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}

int hdcr_apply_coarse(const hdcr_coarse_desc* desc, hdcr_dtype dtype, const void* A, const void* v, void* out,
                      int32_t nrhs, hipStream_t stream) {
    int e = check_coarse_desc(desc);
    if (e) return e;
    if (dtype != HDCR_C128 && dtype != HDCR_C64 && dtype != HDCR_BF16C)
        return fail(HDCR_EINVAL, "hdcr_apply_coarse: bad dtype");
    if (nrhs < 1 || nrhs > 65535) return fail(HDCR_EINVAL, "hdcr_apply_coarse: nrhs in [1, 65535]");
    const hdcr_dtype vdt = (dtype == HDCR_C128) ? HDCR_C128 : HDCR_C64;
    if ((e = check_ptr(A, 4, "A")) || (e = check_ptr(v, csize(vdt), "v")) || (e = check_ptr(out, csize(vdt), "out")))
        return e;
    const CoarseGeom c = make_coarse_geom(desc);
    const size_t vb = (size_t)nrhs * c.Nc * c.Nb * csize(vdt);
    const char* pv = static_cast<const char*>(v);
    const char* po = static_cast<const char*>(out);
    if (pv < po + vb && po < pv + vb) return fail(HDCR_EINVAL, "hdcr_apply_coarse: v and out overlap");
    if (dtype == HDCR_C128)
        launch_coarse_apply<double>(c, static_cast<const double2*>(A), static_cast<const double2*>(v),
                                    static_cast<double2*>(out), nrhs, stream);
    else if (dtype == HDCR_C64)
        launch_coarse_apply<float>(c, static_cast<const float2*>(A), static_cast<const float2*>(v),
                                   static_cast<float2*>(out), nrhs, stream);
    else
        launch_coarse_apply_bf16(c, static_cast<const uint16_t*>(A), static_cast<const float2*>(v),
                                 static_cast<float2*>(out), nrhs, stream);
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}


int hdcr_apply_coarse_batched(const hdcr_coarse_desc* desc, const void* A, const void* v, void* out, int32_t nrhs,
                              int32_t variant, int32_t rhs_terms, hipStream_t stream) {
    int e = check_batched(desc, A, v, out, nrhs, "hdcr_apply_coarse_batched");
    if (e) return e;
    if (variant < 0 || variant > coarse_mfma_variants())
        return fail(HDCR_EINVAL, "hdcr_apply_coarse_batched: variant out of range");
    if (rhs_terms < 1 || rhs_terms > 3) return fail(HDCR_EINVAL, "hdcr_apply_coarse_batched: rhs_terms must be 1, 2 or 3");
    const CoarseGeom c = make_coarse_geom(desc);
    if (variant == 0) variant = tuned_variant(c, nrhs, rhs_terms);
    if (!coarse_mfma_eligible(c, variant, rhs_terms))
        return fail(HDCR_EINVAL, "hdcr_apply_coarse_batched: variant " + std::to_string(variant) + " with " +
                                     std::to_string(rhs_terms) +
                                     " term(s) does not apply to this shape (waves per site <= Nb / 8; variants 7 to "
                                     "9 need Nb = 64; 2 or 3 terms need variant 9)");
    launch_coarse_mfma(c, variant, rhs_terms, static_cast<const uint32_t*>(A), static_cast<const float2*>(v),
                       static_cast<float2*>(out), nrhs, stream);
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}

int hdcr_tune_coarse_batched(const hdcr_coarse_desc* desc, const void* A, const void* v, void* out, int32_t nrhs,
                             int32_t rhs_terms, int32_t* best, double* ms, hipStream_t stream) {
    int e = check_batched(desc, A, v, out, nrhs, "hdcr_tune_coarse_batched");
    if (e) return e;
    if (rhs_terms < 1 || rhs_terms > 3) return fail(HDCR_EINVAL, "hdcr_tune_coarse_batched: rhs_terms must be 1, 2 or 3");
    const CoarseGeom c = make_coarse_geom(desc);
    const int nv = coarse_mfma_variants();
    constexpr int REPS = 7;
    hipEvent_t ev[REPS + 1];
    for (int i = 0; i <= REPS; ++i) HDCR_HIP_CHECK(hipEventCreate(&ev[i]));
    int win = 0;
    double win_ms = 0;
    for (int k = 1; k <= nv; ++k) {
        if (!coarse_mfma_eligible(c, k, rhs_terms)) {
            if (ms) ms[k - 1] = -1.0;
            continue;
        }
        const uint32_t* Au = static_cast<const uint32_t*>(A);
        launch_coarse_mfma(c, k, rhs_terms, Au, static_cast<const float2*>(v), static_cast<float2*>(out), nrhs,
                           stream);  // warm-up
        HDCR_HIP_CHECK(hipEventRecord(ev[0], stream));
        for (int i = 0; i < REPS; ++i) {
            launch_coarse_mfma(c, k, rhs_terms, Au, static_cast<const float2*>(v), static_cast<float2*>(out), nrhs,
                               stream);
            HDCR_HIP_CHECK(hipEventRecord(ev[i + 1], stream));
        }
        HDCR_HIP_CHECK(hipGetLastError());
        HDCR_HIP_CHECK(hipEventSynchronize(ev[REPS]));
        std::vector<double> t(REPS);
        for (int i = 0; i < REPS; ++i) {
            float f = 0;
            HDCR_HIP_CHECK(hipEventElapsedTime(&f, ev[i], ev[i + 1]));
            t[i] = f;
        }
        std::sort(t.begin(), t.end());
        const double med = t[REPS / 2];
        if (ms) ms[k - 1] = med;
        if (win == 0 || med < win_ms) {
            win = k;
            win_ms = med;
        }
    }
    for (int i = 0; i <= REPS; ++i) (void)hipEventDestroy(ev[i]);
    int dev = 0;
    HDCR_HIP_CHECK(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(tune_mutex);
        tune_table[std::make_tuple(c.Nc, c.Nb, (int)nrhs, (int)rhs_terms, dev)] = win;
    }
    if (best) *best = win;
    return HDCR_OK;
}
}  // extern "C"
