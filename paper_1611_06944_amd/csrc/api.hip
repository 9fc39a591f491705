// C-ABI entry points: argument validation, workspace sizing and dispatch.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>

#include "twolevel.h"

namespace hdcr {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

int fail(int code, const std::string& msg) {
    set_error(msg);
    return code;
}

FineGeom make_geom(const hdcr_fine_desc* d) {
    FineGeom g;
    for (int i = 0; i < 4; ++i) {
        g.L[i] = d->L[i];
        g.bc[i] = d->bc[i];
    }
    g.Ls = d->Ls;
    g.V4 = d->L[0] * d->L[1] * d->L[2] * d->L[3];
    g.N5 = g.V4 * g.Ls;
    int st = 1;
    for (int i = 0; i < 4; ++i) {
        g.stride[i] = st;
        g.wrap[i] = (d->L[i] - 1) * st;
        st *= d->L[i];
    }
    const double b = (d->cayley_b == 0.0) ? 1.0 : d->cayley_b;
    g.diag = b * (4.0 - d->M5) + 1.0;
    g.hop = -0.5 * b;
    g.mf = d->mf;
    g.tune = d->tune;
    choose_traversal(g, 0, 0);
    return g;
}

void choose_traversal(FineGeom& g, int tslab, int ysplit, int xsplit) {
    const int Lt = g.L[3], Ly = g.L[1];
    // the caller's traversal choices replace the defaults
    if (g.tune.tslab) tslab = g.tune.tslab;
    if (g.tune.ysplit) ysplit = g.tune.ysplit;
    if (g.tune.xsplit) xsplit = g.tune.xsplit;
    if (xsplit < 1 || g.L[0] % xsplit != 0) xsplit = 1;
    if (tslab <= 0) {
        // one slab per XCD when Lt allows it, else the whole t extent
        tslab = (Lt % NUM_XCD == 0) ? Lt / NUM_XCD : Lt;
        if (tslab < 1) tslab = 1;
    }
    if (Lt % tslab != 0) tslab = Lt;
    if (ysplit <= 0) {
        // y parts of about 8 rows: the z-neighbour re-reads of a slab stay
        // within the XCD's L2 (measured best at 24^4 x 16)
        ysplit = Ly / 8;
        if (ysplit < 1) ysplit = 1;
        while (ysplit > 1 && Ly % ysplit != 0) --ysplit;
    }
    if (Ly % ysplit != 0) ysplit = 1;
    g.tslab = tslab;
    g.xsplit = xsplit;
    g.ysplit = ysplit;
    g.variant = g.tune.dslash_variant;
}

int check_fine_desc(const hdcr_fine_desc* d) {
    if (!d) return fail(HDCR_EINVAL, "null fine descriptor");
    int64_t v = 1;
    for (int i = 0; i < 4; ++i) {
        if (d->L[i] < 1) return fail(HDCR_EINVAL, "lattice extent L[" + std::to_string(i) + "] must be >= 1");
        if (d->bc[i] != 1 && d->bc[i] != -1)
            return fail(HDCR_EINVAL, "bc[" + std::to_string(i) + "] must be +1 or -1");
        v *= d->L[i];
    }
    if (d->Ls < 1) return fail(HDCR_EINVAL, "Ls must be >= 1");
    // kernels address a whole FP64 field with 32-bit byte offsets
    if (v * d->Ls * 12 * 16 >= (int64_t(1) << 32) || v * 36 * 16 >= (int64_t(1) << 32))
        return fail(HDCR_EINVAL, "lattice too large (an FP64 fine field and gauge field must stay below 4 GiB)");
    if (!std::isfinite(d->M5) || !std::isfinite(d->mf)) return fail(HDCR_EINVAL, "M5 and mf must be finite");
    if (!std::isfinite(d->cayley_b) || d->cayley_b < 0.0)
        return fail(HDCR_EINVAL, "cayley_b must be finite and >= 0 (0 selects b = 1)");
    return HDCR_OK;
}

int check_ptr(const void* p, size_t align, const char* name) {
    if (!p) return fail(HDCR_EINVAL, std::string("null pointer: ") + name);
    if (reinterpret_cast<uintptr_t>(p) % align)
        return fail(HDCR_EINVAL, std::string("misaligned pointer: ") + name);
    return HDCR_OK;
}

static size_t csize(hdcr_dtype dt) { return dt == HDCR_C128 ? 16 : dt == HDCR_C64 ? 8 : 4; }

}  // namespace hdcr

using namespace hdcr;

extern "C" {

const char* hdcr_strerror(int code) {
    switch (code) {
        case HDCR_OK: return "success";
        case HDCR_EINVAL: return "invalid argument";
        case HDCR_EHIP: return "HIP runtime error";
        case HDCR_ENOMEM: return "workspace too small";
        case HDCR_ENOTCONV: return "not converged within maxiter";
        case HDCR_EBREAKDOWN: return "Krylov breakdown";
        case HDCR_ENAN: return "NaN or Inf in the residual";
        case HDCR_ERANK: return "block basis rank deficient";
        default: return "unknown status";
    }
}

const char* hdcr_last_error(void) { return hdcr::last_error_cstr(); }

int hdcr_apply_fine(const hdcr_fine_desc* desc, hdcr_dtype dtype, const void* U, const void* psi, void* out,
                    hipStream_t stream) {
    int e = check_fine_desc(desc);
    if (e) return e;
    if (dtype != HDCR_C128 && dtype != HDCR_C64 && dtype != HDCR_F16C)
        return fail(HDCR_EINVAL, "hdcr_apply_fine: dtype must be C128, C64 or F16C");
    const size_t cs = csize(dtype);
    const size_t us = dtype == HDCR_F16C ? 8 : cs;  // F16C fields take C64 links
    if ((e = check_ptr(U, us, "U")) || (e = check_ptr(psi, cs, "psi")) || (e = check_ptr(out, cs, "out"))) return e;
    const FineGeom g = make_geom(desc);
    const size_t fbytes = (size_t)12 * g.N5 * cs;
    if (overlap(psi, fbytes, out, fbytes)) return fail(HDCR_EINVAL, "hdcr_apply_fine: psi and out overlap");
    if (dtype == HDCR_F16C) {
        if (!dslash_h16_ok(g)) return fail(HDCR_EINVAL, "hdcr_apply_fine: F16C needs Ls = 16 and even extents");
        launch_dslash_h16(g, (const float2*)U, psi, out, stream);
    } else if (dtype == HDCR_C128)
        launch_dslash<double>(g, (const double2*)U, (const double2*)psi, (double2*)out, stream);
    else
        launch_dslash<float>(g, (const float2*)U, (const float2*)psi, (float2*)out, stream);
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}

int hdcr_apply_cf(const hdcr_fine_desc* desc, hdcr_dtype dtype, const double* beta, double R, const void* U,
                  const void* psi, void* out, hipStream_t stream) {
    int e = check_fine_desc(desc);
    if (e) return e;
    if (dtype != HDCR_C128 && dtype != HDCR_C64) return fail(HDCR_EINVAL, "hdcr_apply_cf: dtype must be C128 or C64");
    const int Ls = desc->Ls, m = Ls - 1;
    if (Ls < 2 || Ls > CF_MAX_LS)
        return fail(HDCR_EINVAL, "hdcr_apply_cf: Ls (pole slices + 1) must be in [2, " + std::to_string(CF_MAX_LS) + "]");
    if (desc->cayley_b != 0.0 && desc->cayley_b != 1.0)
        return fail(HDCR_EINVAL, "hdcr_apply_cf: the Wilson kernel has no Cayley scale (cayley_b must be 0 or 1)");
    if (!beta) return fail(HDCR_EINVAL, "hdcr_apply_cf: null beta");
    for (int i = 0; i < m; ++i)
        if (!std::isfinite(beta[i]) || !(beta[i] > 0.0))
            return fail(HDCR_EINVAL, "hdcr_apply_cf: beta[" + std::to_string(i) + "] must be finite and > 0");
    if (!std::isfinite(R)) return fail(HDCR_EINVAL, "hdcr_apply_cf: R must be finite");
    const size_t cs = csize(dtype);
    if ((e = check_ptr(U, cs, "U")) || (e = check_ptr(psi, cs, "psi")) || (e = check_ptr(out, cs, "out"))) return e;
    const FineGeom g = make_geom(desc);
    const size_t fbytes = (size_t)12 * g.N5 * cs;
    if (overlap(psi, fbytes, out, fbytes)) return fail(HDCR_EINVAL, "hdcr_apply_cf: psi and out overlap");
    // the printed matrix continued to m pole slices: (-1)^i H_W on slice i < m,
    // R gamma5 + beta_0 H_W on slice m; slices i, i + 1 coupled by
    // 1/sqrt(beta_i beta_(i+1)) (i < m - 1) and 1/sqrt(beta_(m-1)) (i = m - 1)
    CfCoef k{};
    for (int i = 0; i < Ls; ++i) {
        k.sigma[i] = (i < m) ? ((i % 2) ? -1.0 : 1.0) : beta[0];
        const double c_up = (i < m - 1) ? 1.0 / std::sqrt(beta[i] * beta[i + 1]) : (i == m - 1 ? 1.0 / std::sqrt(beta[i]) : 0.0);
        k.cup[i] = c_up;
        if (i + 1 < Ls) k.cdn[i + 1] = c_up;
    }
    k.cdn[0] = 0.0;
    k.R = R;
    k.wdiag = 4.0 - desc->M5;
    k.sites = Ls <= 16 ? 16 : 256 / Ls;
    if (dtype == HDCR_C128)
        launch_cf<double>(g, k, (const double2*)U, (const double2*)psi, (double2*)out, stream);
    else
        launch_cf<float>(g, k, (const float2*)U, (const float2*)psi, (float2*)out, stream);
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}

int hdcr_fermion_force(const hdcr_fine_desc* desc, hdcr_dtype dtype, const void* U, const void* chi, const void* psi,
                       void* W, void* T, hipStream_t stream) {
    int e = check_fine_desc(desc);
    if (e) return e;
    if (dtype != HDCR_C128 && dtype != HDCR_C64)
        return fail(HDCR_EINVAL, "hdcr_fermion_force: dtype must be C128 or C64");
    if (!W && !T) return fail(HDCR_EINVAL, "hdcr_fermion_force: W and T are both NULL");
    const size_t cs = csize(dtype);
    if ((e = check_ptr(U, cs, "U")) || (e = check_ptr(chi, cs, "chi")) || (e = check_ptr(psi, cs, "psi"))) return e;
    if ((W && (e = check_ptr(W, cs, "W"))) || (T && (e = check_ptr(T, cs, "T")))) return e;
    const FineGeom g = make_geom(desc);
    const size_t fbytes = (size_t)12 * g.N5 * cs, gbytes = (size_t)36 * g.V4 * cs;
    for (void* o : {W, T}) {
        if (!o) continue;
        if (overlap(o, gbytes, U, gbytes) || overlap(o, gbytes, chi, fbytes) || overlap(o, gbytes, psi, fbytes))
            return fail(HDCR_EINVAL, "hdcr_fermion_force: an output overlaps an input");
    }
    if (W && T && overlap(W, gbytes, T, gbytes)) return fail(HDCR_EINVAL, "hdcr_fermion_force: W and T overlap");
    // the caller's work split (tune.force_*; 0 = the default choice)
    const hdcr_tuning& tu = desc->tune;
    if (tu.force_sum < 0 || tu.force_sum > 2)
        return fail(HDCR_EINVAL, "hdcr_fermion_force: tune.force_sum must be 0, 1 (DPP) or 2 (LDS)");
    const ForceShape f =
        choose_force_shape(g, (int)cs, tu.force_r, tu.force_ms, tu.force_p, tu.force_sum == 0 ? -1 : tu.force_sum - 1);
    if (!force_shape_ok(g, (int)cs, f))
        return fail(HDCR_EINVAL, "hdcr_fermion_force: unsupported work split (tune.force_r/ms/p)");
    if (dtype == HDCR_C128)
        launch_link_force<double>(g, f, (const double2*)U, (const double2*)chi, (const double2*)psi, (double2*)W,
                                  (double2*)T, stream);
    else
        launch_link_force<float>(g, f, (const float2*)U, (const float2*)chi, (const float2*)psi, (float2*)W,
                                 (float2*)T, stream);
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}

int hdcr_vec_dot(hdcr_dtype dtype, int64_t n, const void* x, const void* y, double* out, void* work, size_t work_bytes,
                 hipStream_t stream) {
    if (dtype != HDCR_C128 && dtype != HDCR_C64) return fail(HDCR_EINVAL, "hdcr_vec_dot: dtype must be C128 or C64");
    if (n < 0) return fail(HDCR_EINVAL, "hdcr_vec_dot: n < 0");
    if (!out) return fail(HDCR_EINVAL, "hdcr_vec_dot: null out");
    int e;
    if (n > 0 && ((e = check_ptr(x, csize(dtype), "x")) || (e = check_ptr(y, csize(dtype), "y")))) return e;
    if ((e = check_ptr(work, 256, "work"))) return e;
    if (work_bytes < HDCR_DOT_WORK_BYTES) return fail(HDCR_ENOMEM, "hdcr_vec_dot: work smaller than HDCR_DOT_WORK_BYTES");
    double2* scratch = static_cast<double2*>(work);
    if (dtype == HDCR_C128)
        launch_dot<double>(n, (const double2*)x, (const double2*)y, scratch, scratch + REDUCE_BLOCKS, stream);
    else
        launch_dot<float>(n, (const float2*)x, (const float2*)y, scratch, scratch + REDUCE_BLOCKS, stream);
    HDCR_HIP_CHECK(hipGetLastError());
    double2 h;
    HDCR_HIP_CHECK(hipMemcpyAsync(&h, scratch + REDUCE_BLOCKS, sizeof(h), hipMemcpyDeviceToHost, stream));
    HDCR_HIP_CHECK(hipStreamSynchronize(stream));
    out[0] = h.x;
    out[1] = h.y;
    return HDCR_OK;
}

int hdcr_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t stream) {
    int e;
    if (bytes % 16) return fail(HDCR_EINVAL, "hdcr_stream_copy: bytes must be a multiple of 16");
    if (bytes == 0) return HDCR_OK;
    if ((e = check_ptr(src, 16, "src")) || (e = check_ptr(dst, 16, "dst"))) return e;
    if (overlap(src, bytes, dst, bytes)) return fail(HDCR_EINVAL, "hdcr_stream_copy: src and dst overlap");
    launch_stream_copy(src, dst, bytes, stream);
    HDCR_HIP_CHECK(hipGetLastError());
    return HDCR_OK;
}

size_t hdcr_workspace_bytes(int which, const hdcr_coarse_desc* desc, const hdcr_solve_params* params) {
    if (!desc || check_fine_desc(&desc->fine)) return 0;
    const FineGeom g = make_geom(&desc->fine);
    switch (which) {
        case HDCR_WS_SOLVE:
            if (!params) return 0;
            if (params->precond == HDCR_PRECOND_NONE) return cr_workspace_bytes(g);
            if (check_coarse_desc(desc) || check_two_level_params(params)) return 0;
            return two_level_workspace_bytes(make_coarse_geom(desc), params);
        case HDCR_WS_VCYCLE:
            if (!params || check_coarse_desc(desc) || check_two_level_params(params)) return 0;
            return vcycle_workspace_bytes(make_coarse_geom(desc), params);
        case HDCR_WS_SMOOTH:
            return (size_t)4 * 12 * g.N5 * 16 + 4 * 256;
        case HDCR_WS_SUBSPACE:
            return hdcr_subspace_workspace_bytes(&desc->fine, (params && params->inner_dtype == HDCR_C64) ? HDCR_C64
                                                                                                         : HDCR_C128);
        case HDCR_WS_BUILD:
            if (check_coarse_desc(desc)) return 0;
            return build_workspace_bytes(make_coarse_geom(desc));
        case HDCR_WS_COARSE:
            if (!params || check_coarse_desc(desc)) return 0;
            if (params->coarse_dtype == HDCR_C128) return coarse_cr_bytes<double>(make_coarse_geom(desc));
            if (params->coarse_dtype == HDCR_C64 || params->coarse_dtype == HDCR_BF16C)
                return coarse_cr_bytes<float>(make_coarse_geom(desc));
            return 0;
        default:
            return 0;
    }
}

int hdcr_solve(const hdcr_coarse_desc* desc, const hdcr_solve_params* params, const void* U, const void* basis,
               const void* A, const hdcr_coarse_deflation* defl, const void* b, void* x, hdcr_solve_stats* stats,
               double* history, int32_t history_cap, void* work, size_t work_bytes, hipStream_t stream) {
    if (!desc || !params) return fail(HDCR_EINVAL, "hdcr_solve: null descriptor or params");
    int e = check_fine_desc(&desc->fine);
    if (e) return e;
    if ((e = check_ptr(U, 16, "U")) || (e = check_ptr(b, 16, "b")) || (e = check_ptr(x, 16, "x")) ||
        (e = check_ptr(work, 256, "work")))
        return e;
    if (!(params->tol > 0) || params->maxiter < 0) return fail(HDCR_EINVAL, "hdcr_solve: tol must be > 0, maxiter >= 0");
    if (history_cap < 0 || (history_cap > 0 && !history)) return fail(HDCR_EINVAL, "hdcr_solve: bad history buffer");
    const FineGeom g = make_geom(&desc->fine);
    const size_t fbytes = (size_t)12 * g.N5 * 16;
    if (overlap(b, fbytes, x, fbytes)) return fail(HDCR_EINVAL, "hdcr_solve: b and x overlap");
    if (params->precond == HDCR_PRECOND_NONE) {
        if (work_bytes < cr_workspace_bytes(g)) return fail(HDCR_ENOMEM, "hdcr_solve: workspace too small");
        return cr_solve(g, params, (const double2*)U, (const double2*)b, (double2*)x, stats, history, history_cap,
                        work, work_bytes, stream);
    }
    if (params->precond != HDCR_PRECOND_TWO_LEVEL) return fail(HDCR_EINVAL, "hdcr_solve: unknown precond");
    if ((e = check_coarse_desc(desc))) return e;
    if ((e = check_two_level_params(params))) return e;
    if ((e = check_ptr(basis, 16, "basis")) || (e = check_ptr(A, 4, "A"))) return e;
    const CoarseGeom c = make_coarse_geom(desc);
    if (params->inner_dtype == HDCR_F16C && !dslash_h16_ok(c.f))
        return fail(HDCR_EINVAL, "hdcr_solve: inner F16C needs Ls = 16 and even extents");
    if (defl && (e = check_deflation(c, defl, params->inner_dtype == HDCR_C128 ? HDCR_C128 : HDCR_C64, "hdcr_solve")))
        return e;
    if (work_bytes < two_level_workspace_bytes(c, params)) return fail(HDCR_ENOMEM, "hdcr_solve: workspace too small");
    return two_level_solve(c, params, (const double2*)U, basis, A, defl, (const double2*)b, (double2*)x, stats,
                           history, history_cap, work, work_bytes, stream);
}

}  // extern "C"
