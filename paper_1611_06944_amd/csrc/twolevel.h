// Two-level solver (Sec. 4): coarse CR, Chebyshev smoother, the symmetric
// two-level cycle, flexible GCR, and the subspace filter.
#pragma once

#include <vector>

#include "coarse.h"
#include "solver.h"
#include "vec.h"

namespace hdcr {

// Event-timed phases of a solve.
struct PhaseTimer {
    enum Phase { FINE = 0, COARSE = 1, OUTER = 2 };
    struct Rec {
        hipEvent_t a, b;
        int phase;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipStream_t s = nullptr;
    bool on = false;
    int open_phase = -1;
    hipEvent_t open_ev = nullptr;
    hipEvent_t get();
    void begin(int phase);
    void end();
    void totals(double out[3]);  // call after the stream has been synchronised
    ~PhaseTimer();
};

template <typename T> size_t coarse_cr_bytes(const CoarseGeom& c);
template <typename T> CoarseCRWork<T> coarse_cr_carve(Carver& w, const CoarseGeom& c);

// x = CR_A(b) from x = 0: exactly maxiter iterations if tol <= 0, else until
// |r| <= tol |b| or maxiter.  Asynchronous except that the tolerance mode may
// synchronise to decide how many iterations to enqueue; *iters gets the count
// (after the stream has been synchronised) through flags[1].
// defl (may be null): start from the Galerkin projection on the deflation space.
// reason (may be null; tolerance mode only): why the iteration stopped early, 0
// (tolerance or maxiter), 2 (near-breakdown: |<r,Ar>| < eps |r||Ar|) or 3 (not finite).
template <typename T>
int coarse_cr(const CoarseGeom& c, hdcr_dtype A_dtype, const void* A, const C2<T>* b, C2<T>* x, int maxiter,
              double tol, const CoarseCRWork<T>& w, int hint, hipStream_t s, int* iters,
              const DeflView<T>* defl = nullptr, int* reason = nullptr);

// Chebyshev smoother out (+)= p(H^2) H in, p the order-term Chebyshev interpolant
// of 1/y on [lo, hi] (Sec. 4); tmp: 4 fine vectors of precision T.
template <typename T>
void cheb_smoother(const FineGeom& g, const C2<T>* U, const C2<T>* in, C2<T>* out, bool accumulate,
                   C2<T>* const tmp[4], int order, double lo, double hi, hipStream_t s);
// The same with FP16 storage of the smoother's fields (Ls = 16, even extents,
// order >= 2): in is scaled to unit RMS per entry and rounded to FP16 (the
// smoother is linear), the recurrence runs through the FP16-storage stencil,
// and the result is scaled back into the FP32 out.  h: six FP16 fields of
// 12 N5 entries (4 bytes each); part: REDUCE_BLOCKS doubles; S: one double.
void cheb_smoother_h16(const FineGeom& g, const float2* U, const float2* in, float2* out, bool accumulate,
                       void* const h[6], double* part, double* S, int order, double lo, double hi, hipStream_t s);

void cheby_coeffs(int n, double lo, double hi, double* c);

int check_two_level_params(const hdcr_solve_params* p);
size_t two_level_workspace_bytes(const CoarseGeom& c, const hdcr_solve_params* p);
// defl: the coarse deflation space (may be null), vectors in the inner precision
int check_deflation(const CoarseGeom& c, const hdcr_coarse_deflation* d, hdcr_dtype dtype, const char* where);
int two_level_solve(const CoarseGeom& c, const hdcr_solve_params* p, const double2* U, const void* basis,
                    const void* A, const hdcr_coarse_deflation* defl, const double2* b, double2* x,
                    hdcr_solve_stats* st, double* history, int hcap, void* work, size_t work_bytes, hipStream_t s);
size_t vcycle_workspace_bytes(const CoarseGeom& c, const hdcr_solve_params* p);
int vcycle_apply(const CoarseGeom& c, const hdcr_solve_params* p, const double2* U, const void* basis, const void* A,
                 const hdcr_coarse_deflation* defl, const double2* r, double2* e, void* work, size_t work_bytes,
                 hipStream_t s);

}  // namespace hdcr
