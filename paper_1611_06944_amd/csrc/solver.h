// Host-side solver plumbing shared by the solver sources.
#pragma once

#include "internal.h"

namespace hdcr {

// Carves aligned sub-buffers out of the caller's workspace.  With base ==
// nullptr it only counts bytes (used by hdcr_workspace_bytes).
class Carver {
  public:
    Carver(void* base, size_t cap) : base_(static_cast<char*>(base)), cap_(cap) {}
    template <typename T> T* take(size_t count) {
        off_ = (off_ + 255) & ~size_t(255);
        T* p = base_ ? reinterpret_cast<T*>(base_ + off_) : nullptr;
        off_ += count * sizeof(T);
        return p;
    }
    size_t used() const { return (off_ + 255) & ~size_t(255); }
    bool ok() const { return base_ != nullptr && off_ <= cap_; }

  private:
    char* base_;
    size_t cap_;
    size_t off_ = 0;
};

// true if the byte ranges [a, a + na) and [b, b + nb) intersect
inline bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}

// Sums nq rows of REDUCE_BLOCKS partials (row q at partials + q*REDUCE_BLOCKS)
// in fixed order; S[d0] = row 0, S[d1] = row 1 (if nq == 2).  Afterwards, if
// csrc >= 0, S[cdst] = S[csrc] (old value of csrc).
void launch_finalize_real(const double* partials, int nq, double* S, int d0, int d1, int csrc, int cdst,
                          hipStream_t s);

size_t cr_workspace_bytes(const FineGeom& g);
int cr_solve(const FineGeom& g, const hdcr_solve_params* prm, const double2* U, const double2* b, double2* x,
             hdcr_solve_stats* st, double* history, int hcap, void* work, size_t work_bytes, hipStream_t s);

}  // namespace hdcr
