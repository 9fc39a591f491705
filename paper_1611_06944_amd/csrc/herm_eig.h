// Eigenvalues and eigenvectors of a small complex Hermitian matrix (host code,
// no HIP), by cyclic Jacobi rotations.  Used for the Rayleigh-Ritz steps of the
// coarse deflation set-up, whose matrices are at most 64 x 64.
//
// A rotation on the index pair (p, q) with H_pq = r e (r = |H_pq|, |e| = 1) is the
// unitary G with columns g_p = (c, -s conj(e)) and g_q = (s e, c) in rows (p, q);
// (G^dag H G)_pq = e [r (c^2 - s^2) + (H_pp - H_qq) s c] vanishes for t = s / c the
// smaller root of t^2 + 2 th t - 1 = 0, th = (H_qq - H_pp) / (2 r).
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

namespace hdcr {

// H: m x m, row-major, Hermitian (only its Hermitian part is used).  On return
// lam holds the eigenvalues in ascending order and V (row-major, m x m) the
// eigenvectors as columns: H V[:, j] = lam[j] V[:, j].  Returns the number of
// sweeps, or -1 if the off-diagonal part did not fall below the tolerance.
inline int herm_eig(int m, const std::complex<double>* H_in, double* lam, std::complex<double>* V) {
    typedef std::complex<double> cd;
    std::vector<cd> H(H_in, H_in + (size_t)m * m);
    for (int i = 0; i < m; ++i)
        for (int j = i; j < m; ++j) {
            const cd hij = 0.5 * (H[(size_t)i * m + j] + std::conj(H[(size_t)j * m + i]));
            H[(size_t)i * m + j] = hij;
            H[(size_t)j * m + i] = std::conj(hij);
        }
    std::vector<cd> Q((size_t)m * m, cd(0.0, 0.0));
    for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;
    double fro = 0.0;
    for (size_t i = 0; i < (size_t)m * m; ++i) fro += std::norm(H[i]);
    fro = std::sqrt(fro);
    const double tol = 1e-15 * (fro > 0 ? fro : 1.0);
    int sweep = 0, status = -1;
    for (; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j)
                if (i != j) off += std::norm(H[(size_t)i * m + j]);
        if (std::sqrt(off) <= tol) {
            status = sweep;
            break;
        }
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                const cd hpq = H[(size_t)p * m + q];
                const double r = std::abs(hpq);
                if (r <= 1e-300) continue;
                const cd e = hpq / r;
                const double a = H[(size_t)p * m + p].real(), b = H[(size_t)q * m + q].real();
                const double th = (b - a) / (2.0 * r);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                const cd gpp = c, gqp = -s * std::conj(e), gpq = s * e, gqq = c;
                // H <- H G (columns p, q), Q <- Q G
                for (int k = 0; k < m; ++k) {
                    const cd hp = H[(size_t)k * m + p], hq = H[(size_t)k * m + q];
                    H[(size_t)k * m + p] = hp * gpp + hq * gqp;
                    H[(size_t)k * m + q] = hp * gpq + hq * gqq;
                    const cd vp = Q[(size_t)k * m + p], vq = Q[(size_t)k * m + q];
                    Q[(size_t)k * m + p] = vp * gpp + vq * gqp;
                    Q[(size_t)k * m + q] = vp * gpq + vq * gqq;
                }
                // H <- G^dag H (rows p, q)
                for (int k = 0; k < m; ++k) {
                    const cd hp = H[(size_t)p * m + k], hq = H[(size_t)q * m + k];
                    H[(size_t)p * m + k] = std::conj(gpp) * hp + std::conj(gqp) * hq;
                    H[(size_t)q * m + k] = std::conj(gpq) * hp + std::conj(gqq) * hq;
                }
                H[(size_t)p * m + q] = H[(size_t)q * m + p] = 0.0;
                H[(size_t)p * m + p] = H[(size_t)p * m + p].real();
                H[(size_t)q * m + q] = H[(size_t)q * m + q].real();
            }
    }
    std::vector<int> order(m);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(),
              [&](int i, int j) { return H[(size_t)i * m + i].real() < H[(size_t)j * m + j].real(); });
    for (int j = 0; j < m; ++j) {
        lam[j] = H[(size_t)order[j] * m + order[j]].real();
        for (int i = 0; i < m; ++i) V[(size_t)i * m + j] = Q[(size_t)i * m + order[j]];
    }
    return status;
}

}  // namespace hdcr
