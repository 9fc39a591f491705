// FP64 CPU oracle for the HDCR hot path -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, obviously-correct loops over the canonical site-major layout
//   fermion  psi[t][z][y][x][s][spin][colour]   (std::complex<double>)
//   gauge    U[t][z][y][x][mu][row][col]         mu = x, y, z, t
//   coarse   v[site_c][k], A[site_c][d][j][k]    d in D9 = (0,+x,+y,+z,+t,-x,-y,-z,-t)
//
// Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
// may load this library. It shares no source, header or helper with the HIP
// library, and it never calls it.
//
// What each routine follows (Yamaguchi & Boyle, "Hierarchically deflated
// conjugate residual", Lattice 2016):
//   * H = gamma5 R5 D_dwf = Gamma5 D_dwf, the Hermitian indefinite domain wall
//     operator (Sec. 3). The paper does not write D_dwf out; the oracle uses
//     the Cayley form with c = 0 that Sec. 3 names, scale b = mob_b (b = 1: the
//     Shamir kernel):
//       (D psi)(x,s) = (b (4 - M5) + 1) psi(x,s)
//          - b/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu,s) + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu,s) ]
//          - P- psi(x,s+1) - P+ psi(x,s-1)
//       with the walls  -P- psi(x,Ls) -> +mf P- psi(x,0)  and  -P+ psi(x,-1) -> +mf P+ psi(x,Ls-1),
//       P+- = (1 +- g5)/2, a boundary-crossing 4d hop picks up bc[mu] (+1 periodic, -1 antiperiodic),
//     and (H psi)(x,s) = g5 (D psi)(x, Ls-1-s).
//   * chiral split of the subspace vectors into the two Gamma5 eigenspaces (Sec. 4),
//   * block-restricted vectors phi^b_k (Sec. 4, first display) made orthonormal per
//     block and chirality (Q of a thin QR, positive real R diagonal), so that
//     P_S = sum |phi^b_k><phi^b_k| is a projector (Sec. 4, projector display),
//   * restriction P^dag and prolongation P,
//   * little Dirac operator A^{ab}_{jk} = <phi^a_j | H | phi^b_k> (Sec. 4, little
//     Dirac operator display), split into the 9 nearest-neighbour blocks,
//   * the coarse 9-point apply.
// The Krylov solvers, the Chebyshev polynomials and the two-level cycle live in
// the Python half of the oracle (oracle/__init__.py) on top of these routines.

#include <complex>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

typedef std::complex<double> cd;

namespace {

struct Geom {
    int L[4];
    int Ls;
    long V4;
    explicit Geom(const int* dims) {
        for (int i = 0; i < 4; ++i) L[i] = dims[i];
        Ls = dims[4];
        V4 = (long)L[0] * L[1] * L[2] * L[3];
    }
    long site(const int x[4]) const {
        return (((long)x[3] * L[2] + x[2]) * L[1] + x[1]) * L[0] + x[0];
    }
    void coords(long i, int x[4]) const {
        x[0] = (int)(i % L[0]); i /= L[0];
        x[1] = (int)(i % L[1]); i /= L[1];
        x[2] = (int)(i % L[2]); i /= L[2];
        x[3] = (int)i;
    }
    // index of component (spin, colour) of the 5d site (x4, s)
    long idx(long x4, int s, int spin, int col) const {
        return ((x4 * Ls + s) * 4 + spin) * 3 + col;
    }
    long fdof() const { return V4 * Ls * 12; }
};

typedef cd Mat4[4][4];

void mat4_mul(const Mat4 a, const Mat4 b, Mat4 c) {
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cd s = 0;
            for (int k = 0; k < 4; ++k) s += a[i][k] * b[k][j];
            c[i][j] = s;
        }
}

// Chiral basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] for k = x, y, z;
// gamma_t = [[0, 1], [1, 0]]; gamma_5 = gamma_x gamma_y gamma_z gamma_t.
struct Gammas {
    Mat4 g[5];
    Gammas() {
        const cd I(0.0, 1.0);
        cd sig[3][2][2];
        sig[0][0][0] = 0; sig[0][0][1] = 1; sig[0][1][0] = 1; sig[0][1][1] = 0;
        sig[1][0][0] = 0; sig[1][0][1] = -I; sig[1][1][0] = I; sig[1][1][1] = 0;
        sig[2][0][0] = 1; sig[2][0][1] = 0; sig[2][1][0] = 0; sig[2][1][1] = -1;
        for (int m = 0; m < 5; ++m)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) g[m][a][b] = 0;
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    g[k][a][2 + b] = -I * sig[k][a][b];
                    g[k][2 + a][b] = I * sig[k][a][b];
                }
        for (int a = 0; a < 2; ++a) {
            g[3][a][2 + a] = 1;
            g[3][2 + a][a] = 1;
        }
        Mat4 t1, t2;
        mat4_mul(g[0], g[1], t1);
        mat4_mul(t1, g[2], t2);
        mat4_mul(t2, g[3], g[4]);
    }
};

const Gammas& gam() {
    static const Gammas G;
    return G;
}

// y[spin][col] += coef * sum_spin' M[spin][spin'] * x[spin'][col]
inline void spin_mul_acc(cd* y, const Mat4 M, const cd* x, cd coef) {
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c) {
            cd s = 0;
            for (int b = 0; b < 4; ++b) s += M[a][b] * x[b * 3 + c];
            y[a * 3 + c] += coef * s;
        }
}

// chi[spin][row] = sum_col U[row][col] psi[spin][col]   (dag = false)
// chi[spin][row] = sum_col conj(U[col][row]) psi[spin][col]   (dag = true)
inline void colour_mul(cd* chi, const cd* U, const cd* psi, bool dag) {
    for (int a = 0; a < 4; ++a)
        for (int r = 0; r < 3; ++r) {
            cd s = 0;
            for (int c = 0; c < 3; ++c) {
                cd u = dag ? std::conj(U[c * 3 + r]) : U[r * 3 + c];
                s += u * psi[a * 3 + c];
            }
            chi[a * 3 + r] = s;
        }
}

// One 5d site of D_dwf, each term added to acc[cls] where cls is its hop class:
//   0 = diagonal, fifth-dimension hops and 4d hops inside a block,
//   1+mu = forward mu hop whose source lies across the +mu face of the block,
//   5+mu = backward mu hop whose source lies across the -mu face.
// With block == nullptr every term goes to class 0.
void dwf_site(const Geom& g, const int bc[4], double M5, double mf, double mob_b, const int* block,
              const cd* U, const cd* in, long x4, int s, cd acc[9][12]) {
    const Gammas& G = gam();
    int x[4];
    g.coords(x4, x);
    const cd* psi = in + g.idx(x4, s, 0, 0);
    for (int c = 0; c < 12; ++c) acc[0][c] += (mob_b * (4.0 - M5) + 1.0) * psi[c];

    Mat4 one_m[4], one_p[4];
    for (int mu = 0; mu < 4; ++mu)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                cd d = (a == b) ? 1.0 : 0.0;
                one_m[mu][a][b] = d - G.g[mu][a][b];
                one_p[mu][a][b] = d + G.g[mu][a][b];
            }

    cd chi[12];
    for (int mu = 0; mu < 4; ++mu) {
        // forward hop: -b/2 (1 - g_mu) U_mu(x) psi(x + mu)
        int xp[4] = {x[0], x[1], x[2], x[3]};
        xp[mu] = (x[mu] + 1) % g.L[mu];
        double sgn_p = (x[mu] == g.L[mu] - 1) ? (double)bc[mu] : 1.0;
        int cls_p = (block && (x[mu] % block[mu] == block[mu] - 1)) ? 1 + mu : 0;
        colour_mul(chi, U + (x4 * 4 + mu) * 9, in + g.idx(g.site(xp), s, 0, 0), false);
        spin_mul_acc(acc[cls_p], one_m[mu], chi, cd(-0.5 * mob_b * sgn_p));

        // backward hop: -b/2 (1 + g_mu) U_mu(x - mu)^dag psi(x - mu)
        int xm[4] = {x[0], x[1], x[2], x[3]};
        xm[mu] = (x[mu] - 1 + g.L[mu]) % g.L[mu];
        double sgn_m = (x[mu] == 0) ? (double)bc[mu] : 1.0;
        int cls_m = (block && (x[mu] % block[mu] == 0)) ? 5 + mu : 0;
        long xm4 = g.site(xm);
        colour_mul(chi, U + (xm4 * 4 + mu) * 9, in + g.idx(xm4, s, 0, 0), true);
        spin_mul_acc(acc[cls_m], one_p[mu], chi, cd(-0.5 * mob_b * sgn_m));
    }

    // fifth dimension: -P- psi(x,s+1) - P+ psi(x,s-1), mass mf on the walls
    Mat4 Pm, Pp;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            cd d = (a == b) ? 1.0 : 0.0;
            Pm[a][b] = 0.5 * (d - G.g[4][a][b]);
            Pp[a][b] = 0.5 * (d + G.g[4][a][b]);
        }
    if (s + 1 < g.Ls)
        spin_mul_acc(acc[0], Pm, in + g.idx(x4, s + 1, 0, 0), cd(-1.0));
    else
        spin_mul_acc(acc[0], Pm, in + g.idx(x4, 0, 0, 0), cd(mf));
    if (s >= 1)
        spin_mul_acc(acc[0], Pp, in + g.idx(x4, s - 1, 0, 0), cd(-1.0));
    else
        spin_mul_acc(acc[0], Pp, in + g.idx(x4, g.Ls - 1, 0, 0), cd(mf));
}

// gamma5 times a 12-component spinor
inline void g5_mul(cd* y, const cd* x) {
    const Gammas& G = gam();
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 3; ++c) {
            cd s = 0;
            for (int b = 0; b < 4; ++b) s += G.g[4][a][b] * x[b * 3 + c];
            y[a * 3 + c] = s;
        }
}

struct CGeom {
    int C[4];  // coarse extents
    int B[4];  // block extents
    long Nc;
    CGeom(const Geom& g, const int* block) {
        for (int i = 0; i < 4; ++i) {
            B[i] = block[i];
            C[i] = g.L[i] / block[i];
        }
        Nc = (long)C[0] * C[1] * C[2] * C[3];
    }
    long csite(const int c[4]) const {
        return (((long)c[3] * C[2] + c[2]) * C[1] + c[1]) * C[0] + c[0];
    }
    void ccoords(long i, int c[4]) const {
        c[0] = (int)(i % C[0]); i /= C[0];
        c[1] = (int)(i % C[1]); i /= C[1];
        c[2] = (int)(i % C[2]); i /= C[2];
        c[3] = (int)i;
    }
    long block_of(const int x[4]) const {
        int c[4] = {x[0] / B[0], x[1] / B[1], x[2] / B[2], x[3] / B[3]};
        return csite(c);
    }
    // coarse neighbour a + d, d in D9 order, coarse-periodic
    long neighbour(long a, int d) const {
        if (d == 0) return a;
        int c[4];
        ccoords(a, c);
        int mu = (d - 1) % 4;
        int step = (d <= 4) ? 1 : -1;
        c[mu] = (c[mu] + step + C[mu]) % C[mu];
        return csite(c);
    }
    long bvol() const { return (long)B[0] * B[1] * B[2] * B[3]; }
    // the fine 4d sites of block a, in lexicographic order
    void block_sites(const Geom& g, long a, std::vector<long>& out) const {
        int c[4];
        ccoords(a, c);
        out.clear();
        for (int t = 0; t < B[3]; ++t)
            for (int z = 0; z < B[2]; ++z)
                for (int y = 0; y < B[1]; ++y)
                    for (int x = 0; x < B[0]; ++x) {
                        int xx[4] = {c[0] * B[0] + x, c[1] * B[1] + y, c[2] * B[2] + z, c[3] * B[3] + t};
                        out.push_back(g.site(xx));
                    }
    }
};

}  // namespace

extern "C" {

// gamma matrix mu (0..3 = x, y, z, t; 4 = gamma5), 4x4 row-major complex
void or_gamma(int mu, double* out) {
    const Gammas& G = gam();
    cd* o = reinterpret_cast<cd*>(out);
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) o[a * 4 + b] = G.g[mu][a][b];
}

// out = D_dwf in  (dims = Lx, Ly, Lz, Lt, Ls)
void or_apply_dw(const int* dims, const int* bc, double M5, double mf, double mob_b, const double* U_, const double* in_,
                 double* out_) {
    Geom g(dims);
    const cd* U = reinterpret_cast<const cd*>(U_);
    const cd* in = reinterpret_cast<const cd*>(in_);
    cd* out = reinterpret_cast<cd*>(out_);
#pragma omp parallel for schedule(static)
    for (long x4 = 0; x4 < g.V4; ++x4)
        for (int s = 0; s < g.Ls; ++s) {
            cd acc[9][12];
            for (int k = 0; k < 9; ++k)
                for (int c = 0; c < 12; ++c) acc[k][c] = 0;
            dwf_site(g, bc, M5, mf, mob_b, nullptr, U, in, x4, s, acc);
            for (int c = 0; c < 12; ++c) out[g.idx(x4, s, 0, 0) + c] = acc[0][c];
        }
}

// out = H in = gamma5 R5 D_dwf in
void or_apply_h(const int* dims, const int* bc, double M5, double mf, double mob_b, const double* U_, const double* in_,
                double* out_) {
    Geom g(dims);
    const cd* U = reinterpret_cast<const cd*>(U_);
    const cd* in = reinterpret_cast<const cd*>(in_);
    cd* out = reinterpret_cast<cd*>(out_);
#pragma omp parallel for schedule(static)
    for (long x4 = 0; x4 < g.V4; ++x4)
        for (int s = 0; s < g.Ls; ++s) {
            cd acc[9][12];
            for (int k = 0; k < 9; ++k)
                for (int c = 0; c < 12; ++c) acc[k][c] = 0;
            dwf_site(g, bc, M5, mf, mob_b, nullptr, U, in, x4, s, acc);
            g5_mul(out + g.idx(x4, g.Ls - 1 - s, 0, 0), acc[0]);
        }
}

// (H in) at nsel selected 5d output sites: sel[i] = site4 * Ls + s; out_sel[i][12].
// Used for spot checks on lattices too large to apply H to in full.
void or_apply_h_sites(const int* dims, const int* bc, double M5, double mf, double mob_b, const double* U_, const double* in_,
                      long nsel, const long* sel, double* out_) {
    Geom g(dims);
    const cd* U = reinterpret_cast<const cd*>(U_);
    const cd* in = reinterpret_cast<const cd*>(in_);
    cd* out = reinterpret_cast<cd*>(out_);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < nsel; ++i) {
        const long x4 = sel[i] / g.Ls;
        const int s_out = (int)(sel[i] % g.Ls);
        cd acc[9][12];
        for (int k = 0; k < 9; ++k)
            for (int c = 0; c < 12; ++c) acc[k][c] = 0;
        dwf_site(g, bc, M5, mf, mob_b, nullptr, U, in, x4, g.Ls - 1 - s_out, acc);
        g5_mul(out + i * 12, acc[0]);
    }
}

// out9[cls] = H^(cls) in: H split by hop class relative to blocks of extent `block`
// (nine full fields, D9 order). Summing the nine gives H in.
void or_apply_h_classes(const int* dims, const int* bc, double M5, double mf, double mob_b, const int* block,
                        const double* U_, const double* in_, double* out9_) {
    Geom g(dims);
    const cd* U = reinterpret_cast<const cd*>(U_);
    const cd* in = reinterpret_cast<const cd*>(in_);
    cd* out9 = reinterpret_cast<cd*>(out9_);
    const long n = g.fdof();
#pragma omp parallel for schedule(static)
    for (long x4 = 0; x4 < g.V4; ++x4)
        for (int s = 0; s < g.Ls; ++s) {
            cd acc[9][12];
            for (int k = 0; k < 9; ++k)
                for (int c = 0; c < 12; ++c) acc[k][c] = 0;
            dwf_site(g, bc, M5, mf, mob_b, block, U, in, x4, s, acc);
            for (int k = 0; k < 9; ++k) g5_mul(out9 + k * n + g.idx(x4, g.Ls - 1 - s, 0, 0), acc[k]);
        }
}

// Chirally split, block-orthonormal basis (Sec. 4).
//   vecs:  nvec fine fields (the subspace vectors phi_k)
//   basis: Nb = 2*nvec fine fields; basis field k holds, on every block b, the
//          block vector phi^b_k; k < nvec: Gamma5 = +1 half, k >= nvec: -1 half.
//   mode 0: Gamma5 = gamma5 R5 (the full 5d reflection);
//   mode 1: the 4d gamma5 on every slice (alternative reading, kept for comparison).
// Per block and chirality the vectors are orthonormalised in index order by
// modified Gram-Schmidt applied twice (the Q of the thin QR with a positive real
// R diagonal). Returns 0, or 4 if some vector is numerically dependent
// (remaining norm below 1e-12 of its chiral projection's norm).
int or_block_basis(const int* dims, const int* block, int nvec, int mode, const double* vecs_,
                   double* basis_) {
    Geom g(dims);
    CGeom cg(g, block);
    const cd* vecs = reinterpret_cast<const cd*>(vecs_);
    cd* basis = reinterpret_cast<cd*>(basis_);
    const long n = g.fdof();
    const long nb_dof = cg.bvol() * g.Ls * 12;
    int status = 0;
    for (long k = 0; k < 2L * nvec * n; ++k) basis[k] = 0;
#pragma omp parallel for schedule(dynamic)
    for (long a = 0; a < cg.Nc; ++a) {
        std::vector<long> sites;
        cg.block_sites(g, a, sites);
        std::vector<cd> q((size_t)nvec * nb_dof);
        std::vector<cd> w(nb_dof), tmp(12);
        for (int h = 0; h < 2; ++h) {
            const double hs = (h == 0) ? 1.0 : -1.0;
            for (int k = 0; k < nvec; ++k) {
                const cd* v = vecs + (long)k * n;
                // w = (v + h Gamma5 v)/2 restricted to block a
                long p = 0;
                for (long i = 0; i < (long)sites.size(); ++i)
                    for (int s = 0; s < g.Ls; ++s) {
                        int sr = (mode == 0) ? g.Ls - 1 - s : s;
                        g5_mul(tmp.data(), v + g.idx(sites[i], sr, 0, 0));
                        for (int c = 0; c < 12; ++c)
                            w[p++] = 0.5 * (v[g.idx(sites[i], s, 0, 0) + c] + hs * tmp[c]);
                    }
                double n0 = 0;
                for (long i = 0; i < nb_dof; ++i) n0 += std::norm(w[i]);
                n0 = std::sqrt(n0);
                for (int pass = 0; pass < 2; ++pass)
                    for (int j = 0; j < k; ++j) {
                        const cd* qj = q.data() + (long)j * nb_dof;
                        cd r = 0;
                        for (long i = 0; i < nb_dof; ++i) r += std::conj(qj[i]) * w[i];
                        for (long i = 0; i < nb_dof; ++i) w[i] -= r * qj[i];
                    }
                double nr = 0;
                for (long i = 0; i < nb_dof; ++i) nr += std::norm(w[i]);
                nr = std::sqrt(nr);
                if (!(nr > 1e-12 * n0)) {
#pragma omp critical
                    status = 4;
                    nr = 1.0;
                }
                cd* qk = q.data() + (long)k * nb_dof;
                for (long i = 0; i < nb_dof; ++i) qk[i] = w[i] / nr;
                // scatter into the basis field h*nvec + k
                cd* dst = basis + (long)(h * nvec + k) * n;
                p = 0;
                for (long i = 0; i < (long)sites.size(); ++i)
                    for (int s = 0; s < g.Ls; ++s)
                        for (int c = 0; c < 12; ++c) dst[g.idx(sites[i], s, 0, 0) + c] = qk[p++];
            }
        }
    }
    return status;
}

// v[a][k] = <phi^a_k, psi> = sum_{x in a, s} conj(basis_k(x,s)) . psi(x,s)   (restriction P^dag)
void or_restrict(const int* dims, const int* block, int nb, const double* basis_, const double* psi_,
                 double* v_) {
    Geom g(dims);
    CGeom cg(g, block);
    const cd* basis = reinterpret_cast<const cd*>(basis_);
    const cd* psi = reinterpret_cast<const cd*>(psi_);
    cd* v = reinterpret_cast<cd*>(v_);
    const long n = g.fdof();
#pragma omp parallel for schedule(static)
    for (long a = 0; a < cg.Nc; ++a) {
        std::vector<long> sites;
        cg.block_sites(g, a, sites);
        for (int k = 0; k < nb; ++k) {
            cd acc = 0;
            for (long x4 : sites)
                for (int s = 0; s < g.Ls; ++s)
                    for (int c = 0; c < 12; ++c) {
                        long i = g.idx(x4, s, 0, 0) + c;
                        acc += std::conj(basis[(long)k * n + i]) * psi[i];
                    }
            v[a * nb + k] = acc;
        }
    }
}

// psi(x,s) = sum_k phi^{b(x)}_k(x,s) v[b(x)][k]   (prolongation P)
void or_prolong(const int* dims, const int* block, int nb, const double* basis_, const double* v_,
                double* psi_) {
    Geom g(dims);
    CGeom cg(g, block);
    const cd* basis = reinterpret_cast<const cd*>(basis_);
    const cd* v = reinterpret_cast<const cd*>(v_);
    cd* psi = reinterpret_cast<cd*>(psi_);
    const long n = g.fdof();
#pragma omp parallel for schedule(static)
    for (long x4 = 0; x4 < g.V4; ++x4) {
        int x[4];
        g.coords(x4, x);
        long a = cg.block_of(x);
        for (int s = 0; s < g.Ls; ++s)
            for (int c = 0; c < 12; ++c) {
                long i = g.idx(x4, s, 0, 0) + c;
                cd acc = 0;
                for (int k = 0; k < nb; ++k) acc += basis[(long)k * n + i] * v[a * nb + k];
                psi[i] = acc;
            }
    }
}

// Columns kcols[0..ncols) of the little Dirac operator, by definition:
//   A[a][d][j][k] = <phi^a_j | H^(d) | phi^{a+d}_k>,
// where H^(d) collects the hops from block a+d into block a across the face d
// (d = 0: everything inside a). The basis field k carries phi^b_k on every block b,
// so applying the class-split H to it once gives, on block a, class d exactly
// H^(d) phi^{a+d}_k.  Output A_cols[c][a][d][j] (complex), c < ncols.
void or_coarse_columns(const int* dims, const int* bc, double M5, double mf, double mob_b, const int* block, int nb,
                       const double* U_, const double* basis_, int ncols, const int* kcols, double* out_) {
    Geom g(dims);
    CGeom cg(g, block);
    const cd* basis = reinterpret_cast<const cd*>(basis_);
    cd* out = reinterpret_cast<cd*>(out_);
    const long n = g.fdof();
    std::vector<cd> cls((size_t)9 * n);
    for (int c = 0; c < ncols; ++c) {
        int k = kcols[c];
        or_apply_h_classes(dims, bc, M5, mf, mob_b, block, U_, basis_ + 2L * k * n,
                           reinterpret_cast<double*>(cls.data()));
#pragma omp parallel for schedule(static)
        for (long a = 0; a < cg.Nc; ++a) {
            std::vector<long> sites;
            cg.block_sites(g, a, sites);
            for (int d = 0; d < 9; ++d)
                for (int j = 0; j < nb; ++j) {
                    cd acc = 0;
                    for (long x4 : sites)
                        for (int s = 0; s < g.Ls; ++s)
                            for (int cc = 0; cc < 12; ++cc) {
                                long i = g.idx(x4, s, 0, 0) + cc;
                                acc += std::conj(basis[(long)j * n + i]) * cls[(size_t)d * n + i];
                            }
                    out[(((long)c * cg.Nc + a) * 9 + d) * nb + j] = acc;
                }
        }
    }
}

// Full little Dirac operator A[a][d][j][k].
void or_coarse_build(const int* dims, const int* bc, double M5, double mf, double mob_b, const int* block, int nb,
                     const double* U_, const double* basis_, double* A_) {
    Geom g(dims);
    CGeom cg(g, block);
    cd* A = reinterpret_cast<cd*>(A_);
    std::vector<cd> col((size_t)cg.Nc * 9 * nb);
    for (int k = 0; k < nb; ++k) {
        or_coarse_columns(dims, bc, M5, mf, mob_b, block, nb, U_, basis_, 1, &k, reinterpret_cast<double*>(col.data()));
        for (long a = 0; a < cg.Nc; ++a)
            for (int d = 0; d < 9; ++d)
                for (int j = 0; j < nb; ++j)
                    A[((a * 9 + d) * nb + j) * nb + k] = col[(a * 9 + d) * nb + j];
    }
}

// out[r][a] = sum_d A[a][d] v[r][a+d]   (coarse-periodic; cdims = coarse extents x, y, z, t)
void or_coarse_apply(const int* cdims, int nb, int nrhs, const double* A_, const double* v_, double* out_) {
    int blk1[4] = {1, 1, 1, 1};
    int d5[5] = {cdims[0], cdims[1], cdims[2], cdims[3], 1};
    Geom g(d5);
    CGeom cg(g, blk1);
    const cd* A = reinterpret_cast<const cd*>(A_);
    const cd* v = reinterpret_cast<const cd*>(v_);
    cd* out = reinterpret_cast<cd*>(out_);
    for (int r = 0; r < nrhs; ++r) {
#pragma omp parallel for schedule(static)
        for (long a = 0; a < cg.Nc; ++a)
            for (int j = 0; j < nb; ++j) {
                cd acc = 0;
                for (int d = 0; d < 9; ++d) {
                    long b = cg.neighbour(a, d);
                    for (int k = 0; k < nb; ++k)
                        acc += A[((a * 9 + d) * nb + j) * nb + k] * v[((long)r * cg.Nc + b) * nb + k];
                }
                out[((long)r * cg.Nc + a) * nb + j] = acc;
            }
    }
}

}  // extern "C"
