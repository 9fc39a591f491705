// Driver of the C++ oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
// (test infrastructure): calls every exported routine on small lattices, among them odd
// extents, extent 1 and one-site blocks, and checks that every output is finite.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
void or_gamma(int mu, double* out);
void or_apply_dw(const int* dims, const int* bc, double M5, double mf, double mob_b, const double* U, const double* in,
                 double* out);
void or_apply_h(const int* dims, const int* bc, double M5, double mf, double mob_b, const double* U, const double* in,
                double* out);
void or_apply_h_sites(const int* dims, const int* bc, double M5, double mf, double mob_b, const double* U,
                      const double* in, long nsel, const long* sel, double* out);
void or_apply_h_classes(const int* dims, const int* bc, double M5, double mf, double mob_b, const int* block,
                        const double* U, const double* in, double* out9);
int or_block_basis(const int* dims, const int* block, int nvec, int mode, const double* vecs, double* basis);
void or_restrict(const int* dims, const int* block, int nb, const double* basis, const double* psi, double* v);
void or_prolong(const int* dims, const int* block, int nb, const double* basis, const double* v, double* psi);
void or_coarse_columns(const int* dims, const int* bc, double M5, double mf, double mob_b, const int* block, int nb,
                       const double* U, const double* basis, int ncols, const int* kcols, double* out);
void or_coarse_build(const int* dims, const int* bc, double M5, double mf, double mob_b, const int* block, int nb,
                     const double* U, const double* basis, double* A);
void or_coarse_apply(const int* cdims, int nb, int nrhs, const double* A, const double* v, double* out);
}

static unsigned long long state = 12345;
static double rnd() {
    state = state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(state >> 11) / 9007199254740992.0 - 0.5;
}
static std::vector<double> random_doubles(size_t n) {
    std::vector<double> v(n);
    for (auto& x : v) x = rnd();
    return v;
}
static bool finite(const std::vector<double>& v) {
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

static int run_case(const int L[4], int Ls, const int block[4], int nvec) {
    const int dims[5] = {L[0], L[1], L[2], L[3], Ls};
    const int bc[4] = {1, -1, 1, -1};
    const long V4 = (long)L[0] * L[1] * L[2] * L[3];
    const long nf = V4 * Ls * 12 * 2;  // doubles in a fine field
    const int nb = 2 * nvec;
    int cd[4];
    long nc = 1;
    for (int i = 0; i < 4; ++i) {
        cd[i] = L[i] / block[i];
        nc *= cd[i];
    }
    std::vector<double> U = random_doubles(V4 * 36 * 2), in = random_doubles(nf), out(nf), out9(9 * nf);
    or_apply_dw(dims, bc, 1.8, 0.05, 1.3, U.data(), in.data(), out.data());
    if (!finite(out)) return 1;
    or_apply_h(dims, bc, 1.8, 0.05, 1.0, U.data(), in.data(), out.data());
    if (!finite(out)) return 2;
    std::vector<long> sel = {0, V4 * Ls - 1, (V4 * Ls) / 2};
    std::vector<double> hs(sel.size() * 24);
    or_apply_h_sites(dims, bc, 1.8, 0.05, 1.0, U.data(), in.data(), (long)sel.size(), sel.data(), hs.data());
    if (!finite(hs)) return 3;
    or_apply_h_classes(dims, bc, 1.8, 0.05, 1.0, block, U.data(), in.data(), out9.data());
    if (!finite(out9)) return 4;
    std::vector<double> vecs = random_doubles(nvec * nf), basis(nb * nf);
    if (or_block_basis(dims, block, nvec, 0, vecs.data(), basis.data()) != 0) return 5;
    if (!finite(basis)) return 6;
    std::vector<double> v(nc * nb * 2), psi(nf);
    or_restrict(dims, block, nb, basis.data(), in.data(), v.data());
    or_prolong(dims, block, nb, basis.data(), v.data(), psi.data());
    if (!finite(v) || !finite(psi)) return 7;
    std::vector<double> A(nc * 9 * nb * nb * 2);
    or_coarse_build(dims, bc, 1.8, 0.05, 1.0, block, nb, U.data(), basis.data(), A.data());
    const int kcols[2] = {0, nb - 1};
    std::vector<double> cols(2 * nc * 9 * nb * 2);
    or_coarse_columns(dims, bc, 1.8, 0.05, 1.0, block, nb, U.data(), basis.data(), 2, kcols, cols.data());
    if (!finite(A) || !finite(cols)) return 8;
    std::vector<double> vv = random_doubles(3 * nc * nb * 2), vo(3 * nc * nb * 2);
    or_coarse_apply(cd, nb, 3, A.data(), vv.data(), vo.data());
    if (!finite(vo)) return 9;
    return 0;
}

int main() {
    std::vector<double> g(32);
    for (int mu = 0; mu < 5; ++mu) or_gamma(mu, g.data());
    const int L1[4] = {2, 2, 2, 4}, B1[4] = {2, 2, 2, 2};
    const int L2[4] = {3, 1, 2, 2}, B2[4] = {3, 1, 1, 2};
    const int L3[4] = {2, 2, 2, 2}, B3[4] = {1, 1, 1, 1};
    int rc;
    if ((rc = run_case(L1, 4, B1, 2))) return 10 + rc;
    if ((rc = run_case(L2, 3, B2, 3))) return 20 + rc;
    if ((rc = run_case(L3, 2, B3, 12))) return 30 + rc;   // one-site blocks at full rank (24 dof / 2)
    std::printf("oracle sanitizer run ok\n");
    return 0;
}
