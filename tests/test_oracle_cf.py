"""Pins of the oracle's continued-fraction overlap operator (Sec. 3, the continued-fraction
matrix): the Wilson kernel H_W against the domain wall oracle at Ls = 1, the 5d matrix against
an independent dense construction on 2^4 and against its free-field momentum form, Hermiticity
(real spectrum of both signs) and gauge covariance; the per-site form against the whole-field
form."""
import numpy as np
import pytest

import hdcr_inputs as hi
import oracle
from tests import dense_ref

BETA3 = [0.8, 1.7, 0.45]   # three pole slices (Ls = 4); any positive values define a valid matrix
R = 0.37


def test_wilson_kernel_matches_dwf_oracle_at_ls1():
    """At Ls = 1 both fifth-dimension hops of D_dwf land on the slice itself with the wall factor mf,
    so D_dwf = D_W(-M5) + (1 + mf) and H = gamma5 D_dwf: H_W = H - (1 + mf) gamma5."""
    L = (4, 2, 2, 4)
    for mf, bc in ((0.3, (1, 1, 1, -1)), (-0.2, (-1, 1, -1, 1))):
        p = oracle.Params(L, 1, M5=1.6, mf=mf, bc=bc)
        U = hi.gauge_field(L, seed=2)
        x = hi.gaussian_fermion(L, 1, seed=3)
        ref = oracle.apply_h(U, x, p) - (1 + mf) * np.einsum("ij,...jc->...ic", oracle.gamma(4), x)
        np.testing.assert_allclose(oracle.apply_hw(U, x, 1.6, bc), ref, atol=1e-13)


def test_cf_matches_dense_construction():
    L, bc, M5 = (2, 2, 2, 2), (1, -1, 1, -1), 1.4
    U = hi.gauge_field(L, seed=4)
    A = dense_ref.dense_cf(U, L, M5, bc, BETA3, R)
    Ls = len(BETA3) + 1
    rng = np.random.default_rng(5)
    for _ in range(3):
        x = rng.standard_normal((2, 2, 2, 2, Ls, 4, 3)) + 1j * rng.standard_normal((2, 2, 2, 2, Ls, 4, 3))
        np.testing.assert_allclose(oracle.apply_cf(U, x, M5, BETA3, R, bc).ravel(), A @ x.ravel(), atol=1e-12)
    # the dense matrix is Hermitian and indefinite (Sec. 3)
    assert np.abs(A - A.conj().T).max() < 1e-13
    ev = np.linalg.eigvalsh(A)
    assert ev[0] < 0 < ev[-1]


@pytest.mark.parametrize("beta", [[1.0], [0.6, 1.9], BETA3])
def test_cf_free_field_momentum_form(beta):
    """Unit links: a plane wave e^{ipx} chi(s, spin) delta(colour) maps to e^{ipx} (A(p) chi)."""
    L, bc, M5 = (4, 2, 2, 4), (1, 1, 1, -1), 1.8
    U = hi.gauge_field(L, eps=0.0)
    Ls = len(beta) + 1
    rng = np.random.default_rng(6)
    for p in dense_ref.momenta(L, bc)[::5]:
        chi = rng.standard_normal(4 * Ls) + 1j * rng.standard_normal(4 * Ls)
        f = dense_ref.plane_wave(L, Ls, p, chi, colour=1)
        got = oracle.apply_cf(U, f, M5, beta, R, bc)
        want = dense_ref.plane_wave(L, Ls, p, dense_ref.free_cf_momentum(p, M5, beta, R) @ chi, colour=1)
        np.testing.assert_allclose(got, want, atol=1e-12)


def test_cf_hermitian_and_gauge_covariant():
    L, bc, M5 = (4, 4, 2, 4), (1, 1, 1, -1), 1.8
    U = hi.gauge_field(L, seed=7)
    Ls = len(BETA3) + 1
    x, y = hi.gaussian_fermion(L, Ls, seed=8), hi.gaussian_fermion(L, Ls, seed=9)
    a = np.vdot(x, oracle.apply_cf(U, y, M5, BETA3, R, bc))
    b = np.vdot(oracle.apply_cf(U, x, M5, BETA3, R, bc), y)
    assert abs(a - b) <= 1e-12 * abs(a)
    # U_mu(x) -> G(x) U_mu(x) G(x + mu)^dag, psi(x, s) -> G(x) psi(x, s)
    G = hi.gauge_transform(L, seed=10)
    axis = {0: 3, 1: 2, 2: 1, 3: 0}
    Ug = np.empty_like(U)
    for mu in range(4):
        Gp = np.roll(G, -1, axis=axis[mu])
        Ug[..., mu, :, :] = G @ U[..., mu, :, :] @ np.conj(np.swapaxes(Gp, -1, -2))
    xg = np.einsum("tzyxab,tzyxsjb->tzyxsja", G, x)
    lhs = oracle.apply_cf(Ug, xg, M5, BETA3, R, bc)
    rhs = np.einsum("tzyxab,tzyxsjb->tzyxsja", G, oracle.apply_cf(U, x, M5, BETA3, R, bc))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_cf_sites_matches_full_apply():
    """The per-site form equals the whole-field form on every site of a small lattice with
    odd extents and both boundary-condition patterns (Ls = 6), and on a sample of a larger one."""
    for L, bc, m in (((3, 2, 5, 3), (-1, 1, -1, 1), 5), ((4, 4, 4, 6), (1, 1, 1, -1), 8)):
        beta = list(0.3 + np.arange(m) * 0.17)
        U = hi.gauge_field(L, seed=7)
        x = hi.gaussian_fermion(L, m + 1, seed=8)
        full = oracle.apply_cf(U, x, 1.7, beta, 0.45, bc)
        n5 = int(np.prod(L)) * (m + 1)
        sel = np.arange(n5) if n5 < 2000 else np.random.default_rng(3).choice(n5, 700, replace=False)
        got = oracle.apply_cf_sites(U, x, 1.7, beta, 0.45, sel, bc)
        ref = full.reshape(-1, 4, 3)[sel]
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
