"""Pins of the oracle's fine operator H = Gamma5 D_dwf (Sec. 3) against facts fixed
outside the oracle: Clifford algebra, a dense shift-operator construction, the
free-field spectrum in closed form, gauge covariance, the Ls = 1 Wilson
reduction and Hermiticity."""
import numpy as np
import pytest

import hdcr_inputs as hi
import oracle
from tests import dense_ref


def test_gamma_matrices_chiral_basis():
    g, g5 = dense_ref.chiral_gammas()
    for mu in range(4):
        np.testing.assert_allclose(oracle.gamma(mu), g[mu], atol=0)
    np.testing.assert_allclose(oracle.gamma(4), np.diag([1, 1, -1, -1]), atol=1e-15)
    # Euclidean Clifford algebra, Hermitian gammas
    for mu in range(4):
        gm = oracle.gamma(mu)
        np.testing.assert_allclose(gm, gm.conj().T, atol=0)
        for nu in range(4):
            gn = oracle.gamma(nu)
            np.testing.assert_allclose(gm @ gn + gn @ gm, 2.0 * (mu == nu) * np.eye(4), atol=1e-15)
        np.testing.assert_allclose(gm @ oracle.gamma(4) + oracle.gamma(4) @ gm, 0, atol=1e-15)


@pytest.mark.parametrize("L,Ls", [((2, 2, 2, 2), 4), ((2, 2, 2, 4), 3), ((3, 2, 2, 2), 1)])
def test_dwf_matches_dense_shift_construction(L, Ls):
    p = oracle.Params(L, Ls, M5=1.8, mf=0.07)
    U = hi.gauge_field(L, seed=11)
    D = dense_ref.dense_dwf(U, L, Ls, p.M5, p.mf, p.bc)
    psi = hi.gaussian_fermion(L, Ls, seed=3)
    np.testing.assert_allclose(oracle.apply_dw(U, psi, p).ravel(), D @ psi.ravel(), rtol=0, atol=1e-12)
    H = dense_ref.dense_gamma5R5(L, Ls) @ D
    np.testing.assert_allclose(oracle.apply_h(U, psi, p).ravel(), H @ psi.ravel(), rtol=0, atol=1e-12)
    # the full dense matrix from the oracle equals the shift construction
    if L == (2, 2, 2, 2):
        Ho = dense_ref.dense_from_apply(lambda v: oracle.apply_h(U, v, p), p.fshape)
        np.testing.assert_allclose(Ho, H, atol=1e-13)
        np.testing.assert_allclose(Ho, Ho.conj().T, atol=1e-13)


@pytest.mark.parametrize("b", [1.0, 1.7])   # b != 1: the Cayley form with c = 0 (Sec. 3)
def test_free_field_spectrum_closed_form(b):
    L, Ls = (2, 2, 2, 4), 4
    p = oracle.Params(L, Ls, M5=1.8, mf=0.05, b=b)
    U = hi.gauge_field(L, eps=0.0)
    Ho = dense_ref.dense_from_apply(lambda v: oracle.apply_h(U, v, p), p.fshape)
    ev = np.linalg.eigvalsh(Ho)
    ref = dense_ref.free_spectrum(L, Ls, p.M5, p.mf, p.bc, b)
    np.testing.assert_allclose(ev, ref, atol=1e-12)


@pytest.mark.parametrize("b", [1.0, 1.7])
def test_free_field_ls1_wilson_closed_form(b):
    """Ls = 1: H = gamma5 (b D_W(-M5) + 1 + mf); eigenvalues +-sqrt(a^2 + b^2 sum sin^2 p),
    a = b (sum (1 - cos p) - M5) + 1 + mf, each sign twice (spin) times three colours."""
    L, Ls = (2, 2, 2, 4), 1
    p = oracle.Params(L, Ls, M5=1.8, mf=0.05, b=b)
    U = hi.gauge_field(L, eps=0.0)
    Ho = dense_ref.dense_from_apply(lambda v: oracle.apply_h(U, v, p), p.fshape)
    ev = np.linalg.eigvalsh(Ho)
    ref = []
    for mom in dense_ref.momenta(L, p.bc):
        a = b * (np.sum(1 - np.cos(mom)) - p.M5) + 1.0 + p.mf
        w = np.sqrt(a * a + b * b * np.sum(np.sin(mom) ** 2))
        ref += [w] * 6 + [-w] * 6
    np.testing.assert_allclose(ev, np.sort(ref), atol=1e-12)


@pytest.mark.parametrize("b", [1.0, 1.5])
def test_free_field_plane_wave_action(b):
    """On a plane wave e^{ipx} chi, H acts as the 4Ls x 4Ls matrix H(p) (momentum space)."""
    L, Ls = (4, 4, 4, 6), 6
    p = oracle.Params(L, Ls, M5=1.8, mf=0.01, b=b)
    U = hi.gauge_field(L, eps=0.0)
    rng = np.random.default_rng(7)
    for mom in [np.array([0.0, 0.0, 0.0, np.pi / 6]),
                np.array([np.pi / 2, np.pi, 3 * np.pi / 2, 5 * np.pi / 6]),
                np.array([np.pi / 2, 0.0, np.pi, 2 * np.pi * 4.5 / 6])]:
        chi = rng.standard_normal(4 * Ls) + 1j * rng.standard_normal(4 * Ls)
        f = dense_ref.plane_wave(L, Ls, mom, chi, colour=1)
        hp = dense_ref.free_h_momentum(mom, Ls, p.M5, p.mf, b)
        ref = dense_ref.plane_wave(L, Ls, mom, hp @ chi, colour=1)
        np.testing.assert_allclose(oracle.apply_h(U, f, p), ref, atol=1e-12)


@pytest.mark.parametrize("b", [1.0, 1.5])
def test_hermiticity_and_gamma5(b):
    L, Ls = (4, 4, 4, 4), 8
    p = oracle.Params(L, Ls, b=b)
    U = hi.gauge_field(L)
    x = hi.gaussian_fermion(L, Ls, seed=21)
    y = hi.gaussian_fermion(L, Ls, seed=22)
    Hy = oracle.apply_h(U, y, p)
    Hx = oracle.apply_h(U, x, p)
    assert abs(oracle.vdot(x, Hy) - oracle.vdot(Hx, y)) <= 1e-14 * oracle.norm(x) * oracle.norm(Hy)
    # Gamma5^2 = 1 and D = Gamma5 H
    g5x = oracle.apply_gamma5_field(x)
    np.testing.assert_allclose(oracle.apply_gamma5_field(g5x), x, atol=0)
    np.testing.assert_allclose(oracle.apply_gamma5_field(Hx), oracle.apply_dw(U, x, p), atol=1e-13)


def test_gauge_covariance():
    """H[U^V](V psi) = V H[U] psi with U^V_mu(x) = V(x) U_mu(x) V(x+mu)^dag."""
    L, Ls = (4, 4, 4, 4), 4
    p = oracle.Params(L, Ls)
    U = hi.gauge_field(L)
    V = hi.gauge_transform(L)
    psi = hi.gaussian_fermion(L, Ls, seed=4)
    axis = {0: 3, 1: 2, 2: 1, 3: 0}
    UV = np.empty_like(U)
    for mu in range(4):
        Vp = np.roll(V, -1, axis=axis[mu])
        UV[..., mu, :, :] = V @ U[..., mu, :, :] @ np.conj(np.swapaxes(Vp, -1, -2))
    Vpsi = np.einsum("tzyxab,tzyxsib->tzyxsia", V, psi)
    lhs = oracle.apply_h(UV, Vpsi, p)
    rhs = np.einsum("tzyxab,tzyxsib->tzyxsia", V, oracle.apply_h(U, psi, p))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_hop_classes_sum_to_h():
    L, Ls = (4, 4, 2, 4), 4
    p = oracle.Params(L, Ls)
    U = hi.gauge_field(L)
    psi = hi.gaussian_fermion(L, Ls, seed=9)
    cls = oracle.apply_h_classes(U, psi, p, block=(2, 2, 1, 4))
    np.testing.assert_allclose(cls.sum(axis=0), oracle.apply_h(U, psi, p), atol=1e-13)
    # extent-1 blocks in z: every z hop crosses a face; extent = L in t: the t hops that
    # wrap the lattice cross the (only) block's face
    assert np.abs(cls[3]).max() > 0 and np.abs(cls[7]).max() > 0


def test_apply_h_sites_matches_full_apply():
    L, Ls = (4, 2, 6, 4), 6
    p = oracle.Params(L, Ls)
    U = hi.gauge_field(L)
    psi = hi.gaussian_fermion(L, Ls, seed=2)
    full = oracle.apply_h(U, psi, p).reshape(-1, Ls, 4, 3)
    sel = np.array([0, 5, 17, 191, 4 * 2 * 6 * 4 * 6 - 1])
    got = oracle.apply_h_sites(U, psi, p, sel)
    np.testing.assert_array_equal(got, full.reshape(-1, 4, 3)[sel])
