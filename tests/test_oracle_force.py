"""Pins of the oracle's link gradient and su(3) force of L = Re <chi, H psi>
(the HMC fermion force that motivates the solver, Sec. 1 and Sec. 5).

* L is linear in (Re U, Im U) (every hop holds U or U^dag once), so the central
  difference of L in one real link coordinate has no truncation error: at
  eps = 1e-6 it differs from the exact derivative only by the rounding of the
  two losses, bounded here by 64 u S / eps with u = 2^-53 and S = sum |chi| |H psi|.
* The force T = P_TA(U W^dag) is checked against the group derivative
  dL/deps of U -> exp(eps X) U (X traceless anti-Hermitian): the central
  difference of a smooth function, truncation O(eps^2).
* Gauge covariance: T[U^V, V chi, V psi] = V T V^dag.
"""
import numpy as np
import pytest

import hdcr_inputs as hi
import oracle

U53 = 2.0 ** -53
EPS = 1e-6


def _setup(L, Ls, bc=(1, 1, 1, -1), mf=0.1, seed=1, b=1.0):
    p = oracle.Params(L, Ls, M5=1.8, mf=mf, bc=bc, b=b)
    U = hi.gauge_field(L, seed=seed)
    chi = hi.gaussian_fermion(L, Ls, seed=3)
    psi = hi.gaussian_fermion(L, Ls, seed=4)
    return p, U, chi, psi


def _fd_bound(U, chi, psi, p):
    S = float(np.sum(np.abs(chi) * np.abs(oracle.apply_h(U, psi, p))))
    return 64 * U53 * S / EPS


@pytest.mark.parametrize("L,Ls,bc,b", [((2, 2, 2, 4), 4, (1, 1, 1, -1), 1.0),   # extent 2: both hops of a link coincide
                                       ((3, 2, 2, 3), 3, (1, -1, 1, -1), 1.0),  # odd extents and Ls, antiperiodic in y
                                       ((2, 3, 1, 2), 2, (-1, 1, 1, -1), 1.0),  # extent 1: a site is its own neighbour
                                       ((2, 2, 3, 2), 3, (1, 1, 1, -1), 1.6)])  # Cayley scale b != 1 (Sec. 3)
def test_link_grad_matches_finite_differences(L, Ls, bc, b):
    p, U, chi, psi = _setup(L, Ls, bc, b=b)
    W = oracle.link_grad(U, chi, psi, p)
    bound = _fd_bound(U, chi, psi, p)
    rng = np.random.default_rng(7)
    idx = [tuple(int(rng.integers(0, n)) for n in U.shape) for _ in range(24)]
    # every direction at the last site (boundary-crossing links)
    idx += [(L[3] - 1, L[2] - 1, L[1] - 1, L[0] - 1, mu, 1, 2) for mu in range(4)]
    for ix in idx:
        E = np.zeros_like(U)
        E[ix] = 1.0
        dre = (oracle.loss(U + EPS * E, chi, psi, p) - oracle.loss(U - EPS * E, chi, psi, p)) / (2 * EPS)
        dim = (oracle.loss(U + 1j * EPS * E, chi, psi, p) - oracle.loss(U - 1j * EPS * E, chi, psi, p)) / (2 * EPS)
        assert abs(W[ix] - (dre + 1j * dim)) <= bound, (ix, W[ix], dre + 1j * dim, bound)


def _random_su3_algebra(rng):
    """X = i sum_a w_a lambda_a / 2: traceless anti-Hermitian."""
    h = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    h = 0.5 * (h + h.conj().T)
    h -= np.trace(h) / 3 * np.eye(3)
    return 1j * h


def _expm_ah(X, eps):
    """exp(eps X) for anti-Hermitian X (X = i H, H Hermitian)."""
    w, v = np.linalg.eigh(-1j * X)
    return (v * np.exp(1j * eps * w)) @ v.conj().T


def test_force_is_the_group_derivative():
    L, Ls = (2, 2, 2, 4), 4
    p, U, chi, psi = _setup(L, Ls)
    T = oracle.force(U, oracle.link_grad(U, chi, psi, p))
    rng = np.random.default_rng(3)
    bound = _fd_bound(U, chi, psi, p)
    for _ in range(12):
        site = tuple(int(rng.integers(0, n)) for n in U.shape[:4])
        mu = int(rng.integers(0, 4))
        X = _random_su3_algebra(rng)
        Up, Um = U.copy(), U.copy()
        Up[site + (mu,)] = _expm_ah(X, EPS) @ U[site + (mu,)]
        Um[site + (mu,)] = _expm_ah(X, -EPS) @ U[site + (mu,)]
        fd = (oracle.loss(Up, chi, psi, p) - oracle.loss(Um, chi, psi, p)) / (2 * EPS)
        exact = np.trace(X @ T[site + (mu,)]).real
        assert abs(fd - exact) <= bound + 1e-9 * abs(exact), (fd, exact)


def test_force_traceless_antihermitian():
    L, Ls = (3, 2, 2, 3), 3
    p, U, chi, psi = _setup(L, Ls, (1, -1, 1, -1))
    T = oracle.force(U, oracle.link_grad(U, chi, psi, p))
    np.testing.assert_allclose(T + np.conj(np.swapaxes(T, -1, -2)), 0, atol=1e-13)
    np.testing.assert_allclose(np.trace(T, axis1=-2, axis2=-1), 0, atol=1e-13)
    assert np.abs(T).max() > 0.1


def test_force_gauge_covariant():
    """T[U^V, V chi, V psi] = V T[U, chi, psi] V^dag (L is gauge invariant)."""
    L, Ls = (4, 2, 2, 4), 4
    p, U, chi, psi = _setup(L, Ls)
    V = hi.gauge_transform(L)
    axis = {0: 3, 1: 2, 2: 1, 3: 0}
    UV = np.empty_like(U)
    for mu in range(4):
        Vp = np.roll(V, -1, axis=axis[mu])
        UV[..., mu, :, :] = V @ U[..., mu, :, :] @ np.conj(np.swapaxes(Vp, -1, -2))
    rot = lambda f: np.einsum("tzyxab,tzyxsib->tzyxsia", V, f)
    T = oracle.force(U, oracle.link_grad(U, chi, psi, p))
    TV = oracle.force(UV, oracle.link_grad(UV, rot(chi), rot(psi), p))
    Vd = np.conj(np.swapaxes(V, -1, -2))
    np.testing.assert_allclose(TV, V[..., None, :, :] @ T @ Vd[..., None, :, :], atol=1e-12)
    assert abs(oracle.loss(UV, rot(chi), rot(psi), p) - oracle.loss(U, chi, psi, p)) <= 1e-10


def test_psi_gradient_is_h_chi():
    """dL/dRe psi + i dL/dIm psi = H chi (H Hermitian), by finite differences."""
    L, Ls = (2, 2, 2, 2), 4
    p, U, chi, psi = _setup(L, Ls)
    g = oracle.apply_h(U, chi, p)
    bound = _fd_bound(U, chi, psi, p)
    rng = np.random.default_rng(5)
    for _ in range(10):
        ix = tuple(int(rng.integers(0, n)) for n in psi.shape)
        E = np.zeros_like(psi)
        E[ix] = 1.0
        dre = (oracle.loss(U, chi, psi + EPS * E, p) - oracle.loss(U, chi, psi - EPS * E, p)) / (2 * EPS)
        dim = (oracle.loss(U, chi, psi + 1j * EPS * E, p) - oracle.loss(U, chi, psi - 1j * EPS * E, p)) / (2 * EPS)
        assert abs(g[ix] - (dre + 1j * dim)) <= bound


def test_link_grad_at_matches_whole_field():
    """The link-by-link form used for sampled checks on large lattices agrees with the whole-field form."""
    L, Ls = (3, 2, 2, 3), 3
    p, U, chi, psi = _setup(L, Ls, (1, -1, 1, -1))
    W = oracle.link_grad(U, chi, psi, p)
    links = [(t, z, y, x, mu) for t in range(3) for z in range(2) for y in range(2) for x in range(3)
             for mu in range(4)]
    got = oracle.link_grad_at(U, chi, psi, p, links)
    ref = np.stack([W[l] for l in links])
    np.testing.assert_allclose(got, ref, atol=1e-13)
