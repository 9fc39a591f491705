"""Pins of the oracle's Krylov solvers, Chebyshev polynomials and two-level cycle
(Secs. 3-4) against library routines, closed forms and exact dense identities."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
from numpy.polynomial import chebyshev as npcheb

import hdcr_inputs as hi
import oracle
from tests import dense_ref
from tests.test_oracle_coarse import _dense_P


def test_cheby_coeffs_match_numpy_interpolation():
    lo, hi_ = 1.0, 64.0
    for n in (2, 5, 10, 13):
        c = oracle.cheby_coeffs(n, lo, hi_)
        ref = npcheb.chebinterpolate(lambda t: 1.0 / (0.5 * (hi_ + lo) + 0.5 * (hi_ - lo) * t), n - 1)
        mine = c.copy()
        mine[0] *= 0.5
        np.testing.assert_allclose(mine, ref, rtol=1e-12, atol=1e-15)
        y = np.linspace(lo, hi_, 7)
        np.testing.assert_allclose(oracle.cheby_eval(c, lo, hi_, y),
                                   npcheb.chebval((2 * y - hi_ - lo) / (hi_ - lo), ref), rtol=1e-12)


def test_cheby_golden_order10():
    """Stored coefficients of the paper's smoother polynomial (order 10, [1, 64], Sec. 4)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "cheby_order10_1_64.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    ref = np.array([float(r[1]) for r in rows])
    np.testing.assert_allclose(oracle.cheby_coeffs(10, 1.0, 64.0), ref, rtol=1e-14)


def _free_dense(L, Ls, mf=0.05):
    p = oracle.Params(L, Ls, M5=1.8, mf=mf)
    U = hi.gauge_field(L, eps=0.0)
    H = dense_ref.dense_gamma5R5(L, Ls) @ dense_ref.dense_dwf(U, L, Ls, p.M5, p.mf, p.bc)
    return p, U, H


def test_smoother_scalar_action_on_eigenvectors():
    L, Ls = (2, 2, 2, 4), 4
    p, U, H = _free_dense(L, Ls)
    lam, vec = np.linalg.eigh(H)
    coef = npcheb.chebinterpolate(lambda t: 1.0 / (32.5 + 31.5 * t), 9)
    for i in [0, 100, 700, len(lam) - 1]:
        v = vec[:, i].reshape(p.fshape)
        s = oracle.smoother(lambda f: oracle.apply_h(U, f, p), v, order=10, lo=1.0, hi=64.0)
        pl = npcheb.chebval((2 * lam[i] ** 2 - 65.0) / 63.0, coef)
        np.testing.assert_allclose(s, lam[i] * pl * v, atol=1e-12)


def test_filter_gain_closed_form():
    """T_d(yhat) acts on an eigenvector of H^2 as the scalar T_d((2 lam^2 - hi - lo)/(hi - lo))."""
    L, Ls = (2, 2, 2, 4), 4
    p, U, H = _free_dense(L, Ls)
    lam, vec = np.linalg.eigh(H)
    lo, hi_ = 2.0, 70.0
    for d in (1, 2, 7, 20):
        for i in [np.argmin(np.abs(lam)), 400]:
            v = vec[:, i].reshape(p.fshape)
            f = oracle.cheby_filter(lambda g: oracle.apply_h(U, g, p), v, d, lo, hi_, normalise=False)
            c = np.zeros(d + 1)
            c[d] = 1.0
            gain = npcheb.chebval((2 * lam[i] ** 2 - hi_ - lo) / (hi_ - lo), c)
            np.testing.assert_allclose(f, gain * v, atol=1e-11 * max(1.0, abs(gain)))
    # below lambda_cut the gain is cosh(d acosh|yhat|) > 1
    i = np.argmin(np.abs(lam))
    yh = (2 * lam[i] ** 2 - hi_ - lo) / (hi_ - lo)
    assert yh < -1


def test_power_max():
    L, Ls = (2, 2, 2, 4), 4
    p, U, H = _free_dense(L, Ls)
    lam = np.linalg.eigvalsh(H)
    est = oracle.power_max(lambda f: oracle.apply_h(U, f, p), hi.gaussian_fermion(L, Ls, seed=3), iters=200)
    assert abs(est - np.max(lam ** 2)) < 1e-3 * np.max(lam ** 2)


def test_cr_matches_dense_solve():
    L, Ls = (2, 2, 2, 2), 4
    p = oracle.Params(L, Ls, M5=1.8, mf=0.05)
    U = hi.gauge_field(L)
    H = dense_ref.dense_gamma5R5(L, Ls) @ dense_ref.dense_dwf(U, L, Ls, p.M5, p.mf, p.bc)
    b = hi.gaussian_fermion(L, Ls, seed=0)
    res = oracle.cr(lambda f: oracle.apply_h(U, f, p), b, tol=1e-10, maxiter=5000)
    assert res.status == 0 and res.true_rel <= 1e-10
    xs = np.linalg.solve(H, b.ravel())
    kappa = np.linalg.cond(H)
    assert np.linalg.norm(res.x.ravel() - xs) <= kappa * 1e-10 * np.linalg.norm(xs)
    h = np.array(res.history)
    assert np.all(np.diff(h) <= 1e-12 * h[:-1])   # minimal residual: non-increasing


def test_cr_residuals_match_scipy_gmres():
    """CR and unrestarted GMRES both minimise |b - H x| over the same Krylov space, so on a
    Hermitian operator their residual norms agree iteration by iteration (scipy's MINRES
    would be the textbook twin but takes real symmetric operators only)."""
    L, Ls = (4, 4, 4, 4), 8
    p = oracle.Params(L, Ls)
    U = hi.gauge_field(L)
    b = hi.gaussian_fermion(L, Ls, seed=0)
    ap = lambda f: oracle.apply_h(U, f, p)
    res = oracle.cr(ap, b, tol=1e-12, maxiter=30, check_true=False)
    n = b.size
    op = spla.LinearOperator((n, n), matvec=lambda v: ap(v.reshape(b.shape)).ravel(), dtype=complex)
    hist = []
    spla.gmres(op, b.ravel(), rtol=1e-30, atol=0.0, restart=30, maxiter=1,
               callback=lambda rk: hist.append(rk), callback_type="pr_norm")
    bn = oracle.norm(b)
    k = min(len(hist), len(res.history), 30)
    assert k >= 25
    np.testing.assert_allclose(np.array(res.history[:k]) / bn, np.array(hist[:k]), rtol=1e-6)


def test_cr_solution_true_residual_cfg_small():
    """4^4 x 8, M5 = 1.8, mf = 0.01, antiperiodic t, source seed 0: solve to 1e-8."""
    L, Ls = (4, 4, 4, 4), 8
    p = oracle.Params(L, Ls, M5=1.8, mf=0.01)
    U = hi.gauge_field(L)
    b = hi.gaussian_fermion(L, Ls, seed=0)
    ap = lambda f: oracle.apply_h(U, f, p)
    res = oracle.cr(ap, b, tol=1e-8, maxiter=10000)
    assert res.status == 0
    assert oracle.norm(b - ap(res.x)) <= 1e-8 * oracle.norm(b)


def test_fgcr_identity_preconditioner_equals_cr():
    L, Ls = (4, 4, 4, 4), 4
    p = oracle.Params(L, Ls)
    U = hi.gauge_field(L)
    b = hi.gaussian_fermion(L, Ls, seed=0)
    ap = lambda f: oracle.apply_h(U, f, p)
    r1 = oracle.cr(ap, b, tol=1e-14, maxiter=20, check_true=False)
    r2 = oracle.fgcr(ap, lambda r: r, b, tol=1e-14, maxiter=20, restart=20)
    np.testing.assert_allclose(np.array(r2.history[:20]), np.array(r1.history[:20]), rtol=1e-10)
    np.testing.assert_allclose(r2.x, r1.x, atol=1e-10 * oracle.norm(r1.x))


def test_cr_breakdown_source():
    """b = sqrt|l-| u+ + sqrt(l+) u- has <b, H b> = 0: CR must report breakdown."""
    L, Ls = (2, 2, 2, 4), 4
    p, U, H = _free_dense(L, Ls)
    lam, vec = np.linalg.eigh(H)
    ip = np.argmax(lam)
    im = np.argmin(lam)
    b = (np.sqrt(-lam[im]) * vec[:, ip] + np.sqrt(lam[ip]) * vec[:, im]).reshape(p.fshape)
    res = oracle.cr(lambda f: oracle.apply_h(U, f, p), b, tol=1e-8, maxiter=100)
    assert res.status == 2


def test_two_level_cycle_identities():
    """With an exact coarse inverse Q = P A^-1 P^dag (Sec. 4):
    QHQ = Q, QHP = P, P_L^2 = P_L, P_L^dag = P_R, P_L H = H P_R, P_L H P = 0, and the
    symmetric cycle equals S P_L + P_R S + Q - S P_L H S and satisfies
    1 - B H = (1 - S H)(1 - Q H)(1 - S H)."""
    L, Ls, block, nvec = (2, 2, 2, 2), 4, (1, 1, 1, 1), 6
    p = oracle.Params(L, Ls, M5=1.8, mf=0.05)
    cs = oracle.Coarse(p, block, nvec)
    U = hi.gauge_field(L)
    vecs = [hi.gaussian_fermion(L, Ls, seed=100 + k) for k in range(nvec)]
    basis, st = oracle.block_basis(vecs, cs)
    A = oracle.coarse_build(U, basis, cs)
    H = dense_ref.dense_gamma5R5(L, Ls) @ dense_ref.dense_dwf(U, L, Ls, p.M5, p.mf, p.bc)
    P = _dense_P(basis, cs)
    Ad = oracle.coarse_dense(A, cs.cdims)
    Q = P @ np.linalg.solve(Ad, P.conj().T)
    n = H.shape[0]
    I = np.eye(n)
    PL = I - H @ Q
    PR = I - Q @ H
    np.testing.assert_allclose(Q @ H @ Q, Q, atol=1e-10)
    np.testing.assert_allclose(Q @ H @ P, P, atol=1e-10)
    np.testing.assert_allclose(PL @ PL, PL, atol=1e-10)
    np.testing.assert_allclose(PL.conj().T, PR, atol=1e-10)
    np.testing.assert_allclose(PL @ H, H @ PR, atol=1e-10)
    np.testing.assert_allclose(PL @ H @ P, 0, atol=1e-10)

    ap = lambda f: oracle.apply_h(U, f, p)
    S = dense_ref.dense_from_apply(lambda f: oracle.smoother(ap, f, 10, 1.0, 64.0), p.fshape)
    exact = lambda v, cdims: np.linalg.solve(Ad, v.ravel()).reshape(v.shape)
    B = dense_ref.dense_from_apply(
        lambda f: oracle.vcycle(ap, A, basis, cs, f, coarse_solve=exact), p.fshape)
    Mouter = S @ PL + PR @ S + Q - S @ PL @ H @ S
    np.testing.assert_allclose(B, Mouter, atol=1e-9)
    np.testing.assert_allclose(I - B @ H, (I - S @ H) @ (I - Q @ H) @ (I - S @ H), atol=1e-9)
    np.testing.assert_allclose(B, B.conj().T, atol=1e-9)


def test_hdcr_oracle_converges():
    L, Ls, block, nvec = (4, 4, 4, 4), 8, (2, 2, 2, 2), 4
    p = oracle.Params(L, Ls)
    cs = oracle.Coarse(p, block, nvec)
    U = hi.gauge_field(L)
    ap = lambda f: oracle.apply_h(U, f, p)
    lmax = oracle.power_max(ap, hi.gaussian_fermion(L, Ls, seed=99), iters=30) * 1.1
    vecs = [oracle.cheby_filter(ap, e, 12, 0.05 * lmax, lmax) for e in hi.subspace_noise(L, Ls, nvec)]
    basis, st = oracle.block_basis(vecs, cs)
    A = oracle.coarse_build(U, basis, cs)
    b = hi.gaussian_fermion(L, Ls, seed=0)
    res = oracle.fgcr(ap, lambda r: oracle.vcycle(ap, A, basis, cs, r), b, tol=1e-8, maxiter=100)
    assert res.status == 0 and res.true_rel <= 1e-8
    ref = oracle.cr(ap, b, tol=1e-10, maxiter=10000)
    np.testing.assert_allclose(res.x, ref.x, atol=1e-6 * oracle.norm(ref.x))
    assert res.iters < ref.iters


# ---------------------------------------------------------------------------
# coarse-space eigenvector deflation (Sec. 5 names it for the coarse cost)
# ---------------------------------------------------------------------------

def _small_coarse(nvec=4):
    L, Ls, block = (4, 4, 4, 4), 4, (2, 2, 2, 2)
    p = oracle.Params(L, Ls, M5=1.8, mf=0.01)
    cs = oracle.Coarse(p, block, nvec)
    U = hi.gauge_field(L, seed=1)
    vecs = hi.subspace_noise(L, Ls, nvec)
    basis, st = oracle.block_basis(vecs, cs)
    assert st == 0
    return cs, oracle.coarse_build(U, basis, cs)


def test_coarse_deflation_matches_dense_eigenpairs():
    """The Ritz pairs of the filtered subspace iteration are the k eigenpairs of smallest
    |lambda| of the dense coarse matrix (numpy eigh of the matrix assembled column by column)."""
    cs, A = _small_coarse()
    k, m = 6, 12
    V0 = [hi.gaussian_coarse(cs.nc, cs.nb, seed=40 + i) for i in range(m)]
    theta, V, W = oracle.coarse_deflation(A, cs.cdims, V0, k, degree=40, iters=4, cut=0.05)
    D = oracle.coarse_dense(A, cs.cdims)
    ev, evec = np.linalg.eigh(D)
    ref = ev[np.argsort(np.abs(ev))[:k]]
    anorm = np.abs(ev).max()
    np.testing.assert_allclose(np.sort(theta), np.sort(ref), atol=1e-9 * anorm)
    G = np.array([[oracle.vdot(a, b) for b in V] for a in V])
    np.testing.assert_allclose(G, np.eye(k), atol=1e-12)
    for th, v, w in zip(theta, V, W):
        np.testing.assert_allclose(w, oracle.coarse_apply(A, v, cs.cdims), atol=1e-12 * anorm)
        assert oracle.norm(w - th * v) <= 1e-7 * anorm


def test_coarse_deflation_keeps_only_converged_pairs():
    """A block filtered too little to be an invariant subspace of A yields Ritz pairs of A that
    are not eigenpairs; only pairs with residual |A y - theta y| <= 1e-2 |theta| are returned.
    For a Hermitian matrix every such theta lies within its residual of an eigenvalue (checked
    against the dense matrix), and more passes find more pairs."""
    cs, A = _small_coarse()
    m = 12
    V0 = [hi.gaussian_coarse(cs.nc, cs.nb, seed=40 + i) for i in range(m)]
    D = oracle.coarse_dense(A, cs.cdims)
    ev = np.linalg.eigvalsh(D)
    found = []
    for iters in (2, 3):
        theta, V, W = oracle.coarse_deflation(A, cs.cdims, V0, m, degree=40, iters=iters, cut=0.05)
        found.append(len(theta))
        assert np.all(np.diff(np.abs(theta)) >= 0)
        for th, v, w in zip(theta, V, W):
            y = v.reshape(-1)
            r = np.linalg.norm(D @ y - th * y)
            assert abs(np.linalg.norm(y) - 1.0) <= 1e-12
            assert r <= oracle.DEFL_RES_TOL * abs(th) * (1 + 1e-9)
            assert np.min(np.abs(ev - th)) <= r * (1 + 1e-9) + 1e-12
    assert 0 < found[0] < found[1] < m


def test_deflated_coarse_cr():
    """The Galerkin start leaves a residual orthogonal to the deflation space; the deflated
    solve reaches the same solution in no more iterations."""
    cs, A = _small_coarse()
    k, m = 6, 12
    V0 = [hi.gaussian_coarse(cs.nc, cs.nb, seed=40 + i) for i in range(m)]
    defl = oracle.coarse_deflation(A, cs.cdims, V0, k, degree=40, iters=4, cut=0.05)
    b = hi.gaussian_coarse(cs.nc, cs.nb, seed=7)
    theta, V = defl[0], defl[1]
    x0 = sum((oracle.vdot(v, b) / th) * v for th, v in zip(theta, V))
    r0 = b - oracle.coarse_apply(A, x0, cs.cdims)
    for v in V:
        assert abs(oracle.vdot(v, r0)) <= 1e-10 * oracle.norm(b)
    plain = oracle.coarse_cr(A, b, cs.cdims, tol=1e-10, maxiter=5000)
    defl_res = oracle.coarse_cr(A, b, cs.cdims, tol=1e-10, maxiter=5000, defl=defl)
    assert plain.status == 0 and defl_res.status == 0
    assert defl_res.iters <= plain.iters
    np.testing.assert_allclose(defl_res.x, plain.x, atol=1e-7 * oracle.norm(plain.x))
