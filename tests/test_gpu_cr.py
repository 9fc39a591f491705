"""GPU plain conjugate residual (Sec. 3) through hdcr_solve, against the oracle's CR:
same residual history, true residual <= 1e-8 under the oracle's H, and the error
paths (zero source, maxiter, NaN source, exact breakdown)."""
import numpy as np
import pytest

import hdcr_inputs as hi
import oracle
from paper_1611_06944_amd import Lattice, default_params, pack_fermion, pack_gauge, solve, unpack_fermion, _abi
from tests import dense_ref
from tests.gpu_util import log, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu


def _run(lat, U, b, **kw):
    return solve(lat, to_dev(pack_gauge(U)), to_dev(pack_fermion(b)), params=default_params(**kw))


def test_cr_small_config_matches_oracle():
    """4^4 x 8, M5 = 1.8, mf = 0.01, antiperiodic t, complex128, source seed 0, tol 1e-8."""
    torch_dev()
    L, Ls = (4, 4, 4, 4), 8
    log("CR 4^4x8 vs oracle")
    p = oracle.Params(L, Ls, M5=1.8, mf=0.01)
    lat = Lattice(L, Ls, M5=1.8, mf=0.01)
    U = hi.gauge_field(L, seed=1)
    b = hi.gaussian_fermion(L, Ls, seed=0)
    x, st, hist = _run(lat, U, b, tol=1e-8)
    assert st["status"] == 0
    xs = unpack_fermion(to_host(x), L, Ls)
    ap = lambda f: oracle.apply_h(U, f, p)
    true = oracle.norm(b - ap(xs)) / oracle.norm(b)
    assert true <= 1e-8
    assert abs(st["true_rel_residual"] - true) <= 1e-3 * true
    ref = oracle.cr(ap, b, tol=1e-8, maxiter=10000)
    # the same minimal-residual sequence, up to rounding
    k = min(len(hist), len(ref.history), 60)
    np.testing.assert_allclose(np.array(hist[:k]), np.array(ref.history[:k]) / oracle.norm(b), rtol=1e-6)
    assert abs(st["outer_iters"] - ref.iters) <= 2
    # both solutions solve the system to 1e-8, so they agree to ~kappa * 1e-8
    assert oracle.norm(xs - ref.x) <= 1e-5 * oracle.norm(ref.x)


def test_cr_zero_source_and_maxiter():
    torch_dev()
    L, Ls = (2, 2, 2, 4), 4
    log("CR edge cases")
    lat = Lattice(L, Ls)
    U = hi.gauge_field(L, seed=1)
    x, st, _ = _run(lat, U, np.zeros((4, 2, 2, 2, 4, 4, 3), dtype=complex))
    assert st["status"] == 0 and np.all(to_host(x) == 0)
    b = hi.gaussian_fermion(L, Ls, seed=0)
    x, st, hist = _run(lat, U, b, maxiter=3)
    assert st["status"] == _abi.HDCR_ENOTCONV and st["outer_iters"] == 3 and len(hist) == 3


def test_cr_nan_source():
    torch_dev()
    L, Ls = (2, 2, 2, 4), 4
    log("CR NaN source")
    lat = Lattice(L, Ls)
    U = hi.gauge_field(L, seed=1)
    b = hi.gaussian_fermion(L, Ls, seed=0)
    b[0, 0, 0, 0, 0, 0, 0] = np.nan
    x, st, _ = _run(lat, U, b)
    assert st["status"] == _abi.HDCR_ENAN


def test_cr_exact_breakdown():
    """b = sqrt|l-| u+ + sqrt(l+) u- (free field eigenvectors) has <b, H b> = 0."""
    torch_dev()
    L, Ls = (2, 2, 2, 4), 4
    log("CR breakdown source")
    p = oracle.Params(L, Ls, M5=1.8, mf=0.05)
    lat = Lattice(L, Ls, M5=1.8, mf=0.05)
    U = hi.gauge_field(L, eps=0.0)
    H = dense_ref.dense_gamma5R5(L, Ls) @ dense_ref.dense_dwf(U, L, Ls, p.M5, p.mf, p.bc)
    lam, vec = np.linalg.eigh(H)
    ip, im = np.argmax(lam), np.argmin(lam)
    b = (np.sqrt(-lam[im]) * vec[:, ip] + np.sqrt(lam[ip]) * vec[:, im]).reshape(p.fshape)
    x, st, _ = _run(lat, U, b)
    assert st["status"] == _abi.HDCR_EBREAKDOWN


def test_cr_resume_from_nonzero_x0():
    """Resuming from an initial guess (the x argument of hdcr_solve holds x0 on entry): CR
    starts from r = b - H x0.  x0 is the 40-iteration iterate of a first solve plus a Gaussian
    perturbation of 1e-3 of its norm; the residual history follows the oracle's CR from the same
    x0, and the solution meets 1e-8 under the oracle's H."""
    torch = torch_dev()
    L, Ls = (4, 4, 4, 4), 8
    log("CR from x0 != 0")
    p = oracle.Params(L, Ls, M5=1.8, mf=0.01)
    lat = Lattice(L, Ls, M5=1.8, mf=0.01)
    U = hi.gauge_field(L, seed=1)
    b = hi.gaussian_fermion(L, Ls, seed=0)
    ap = lambda f: oracle.apply_h(U, f, p)
    x40 = oracle.cr(ap, b, tol=1e-30, maxiter=40, check_true=False).x
    x0 = x40 + 1e-3 * oracle.norm(x40) / np.sqrt(x40.size) * hi.gaussian_fermion(L, Ls, seed=17)
    x = to_dev(pack_fermion(x0))
    x, st, hist = solve(lat, to_dev(pack_gauge(U)), to_dev(pack_fermion(b)), x=x, params=default_params(tol=1e-8))
    assert st["status"] == 0
    xs = unpack_fermion(to_host(x), L, Ls)
    bn = oracle.norm(b)
    assert oracle.norm(b - ap(xs)) <= 1e-8 * bn
    ref = oracle.cr(ap, b, tol=1e-8, maxiter=10000, x0=x0)
    k = min(len(hist), len(ref.history), 60)
    np.testing.assert_allclose(np.array(hist[:k]), np.array(ref.history[:k]) / bn, rtol=1e-6)
    assert abs(st["outer_iters"] - ref.iters) <= 2
    # the guess was used: fewer iterations than from zero, whose count is pinned above
    assert st["outer_iters"] < oracle.cr(ap, b, tol=1e-8, maxiter=10000).iters
    # an exact solution as x0 returns at once with no iteration
    x, st, _ = solve(lat, to_dev(pack_gauge(U)), to_dev(pack_fermion(b)), x=to_dev(pack_fermion(xs)),
                     params=default_params(tol=1e-8))
    assert st["status"] == 0 and st["outer_iters"] == 0
