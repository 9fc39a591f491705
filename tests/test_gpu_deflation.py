"""GPU coarse-space eigenvector deflation (Sec. 5 names it for the coarse-solve cost) against
the FP64 oracle, through the C-ABI: the filtered subspace iteration in A^2 with Rayleigh-Ritz
steps, the deflated (Galerkin-start) coarse CR, and the deflated two-level cycle and solve.

The coarse operators come from Chebyshev-filtered subspace vectors, as in the solver, so
their lowest modes are separated from the rest of the spectrum and the set-up converges
(the oracle's own pins check the eigenpairs against the dense matrix).

Tolerances.  Both sides run the same steps from the same start block, but the
eigenvector phases of the small dense eigenproblems (Jacobi on the device side,
LAPACK in the oracle) and the Gram-Schmidt form (classical twice against modified
twice) differ, so vectors are compared through phase-free quantities: the Ritz
values, |<v_gpu, v_oracle>| and the Galerkin start x0 = V diag(1/theta) V^dag b,
which depends only on the converged eigenpairs.  FP64: eigenvalues to 1e-9 |A| (the
oracle's pin against the dense matrix), x0 and the fixed-iteration CR iterates to
1e-8 (eigenvector residuals are ~1e-15 |A| and the gap above the deflated cluster is
>= 0.02 |A|, so the eigenvectors agree to ~1e-12; the margin covers the CR's
amplification of rounding over a few iterations).  FP32 (C64 and BF16 storage of A):
the eigenpairs are those of the stored operator, so they are compared with the dense
eigenvalues of the exported storage to 1e-4 |A| (FP32 Gram-Schmidt leaves the block
orthonormal to ~1e-6, and Ritz values are accurate to the square of that)."""
import numpy as np
import pytest

import hdcr_inputs as hi
import oracle
import paper_1611_06944_amd as hd
from tests.gpu_util import log, max_rel_elem, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

DEG, ITERS, CUT, PITERS = 40, 4, 0.05, 30

CASES = [
    # L, Ls, block, nvec, m, k
    ((4, 4, 4, 4), 8, (2, 2, 2, 2), 4, 12, 6),   # n = 128
    ((8, 8, 8, 8), 8, (2, 2, 2, 2), 4, 18, 7),   # n = 2048: ragged Gram tiles and rotation chunks
]
# Nb = 64, n = 1024: with BF16C storage the set-up's block applies run on the matrix cores
CASE_NB64 = ((8, 8, 8, 8), 4, (4, 4, 4, 4), 32, 40, 12)

_cache = {}


def _problem(L, Ls, block, nvec):
    key = (L, Ls, block, nvec)
    if key not in _cache:
        p = oracle.Params(L, Ls, M5=1.8, mf=0.01)
        cs = oracle.Coarse(p, block, nvec)
        lat = hd.Lattice(L, Ls, M5=1.8, mf=0.01, block=block, nvec=nvec)
        U = hi.gauge_field(L, seed=1)
        ap = lambda f: oracle.apply_h(U, f, p)
        lmax = oracle.power_max(ap, hi.gaussian_fermion(L, Ls, seed=99), iters=30) * 1.1
        vecs = [oracle.cheby_filter(ap, e, 12, 0.05 * lmax, lmax) for e in hi.subspace_noise(L, Ls, nvec)]
        basis_ref, st = oracle.block_basis(vecs, cs)
        assert st == 0
        A_ref = oracle.coarse_build(U, basis_ref, cs)
        _cache[key] = (p, cs, lat, U, vecs, basis_ref, A_ref)
    return _cache[key]


def _gpu_coarse(lat, U, vecs, dt):
    return hd.build_coarse(lat, to_dev(hd.pack_gauge(U)), to_dev(np.stack([hd.pack_fermion(v) for v in vecs])), dt)


def _v0(cs, m):
    return [hi.gaussian_coarse(cs.nc, cs.nb, seed=40 + i) for i in range(m)]


def _dense_storage(lat, cs, A, dt):
    """Dense matrix of the operator as the library stores it (for the FP32 checks)."""
    return oracle.coarse_dense(to_host(hd.export_coarse(lat, A, dt)), cs.cdims)


@pytest.mark.parametrize("L,Ls,block,nvec,m,k", CASES)
def test_deflation_fp64_matches_oracle_and_dense(L, Ls, block, nvec, m, k):
    torch = torch_dev()
    log(f"deflation fp64 L={L} Ls={Ls} m={m} k={k}")
    p, cs, lat, U, vecs, basis_ref, A_ref = _problem(L, Ls, block, nvec)
    V0 = _v0(cs, m)
    th_ref, V_ref, _ = oracle.coarse_deflation(A_ref, cs.cdims, V0, k, degree=DEG, iters=ITERS, cut=CUT,
                                               power_iters=PITERS)
    D = oracle.coarse_dense(A_ref, cs.cdims)
    ev = np.linalg.eigvalsh(D)
    anorm = np.abs(ev).max()
    _, A = _gpu_coarse(lat, U, vecs, hd.C128)
    d = hd.build_deflation(lat, A, hd.C128, to_dev(np.stack(V0)), k, degree=DEG, iters=ITERS, cut=CUT,
                           power_iters=PITERS)
    assert d.k == k
    th = to_host(d.theta)
    np.testing.assert_array_equal(th, np.array(d.theta_host))
    # ascending |theta|, the k eigenvalues of smallest |lambda|, the oracle's Ritz values
    assert np.all(np.diff(np.abs(th)) >= 0)
    np.testing.assert_allclose(np.sort(th), np.sort(ev[np.argsort(np.abs(ev))[:k]]), atol=1e-9 * anorm)
    np.testing.assert_allclose(th, th_ref, atol=1e-9 * anorm)
    V, W = to_host(d.V).reshape(k, -1), to_host(d.W).reshape(k, -1)
    np.testing.assert_allclose(V.conj() @ V.T, np.eye(k), atol=1e-12)
    for i in range(k):
        np.testing.assert_allclose(W[i], D @ V[i], atol=1e-12 * anorm)
        assert np.linalg.norm(D @ V[i] - th[i] * V[i]) <= 1e-8 * anorm
        assert abs(abs(np.vdot(V_ref[i].ravel(), V[i])) - 1.0) <= 1e-8


def test_deflation_keeps_only_converged_pairs():
    """A block filtered too little (degree 40, 2 passes, k = m = 12) leaves Ritz pairs of A that
    are not eigenpairs; the set-up returns only those with |A y - theta y| <= 1e-2 |theta|, fewer
    than asked for, each within its residual of an eigenvalue of the dense operator, in
    ascending |theta| (FP64 storage; the oracle applies the same rule)."""
    torch = torch_dev()
    L, Ls, block, nvec, m, _ = CASES[0]
    log(f"deflation, unconverged block L={L} m={m}")
    p, cs, lat, U, vecs, basis_ref, A_ref = _problem(L, Ls, block, nvec)
    _, A = _gpu_coarse(lat, U, vecs, hd.C128)
    D = oracle.coarse_dense(A_ref, cs.cdims)
    ev = np.linalg.eigvalsh(D)
    V0 = _v0(cs, m)
    d = hd.build_deflation(lat, A, hd.C128, to_dev(np.stack(V0)), m, degree=40, iters=2, cut=CUT, power_iters=PITERS)
    th_ref, _, _ = oracle.coarse_deflation(A_ref, cs.cdims, V0, m, degree=40, iters=2, cut=CUT, power_iters=PITERS)
    log(f"  found {d.k} of {m} (oracle {len(th_ref)})")
    assert 0 < d.k < m and abs(d.k - len(th_ref)) <= 1
    th = np.array(d.theta_host)
    assert np.all(np.diff(np.abs(th)) >= 0)
    V = to_host(d.V).reshape(d.k, -1)
    W = to_host(d.W).reshape(d.k, -1)
    for q in range(d.k):
        r = np.linalg.norm(D @ V[q] - th[q] * V[q])
        assert np.linalg.norm(W[q] - D @ V[q]) <= 1e-12 * np.abs(ev).max()
        assert r <= 1e-2 * abs(th[q]) * (1 + 1e-6)
        assert np.min(np.abs(ev - th[q])) <= r * (1 + 1e-9) + 1e-12


@pytest.mark.parametrize("L,Ls,block,nvec,m,k", CASES)
def test_deflated_coarse_cr_parity(L, Ls, block, nvec, m, k):
    """hdcr_coarse_solve against the oracle's coarse_cr: from 0 (1e-10), the Galerkin start
    alone (maxiter 0: V^dag r0 = 0) and 8 fixed iterations from it."""
    torch = torch_dev()
    log(f"deflated coarse CR L={L} Ls={Ls} m={m} k={k}")
    p, cs, lat, U, vecs, basis_ref, A_ref = _problem(L, Ls, block, nvec)
    V0 = _v0(cs, m)
    defl_ref = oracle.coarse_deflation(A_ref, cs.cdims, V0, k, degree=DEG, iters=ITERS, cut=CUT,
                                       power_iters=PITERS)
    _, A = _gpu_coarse(lat, U, vecs, hd.C128)
    d = hd.build_deflation(lat, A, hd.C128, to_dev(np.stack(V0)), k, degree=DEG, iters=ITERS, cut=CUT,
                           power_iters=PITERS)
    b = hi.gaussian_coarse(cs.nc, cs.nb, seed=7)
    bd = to_dev(b)
    # plain CR, fixed iterations
    x, it = hd.coarse_solve(lat, A, hd.C128, bd, maxiter=8, tol=0.0)
    ref = oracle.coarse_cr(A_ref, b, cs.cdims, tol=0.0, maxiter=8).x
    assert it == 8
    assert max_rel_elem(to_host(x), ref) <= 1e-10
    # Galerkin start only
    x0, it = hd.coarse_solve(lat, A, hd.C128, bd, maxiter=0, tol=0.0, defl=d)
    assert it == 0
    x0_ref = sum((oracle.vdot(v, b) / t) * v for t, v in zip(defl_ref[0], defl_ref[1]))
    assert max_rel_elem(to_host(x0), x0_ref) <= 1e-8
    r0 = b.ravel() - oracle.coarse_dense(A_ref, cs.cdims) @ to_host(x0).ravel()
    Vh = to_host(d.V).reshape(k, -1)
    assert np.max(np.abs(Vh.conj() @ r0)) <= 1e-10 * np.linalg.norm(b)
    # deflated CR, fixed iterations
    x, it = hd.coarse_solve(lat, A, hd.C128, bd, maxiter=8, tol=0.0, defl=d)
    ref = oracle.coarse_cr(A_ref, b, cs.cdims, tol=0.0, maxiter=8, defl=defl_ref).x
    assert it == 8
    assert max_rel_elem(to_host(x), ref) <= 1e-8
    # to tolerance: the deflated solve needs fewer iterations and meets the tolerance
    _, it_plain = hd.coarse_solve(lat, A, hd.C128, bd, maxiter=500, tol=1e-2)
    xd, it_defl = hd.coarse_solve(lat, A, hd.C128, bd, maxiter=500, tol=1e-2, defl=d)
    ref_plain = oracle.coarse_cr(A_ref, b, cs.cdims, tol=1e-2, maxiter=500)
    ref_defl = oracle.coarse_cr(A_ref, b, cs.cdims, tol=1e-2, maxiter=500, defl=defl_ref)
    log(f"  coarse CR to 1e-2: plain {it_plain} (oracle {ref_plain.iters}), deflated {it_defl} "
        f"(oracle {ref_defl.iters})")
    assert it_plain == ref_plain.iters and it_defl == ref_defl.iters
    assert it_defl < it_plain
    res = b.ravel() - oracle.coarse_dense(A_ref, cs.cdims) @ to_host(xd).ravel()
    assert np.linalg.norm(res) <= 1.0001e-2 * np.linalg.norm(b)


@pytest.mark.parametrize("dt,case", [("c64", 1), ("bf16", 1), ("bf16", 2)])
def test_deflation_fp32_storage(dt, case):
    """Set-up with A in C64 or BF16C storage (FP32 vectors): Ritz values of the stored
    operator, orthonormal V, W = A V, and the deflated FP32 coarse CR converging.  With
    BF16C and Nb = 64 the set-up's block applies run on the matrix cores with the
    vectors split into three bf16 terms."""
    torch = torch_dev()
    L, Ls, block, nvec, m, k = CASES[1] if case == 1 else CASE_NB64
    log(f"deflation {dt} L={L} m={m} k={k}")
    p, cs, lat, U, vecs, basis_ref, A_ref = _problem(L, Ls, block, nvec)
    code = hd.C64 if dt == "c64" else hd.BF16C
    _, A = _gpu_coarse(lat, U, vecs, code)
    Ds = _dense_storage(lat, cs, A, code)
    ev = np.linalg.eigvalsh(0.5 * (Ds + Ds.conj().T))
    anorm = np.abs(ev).max()
    d = hd.build_deflation(lat, A, code, to_dev(np.stack(_v0(cs, m))), k, degree=DEG, iters=ITERS, cut=CUT,
                           power_iters=PITERS)
    assert d.V.dtype == torch.complex64 and d.k == k
    th = to_host(d.theta)
    np.testing.assert_allclose(np.sort(th), np.sort(ev[np.argsort(np.abs(ev))[:k]]), atol=1e-4 * anorm)
    V = to_host(d.V).reshape(k, -1).astype(np.complex128)
    W = to_host(d.W).reshape(k, -1).astype(np.complex128)
    np.testing.assert_allclose(V.conj() @ V.T, np.eye(k), atol=1e-5)
    for i in range(k):
        assert np.linalg.norm(W[i] - Ds @ V[i]) <= 1e-5 * anorm
        assert np.linalg.norm(Ds @ V[i] - th[i] * V[i]) <= 1e-3 * anorm
    b = hi.gaussian_coarse(cs.nc, cs.nb, seed=7)
    bd = to_dev(b, torch.complex64)
    _, it_plain = hd.coarse_solve(lat, A, code, bd, maxiter=500, tol=1e-2)
    xd, it_defl = hd.coarse_solve(lat, A, code, bd, maxiter=500, tol=1e-2, defl=d)
    log(f"  {dt} coarse CR to 1e-2: plain {it_plain}, deflated {it_defl}")
    assert it_defl < it_plain
    res = b.ravel() - Ds @ to_host(xd).ravel().astype(np.complex128)
    assert np.linalg.norm(res) <= 1.01e-2 * np.linalg.norm(b)


@pytest.mark.parametrize("inner", ["c128", "c64"])
def test_deflated_vcycle_parity(inner):
    """The two-level cycle with a deflated coarse solve of exactly 6 iterations against the
    oracle's vcycle with its own deflation space (FP64 1e-8; FP32 1e-4, the FP32 set-up's
    eigenvectors agreeing with the FP64 ones to ~1e-5)."""
    torch = torch_dev()
    L, Ls, block, nvec, m, k = CASES[0]
    log(f"deflated vcycle inner={inner}")
    p, cs, lat, U, vecs, basis_ref, A_ref = _problem(L, Ls, block, nvec)
    V0 = _v0(cs, m)
    defl_ref = oracle.coarse_deflation(A_ref, cs.cdims, V0, k, degree=DEG, iters=ITERS, cut=CUT,
                                       power_iters=PITERS)
    r = hi.gaussian_fermion(L, Ls, seed=5)
    ap = lambda f: oracle.apply_h(U, f, p)
    ref = oracle.vcycle(ap, A_ref, basis_ref, cs, r, order=10, lo=1.0, hi=64.0, ctol=0.0, cmaxiter=6, defl=defl_ref)
    cdt = hd.C128 if inner == "c128" else hd.C64
    basis, A = _gpu_coarse(lat, U, vecs, cdt)
    d = hd.build_deflation(lat, A, cdt, to_dev(np.stack(V0)), k, degree=DEG, iters=ITERS, cut=CUT,
                           power_iters=PITERS)
    prm = hd.default_params(inner_dtype=cdt, coarse_dtype=cdt, coarse_tol=0.0, coarse_maxiter=6)
    e = hd.unpack_fermion(to_host(hd.vcycle(lat, to_dev(hd.pack_gauge(U)), basis, A, to_dev(hd.pack_fermion(r)), prm,
                                            defl=d)), L, Ls)
    assert max_rel_elem(e, ref) <= (1e-8 if inner == "c128" else 1e-4)
    # without deflation the cycle differs (the deflation is really applied)
    e0 = hd.unpack_fermion(to_host(hd.vcycle(lat, to_dev(hd.pack_gauge(U)), basis, A, to_dev(hd.pack_fermion(r)),
                                             prm)), L, Ls)
    assert max_rel_elem(e0, ref) > 1e-6


@pytest.mark.parametrize("inner", ["c128", "c64"])
def test_hdcr_solve_deflated_converges(inner):
    """The full HDCR solve with the deflated coarse solve reaches the tolerance, with fewer
    coarse iterations than without deflation."""
    torch = torch_dev()
    L, Ls, block, nvec, m, k = CASES[1]
    log(f"deflated HDCR solve inner={inner}")
    p, cs, lat, U, vecs, basis_ref, A_ref = _problem(L, Ls, block, nvec)
    cdt = hd.C128 if inner == "c128" else hd.C64
    basis, A = _gpu_coarse(lat, U, vecs, cdt)
    d = hd.build_deflation(lat, A, cdt, to_dev(np.stack(_v0(cs, m))), k, degree=DEG, iters=ITERS, cut=CUT,
                           power_iters=PITERS)
    Ud = to_dev(hd.pack_gauge(U))
    b = to_dev(hd.pack_fermion(hi.gaussian_fermion(L, Ls, seed=11)))
    prm = hd.default_params(precond=hd.PRECOND_TWO_LEVEL, tol=1e-8, maxiter=200, inner_dtype=cdt, coarse_dtype=cdt,
                            coarse_tol=0.05, coarse_maxiter=200, cheb_lo=1.0, cheb_hi=64.0)
    _, st0, _ = hd.solve(lat, Ud, b, params=prm, basis=basis, A=A)
    x, st1, _ = hd.solve(lat, Ud, b, params=prm, basis=basis, A=A, defl=d)
    log(f"  plain: outer {st0['outer_iters']} coarse {st0['coarse_iters']}; deflated: outer {st1['outer_iters']} "
        f"coarse {st1['coarse_iters']}")
    assert st0["status"] == 0 and st1["status"] == 0
    assert st1["true_rel_residual"] <= 1e-8
    assert st1["coarse_iters"] < st0["coarse_iters"]
    # the true residual, from the oracle's operator
    xh = hd.unpack_fermion(to_host(x), L, Ls)
    bh = hd.unpack_fermion(to_host(b), L, Ls)
    assert oracle.norm(bh - oracle.apply_h(U, xh, p)) <= 1.01e-8 * oracle.norm(bh)
