"""Pins of the oracle's coarse space (Sec. 4): chiral split, block orthonormal basis,
restriction/prolongation, little Dirac operator and coarse apply, against numpy QR,
projector identities and dense brute force P^dag H P."""
import itertools

import numpy as np
import pytest

import hdcr_inputs as hi
import oracle
from tests import dense_ref


def _setup(L, Ls, block, nvec, seed=1, mf=0.01):
    p = oracle.Params(L, Ls, M5=1.8, mf=mf)
    cs = oracle.Coarse(p, block, nvec)
    U = hi.gauge_field(L, seed=seed)
    vecs = [hi.gaussian_fermion(L, Ls, seed=100 + k) for k in range(nvec)]
    basis, st = oracle.block_basis(vecs, cs)
    assert st == 0
    return p, cs, U, vecs, basis


def _block_mask(L, block, a):
    """Boolean mask [t,z,y,x] of the fine sites in coarse site a."""
    C = [l // b for l, b in zip(L, block)]
    c = [a % C[0], (a // C[0]) % C[1], (a // (C[0] * C[1])) % C[2], a // (C[0] * C[1] * C[2])]
    Lx, Ly, Lz, Lt = L
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    return ((x // block[0] == c[0]) & (y // block[1] == c[1]) & (z // block[2] == c[2]) & (t // block[3] == c[3]))


def _g5r5(f):
    """Gamma5 = gamma5 R5 in numpy: reverse s and flip the sign of spins 2, 3."""
    sgn = np.array([1, 1, -1, -1])[:, None]
    return f[..., ::-1, :, :] * sgn


def test_block_basis_matches_numpy_qr():
    L, Ls, block, nvec = (4, 4, 2, 2), 4, (2, 2, 2, 2), 5
    p, cs, U, vecs, basis = _setup(L, Ls, block, nvec)
    for a in [0, 3, cs.nc - 1]:
        m = _block_mask(L, block, a)
        for h, sgn in enumerate([1.0, -1.0]):
            cols = [(0.5 * (v + sgn * _g5r5(v)))[m].ravel() for v in vecs]
            Q, R = np.linalg.qr(np.stack(cols, axis=1))
            ph = np.diag(R) / np.abs(np.diag(R))
            Q = Q * ph[None, :]
            got = np.stack([basis[h * nvec + k][m].ravel() for k in range(nvec)], axis=1)
            np.testing.assert_allclose(got, Q, atol=1e-13)
    # every basis field (phi^a_k on all blocks a) is a Gamma5 eigenvector of its
    # chirality: +1 for k < nvec, -1 for k >= nvec
    for k in range(cs.nb):
        sgn = 1.0 if k < nvec else -1.0
        np.testing.assert_allclose(_g5r5(basis[k]), sgn * basis[k], atol=1e-14)
        assert oracle.norm(basis[k]) > 0.5


def test_projector_identities_and_span():
    L, Ls, block, nvec = (4, 4, 4, 4), 4, (2, 2, 2, 2), 4
    p, cs, U, vecs, basis = _setup(L, Ls, block, nvec)
    rng = np.random.default_rng(3)
    v = rng.standard_normal((cs.nc, cs.nb)) + 1j * rng.standard_normal((cs.nc, cs.nb))
    # P^dag P = 1
    np.testing.assert_allclose(oracle.restrict(basis, oracle.prolong(basis, v, cs), cs), v, atol=1e-13)
    # P_S = P P^dag is a projector
    psi = hi.gaussian_fermion(L, Ls, seed=8)
    ps = oracle.prolong(basis, oracle.restrict(basis, psi, cs), cs)
    ps2 = oracle.prolong(basis, oracle.restrict(basis, ps, cs), cs)
    np.testing.assert_allclose(ps2, ps, atol=1e-12)
    # span{phi_k} is contained in span{phi^b_k} (Sec. 4, span display)
    for vk in vecs:
        np.testing.assert_allclose(oracle.prolong(basis, oracle.restrict(basis, vk, cs), cs), vk, atol=1e-12)
    # adjointness <P v, psi> = <v, P^dag psi>
    lhs = oracle.vdot(oracle.prolong(basis, v, cs), psi)
    rhs = oracle.vdot(v, oracle.restrict(basis, psi, cs))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # Gamma5 P = P Gamma5c with Gamma5c = diag(+1 x nvec, -1 x nvec)
    g5c = np.concatenate([np.ones(nvec), -np.ones(nvec)])
    np.testing.assert_allclose(_g5r5(oracle.prolong(basis, v, cs)), oracle.prolong(basis, v * g5c, cs),
                               atol=1e-13)


def _dense_P(basis, cs):
    """Dense prolongation matrix: column a*nb + k is phi^a_k (basis field k on block a)."""
    L = cs.p.L
    n = basis[0].size
    P = np.zeros((n, cs.nc * cs.nb), dtype=complex)
    for a in range(cs.nc):
        m = _block_mask(L, cs.block, a)
        for k in range(cs.nb):
            f = np.zeros_like(basis[k])
            f[m] = basis[k][m]
            P[:, a * cs.nb + k] = f.ravel()
    return P


@pytest.mark.parametrize("block,nvec", [((1, 1, 1, 1), 4), ((2, 2, 2, 2), 4), ((1, 1, 1, 1), 24),
                                        ((2, 1, 2, 1), 3)])
def test_coarse_build_dense_brute_force(block, nvec):
    L, Ls = (2, 2, 2, 2), 4
    p, cs, U, vecs, basis = _setup(L, Ls, block, nvec, mf=0.05)
    A = oracle.coarse_build(U, basis, cs)
    H = dense_ref.dense_gamma5R5(L, Ls) @ dense_ref.dense_dwf(U, L, Ls, p.M5, p.mf, p.bc)
    P = _dense_P(basis, cs)
    Ad = oracle.coarse_dense(A, cs.cdims)
    np.testing.assert_allclose(Ad, P.conj().T @ H @ P, atol=1e-12)
    if nvec * 2 == 12 * Ls * int(np.prod(block)):
        # full-rank special case: P unitary, so A and H share their spectrum
        np.testing.assert_allclose(np.linalg.eigvalsh(Ad), np.linalg.eigvalsh(H), atol=1e-11)
    # Gamma5c A = P^dag (Gamma5 H) P = P^dag D P
    g5c = np.tile(np.concatenate([np.ones(nvec), -np.ones(nvec)]), cs.nc)
    D = dense_ref.dense_dwf(U, L, Ls, p.M5, p.mf, p.bc)
    np.testing.assert_allclose(g5c[:, None] * Ad, P.conj().T @ D @ P, atol=1e-12)


def test_coarse_build_nondegenerate_neighbours():
    """Coarse extent 3: each A[a][d] is exactly <phi^a_j | H | phi^(a+d)_k>."""
    L, Ls, block, nvec = (6, 6, 6, 6), 4, (2, 2, 2, 2), 3
    p, cs, U, vecs, basis = _setup(L, Ls, block, nvec)
    kc = [0, 4]
    cols = oracle.coarse_columns(U, basis, cs, kc)
    rng = np.random.default_rng(0)
    C = cs.cdims
    for a in rng.choice(cs.nc, size=3, replace=False):
        c = [a % C[0], (a // C[0]) % C[1], (a // (C[0] * C[1])) % C[2], a // (C[0] * C[1] * C[2])]
        for d in range(9):
            cc = list(c)
            if d > 0:
                mu = (d - 1) % 4
                cc[mu] = (cc[mu] + (1 if d <= 4 else -1)) % C[mu]
            b = ((cc[3] * C[2] + cc[2]) * C[1] + cc[1]) * C[0] + cc[0]
            mb = _block_mask(L, block, b)
            ma = _block_mask(L, block, a)
            for ci, k in enumerate(kc):
                f = np.zeros_like(basis[k])
                f[mb] = basis[k][mb]
                hf = oracle.apply_h(U, f, p)
                for j in range(cs.nb):
                    ref = np.vdot(basis[j][ma].ravel(), hf[ma].ravel())
                    assert abs(cols[ci, a, d, j] - ref) <= 1e-12 * (1 + abs(ref))


def test_coarse_hermiticity_and_apply():
    L, Ls, block, nvec = (4, 4, 4, 6), 4, (2, 2, 2, 2), 3
    p, cs, U, vecs, basis = _setup(L, Ls, block, nvec)
    A = oracle.coarse_build(U, basis, cs)
    C = cs.cdims
    for a in range(cs.nc):
        np.testing.assert_allclose(A[a, 0], A[a, 0].conj().T, atol=1e-13)
        c = [a % C[0], (a // C[0]) % C[1], (a // (C[0] * C[1])) % C[2], a // (C[0] * C[1] * C[2])]
        for mu in range(4):
            cc = list(c)
            cc[mu] = (cc[mu] + 1) % C[mu]
            b = ((cc[3] * C[2] + cc[2]) * C[1] + cc[1]) * C[0] + cc[0]
            np.testing.assert_allclose(A[a, 1 + mu], A[b, 5 + mu].conj().T, atol=1e-13)
    # coarse apply equals the dense coarse matrix, single and multiple right-hand sides
    Ad = oracle.coarse_dense(A, C)
    v = hi.gaussian_coarse(cs.nc, cs.nb, seed=5, nrhs=3)
    out = oracle.coarse_apply(A, v, C)
    for r in range(3):
        np.testing.assert_allclose(out[r].ravel(), Ad @ v[r].ravel(), atol=1e-12)
    # Galerkin action identity A v = P^dag H P v
    w = oracle.restrict(basis, oracle.apply_h(U, oracle.prolong(basis, v[0], cs), p), cs)
    np.testing.assert_allclose(out[0], w, atol=1e-12)


def test_rank_deficient_block_is_reported():
    L, Ls, block, nvec = (2, 2, 2, 2), 4, (2, 2, 2, 2), 3
    p = oracle.Params(L, Ls)
    cs = oracle.Coarse(p, block, nvec)
    v0 = hi.gaussian_fermion(L, Ls, seed=1)
    vecs = [v0, hi.gaussian_fermion(L, Ls, seed=2), 2.0 * v0]
    _, st = oracle.block_basis(vecs, cs)
    assert st == oracle.ERANK
