"""FP64 CPU oracle for the HDCR hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_1611_06944_amd``) and never imports it.

Arrays are numpy complex128 in the canonical site-major layout
``psi[t, z, y, x, s, spin, colour]`` / ``U[t, z, y, x, mu, row, col]``.
Coarse vectors are ``v[site_c, k]`` and the little Dirac operator is
``A[site_c, d, j, k]`` with d in D9 = (0, +x, +y, +z, +t, -x, -y, -z, -t).

The operator-level routines (H, the hop-class split of H, the block basis,
restriction, prolongation, the little Dirac operator and the coarse apply)
are plain C++ loops in ``hdcr_oracle.cpp``.  This module adds, in numpy:

* conjugate residual for Hermitian indefinite H (Sec. 3),
* Chebyshev interpolation of 1/y and the smoother S = p(H^2) H (Sec. 4,
  order-10 smoother on [1, 64]),
* the high-order Chebyshev low-pass filter used to generate the subspace
  (Sec. 4 and the Fig. 1 caption),
* the coarse Krylov solve Q = P A^-1 P^dag (Sec. 4, coarse-inverse display),
* the symmetric two-level cycle (Sec. 4, the M_outer display) and the
  flexible (variable-preconditioned) GCR outer iteration (Sec. 4),
* the Hermitian Wilson kernel H_W = gamma5 D_W(-M5) and the continued-fraction
  form of the overlap operator as a 5d matrix (Sec. 3, the continued-fraction
  display), with its coefficients beta_i and R as inputs.

Each function names the passage it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hdcr_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ERANK = 4


def build(force: bool = True) -> str:
    """Compile the C++ half of the oracle (g++ -O3 -fopenmp)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["g++", "-O3", "-march=x86-64-v2", "-fopenmp", "-std=c++17", "-shared", "-fPIC",
               _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        _lib = ctypes.CDLL(_LIB_PATH)
    return _lib


@dataclass
class Params:
    """Fine-lattice parameters: L = (Lx, Ly, Lz, Lt), Ls, M5, mf, bc per direction, and
    b, the scale of the 4d part in the Cayley form with c = 0 (Sec. 3; b = 1 is Shamir)."""
    L: tuple
    Ls: int
    M5: float = 1.8
    mf: float = 0.01
    bc: tuple = (1, 1, 1, -1)
    b: float = 1.0

    @property
    def dims(self):
        return (ctypes.c_int * 5)(*[int(v) for v in self.L], int(self.Ls))

    @property
    def cbc(self):
        return (ctypes.c_int * 4)(*[int(v) for v in self.bc])

    @property
    def fshape(self):
        Lx, Ly, Lz, Lt = self.L
        return (Lt, Lz, Ly, Lx, self.Ls, 4, 3)


def _dp(a: np.ndarray):
    assert a.dtype == np.complex128 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def gamma(mu: int) -> np.ndarray:
    """The oracle's gamma matrix (mu = 0..3 for x, y, z, t; 4 for gamma5)."""
    out = np.zeros((4, 4), dtype=np.complex128)
    lib().or_gamma(ctypes.c_int(mu), _dp(out))
    return out


# ----------------------------------------------------------------------------
# Fine operator (Sec. 3): D_dwf and H = Gamma5 D_dwf
# ----------------------------------------------------------------------------

def apply_dw(U, psi, p: Params) -> np.ndarray:
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    lib().or_apply_dw(p.dims, p.cbc, ctypes.c_double(p.M5), ctypes.c_double(p.mf), ctypes.c_double(p.b), _dp(U), _dp(psi), _dp(out))
    return out


def apply_h(U, psi, p: Params) -> np.ndarray:
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    lib().or_apply_h(p.dims, p.cbc, ctypes.c_double(p.M5), ctypes.c_double(p.mf), ctypes.c_double(p.b), _dp(U), _dp(psi), _dp(out))
    return out


def apply_h_sites(U, psi, p: Params, sel) -> np.ndarray:
    """(H psi) at the selected output sites sel = site4 * Ls + s; returns [len(sel), 4, 3]."""
    U, psi = _c(U), _c(psi)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    out = np.empty((len(sel), 4, 3), dtype=np.complex128)
    lib().or_apply_h_sites(p.dims, p.cbc, ctypes.c_double(p.M5), ctypes.c_double(p.mf), ctypes.c_double(p.b), _dp(U), _dp(psi),
                           ctypes.c_long(len(sel)), sel.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dp(out))
    return out


def apply_h_classes(U, psi, p: Params, block) -> np.ndarray:
    """H split by hop class relative to the blocks (9 fields, D9 order)."""
    U, psi = _c(U), _c(psi)
    out = np.empty((9,) + psi.shape, dtype=np.complex128)
    blk = (ctypes.c_int * 4)(*[int(b) for b in block])
    lib().or_apply_h_classes(p.dims, p.cbc, ctypes.c_double(p.M5), ctypes.c_double(p.mf), ctypes.c_double(p.b), blk,
                             _dp(U), _dp(psi), _dp(out))
    return out


def apply_gamma5_field(psi) -> np.ndarray:
    """Gamma5 = gamma5 R5 on a fine field: (Gamma5 psi)(x,s) = gamma5 psi(x, Ls-1-s)."""
    g5 = gamma(4)
    return np.einsum("ab,...sbc->...sac", g5, psi[..., ::-1, :, :])


# ----------------------------------------------------------------------------
# Continued-fraction overlap operator (Sec. 3, the continued-fraction matrix)
# ----------------------------------------------------------------------------

def apply_hw(U, psi, M5: float, bc=(1, 1, 1, -1)) -> np.ndarray:
    """H_W psi = gamma5 D_W(-M5) psi, the Hermitian Wilson kernel of the overlap operator
    (Sec. 3), slice by slice on a field psi[t, z, y, x, s, spin, colour]:

        D_W psi(x) = (4 - M5) psi(x)
                     - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x + mu) + (1 + g_mu) U_mu(x - mu)^dag psi(x - mu)],

    with the factor bc[mu] on a hop that crosses the lattice boundary (the 4d part of the
    domain wall operator's conventions).  Plain numpy: each hop is a shift of the whole
    field by one site along the array axis of mu.
    """
    U, psi = _c(U), _c(psi)
    axis = {0: 3, 1: 2, 2: 1, 3: 0}   # mu -> array axis of (t, z, y, x)
    out = (4.0 - M5) * psi
    eye = np.eye(4)
    for mu in range(4):
        ax, L = axis[mu], psi.shape[axis[mu]]
        g = gamma(mu)
        Umu = U[..., mu, :, :]
        # forward: psi(x + mu), with bc[mu] where x + mu wraps (x = L - 1)
        fwd = np.roll(psi, -1, axis=ax)
        edge = [slice(None)] * psi.ndim
        edge[ax] = L - 1
        fwd[tuple(edge)] *= bc[mu]
        t = np.einsum("tzyxab,tzyxsjb->tzyxsja", Umu, fwd)            # colour: U psi
        out -= 0.5 * np.einsum("ij,tzyxsja->tzyxsia", eye - g, t)     # spin: (1 - g)
        # backward: U_mu(x - mu)^dag psi(x - mu), with bc[mu] where x - mu wraps (x = 0)
        bwd = np.roll(psi, 1, axis=ax)
        Ub = np.roll(Umu, 1, axis=ax)
        edge[ax] = 0
        bwd[tuple(edge)] *= bc[mu]
        t = np.einsum("tzyxba,tzyxsjb->tzyxsja", Ub.conj(), bwd)      # colour: U^dag psi
        out -= 0.5 * np.einsum("ij,tzyxsja->tzyxsia", eye + g, t)     # spin: (1 + g)
    return np.einsum("ij,tzyxsja->tzyxsia", gamma(4), out)


def cf_coefficients(beta):
    """Diagonal signs and couplings of the continued-fraction matrix (Sec. 3) for m = len(beta)
    pole slices plus the last slice (Ls = m + 1), read off the printed matrix and continued to any
    m: slice i < m carries (-1)^i H, slice m carries R gamma5 + beta_0 H; slices i and i + 1 are
    coupled by 1/sqrt(beta_i beta_(i+1)) for i < m - 1 and by 1/sqrt(beta_(m-1)) for i = m - 1.
    Returns (sigma[Ls], c[Ls - 1])."""
    beta = np.asarray(beta, dtype=np.float64)
    m = len(beta)
    assert m >= 1 and np.all(beta > 0)
    sigma = np.array([(-1.0) ** i for i in range(m)] + [beta[0]])
    c = np.array([1.0 / np.sqrt(beta[i] * beta[i + 1]) for i in range(m - 1)] + [1.0 / np.sqrt(beta[m - 1])])
    return sigma, c


def apply_cf(U, psi, M5: float, beta, R: float, bc=(1, 1, 1, -1)) -> np.ndarray:
    """The continued-fraction form of the overlap operator as a 5d Hermitian indefinite matrix
    (Sec. 3): on a field with Ls = len(beta) + 1 slices,

        (A psi)_i = sigma_i H_W psi_i + [i = m] R gamma5 psi_m + c_(i-1) psi_(i-1) + c_i psi_(i+1),

    sigma and c from ``cf_coefficients``, no coupling beyond the first and last slices.  The
    paper gives the structure but neither the beta_i nor R; both are inputs here."""
    psi = _c(psi)
    sigma, c = cf_coefficients(beta)
    m = len(beta)
    assert psi.shape[4] == m + 1
    hw = apply_hw(U, psi, M5, bc)
    out = sigma[None, None, None, None, :, None, None] * hw
    out[..., m, :, :] += R * np.einsum("ij,tzyxjc->tzyxic", gamma(4), psi[..., m, :, :])
    for i in range(m):
        out[..., i, :, :] += c[i] * psi[..., i + 1, :, :]
        out[..., i + 1, :, :] += c[i] * psi[..., i, :, :]
    return out


def apply_cf_sites(U, psi, M5: float, beta, R: float, sel, bc=(1, 1, 1, -1)) -> np.ndarray:
    """``apply_cf`` at the selected output sites only, sel = site4 * Ls + s with
    site4 = ((t Lz + z) Ly + y) Lx + x; returns [len(sel), 4, 3].  The same terms as
    ``apply_cf`` and ``apply_hw``, gathered per output site (for lattices where the whole
    field is too large for the plain numpy form)."""
    U, psi = _c(U), _c(psi)
    Lt, Lz, Ly, Lx, Ls = psi.shape[:5]
    sigma, c = cf_coefficients(beta)
    m = len(beta)
    assert Ls == m + 1
    sel = np.asarray(sel, dtype=np.int64)
    s = sel % Ls
    site = sel // Ls
    x = site % Lx
    y = (site // Lx) % Ly
    z = (site // (Lx * Ly)) % Lz
    t = site // (Lx * Ly * Lz)
    coord = [x, y, z, t]
    ext = [Lx, Ly, Lz, Lt]

    def field(cs, sl):   # psi at coordinates cs = (x, y, z, t), slices sl: [n, 4, 3]
        return psi[cs[3], cs[2], cs[1], cs[0], sl]

    hw = (4.0 - M5) * field(coord, s)
    eye = np.eye(4)
    for mu in range(4):
        g = gamma(mu)
        fw = list(coord)
        fw[mu] = (coord[mu] + 1) % ext[mu]
        sf = np.where(coord[mu] == ext[mu] - 1, bc[mu], 1.0)[:, None, None]
        Uf = U[t, z, y, x, mu]                                              # U_mu(x)
        hop = np.einsum("nab,njb->nja", Uf, field(fw, s)) * sf
        hw -= 0.5 * np.einsum("ij,nja->nia", eye - g, hop)
        bw = list(coord)
        bw[mu] = (coord[mu] - 1) % ext[mu]
        sb = np.where(coord[mu] == 0, bc[mu], 1.0)[:, None, None]
        Ub = U[bw[3], bw[2], bw[1], bw[0], mu]                              # U_mu(x - mu)
        hop = np.einsum("nba,njb->nja", Ub.conj(), field(bw, s)) * sb
        hw -= 0.5 * np.einsum("ij,nja->nia", eye + g, hop)
    out = sigma[s][:, None, None] * np.einsum("ij,nja->nia", gamma(4), hw)
    last = s == m
    out[last] += R * np.einsum("ij,nja->nia", gamma(4), field(coord, s)[last])
    lo = s > 0
    out[lo] += c[s[lo] - 1][:, None, None] * field([q[lo] for q in coord], s[lo] - 1)
    hi_ = s < m
    out[hi_] += c[s[hi_]][:, None, None] * field([q[hi_] for q in coord], s[hi_] + 1)
    return out


# ----------------------------------------------------------------------------
# Coarse space (Sec. 4)
# ----------------------------------------------------------------------------

def loss(U, chi, psi, p: Params) -> float:
    """L = Re <chi, H psi> (the scalar whose gradient the force kernel computes)."""
    return float(np.vdot(_c(chi), apply_h(U, psi, p)).real)


def link_grad(U, chi, psi, p: Params) -> np.ndarray:
    """W_mu(x) = dL/dRe U_mu(x) + i dL/dIm U_mu(x) for L = Re <chi, H psi>.

    The paper motivates the solver by its use inside HMC evolution (Sec. 1 and
    Sec. 5), whose fermion force is this gradient.  Written out from the hop
    terms of D (the Shamir form of Sec. 3 used by apply_h): with
    chi' = Gamma5 chi, chi'(x, s) = gamma5 chi(x, Ls-1-s), only the forward hop
    at x and the backward hop at x + mu contain U_mu(x), so

      W_mu(x) = -b/2 b_mu(x) sum_s [ ((1 - g_mu) chi'(x,s)) (x) psi(x+mu,s)^dag
                                   + psi(x,s) (x) ((1 + g_mu) chi'(x+mu,s))^dag ],

    (x) the spin-traced colour outer product, b the Cayley scale of the 4d part
    (p.b), b_mu(x) = bc[mu] on the link that crosses the boundary
    (x_mu = L_mu - 1), else 1.  Plain numpy, 4x4 gammas.
    """
    U, chi, psi = _c(U), _c(chi), _c(psi)
    Lx, Ly, Lz, Lt = p.L
    g5 = gamma(4)
    eye = np.eye(4, dtype=np.complex128)
    chip = np.einsum("ab,tzyxsbc->tzyxsac", g5, chi[:, :, :, :, ::-1, :, :])
    axis = {0: 3, 1: 2, 2: 1, 3: 0}  # mu -> array axis of (t, z, y, x)
    ext = {0: Lx, 1: Ly, 2: Lz, 3: Lt}
    W = np.zeros(U.shape, dtype=np.complex128)
    for mu in range(4):
        gm = gamma(mu)
        psi_f = np.roll(psi, -1, axis=axis[mu])
        chip_f = np.roll(chip, -1, axis=axis[mu])
        a = np.einsum("ab,tzyxsbc->tzyxsac", eye - gm, chip)
        b = np.einsum("ab,tzyxsbc->tzyxsac", eye + gm, chip_f)
        w = np.einsum("tzyxsac,tzyxsad->tzyxcd", a, psi_f.conj()) + \
            np.einsum("tzyxsac,tzyxsad->tzyxcd", psi, b.conj())
        sign = np.ones(ext[mu])
        sign[-1] = p.bc[mu]
        shape = [1, 1, 1, 1]
        shape[axis[mu]] = ext[mu]
        W[:, :, :, :, mu] = -0.5 * p.b * sign.reshape(shape)[..., None, None] * w
    return W


def link_grad_at(U, chi, psi, p: Params, links) -> np.ndarray:
    """link_grad evaluated only at the listed links [(t, z, y, x, mu), ...]
    (lattices too large for the whole-field version): the same sum over s of
    the two spin-traced outer products, taken link by link.  Returns [n, 3, 3]."""
    g5 = gamma(4)
    eye = np.eye(4, dtype=np.complex128)
    out = np.empty((len(links), 3, 3), dtype=np.complex128)
    for n, (t, z, y, x, mu) in enumerate(links):
        c = [x, y, z, t]
        f = list(c)
        f[mu] = (c[mu] + 1) % p.L[mu]
        X, Xf = (t, z, y, x), (f[3], f[2], f[1], f[0])
        gm = gamma(mu)
        chip = np.einsum("ab,sbc->sac", g5, _c(chi[X])[::-1])
        chipf = np.einsum("ab,sbc->sac", g5, _c(chi[Xf])[::-1])
        a = np.einsum("ab,sbc->sac", eye - gm, chip)
        b = np.einsum("ab,sbc->sac", eye + gm, chipf)
        w = np.einsum("sac,sad->cd", a, np.conj(psi[Xf])) + np.einsum("sac,sad->cd", psi[X], np.conj(b))
        sign = p.bc[mu] if c[mu] == p.L[mu] - 1 else 1
        out[n] = -0.5 * p.b * sign * w
    return out


def force(U, W) -> np.ndarray:
    """su(3) force T_mu(x) = P_TA(U_mu(x) W_mu(x)^dag), P_TA(M) = (M - M^dag)/2 - tr(M - M^dag)/6:
    under U -> exp(eps X) U (X traceless anti-Hermitian) dL/deps = Re tr(X T)."""
    M = _c(U) @ np.conj(np.swapaxes(_c(W), -1, -2))
    A = 0.5 * (M - np.conj(np.swapaxes(M, -1, -2)))
    tr = np.trace(A, axis1=-2, axis2=-1) / 3.0
    return A - tr[..., None, None] * np.eye(3)


@dataclass
class Coarse:
    p: Params
    block: tuple          # block extents (x, y, z, t); blocks span all of Ls
    nvec: int

    @property
    def nb(self):
        return 2 * self.nvec

    @property
    def cdims(self):
        return tuple(int(l) // int(b) for l, b in zip(self.p.L, self.block))

    @property
    def nc(self):
        c = self.cdims
        return c[0] * c[1] * c[2] * c[3]

    @property
    def cblock(self):
        return (ctypes.c_int * 4)(*[int(b) for b in self.block])


def block_basis(vecs, cs: Coarse, mode: int = 0):
    """Chirally split, block-orthonormal basis phi^b_k (Sec. 4).

    Returns (basis[Nb, ...fine field...], status); status 4 = rank deficient.
    """
    vecs = _c(np.stack(vecs) if isinstance(vecs, (list, tuple)) else vecs)
    assert vecs.shape[0] == cs.nvec
    basis = np.empty((cs.nb,) + vecs.shape[1:], dtype=np.complex128)
    st = lib().or_block_basis(cs.p.dims, cs.cblock, ctypes.c_int(cs.nvec), ctypes.c_int(mode), _dp(vecs), _dp(basis))
    return basis, int(st)


def restrict(basis, psi, cs: Coarse) -> np.ndarray:
    basis, psi = _c(basis), _c(psi)
    v = np.empty((cs.nc, cs.nb), dtype=np.complex128)
    lib().or_restrict(cs.p.dims, cs.cblock, ctypes.c_int(cs.nb), _dp(basis), _dp(psi), _dp(v))
    return v


def prolong(basis, v, cs: Coarse) -> np.ndarray:
    basis, v = _c(basis), _c(v)
    psi = np.empty(basis.shape[1:], dtype=np.complex128)
    lib().or_prolong(cs.p.dims, cs.cblock, ctypes.c_int(cs.nb), _dp(basis), _dp(v), _dp(psi))
    return psi


def coarse_build(U, basis, cs: Coarse) -> np.ndarray:
    """Little Dirac operator A[a, d, j, k] = <phi^a_j | H^(d) | phi^(a+d)_k> (Sec. 4)."""
    U, basis = _c(U), _c(basis)
    A = np.empty((cs.nc, 9, cs.nb, cs.nb), dtype=np.complex128)
    p = cs.p
    lib().or_coarse_build(p.dims, p.cbc, ctypes.c_double(p.M5), ctypes.c_double(p.mf), ctypes.c_double(p.b), cs.cblock,
                          ctypes.c_int(cs.nb), _dp(U), _dp(basis), _dp(A))
    return A


def coarse_columns(U, basis, cs: Coarse, kcols) -> np.ndarray:
    """Columns k of A: out[c, a, d, j] = A[a, d, j, kcols[c]]."""
    U, basis = _c(U), _c(basis)
    kc = (ctypes.c_int * len(kcols))(*[int(k) for k in kcols])
    out = np.empty((len(kcols), cs.nc, 9, cs.nb), dtype=np.complex128)
    p = cs.p
    lib().or_coarse_columns(p.dims, p.cbc, ctypes.c_double(p.M5), ctypes.c_double(p.mf), ctypes.c_double(p.b), cs.cblock,
                            ctypes.c_int(cs.nb), _dp(U), _dp(basis), ctypes.c_int(len(kcols)), kc, _dp(out))
    return out


def coarse_apply(A, v, cdims) -> np.ndarray:
    """(A v)(a) = sum_d A[a, d] v(a + d), coarse-periodic. v: [nc, nb] or [nrhs, nc, nb]."""
    A, v = _c(A), _c(v)
    nb = A.shape[-1]
    nrhs = 1 if v.ndim == 2 else v.shape[0]
    out = np.empty_like(v)
    cd = (ctypes.c_int * 4)(*[int(c) for c in cdims])
    lib().or_coarse_apply(cd, ctypes.c_int(nb), ctypes.c_int(nrhs), _dp(A), _dp(v), _dp(out))
    return out


def coarse_dense(A, cdims) -> np.ndarray:
    """The coarse operator as a dense (nc*nb) x (nc*nb) matrix (small lattices only)."""
    nc, _, nb, _ = A.shape
    Cx, Cy, Cz, Ct = cdims
    M = np.zeros((nc * nb, nc * nb), dtype=np.complex128)
    for a in range(nc):
        c = [a % Cx, (a // Cx) % Cy, (a // (Cx * Cy)) % Cz, a // (Cx * Cy * Cz)]
        for d in range(9):
            cc = list(c)
            if d > 0:
                mu = (d - 1) % 4
                cc[mu] = (cc[mu] + (1 if d <= 4 else -1)) % cdims[mu]
            b = ((cc[3] * Cz + cc[2]) * Cy + cc[1]) * Cx + cc[0]
            M[a * nb:(a + 1) * nb, b * nb:(b + 1) * nb] += A[a, d]
    return M


# ----------------------------------------------------------------------------
# Krylov solvers and polynomials
# ----------------------------------------------------------------------------

def vdot(a, b) -> complex:
    """<a, b> = sum conj(a) b."""
    return complex(np.vdot(a.ravel(), b.ravel()))


def norm(a) -> float:
    return float(np.sqrt(np.vdot(a.ravel(), a.ravel()).real))


@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    status: int               # 0 converged, 1 not converged, 2 breakdown
    history: list = field(default_factory=list)   # |r| after each iteration (updated residual)
    applies: int = 0
    true_rel: float = float("nan")


def cr(apply, b, tol=1e-8, maxiter=10000, x0=None, breakdown_tol=1e-13, check_true=True) -> SolveResult:
    """Conjugate residual for a Hermitian (indefinite) operator (Sec. 3).

    r = b - H x;  p = r;  Ar = H r;  Ap = Ar
    repeat:  alpha = Re<r,Ar>/|Ap|^2;  x += alpha p;  r -= alpha Ap
             Ar = H r;  beta = Re<r',Ar'>/Re<r,Ar>;  p = r + beta p;  Ap = Ar + beta Ap
    Stops when the updated |r| <= tol |b|; the true residual is then recomputed and
    the iteration restarted from it if it is not met.  Status 2 on breakdown
    (|<r,Ar>| below rounding level), 1 if maxiter is reached.
    """
    bn = norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    napp = 0
    if x0 is None:
        r = b.copy()
    else:
        r = b - apply(x)
        napp += 1
    hist = []
    if bn == 0.0:
        return SolveResult(x, 0, 0, hist, napp, 0.0)
    it = 0
    status = 1
    while it < maxiter:
        Ar = apply(r)
        napp += 1
        p = r.copy()
        Ap = Ar.copy()
        rAr = vdot(r, Ar).real
        restart = False
        while it < maxiter:
            if abs(rAr) < breakdown_tol * norm(r) * norm(Ar):
                return SolveResult(x, it, 2, hist, napp, norm(b - apply(x)) / bn)
            alpha = rAr / vdot(Ap, Ap).real
            x += alpha * p
            r -= alpha * Ap
            it += 1
            rn = norm(r)
            hist.append(rn)
            if rn <= tol * bn:
                if not check_true:
                    return SolveResult(x, it, 0, hist, napp, float("nan"))
                r = b - apply(x)
                napp += 1
                if norm(r) <= tol * bn:
                    return SolveResult(x, it, 0, hist, napp, norm(r) / bn)
                restart = True
                break
            Ar = apply(r)
            napp += 1
            rAr_new = vdot(r, Ar).real
            beta = rAr_new / rAr
            rAr = rAr_new
            p = r + beta * p
            Ap = Ar + beta * Ap
        if not restart:
            break
    r = b - apply(x)
    return SolveResult(x, it, status, hist, napp + 1, norm(r) / bn)


def cheby_coeffs(n: int, lo: float, hi: float, f=lambda y: 1.0 / y) -> np.ndarray:
    """Chebyshev interpolation coefficients of f on [lo, hi] with n terms (Sec. 4 smoother).

    c_j = (2/n) sum_{k<n} f(y_k) cos(pi j (k+1/2)/n),
    y_k = (hi+lo)/2 + (hi-lo)/2 cos(pi (k+1/2)/n);
    p(y) = sum_{j<n} c_j T_j(yhat) - c_0/2 with yhat = (2y - hi - lo)/(hi - lo).
    "Order 10" is read as n = 10 terms (degree 9).
    """
    k = np.arange(n)
    th = np.pi * (k + 0.5) / n
    yk = 0.5 * (hi + lo) + 0.5 * (hi - lo) * np.cos(th)
    fk = np.array([f(y) for y in yk])
    return np.array([2.0 / n * np.sum(fk * np.cos(j * th)) for j in range(n)])


def cheby_eval(c, lo, hi, y):
    """p(y) = sum c_j T_j(yhat) - c_0/2 (scalar or array y)."""
    yh = (2.0 * np.asarray(y, dtype=float) - hi - lo) / (hi - lo)
    t0 = np.ones_like(yh)
    t1 = yh
    out = c[0] * t0 - 0.5 * c[0]
    if len(c) > 1:
        out = out + c[1] * t1
    for j in range(2, len(c)):
        t0, t1 = t1, 2 * yh * t1 - t0
        out = out + c[j] * t1
    return out


def smoother(apply, r, order=10, lo=1.0, hi=64.0):
    """S r = p(H^2) H r with p the Chebyshev interpolant of 1/y on [lo, hi] (Sec. 4).

    p(H^2) is evaluated by the three-term recurrence T_{j+1} = 2 yhat T_j - T_{j-1}
    with yhat = (2 H^2 - hi - lo)/(hi - lo); 1 + 2 (order - 1) H applications.
    """
    c = cheby_coeffs(order, lo, hi)

    def yhat(v):
        return (2.0 * apply(apply(v)) - (hi + lo) * v) / (hi - lo)

    u = apply(r)
    t0 = u
    out = 0.5 * c[0] * t0
    if order > 1:
        t1 = yhat(u)
        out = out + c[1] * t1
        for j in range(2, order):
            t2 = 2.0 * yhat(t1) - t0
            out = out + c[j] * t2
            t0, t1 = t1, t2
    return out


def cheby_filter(apply, eta, degree: int, lo: float, hi: float, normalise=True):
    """Chebyshev low-pass filter T_d(yhat) eta, yhat = (2 H^2 - hi - lo)/(hi - lo) (Sec. 4).

    [lo, hi] = [lambda_cut^2, lambda_max^2]: modes with H^2 inside the interval
    are bounded by 1, modes below lambda_cut^2 grow like cosh(d acosh|yhat|).
    The result is normalised to unit norm.
    """
    def yhat(v):
        return (2.0 * apply(apply(v)) - (hi + lo) * v) / (hi - lo)

    t0 = eta.copy()
    if degree == 0:
        out = t0
    else:
        t1 = yhat(t0)
        for _ in range(2, degree + 1):
            t0, t1 = t1, 2.0 * yhat(t1) - t0
        out = t1
    if normalise:
        out = out / norm(out)
    return out


def power_max(apply, v0, iters=30):
    """Rayleigh-quotient estimate of the largest eigenvalue of H^2 by power iteration."""
    v = v0 / norm(v0)
    lam = 0.0
    for _ in range(iters):
        w = apply(apply(v))
        lam = vdot(v, w).real
        v = w / norm(w)
    return lam


def coarse_cr(A, v, cdims, tol=1e-2, maxiter=500, defl=None):
    """Coarse solve A c = v by CR from c = 0 (Sec. 4: the subspace inverse by a Krylov method),
    or, with a deflation space ``defl`` (``coarse_deflation``), from the Galerkin start
    c0 = V diag(1/theta) V^dag v, which removes the deflated eigenmodes from the residual.

    tol = 0 runs exactly maxiter iterations (fixed-work mode used for parity).
    """
    x0 = None
    if defl is not None:
        theta, V = defl[0], defl[1]
        x0 = np.zeros_like(v)
        for th, vi in zip(theta, V):
            x0 = x0 + (vdot(vi, v) / th) * vi
    return cr(lambda u: coarse_apply(A, u, cdims), v, tol=tol, maxiter=maxiter, x0=x0, check_true=False)


DEFL_RES_TOL = 1e-2  # largest residual |A y - theta y| / |theta| of a deflated eigenpair (|y| = 1)


def coarse_deflation(A, cdims, V0, k, degree=40, iters=4, cut=0.05, power_iters=30):
    """Low eigenpairs of the little Dirac operator A for deflating the coarse solve (Sec. 5
    names coarse-space eigenvector deflation as the open option for the coarse cost).

    Chebyshev-filtered subspace iteration in A^2 on the start block V0 (m >= k vectors).
    Each pass applies the filter of ``cheby_filter`` on [lo, hi] to every vector, makes the
    block orthonormal (Gram-Schmidt in index order, twice) and rotates it to the Ritz vectors
    of A^2 (eig of (AV)^dag (AV)).  hi = 1.1 lambda_max^2 from ``power_max``; the first pass
    uses lo = cut * hi, later ones lo = the largest Ritz value of A^2 in the block, which
    bounds the part of the spectrum the block does not hold (A^2 is positive definite, so its
    Ritz values never fall below its spectrum, unlike those of the indefinite A).  A final
    Rayleigh-Ritz on A (theta, Y = eig(V^dag A V)) gives the pairs.  A pair counts as found when
    its residual |A y - theta y| (|y| = 1) is at most DEFL_RES_TOL |theta|: a block that is not yet
    an invariant subspace of A can mix eigenvectors of A of opposite sign into a Ritz vector whose
    Rayleigh quotient lies anywhere between them, near zero included, and deflating such a pair
    would divide by that spurious value.  The k found pairs of smallest |theta| (fewer if fewer
    were found) are returned as (theta, V, W = A V).
    """
    apply = lambda u: coarse_apply(A, u, cdims)
    hi = 1.1 * power_max(apply, V0[0], power_iters)
    lo = cut * hi
    V = [np.array(v, dtype=np.complex128) for v in V0]
    m = len(V)
    for _ in range(iters):
        V = [cheby_filter(apply, v, degree, lo, hi, normalise=True) for v in V]
        for i in range(m):
            for _ in range(2):
                for j in range(i):
                    V[i] = V[i] - vdot(V[j], V[i]) * V[j]
            V[i] = V[i] / norm(V[i])
        W = [apply(v) for v in V]
        G2 = np.array([[vdot(W[i], W[j]) for j in range(m)] for i in range(m)])
        mu, Y = np.linalg.eigh(0.5 * (G2 + G2.conj().T))
        V = [sum(Y[i, q] * V[i] for i in range(m)) for q in range(m)]
        lo = min(float(mu.max()), 0.99 * hi)
    W = [apply(v) for v in V]
    G = np.array([[vdot(V[i], W[j]) for j in range(m)] for i in range(m)])
    theta, Y = np.linalg.eigh(0.5 * (G + G.conj().T))
    Vy = [sum(Y[i, q] * V[i] for i in range(m)) for q in range(m)]
    Wy = [sum(Y[i, q] * W[i] for i in range(m)) for q in range(m)]
    found = [q for q in range(m) if norm(Wy[q] - theta[q] * Vy[q]) <= DEFL_RES_TOL * abs(theta[q])]
    order = sorted(found, key=lambda q: abs(theta[q]))[:k]
    return theta[order], [Vy[q] for q in order], [Wy[q] for q in order]


def vcycle(apply, A, basis, cs: Coarse, r, order=10, lo=1.0, hi=64.0, ctol=1e-2, cmaxiter=500,
           coarse_solve=None, defl=None):
    """Two-level cycle B r (Sec. 4, the M_outer display), symmetric form:

    e1 = S r;  e2 = e1 + Q (r - H e1);  e3 = e2 + S (r - H e2),  Q = P A^-1 P^dag.
    Expanding gives S P_L + P_R S + Q - S P_L H S with P_L = 1 - HQ, P_R = 1 - QH.
    The coarse inverse is CR on A (``coarse_cr``, deflated when ``defl`` is given) unless
    ``coarse_solve(v, cdims)`` is given (the tests pass an exact dense solve there).
    """
    e1 = smoother(apply, r, order, lo, hi)
    t = r - apply(e1)
    vc = restrict(basis, t, cs)
    if coarse_solve is None:
        c = coarse_cr(A, vc, cs.cdims, tol=ctol, maxiter=cmaxiter, defl=defl).x
    else:
        c = coarse_solve(vc, cs.cdims)
    e2 = e1 + prolong(basis, c, cs)
    t = r - apply(e2)
    return e2 + smoother(apply, t, order, lo, hi)


def fgcr(apply, precond, b, tol=1e-8, maxiter=200, restart=8, x0=None) -> SolveResult:
    """Flexible (variable-preconditioned) GCR (Sec. 4, outer iteration).

    For i < restart:  z = B r;  w = H z;  orthogonalise w against the stored w_j by
    modified Gram-Schmidt, applying the same combination to z;  normalise;
    alpha = <w, r>;  x += alpha z;  r -= alpha w.  The true residual is recomputed
    at every restart.
    """
    bn = norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply(x) if x0 is not None else b.copy()
    hist = []
    it = 0
    while it < maxiter:
        Z, W = [], []
        for _ in range(restart):
            z = precond(r)
            w = apply(z)
            for zj, wj in zip(Z, W):
                beta = vdot(wj, w)
                w = w - beta * wj
                z = z - beta * zj
            nw = norm(w)
            w = w / nw
            z = z / nw
            alpha = vdot(w, r)
            x = x + alpha * z
            r = r - alpha * w
            Z.append(z)
            W.append(w)
            it += 1
            hist.append(norm(r))
            if hist[-1] <= tol * bn or it >= maxiter:
                break
        r = b - apply(x)
        if norm(r) <= tol * bn:
            return SolveResult(x, it, 0, hist, 0, norm(r) / bn)
    return SolveResult(x, it, 1, hist, 0, norm(b - apply(x)) / bn)
