"""Seeded synthetic inputs shared by the oracle, the GPU tests and the benchmark.

This module draws random numbers and nothing else: it holds none of the
solver's arithmetic (no Dirac operator, no projection, no Krylov step), so
that the CPU oracle and the HIP path can both be fed from it without sharing
any code that computes the method.

Every array is returned in the canonical site-major ("AoS") layout:

* fermion field ``psi[t, z, y, x, s, spin, colour]`` (complex128),
* gauge field   ``U[t, z, y, x, mu, row, col]`` (complex128), mu = x, y, z, t.

The paper's ensemble (a dynamical 2+1 flavour domain wall ensemble,
Sec. 5) is not available; these draws stand in for it:

* links U_mu(x) = exp(i * eps * A) with A = sum_a w_a lambda_a / 2 a random
  Hermitian traceless Gaussian su(3) element (w_a ~ N(0, 1), lambda_a the
  Gell-Mann matrices), eps = 0.3, drawn in (t, z, y, x, mu) order;
* fermion sources: complex Gaussian, real and imaginary parts each N(0, 1),
  drawn in (t, z, y, x, s, spin, colour) order.
"""
from __future__ import annotations

import numpy as np

# Seeds used throughout (links, gauge transformation, source, subspace noise).
LINK_SEED = 1
TRANSFORM_SEED = 2
SOURCE_SEED = 0
SUBSPACE_SEED0 = 100


def _gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    g = np.zeros((8, 3, 3), dtype=np.complex128)
    g[0][0, 1] = g[0][1, 0] = 1
    g[1][0, 1] = -1j
    g[1][1, 0] = 1j
    g[2][0, 0] = 1
    g[2][1, 1] = -1
    g[3][0, 2] = g[3][2, 0] = 1
    g[4][0, 2] = -1j
    g[4][2, 0] = 1j
    g[5][1, 2] = g[5][2, 1] = 1
    g[6][1, 2] = -1j
    g[6][2, 1] = 1j
    g[7][0, 0] = g[7][1, 1] = 1 / np.sqrt(3)
    g[7][2, 2] = -2 / np.sqrt(3)
    return g


def _exp_i_hermitian(a: np.ndarray, eps: float) -> np.ndarray:
    """exp(i * eps * a) for a stack of Hermitian 3x3 matrices, via eigh."""
    w, v = np.linalg.eigh(a)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", v, ph, v.conj())


def random_su3(shape: tuple, rng: np.random.Generator, eps: float) -> np.ndarray:
    """Random SU(3) matrices exp(i*eps*sum_a w_a lambda_a/2), w_a ~ N(0,1)."""
    w = rng.standard_normal(size=tuple(shape) + (8,))
    a = np.einsum("...a,aij->...ij", w, _gell_mann() * 0.5)
    return _exp_i_hermitian(a, eps)


def gauge_field(L, seed: int = LINK_SEED, eps: float = 0.3) -> np.ndarray:
    """Gauge field U[t,z,y,x,mu,3,3]; L = (Lx, Ly, Lz, Lt).

    eps = 0 gives the free field (unit links).
    """
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    if eps == 0.0:
        u = np.zeros((Lt, Lz, Ly, Lx, 4, 3, 3), dtype=np.complex128)
        u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
        return u
    rng = np.random.default_rng(seed)
    return random_su3((Lt, Lz, Ly, Lx, 4), rng, eps)


def gauge_transform(L, seed: int = TRANSFORM_SEED, eps: float = 2.0) -> np.ndarray:
    """A random SU(3) field V[t,z,y,x,3,3] (for gauge-covariance checks)."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    rng = np.random.default_rng(seed)
    return random_su3((Lt, Lz, Ly, Lx), rng, eps)


def gaussian_fermion(L, Ls: int, seed: int = SOURCE_SEED, nrhs: int | None = None) -> np.ndarray:
    """Complex Gaussian fermion field psi[t,z,y,x,s,spin,col] (re, im ~ N(0,1)).

    With ``nrhs`` set, returns a stack of that many independent fields drawn
    one after another from the same stream.
    """
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    shape = (Lt, Lz, Ly, Lx, int(Ls), 4, 3)
    if nrhs is not None:
        shape = (int(nrhs),) + shape
    rng = np.random.default_rng(seed)
    ri = rng.standard_normal(size=shape + (2,))
    return ri[..., 0] + 1j * ri[..., 1]


def subspace_noise(L, Ls: int, nvec: int, seed0: int = SUBSPACE_SEED0) -> list:
    """Gaussian noise vectors eta_k, k < nvec, each from seed ``seed0 + k``."""
    return [gaussian_fermion(L, Ls, seed=seed0 + k) for k in range(nvec)]


def gaussian_coarse(nc: int, nb: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Complex Gaussian coarse vector(s) v[(rhs,) site_c, k]."""
    shape = (int(nc), int(nb)) if nrhs is None else (int(nrhs), int(nc), int(nb))
    rng = np.random.default_rng(seed)
    ri = rng.standard_normal(size=shape + (2,))
    return ri[..., 0] + 1j * ri[..., 1]


def plaquette(U: np.ndarray) -> float:
    """Average plaquette Re tr(U_mu U_nu U_mu^dag U_nu^dag)/3 (a record of the ensemble)."""
    axis = {0: 3, 1: 2, 2: 1, 3: 0}  # mu -> array axis of (t, z, y, x)
    tot = 0.0
    n = 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            umu = U[..., mu, :, :]
            unu = U[..., nu, :, :]
            unu_xpmu = np.roll(unu, -1, axis=axis[mu])
            umu_xpnu = np.roll(umu, -1, axis=axis[nu])
            p = umu @ unu_xpmu @ np.conj(np.swapaxes(umu_xpnu, -1, -2)) @ np.conj(np.swapaxes(unu, -1, -2))
            tot += np.real(np.trace(p, axis1=-2, axis2=-1)).mean() / 3.0
            n += 1
    return tot / n


def gaussian_fermion_device(L, Ls: int, seed: int, device="cuda:0"):
    """Complex Gaussian fermion field drawn on the device with torch's seeded
    generator (re, im ~ N(0, 1)), for large subspace-noise draws that would be
    slow on the host.  Returned in the device layout [12, V4, Ls]."""
    import torch
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    V4 = Lx * Ly * Lz * Lt
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    ri = torch.randn((12, V4, int(Ls), 2), dtype=torch.float64, device=device, generator=g)
    return torch.view_as_complex(ri)
