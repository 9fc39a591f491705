"""Independent dense constructions used to pin the oracle (tests only).

These build the domain wall operator as an explicit matrix from shift
operators and Kronecker products, and the free-field operator in momentum
space. They are written separately from the oracle's site loops so that a
mistake in either shows up as a mismatch.

Index order of a fine field (matches the canonical layout):
    ((site4 * Ls + s) * 4 + spin) * 3 + colour,  site4 = ((t*Lz + z)*Ly + y)*Lx + x.
"""
from __future__ import annotations

import itertools

import numpy as np


def pauli():
    return [np.array([[0, 1], [1, 0]], dtype=complex),
            np.array([[0, -1j], [1j, 0]], dtype=complex),
            np.array([[1, 0], [0, -1]], dtype=complex)]


def chiral_gammas():
    """gamma_k = [[0, -i s_k], [i s_k, 0]] (k = x, y, z), gamma_t = [[0, 1], [1, 0]]."""
    z = np.zeros((2, 2), dtype=complex)
    one = np.eye(2, dtype=complex)
    g = [np.block([[z, -1j * s], [1j * s, z]]) for s in pauli()]
    g.append(np.block([[z, one], [one, z]]))
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    return g, g5


def site_index(x, L):
    Lx, Ly, Lz, Lt = L
    return ((x[3] * Lz + x[2]) * Ly + x[1]) * Lx + x[0]


def dense_dwf(U, L, Ls, M5, mf, bc):
    """Dense D_dwf (Shamir form) from shift operators; U in the canonical layout."""
    g, g5 = chiral_gammas()
    V = L[0] * L[1] * L[2] * L[3]
    n = V * Ls * 12
    D = np.zeros((n, n), dtype=complex)
    Is = np.eye(Ls)
    Pp = 0.5 * (np.eye(4) + g5)
    Pm = 0.5 * (np.eye(4) - g5)
    # U is indexed [t, z, y, x, mu]
    Uf = U.reshape(V, 4, 3, 3)
    for x in itertools.product(*[range(l) for l in L]):
        i = site_index(x, L)
        sl_i = slice(i * Ls * 12, (i + 1) * Ls * 12)
        D[sl_i, sl_i] += (5.0 - M5) * np.eye(Ls * 12)
        for mu in range(4):
            xp = list(x)
            xp[mu] = (x[mu] + 1) % L[mu]
            sp = bc[mu] if x[mu] == L[mu] - 1 else 1.0
            j = site_index(xp, L)
            blk = np.kron(Is, np.kron(np.eye(4) - g[mu], Uf[i, mu]))
            D[sl_i, j * Ls * 12:(j + 1) * Ls * 12] += -0.5 * sp * blk
            xm = list(x)
            xm[mu] = (x[mu] - 1) % L[mu]
            sm = bc[mu] if x[mu] == 0 else 1.0
            j = site_index(xm, L)
            blk = np.kron(Is, np.kron(np.eye(4) + g[mu], Uf[j, mu].conj().T))
            D[sl_i, j * Ls * 12:(j + 1) * Ls * 12] += -0.5 * sm * blk
        # fifth dimension
        D5 = np.zeros((Ls * 4, Ls * 4), dtype=complex)
        for s in range(Ls):
            if s + 1 < Ls:
                D5[s * 4:(s + 1) * 4, (s + 1) * 4:(s + 2) * 4] += -Pm
            else:
                D5[s * 4:(s + 1) * 4, 0:4] += mf * Pm
            if s >= 1:
                D5[s * 4:(s + 1) * 4, (s - 1) * 4:s * 4] += -Pp
            else:
                D5[s * 4:(s + 1) * 4, (Ls - 1) * 4:Ls * 4] += mf * Pp
        D[sl_i, sl_i] += np.kron(D5, np.eye(3))
    return D


def dense_gamma5R5(L, Ls):
    """Gamma5 = gamma5 R5 as a dense matrix."""
    _, g5 = chiral_gammas()
    V = L[0] * L[1] * L[2] * L[3]
    R5 = np.eye(Ls)[::-1]
    return np.kron(np.eye(V), np.kron(R5, np.kron(g5, np.eye(3))))


def free_h_momentum(p, Ls, M5, mf, b=1.0):
    """Free-field H(p) = gamma5 R5 [b D_W(p) x 1_s + D_5] on (s, spin), 4Ls x 4Ls
    (Cayley form with c = 0; b = 1 is the Shamir kernel).

    D_W(p) = (4 - M5 - sum cos p) + i sum gamma_mu sin p_mu.
    """
    g, g5 = chiral_gammas()
    dw = b * ((4.0 - M5 - sum(np.cos(p))) * np.eye(4) + 1j * sum(g[mu] * np.sin(p[mu]) for mu in range(4)))
    Pp = 0.5 * (np.eye(4) + g5)
    Pm = 0.5 * (np.eye(4) - g5)
    D = np.kron(np.eye(Ls), dw) + np.kron(np.eye(Ls), np.eye(4))
    for s in range(Ls):
        if s + 1 < Ls:
            D[s * 4:(s + 1) * 4, (s + 1) * 4:(s + 2) * 4] += -Pm
        else:
            D[s * 4:(s + 1) * 4, 0:4] += mf * Pm
        if s >= 1:
            D[s * 4:(s + 1) * 4, (s - 1) * 4:s * 4] += -Pp
        else:
            D[s * 4:(s + 1) * 4, (Ls - 1) * 4:Ls * 4] += mf * Pp
    G5 = np.kron(np.eye(Ls)[::-1], g5)
    return G5 @ D


def momenta(L, bc):
    """Allowed lattice momenta: 2 pi n / L (periodic) or 2 pi (n + 1/2) / L (antiperiodic)."""
    axes = []
    for l, b in zip(L, bc):
        shift = 0.5 if b < 0 else 0.0
        axes.append([2 * np.pi * (n + shift) / l for n in range(l)])
    return [np.array(p) for p in itertools.product(*axes)]


def free_spectrum(L, Ls, M5, mf, bc, b=1.0):
    """Union over momenta of eig(H(p)), each with colour multiplicity 3."""
    ev = []
    for p in momenta(L, bc):
        e = np.linalg.eigvalsh(free_h_momentum(p, Ls, M5, mf, b))
        ev.extend(list(e) * 3)
    return np.sort(np.array(ev))


def plane_wave(L, Ls, p, chi, colour):
    """Field e^{i p.x} chi(s, spin) delta(colour) in the canonical layout."""
    Lx, Ly, Lz, Lt = L
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    f = np.zeros((Lt, Lz, Ly, Lx, Ls, 4, 3), dtype=complex)
    f[..., colour] = ph[..., None, None] * chi.reshape(Ls, 4)[None, None, None, None]
    return f


def dense_from_apply(apply, shape):
    """Dense matrix of a linear map on fields of the given shape (column by column)."""
    n = int(np.prod(shape))
    M = np.zeros((n, n), dtype=complex)
    e = np.zeros(n, dtype=complex)
    for i in range(n):
        e[:] = 0
        e[i] = 1
        M[:, i] = apply(e.reshape(shape)).ravel()
    return M


def dense_wilson(U, L, M5, bc):
    """Dense 4d D_W(-M5) = (4 - M5) - 1/2 sum_mu [(1 - g) U delta_{x+mu} + (1 + g) U^dag delta_{x-mu}]
    from shift operators, on (site4, spin, colour)."""
    g, _ = chiral_gammas()
    V = L[0] * L[1] * L[2] * L[3]
    D = (4.0 - M5) * np.eye(V * 12, dtype=complex)
    Uf = U.reshape(V, 4, 3, 3)
    for x in itertools.product(*[range(l) for l in L]):
        i = site_index(x, L)
        for mu in range(4):
            xp = list(x)
            xp[mu] = (x[mu] + 1) % L[mu]
            sp = bc[mu] if x[mu] == L[mu] - 1 else 1.0
            j = site_index(xp, L)
            D[i * 12:(i + 1) * 12, j * 12:(j + 1) * 12] += -0.5 * sp * np.kron(np.eye(4) - g[mu], Uf[i, mu])
            xm = list(x)
            xm[mu] = (x[mu] - 1) % L[mu]
            sm = bc[mu] if x[mu] == 0 else 1.0
            j = site_index(xm, L)
            D[i * 12:(i + 1) * 12, j * 12:(j + 1) * 12] += -0.5 * sm * np.kron(np.eye(4) + g[mu], Uf[j, mu].conj().T)
    return D


def dense_cf(U, L, M5, bc, beta, R):
    """The continued-fraction matrix of Sec. 3 as a dense matrix on (site4, s, spin, colour):
    tridiagonal in s with H_W, -H_W, H_W, ... on the first m = len(beta) diagonal blocks,
    R gamma5 + beta_0 H_W on the last, 1/sqrt(beta_i beta_(i+1)) between slices i and i + 1 < m and
    1/sqrt(beta_(m-1)) between slices m - 1 and m."""
    _, g5 = chiral_gammas()
    V = L[0] * L[1] * L[2] * L[3]
    m = len(beta)
    Ls = m + 1
    HW = np.kron(np.eye(V), np.kron(g5, np.eye(3))) @ dense_wilson(U, L, M5, bc)
    T = np.zeros((Ls, Ls))
    for i in range(m - 1):
        T[i, i + 1] = T[i + 1, i] = 1.0 / np.sqrt(beta[i] * beta[i + 1])
    T[m - 1, m] = T[m, m - 1] = 1.0 / np.sqrt(beta[m - 1])
    sig = np.diag([(-1.0) ** i for i in range(m)] + [beta[0]])
    last = np.zeros((Ls, Ls))
    last[m, m] = 1.0
    # order (site4, s, spin*3 + colour): site-major blocks of Ls * 12
    P = np.zeros((V * Ls * 12, V * Ls * 12))
    for v in range(V):
        for s in range(Ls):
            for a in range(12):
                P[(v * Ls + s) * 12 + a, (s * V + v) * 12 + a] = 1.0   # from (s, site4, a) order
    A_s = np.kron(sig, HW) + np.kron(T, np.eye(V * 12)) + R * np.kron(last, np.kron(np.eye(V), np.kron(g5, np.eye(3))))
    return P @ A_s @ P.T


def free_cf_momentum(p, M5, beta, R):
    """Free-field continued-fraction matrix at momentum p on (s, spin): 4 Ls x 4 Ls, with
    H_W(p) = gamma5 [(4 - M5 - sum cos p) + i sum gamma_mu sin p_mu]."""
    g, g5 = chiral_gammas()
    hw = g5 @ ((4.0 - M5 - sum(np.cos(p))) * np.eye(4) + 1j * sum(g[mu] * np.sin(p[mu]) for mu in range(4)))
    m = len(beta)
    Ls = m + 1
    A = np.zeros((4 * Ls, 4 * Ls), dtype=complex)
    for i in range(m):
        A[4 * i:4 * i + 4, 4 * i:4 * i + 4] = (-1.0) ** i * hw
    A[4 * m:, 4 * m:] = R * g5 + beta[0] * hw
    for i in range(m):
        c = 1.0 / np.sqrt(beta[i] * beta[i + 1]) if i < m - 1 else 1.0 / np.sqrt(beta[m - 1])
        A[4 * i:4 * i + 4, 4 * (i + 1):4 * (i + 2)] += c * np.eye(4)
        A[4 * (i + 1):4 * (i + 2), 4 * i:4 * i + 4] += c * np.eye(4)
    return A
