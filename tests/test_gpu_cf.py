"""GPU parity of the continued-fraction overlap operator (Sec. 3, the continued-fraction
matrix) against the FP64 oracle through the C-ABI: element by element at 1e-10 (FP64) and 1e-5
(FP32) over pole counts 1 to 63 (Ls = 2 to 64, so workgroups of 16 whole sites and of 256 / Ls
sites), odd and extent-1 lattices, both boundary conditions; sampled sites at 24^4, the
benchmark's lattice; Hermiticity at 16^4; argument checks before any launch.  Even extents
with Ls <= 16 take the parity-tile kernels (paired slices in FP32 with even Ls), the rest the
one-site-per-work-item kernel; every path is compared."""
import numpy as np
import pytest

import hdcr_inputs as hi
import oracle
import paper_1611_06944_amd as hd
from tests.gpu_util import log, max_rel_elem, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu


def _beta(m, seed):
    rng = np.random.default_rng(seed)
    return list(0.2 + 2.0 * rng.random(m))   # any positive values define the matrix


CASES = [
    # L, m (pole slices), bc, M5, R
    ((4, 4, 4, 4), 1, (1, 1, 1, -1), 1.8, 0.3),
    ((4, 4, 4, 4), 4, (1, 1, 1, -1), 1.8, -0.7),     # the printed four-pole matrix
    ((3, 5, 2, 3), 8, (-1, 1, -1, 1), 1.4, 0.05),    # odd extents; Ls = 9
    ((2, 1, 4, 2), 15, (1, 1, 1, -1), 1.0, 1.3),     # extent 1; Ls = 16
    ((4, 2, 2, 4), 16, (1, -1, 1, -1), 1.8, 0.2),    # Ls = 17: 15 sites per workgroup
    ((2, 2, 2, 4), 63, (1, 1, 1, -1), 1.6, 0.4),     # Ls = 64: 4 sites per workgroup
]


@pytest.mark.parametrize("L,m,bc,M5,R", CASES)
def test_cf_parity(L, m, bc, M5, R):
    torch = torch_dev()
    Ls = m + 1
    log(f"continued fraction L={L} m={m} bc={bc}")
    beta = _beta(m, seed=m)
    U = hi.gauge_field(L, seed=3)
    x = hi.gaussian_fermion(L, Ls, seed=4)
    ref = oracle.apply_cf(U, x, M5, beta, R, bc)
    lat = hd.Lattice(L, Ls, M5=M5, bc=bc)
    for dt, tol in ((torch.complex128, 1e-10), (torch.complex64, 1e-5)):
        out = hd.apply_cf(lat, to_dev(hd.pack_gauge(U), dt), to_dev(hd.pack_fermion(x), dt), beta, R)
        got = hd.unpack_fermion(to_host(out), L, Ls)
        assert max_rel_elem(got, ref) <= tol, dt


@pytest.mark.parametrize("L,m", [((2, 2, 2, 2), 1), ((4, 4, 2, 6), 7), ((4, 2, 6, 4), 15), ((2, 4, 4, 2), 10)])
def test_cf_kernel_paths(L, m):
    """Even extents with Ls <= 16 run on parity tiles: paired slices in FP32 with even Ls
    (the default), one slice per work-item (tune variant 4, and FP64), and the one-site-per-
    work-item kernel (tune variant 2); every path against the oracle at 1e-10 / 1e-5."""
    torch = torch_dev()
    Ls, bc, M5, R = m + 1, (1, -1, 1, -1), 1.7, 0.35
    log(f"continued fraction kernel paths L={L} m={m}")
    beta = _beta(m, seed=50 + m)
    U = hi.gauge_field(L, seed=8)
    x = hi.gaussian_fermion(L, Ls, seed=9)
    ref = oracle.apply_cf(U, x, M5, beta, R, bc)
    for variant in (0, 4, 2):
        lat = hd.Lattice(L, Ls, M5=M5, bc=bc).with_tune(dslash_variant=variant)
        for dt, tol in ((torch.complex128, 1e-10), (torch.complex64, 1e-5)):
            out = hd.apply_cf(lat, to_dev(hd.pack_gauge(U), dt), to_dev(hd.pack_fermion(x), dt), beta, R)
            got = hd.unpack_fermion(to_host(out), L, Ls)
            assert max_rel_elem(got, ref) <= tol, (variant, dt)


def test_cf_parity_12x12x12x12():
    """A lattice of many workgroups (20736 4d sites, Ls = 9), FP64 and FP32, every element."""
    torch = torch_dev()
    L, m, bc, M5, R = (12, 12, 12, 12), 8, (1, 1, 1, -1), 1.8, 0.4
    log(f"continued fraction L={L} m={m}")
    beta = _beta(m, seed=21)
    U = hi.gauge_field(L, seed=5)
    x = hi.gaussian_fermion(L, m + 1, seed=6)
    ref = oracle.apply_cf(U, x, M5, beta, R, bc)
    lat = hd.Lattice(L, m + 1, M5=M5, bc=bc)
    for dt, tol in ((torch.complex128, 1e-10), (torch.complex64, 1e-5)):
        out = hd.apply_cf(lat, to_dev(hd.pack_gauge(U), dt), to_dev(hd.pack_fermion(x), dt), beta, R)
        assert max_rel_elem(hd.unpack_fermion(to_host(out), L, m + 1), ref) <= tol, dt


@pytest.mark.parametrize("m", [8, 15])
def test_cf_parity_full_size_sampled(m):
    """24^4 with 8 and 15 pole slices (the benchmark's shapes: workgroups of 16 and of 16 / Ls
    sites), FP64 and FP32, on 3000 sampled output sites plus the lattice corners (every
    boundary crossing, first and last slice) against the oracle's per-site form."""
    torch = torch_dev()
    L, bc, M5, R = (24, 24, 24, 24), (1, 1, 1, -1), 1.8, 0.3
    Ls = m + 1
    log(f"continued fraction sampled L={L} m={m}")
    beta = _beta(m, seed=30 + m)
    U = hi.gauge_field(L, seed=1)
    x = hi.gaussian_fermion(L, Ls, seed=2)
    lat = hd.Lattice(L, Ls, M5=M5, bc=bc)
    N5 = lat.N5
    rng = np.random.default_rng(9)
    sel = np.unique(np.concatenate([rng.integers(0, N5, 3000), [0, Ls - 1, N5 - 1, N5 - Ls]]))
    ref = oracle.apply_cf_sites(U, x, M5, beta, R, sel, bc)
    for dt, tol in ((torch.complex128, 1e-10), (torch.complex64, 1e-5)):
        out = hd.apply_cf(lat, to_dev(hd.pack_gauge(U), dt), to_dev(hd.pack_fermion(x), dt), beta, R)
        o = to_host(out)                                   # [12, V4, Ls]
        got = o[:, sel // Ls, sel % Ls].T.reshape(-1, 4, 3)
        assert max_rel_elem(got, ref) <= tol, dt
        del out
        torch.cuda.empty_cache()


def test_cf_hermitian_on_device():
    """<x, A y> = <A x, y> at 16^4 with Ls = 13, in FP64 on the device (vec_dot)."""
    torch = torch_dev()
    L, m = (16, 16, 16, 16), 12
    log(f"continued fraction Hermiticity L={L} m={m}")
    beta = _beta(m, seed=31)
    lat = hd.Lattice(L, m + 1, M5=1.8)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(9)
    U = to_dev(hd.pack_gauge(hi.gauge_field(L, seed=7)))
    x = torch.randn((12, lat.V4, m + 1), dtype=torch.complex128, device="cuda:0", generator=g)
    y = torch.randn((12, lat.V4, m + 1), dtype=torch.complex128, device="cuda:0", generator=g)
    a = hd.vec_dot(x, hd.apply_cf(lat, U, y, beta, 0.3))
    b = hd.vec_dot(hd.apply_cf(lat, U, x, beta, 0.3), y)
    assert abs(a - b) <= 1e-12 * abs(a)


def test_cf_argument_checks():
    torch = torch_dev()
    L = (2, 2, 2, 2)
    U = to_dev(hd.pack_gauge(hi.gauge_field(L)))
    x = to_dev(hd.pack_fermion(hi.gaussian_fermion(L, 3, seed=1)))
    lat = hd.Lattice(L, 3)
    for beta, R in (([1.0, -0.5], 0.1), ([1.0, np.nan], 0.1), ([1.0, 2.0], np.inf)):
        with pytest.raises(hd.HDCRError):
            hd.apply_cf(lat, U, x, beta, R)
    with pytest.raises(hd.HDCRError):   # psi and out alias
        hd.apply_cf(lat, U, x, [1.0, 2.0], 0.1, out=x)
    lat1 = hd.Lattice(L, 1)
    x1 = to_dev(hd.pack_fermion(hi.gaussian_fermion(L, 1, seed=1)))
    with pytest.raises(hd.HDCRError):   # no pole slice
        hd.apply_cf(lat1, U, x1, [], 0.1)
