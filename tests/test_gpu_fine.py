"""GPU parity of the fine operator H = Gamma5 D_dwf (Sec. 3) against the FP64 oracle,
through the C-ABI.  FP64 path: 1e-10 relative, FP32 path: 1e-5 relative (element-wise
against the output's scale)."""
import numpy as np
import pytest

import hdcr_inputs as hi
import oracle
from paper_1611_06944_amd import Lattice, apply_fine, pack_fermion, pack_gauge, unpack_fermion
from tests.gpu_util import log, max_rel_elem, rel_err, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

SHAPES = [
    ((2, 2, 2, 2), 4),      # extent 2: both hops of a direction land on the same site
    ((4, 4, 4, 4), 8),      # the small solver configuration
    ((3, 5, 2, 6), 5),      # odd extents and odd Ls, ragged last workgroup
    ((1, 2, 3, 2), 3),      # extent 1: a site is its own neighbour
    ((4, 2, 6, 8), 1),      # Ls = 1 (Wilson limit)
    ((8, 8, 8, 8), 16),     # many workgroups
    ((3, 5, 2, 7), 16),     # tile kernel with DPP fifth-dimension exchange, ragged last workgroup
    ((2, 2, 2, 6), 16),     # parity-tile kernel (FP32): 3 tiles, one workgroup with an empty slot
    ((4, 2, 6, 2), 16),     # parity-tile kernel: extent-2 directions, ragged last workgroup
    ((2, 3, 2, 2), 32),     # tile kernel, fifth-dimension neighbours from memory
    ((2, 2, 1, 3), 64),     # one 4d site per wavefront
]


@pytest.mark.parametrize("L,Ls", SHAPES)
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_apply_fine_parity(L, Ls, prec):
    torch = torch_dev()
    log(f"apply_fine parity L={L} Ls={Ls} prec={prec}")
    mf = 0.07 if Ls > 1 else 0.0
    p = oracle.Params(L, Ls, M5=1.8, mf=mf, bc=(1, -1, 1, -1) if Ls == 5 else (1, 1, 1, -1))
    lat = Lattice(L, Ls, M5=p.M5, mf=p.mf, bc=p.bc)
    U = hi.gauge_field(L, seed=1)
    psi = hi.gaussian_fermion(L, Ls, seed=0)
    ref = oracle.apply_h(U, psi, p)
    dt = torch.complex128 if prec == "c128" else torch.complex64
    Ud = to_dev(pack_gauge(U), dt)
    pd = to_dev(pack_fermion(psi), dt)
    out = apply_fine(lat, Ud, pd)
    torch.cuda.synchronize()
    got = unpack_fermion(to_host(out), L, Ls)
    tol = 1e-10 if prec == "c128" else 1e-5
    assert max_rel_elem(got, ref) <= tol
    assert rel_err(got, ref) <= tol


@pytest.mark.parametrize("L,Ls", [((4, 2, 6, 2), 16),   # parity-tile kernels (FP32 paired, FP64)
                                  ((3, 5, 2, 7), 16),   # tile kernel, odd extents
                                  ((3, 2, 4, 2), 8),    # tile kernel, Ls = 8
                                  ((2, 3, 2, 2), 5)])   # generic kernel
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_apply_fine_cayley_b(L, Ls, prec):
    """The Cayley form with c = 0 and b = 1.5 (Sec. 3: Mobius fermions with c = 0, b != 1)."""
    torch = torch_dev()
    log(f"apply_fine cayley b=1.5 L={L} Ls={Ls} prec={prec}")
    p = oracle.Params(L, Ls, M5=1.8, mf=0.05, bc=(1, -1, 1, -1), b=1.5)
    lat = Lattice(L, Ls, M5=p.M5, mf=p.mf, bc=p.bc, b=1.5)
    U = hi.gauge_field(L, seed=2)
    psi = hi.gaussian_fermion(L, Ls, seed=6)
    ref = oracle.apply_h(U, psi, p)
    dt = torch.complex128 if prec == "c128" else torch.complex64
    out = apply_fine(lat, to_dev(pack_gauge(U), dt), to_dev(pack_fermion(psi), dt))
    torch.cuda.synchronize()
    got = unpack_fermion(to_host(out), L, Ls)
    tol = 1e-10 if prec == "c128" else 1e-5
    assert max_rel_elem(got, ref) <= tol


def test_apply_fine_full_size_sampled():
    """24^4 x 16 (the benchmark's lattice), FP64 and FP32, checked on sampled sites."""
    torch = torch_dev()
    L, Ls = (24, 24, 24, 24), 16
    log(f"apply_fine sampled L={L} Ls={Ls}")
    p = oracle.Params(L, Ls)
    lat = Lattice(L, Ls)
    U = hi.gauge_field(L, seed=1)
    psi = hi.gaussian_fermion(L, Ls, seed=0)
    rng = np.random.default_rng(5)
    N5 = lat.N5
    # random sites plus the lattice corners (every boundary crossing)
    sel = np.unique(np.concatenate([rng.integers(0, N5, 3000), [0, Ls - 1, N5 - 1, N5 - Ls]]))
    ref = oracle.apply_h_sites(U, psi, p, sel)
    for dt, tol in ((torch.complex128, 1e-10), (torch.complex64, 1e-5)):
        Ud = to_dev(pack_gauge(U), dt)
        pd = to_dev(pack_fermion(psi), dt)
        out = apply_fine(lat, Ud, pd)
        torch.cuda.synchronize()
        o = to_host(out)                                  # [12, V4, Ls]
        got = o[:, sel // Ls, sel % Ls].T.reshape(-1, 4, 3)
        assert max_rel_elem(got, ref) <= tol, dt
        del Ud, pd, out
        torch.cuda.empty_cache()
    # FP16 field storage (FP32 links): against the oracle on the same FP16-rounded input, one
    # rounding of each output component (2^-11 |ref|) plus the FP32 arithmetic (2e-5 max|ref|)
    psi16 = psi.real.astype(np.float16).astype(np.float64) + 1j * psi.imag.astype(np.float16).astype(np.float64)
    ref16 = oracle.apply_h_sites(U, psi16, p, sel)
    p16 = torch.view_as_real(to_dev(pack_fermion(psi16), torch.complex64)).to(torch.float16).contiguous()
    out16 = apply_fine(lat, to_dev(pack_gauge(U), torch.complex64), p16)
    o = torch.view_as_complex(out16.to(torch.float32).contiguous()).to("cpu").numpy().astype(np.complex128)
    got = o[:, sel // Ls, sel % Ls].T.reshape(-1, 4, 3)
    e = 2e-5 * np.abs(ref16).max()
    for part in (np.real, np.imag):
        assert np.all(np.abs(part(got) - part(ref16)) <= 2.0 ** -11 * np.abs(part(ref16)) + e)


@pytest.mark.parametrize("Ls", [8, 16])
def test_apply_fine_large_sampled_and_deterministic(Ls):
    """16^4 at Ls = 8 (tile kernel with the fifth-dimension exchange inside groups
    of 8 lanes) and Ls = 16 (parity-tile kernels): sampled sites against the
    oracle, and two launches bitwise equal (the kernels have a fixed order)."""
    torch = torch_dev()
    L = (16, 16, 16, 16)
    log(f"apply_fine sampled L={L} Ls={Ls}")
    p = oracle.Params(L, Ls)
    lat = Lattice(L, Ls)
    U = hi.gauge_field(L, seed=1)
    psi = hi.gaussian_fermion(L, Ls, seed=0)
    rng = np.random.default_rng(6)
    N5 = lat.N5
    sel = np.unique(np.concatenate([rng.integers(0, N5, 4000), [0, Ls - 1, N5 - 1, N5 - Ls]]))
    ref = oracle.apply_h_sites(U, psi, p, sel)
    for dt, tol in ((torch.complex128, 1e-10), (torch.complex64, 1e-5)):
        Ud = to_dev(pack_gauge(U), dt)
        pd = to_dev(pack_fermion(psi), dt)
        out = apply_fine(lat, Ud, pd)
        out2 = apply_fine(lat, Ud, pd)
        torch.cuda.synchronize()
        assert torch.equal(out, out2), dt
        o = to_host(out)
        got = o[:, sel // Ls, sel % Ls].T.reshape(-1, 4, 3)
        assert max_rel_elem(got, ref) <= tol, dt


def test_apply_fine_linearity_and_hermiticity_fp64():
    """<x, H y> = <H x, y> on the device result (1e-12), and H(a x + y) = a Hx + Hy."""
    torch = torch_dev()
    L, Ls = (6, 4, 4, 8), 8
    log(f"apply_fine hermiticity L={L} Ls={Ls}")
    lat = Lattice(L, Ls)
    U = to_dev(pack_gauge(hi.gauge_field(L, seed=3)))
    x = to_dev(pack_fermion(hi.gaussian_fermion(L, Ls, seed=1)))
    y = to_dev(pack_fermion(hi.gaussian_fermion(L, Ls, seed=2)))
    Hx = apply_fine(lat, U, x)
    Hy = apply_fine(lat, U, y)
    lhs = torch.vdot(x.flatten(), Hy.flatten()).item()
    rhs = torch.vdot(Hx.flatten(), y.flatten()).item()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    a = 0.3 - 1.1j
    Hz = apply_fine(lat, U, (a * x + y).contiguous())
    np.testing.assert_allclose(to_host(Hz), to_host(a * Hx + Hy), atol=1e-12 * float(Hx.abs().max()))


@pytest.mark.parametrize("L", [(12, 8, 4, 12), (8, 12, 6, 8)])
def test_traversal_orders_agree(L):
    """The traversal blocking (x split, y split, t slab of the tile lattice) changes only the order
    in which workgroups visit the tiles: FP64, FP32 and FP16-storage applies are bitwise identical
    for every blocking, including splits that do not divide an extent (which fall back to none),
    and for every cap on the resident workgroups per compute unit (tune.wg_per_cu)."""
    torch = torch_dev()
    Ls = 16
    log(f"traversal orders L={L}")
    lat = Lattice(L, Ls, mf=0.05, bc=(1, -1, 1, -1))
    Uh = pack_gauge(hi.gauge_field(L, seed=8))
    xh = pack_fermion(hi.gaussian_fermion(L, Ls, seed=9))
    U64, x64 = to_dev(Uh, torch.complex128), to_dev(xh, torch.complex128)
    U32, x32 = to_dev(Uh, torch.complex64), to_dev(xh, torch.complex64)
    x16 = torch.view_as_real(x32).to(torch.float16).contiguous()
    ref = None
    for xs, ys, ts, cap in ((1, 1, 1, 0), (3, 2, 3, 0), (2, 3, 2, 2), (6, 4, 6, 1), (5, 7, 5, 3), (1, 1, 1, 40)):
        lt = lat.with_tune(xsplit=xs, ysplit=ys, tslab=ts, wg_per_cu=cap)
        outs = (apply_fine(lt, U64, x64), apply_fine(lt, U32, x32), apply_fine(lt, U32, x16).view(torch.int16))
        if ref is None:
            ref = outs
        else:
            assert all(torch.equal(a, b) for a, b in zip(outs, ref)), (xs, ys, ts)


@pytest.mark.parametrize("L,Ls", [((4, 6, 2, 5), 16), ((4, 6, 2, 6), 16), ((3, 2, 4, 2), 8)])
def test_kernel_variants_agree(L, Ls):
    """The kernels of the fine apply give the same result: parity-tile with
    paired slices (FP32, even extents, Ls = 16; variant 0) and with one slice
    per work-item (4), tile kernel with cached (1) and non-temporal (3) stores,
    generic kernel (2)."""
    torch = torch_dev()
    log(f"kernel variants L={L} Ls={Ls}")
    lat = Lattice(L, Ls, mf=0.05)
    Uh = pack_gauge(hi.gauge_field(L, seed=4))
    xh = pack_fermion(hi.gaussian_fermion(L, Ls, seed=3))
    for dt, tol in ((torch.complex128, 1e-14), (torch.complex64, 1e-6)):
        U, x = to_dev(Uh, dt), to_dev(xh, dt)
        outs = []
        for v in (0, 4, 1, 3, 2):
            outs.append(to_host(apply_fine(lat.with_tune(dslash_variant=v), U, x)))
        scale = np.abs(outs[-1]).max()
        for o in outs[:-1]:
            assert np.abs(o - outs[-1]).max() <= tol * scale, dt


def test_stream_copy_exact():
    """The bandwidth-calibration copy moves every byte: sizes with a ragged last chunk, and a
    size that is not a multiple of 16 is refused."""
    torch = torch_dev()
    from paper_1611_06944_amd import HDCRError, stream_copy
    log("stream copy")
    g = torch.Generator(device="cuda:0")
    g.manual_seed(3)
    for nbytes in (16, 4096 * 16 + 48, (1 << 22) + 16 * 257):
        src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda:0", generator=g)
        dst = torch.zeros_like(src)
        stream_copy(src, dst)
        assert torch.equal(src, dst), nbytes
    with pytest.raises(HDCRError):
        stream_copy(src[:40], dst[:40])
