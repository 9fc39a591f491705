"""GPU parity of the gauge-link gradient W and su(3) force T of L = Re <chi, H psi>
(the HMC fermion force, abstract, Sec. 1 and Sec. 5) against the FP64 oracle,
through the C-ABI; finite differences at eps = 1e-6 on the device; the
autograd Function's gradients against the oracle and torch.autograd.gradcheck.

Tolerances: FP64 1e-10, FP32 1e-5, element-wise against the result's scale."""

import numpy as np
import pytest

import hdcr_inputs as hi
import oracle
from paper_1611_06944_amd import Lattice, apply_fine, fermion_force, pack_fermion, pack_gauge
from tests.gpu_util import log, max_rel_elem, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

SHAPES = [
    ((2, 2, 2, 2), 4, (1, 1, 1, -1)),     # extent 2: the forward and backward neighbour coincide
    ((3, 5, 2, 6), 5, (1, -1, 1, -1)),    # odd extents, Ls = 5 (lanes with one and two slices), ragged last workgroup
    ((1, 2, 3, 2), 3, (-1, 1, 1, -1)),    # extent 1: a site is its own neighbour; Ls = 3
    ((4, 2, 6, 2), 1, (1, 1, 1, -1)),     # Ls = 1 (one lane per site)
    ((4, 4, 4, 4), 16, (1, 1, 1, -1)),    # the benchmark's Ls
    ((3, 2, 2, 5), 12, (1, 1, -1, -1)),   # Ls not a power of two
]


def _inputs(L, Ls, bc, seed=1, b=1.0):
    p = oracle.Params(L, Ls, M5=1.8, mf=0.07, bc=bc, b=b)
    lat = Lattice(L, Ls, M5=p.M5, mf=p.mf, bc=p.bc, b=b)
    U = hi.gauge_field(L, seed=seed)
    chi = hi.gaussian_fermion(L, Ls, seed=3)
    psi = hi.gaussian_fermion(L, Ls, seed=4)
    return p, lat, U, chi, psi


def _force(lat, U, chi, psi, dt, **kw):
    torch = torch_dev()
    Ud = to_dev(pack_gauge(U), dt)
    W, T = fermion_force(lat, Ud, to_dev(pack_fermion(chi), dt), to_dev(pack_fermion(psi), dt), **kw)
    torch.cuda.synchronize()
    sh = U.shape
    return (None if W is None else to_host(W).reshape(sh)), (None if T is None else to_host(T).reshape(sh))


@pytest.mark.parametrize("L,Ls,bc", SHAPES)
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_force_parity(L, Ls, bc, prec):
    torch = torch_dev()
    log(f"fermion_force parity L={L} Ls={Ls} bc={bc} prec={prec}")
    p, lat, U, chi, psi = _inputs(L, Ls, bc)
    Wref = oracle.link_grad(U, chi, psi, p)
    Tref = oracle.force(U, Wref)
    dt = torch.complex128 if prec == "c128" else torch.complex64
    W, T = _force(lat, U, chi, psi, dt)
    tol = 1e-10 if prec == "c128" else 1e-5
    assert max_rel_elem(W, Wref) <= tol
    assert max_rel_elem(T, Tref) <= tol
    # either output alone
    W1, T1 = _force(lat, U, chi, psi, dt, want_t=False)
    assert T1 is None and np.array_equal(W1, W)
    W2, T2 = _force(lat, U, chi, psi, dt, want_w=False)
    assert W2 is None and np.array_equal(T2, T)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_force_parity_cayley_b(prec):
    """W and T for the Cayley form with c = 0 and b = 1.5 (Sec. 3)."""
    torch = torch_dev()
    L, Ls = (2, 4, 2, 4), 16
    log(f"fermion_force cayley b=1.5 L={L} Ls={Ls} prec={prec}")
    p, lat, U, chi, psi = _inputs(L, Ls, (1, -1, 1, -1), b=1.5)
    Wref = oracle.link_grad(U, chi, psi, p)
    dt = torch.complex128 if prec == "c128" else torch.complex64
    W, T = _force(lat, U, chi, psi, dt)
    tol = 1e-10 if prec == "c128" else 1e-5
    assert max_rel_elem(W, Wref) <= tol
    assert max_rel_elem(T, oracle.force(U, Wref)) <= tol


WORK_SPLITS = [(r, ms, pp, lds) for r in (2, 4, 8, 16) for ms in (1, 2) for pp in (1, 2) for lds in (0, 1)]


@pytest.mark.parametrize("L,Ls", [((3, 2, 2, 5), 16), ((2, 3, 1, 2), 8), ((2, 1, 3, 2), 6)])
def test_force_every_work_split(L, Ls):
    """Each (lanes per site, direction groups, slices per load, cross-lane sum)
    split of the kernel, FP64 and FP32; Ls = 6 gives lanes with one, two or no
    load units."""
    torch = torch_dev()
    p, lat, U, chi, psi = _inputs(L, Ls, (1, -1, 1, -1))
    Wref = oracle.link_grad(U, chi, psi, p)
    Tref = oracle.force(U, Wref)
    for r, ms, pp, lds in WORK_SPLITS:
        ls = lat.with_tune(force_r=r, force_ms=ms, force_p=pp, force_sum=1 + lds)
        for dt, tol in ((torch.complex128, 1e-10), (torch.complex64, 1e-5)):
            if pp == 2 and dt == torch.complex128:
                continue  # paired slices are an FP32 load shape
            log(f"fermion_force split r={r} ms={ms} p={pp} lds={lds} L={L} Ls={Ls} {dt}")
            W, T = _force(ls, U, chi, psi, dt)
            assert max_rel_elem(W, Wref) <= tol, (r, ms, pp, lds, dt)
            assert max_rel_elem(T, Tref) <= tol, (r, ms, pp, lds, dt)


def test_force_rejects_unsupported_split():
    """A paired-slice load is refused for FP64, and an unknown cross-lane sum for any
    precision (before any launch)."""
    torch = torch_dev()
    from paper_1611_06944_amd import HDCRError
    p, lat, U, chi, psi = _inputs((2, 2, 2, 2), 4, (1, 1, 1, -1))
    with pytest.raises(HDCRError):
        _force(lat.with_tune(force_p=2), U, chi, psi, torch.complex128)
    with pytest.raises(HDCRError):
        _force(lat.with_tune(force_sum=3), U, chi, psi, torch.complex64)


def _sample_links(L, n, rng):
    Lx, Ly, Lz, Lt = L
    links = [tuple(int(v) for v in (rng.integers(Lt), rng.integers(Lz), rng.integers(Ly), rng.integers(Lx),
                                    rng.integers(4))) for _ in range(n)]
    # every direction at the last site (boundary crossings) and at the first
    links += [(Lt - 1, Lz - 1, Ly - 1, Lx - 1, mu) for mu in range(4)] + [(0, 0, 0, 0, mu) for mu in range(4)]
    return links


def _site4(L, t, z, y, x):
    Lx, Ly, Lz, _ = L
    return ((t * Lz + z) * Ly + y) * Lx + x


def test_force_full_size_sampled():
    """16^4 x 16 with Gaussian chi, psi, FP64 and FP32, on sampled links."""
    torch = torch_dev()
    L, Ls = (16, 16, 16, 16), 16
    log(f"fermion_force sampled L={L} Ls={Ls}")
    p, lat, U, chi, psi = _inputs(L, Ls, (1, 1, 1, -1))
    links = _sample_links(L, 400, np.random.default_rng(11))
    Wref = oracle.link_grad_at(U, chi, psi, p, links)
    Uat = np.stack([U[l] for l in links])
    Tref = oracle.force(Uat, Wref)
    idx = [(_site4(L, *l[:4]), l[4]) for l in links]
    for dt, tol in ((torch.complex128, 1e-10), (torch.complex64, 1e-5)):
        Ud = to_dev(pack_gauge(U), dt)
        cd, pd = to_dev(pack_fermion(chi), dt), to_dev(pack_fermion(psi), dt)
        W, T = fermion_force(lat, Ud, cd, pd)
        torch.cuda.synchronize()
        Wh, Th = to_host(W), to_host(T)
        gotW = np.stack([Wh[s, mu] for s, mu in idx])
        gotT = np.stack([Th[s, mu] for s, mu in idx])
        assert max_rel_elem(gotW, Wref) <= tol, dt
        assert max_rel_elem(gotT, Tref) <= tol, dt
        # T is traceless anti-Hermitian everywhere
        Tt = T.reshape(-1, 3, 3)
        ah = (Tt + Tt.conj().transpose(-1, -2)).abs().max().item()
        tr = torch.diagonal(Tt, dim1=-2, dim2=-1).sum(-1).abs().max().item()
        scale = Tt.abs().max().item()
        assert ah <= tol * scale and tr <= 10 * tol * scale, dt
        del Ud, cd, pd, W, T, Tt
        torch.cuda.empty_cache()


def test_force_finite_differences_device():
    """dL/dRe U + i dL/dIm U by central differences at eps = 1e-6 of
    L = Re <chi, H psi>, with H applied by the library in FP64.  L is linear in
    (Re U, Im U), so the difference quotient is exact up to rounding; only the
    5d sites next to the perturbed link change, so (H(U+) - H(U-)) psi is
    formed first and its rounding stays at those sites (bound below)."""
    torch = torch_dev()
    L, Ls = (16, 16, 16, 16), 16
    log(f"fermion_force finite differences L={L} Ls={Ls}")
    p, lat, U, chi, psi = _inputs(L, Ls, (1, 1, 1, -1))
    dt = torch.complex128
    Ud = to_dev(pack_gauge(U), dt)
    cd, pd = to_dev(pack_fermion(chi), dt), to_dev(pack_fermion(psi), dt)
    W, _ = fermion_force(lat, Ud, cd, pd, want_t=False)
    torch.cuda.synchronize()
    Wh = to_host(W)
    eps = 1e-6
    u = 2.0 ** -53
    rng = np.random.default_rng(2)
    links = _sample_links(L, 6, rng)
    cmax, pmax = cd.abs().amax().item(), pd.abs().amax().item()
    for (t, z, y, x, mu) in links:
        a, b = int(rng.integers(3)), int(rng.integers(3))
        s4 = _site4(L, t, z, y, x)
        fd = []
        for dz in (eps, 1j * eps):
            Up, Um = Ud.clone(), Ud.clone()
            Up[s4, mu, a, b] += dz
            Um[s4, mu, a, b] -= dz
            d = apply_fine(lat, Up, pd) - apply_fine(lat, Um, pd)
            fd.append(torch.vdot(cd.flatten(), d.flatten()).real.item() / (2 * eps))
        got = fd[0] + 1j * fd[1]
        # rounding: an entry of H psi is a sum of at most 50 max|psi| in absolute
        # terms, computed with error <= 64 u times that; the two applies differ
        # at 2 * 12 * Ls entries, each weighted by at most max|chi|
        bound = 2 * (2 * 12 * Ls) * cmax * 64 * u * 50 * pmax / (2 * eps)
        assert abs(got - Wh[s4, mu, a, b]) <= bound, ((t, z, y, x, mu, a, b), got, Wh[s4, mu, a, b], bound)


def test_autograd_function_matches_oracle():
    """loss = Re <chi, H psi>: U.grad is the oracle's link gradient, psi.grad = H chi."""
    torch = torch_dev()
    from paper_1611_06944_amd.autograd import apply_h
    L, Ls = (4, 2, 2, 6), 8
    log(f"autograd ApplyH L={L} Ls={Ls}")
    p, lat, U, chi, psi = _inputs(L, Ls, (1, -1, 1, -1))
    dt = torch.complex128
    Ud = to_dev(pack_gauge(U), dt).requires_grad_(True)
    pd = to_dev(pack_fermion(psi), dt).requires_grad_(True)
    cd = to_dev(pack_fermion(chi), dt)
    y = apply_h(lat, Ud, pd)
    loss = torch.vdot(cd.flatten(), y.flatten()).real
    loss.backward()
    torch.cuda.synchronize()
    assert abs(loss.item() - oracle.loss(U, chi, psi, p)) <= 1e-10 * abs(loss.item())
    gU = to_host(Ud.grad).reshape(U.shape)
    assert max_rel_elem(gU, oracle.link_grad(U, chi, psi, p)) <= 1e-10
    gpsi = to_host(pd.grad)
    assert max_rel_elem(gpsi, pack_fermion(oracle.apply_h(U, chi, p))) <= 1e-10


def test_autograd_gradcheck():
    """torch.autograd.gradcheck of ApplyH (complex inputs and output, FP64) on a tiny lattice."""
    torch = torch_dev()
    from paper_1611_06944_amd.autograd import ApplyH
    L, Ls = (2, 2, 1, 2), 2
    log(f"gradcheck ApplyH L={L} Ls={Ls}")
    p, lat, U, chi, psi = _inputs(L, Ls, (1, 1, 1, -1))
    Ud = to_dev(pack_gauge(U), torch.complex128).requires_grad_(True)
    pd = to_dev(pack_fermion(psi), torch.complex128).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: ApplyH.apply(a, b, lat), (Ud, pd), eps=1e-6, atol=1e-7,
                                    rtol=1e-6, fast_mode=True)
