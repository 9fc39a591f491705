"""GPU parity at the benchmark's coarse shape (Sec. 4), element by element against the FP64
oracle, through the C-ABI.

The 24^4 x 16 solve uses 4^4 x Ls = 16 blocks with nvec = 32 subspace vectors (Nb = 64), an
FP16 copy of the basis for restriction and prolongation, and a BF16-stored little Dirac
operator on a 6^4 coarse lattice.  The oracle cannot build that space in seconds, so the same
blocks and vector count are taken on an 8^4 x 16 lattice (coarse 2^4, 24,576 entries per block
and chirality, 8 panels of 4 vectors per chirality in the block orthonormalisation): the basis,
six full columns of A, restriction and prolongation in FP64, FP32 and with the FP16 basis, and
the BF16 single- and multi-right-hand-side coarse applies.  The coarse apply is also checked at
the exact 6^4, Nb = 64 shape with a seeded operator (its cost and code path do not depend on
the values)."""
import numpy as np
import pytest

import hdcr_inputs as hi
import oracle
import paper_1611_06944_amd as hd
from tests.gpu_util import log, max_rel_elem, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

L, LS, BLOCK, NVEC = (8, 8, 8, 8), 16, (4, 4, 4, 4), 32
U24 = 2.0 ** -24   # unit roundoff of FP32


@pytest.fixture(scope="module")
def space():
    torch = torch_dev()
    log(f"bench-shape coarse space L={L} Ls={LS} block={BLOCK} nvec={NVEC}")
    p = oracle.Params(L, LS, M5=1.8, mf=0.01)
    cs = oracle.Coarse(p, BLOCK, NVEC)
    lat = hd.Lattice(L, LS, M5=1.8, mf=0.01, block=BLOCK, nvec=NVEC)
    U = hi.gauge_field(L, seed=1)
    vecs = [hi.gaussian_fermion(L, LS, seed=100 + k) for k in range(NVEC)]
    basis_ref, st = oracle.block_basis(vecs, cs)
    assert st == 0
    Ud = to_dev(hd.pack_gauge(U))
    basis, A = hd.build_coarse(lat, Ud, to_dev(np.stack([hd.pack_fermion(v) for v in vecs])), hd.C128)
    torch.cuda.synchronize()
    return dict(p=p, cs=cs, lat=lat, U=U, vecs=vecs, basis_ref=basis_ref, basis=basis, A=A, Ud=Ud)


def test_basis_bench_shape(space):
    """Chiral split and block orthonormalisation (8 panels per block and chirality) at 1e-10."""
    log("bench-shape basis")
    lat, cs = space["lat"], space["cs"]
    fields = to_host(hd.export_basis(lat, space["basis"]))
    got = np.stack([hd.unpack_fermion(f, L, LS) for f in fields])
    assert max_rel_elem(got, space["basis_ref"]) <= 1e-10


def test_coarse_columns_bench_shape(space):
    """Six full columns of A = P^dag H P (all coarse sites, directions and rows) at 1e-10: the first and
    last vector of each chirality and two inside panels."""
    log("bench-shape A columns")
    lat, cs = space["lat"], space["cs"]
    kcols = [0, 13, 31, 32, 50, 63]
    cols = oracle.coarse_columns(space["U"], space["basis_ref"], cs, kcols)
    Ag = to_host(hd.export_coarse(lat, space["A"], hd.C128))
    for c, k in enumerate(kcols):
        assert max_rel_elem(Ag[:, :, :, k], cols[c]) <= 1e-10, k


def test_restrict_prolong_bench_shape(space):
    """Restriction and prolongation with Nb = 64 (two groups of 16 vectors per chirality per
    restriction workgroup row, four prolongation index pairs): FP64 at 1e-10, FP32 at 1e-5, and
    the FP16 basis copy within 2^-11 sum |phi||psi| (resp. sum |phi||v|) per component plus
    1e-5 of the same sum for the FP32 arithmetic."""
    torch = torch_dev()
    log("bench-shape restrict / prolong")
    lat, cs, basis, basis_ref = space["lat"], space["cs"], space["basis"], space["basis_ref"]
    psi = hi.gaussian_fermion(L, LS, seed=7)
    v = hi.gaussian_coarse(cs.nc, cs.nb, seed=8)
    r_ref = oracle.restrict(basis_ref, psi, cs)
    pr_ref = oracle.prolong(basis_ref, v, cs)
    for dt, tol in ((torch.complex128, 1e-10), (torch.complex64, 1e-5)):
        r = to_host(hd.restrict(lat, basis, to_dev(hd.pack_fermion(psi), dt)))
        assert max_rel_elem(r, r_ref) <= tol, dt
        pr = hd.unpack_fermion(to_host(hd.prolong(lat, basis, to_dev(v, dt))), L, LS)
        assert max_rel_elem(pr, pr_ref) <= tol, dt
    bound_r = (2.0 ** -11 + 1e-5) * oracle.restrict(np.abs(basis_ref), np.abs(psi), cs).real
    bound_p = (2.0 ** -11 + 1e-5) * oracle.prolong(np.abs(basis_ref), np.abs(v), cs).real
    r = to_host(hd.restrict(lat, basis, to_dev(hd.pack_fermion(psi), torch.complex64), half_basis=True))
    err = np.abs(r - r_ref)
    assert np.all(err <= bound_r), float((err / bound_r).max())
    pr = hd.unpack_fermion(to_host(hd.prolong(lat, basis, to_dev(v, torch.complex64), half_basis=True)), L, LS)
    err = np.abs(pr - pr_ref)
    assert np.all(err <= bound_p + 1e-300), float((err / (bound_p + 1e-300)).max())


def _apply_bound(A_log, v, cdims, nb):
    """Element-wise bound of an FP32-accumulated coarse apply of exactly representable A and v:
    each output is a sum of 9 Nb complex products; a complex product carries at most
    sqrt(2) * 2u of relative error and recursive or blocked summation of n terms at most
    (n - 1) u of sum |terms|, so |out - ref| <= (9 Nb + 2) sqrt(2) u sum |A| |v|."""
    n = 9 * nb
    return (n + 2) * np.sqrt(2.0) * U24 * oracle.coarse_apply(np.abs(A_log), np.abs(v), cdims).real


def test_bf16_coarse_apply_real_operator(space):
    """The BF16-stored little Dirac operator of the bench-shape space, applied to one and to three
    right-hand sides (the single-vector wide-load kernel and the multi-vector kernel), against the
    oracle's FP64 apply of the exported bf16 values, element by element within the FP32
    accumulation bound."""
    torch = torch_dev()
    log("bench-shape BF16 coarse apply (built operator)")
    lat, cs = space["lat"], space["cs"]
    Ab = hd.convert_coarse(lat, space["A"], hd.BF16C)
    A_log = to_host(hd.export_coarse(lat, Ab, hd.BF16C))
    v = hi.gaussian_coarse(cs.nc, cs.nb, seed=9, nrhs=3).astype(np.complex64).astype(np.complex128)
    ref = oracle.coarse_apply(A_log, v, cs.cdims)
    bound = _apply_bound(A_log, v, cs.cdims, cs.nb)
    for vv, rr, bb in ((v[0], ref[0], bound[0]), (v, ref, bound)):
        out = to_host(hd.apply_coarse(lat, Ab, hd.BF16C, to_dev(vv, torch.complex64)))
        err = np.abs(out - rr)
        assert np.all(err <= bb), float((err / bb).max())


def test_bf16_coarse_apply_24x24x24x24_coarse_shape():
    """The coarse apply at the benchmark's own shape: 6^4 coarse sites, Nb = 64, BF16 storage, one
    right-hand side (the operator of the HDCR solve's coarse CR) and three, with a seeded Gaussian
    operator rounded to bf16, against the oracle within the FP32 accumulation bound, element by
    element; and the coarse CR's fused apply (one iteration of hdcr_coarse_solve from x = 0 is
    x = alpha b with alpha = <b, A b>/|A b|^2) agrees with the oracle's first CR step."""
    torch = torch_dev()
    Lf, block, nvec = (24, 24, 24, 24), (4, 4, 4, 4), 32
    log(f"BF16 coarse apply at coarse 6^4 Nb=64")
    lat = hd.Lattice(Lf, 16, block=block, nvec=nvec)
    cs = oracle.Coarse(oracle.Params(Lf, 16), block, nvec)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(23)
    raw = torch.randn(hd.coarse_bytes(lat, hd.C128) // 8, dtype=torch.float64, device="cuda:0", generator=g)
    Ab = hd.convert_coarse(lat, raw, hd.BF16C)
    del raw
    A_log = to_host(hd.export_coarse(lat, Ab, hd.BF16C))
    v = hi.gaussian_coarse(cs.nc, cs.nb, seed=24, nrhs=3).astype(np.complex64).astype(np.complex128)
    ref = oracle.coarse_apply(A_log, v, cs.cdims)
    bound = _apply_bound(A_log, v, cs.cdims, cs.nb)
    for vv, rr, bb in ((v[0], ref[0], bound[0]), (v, ref, bound)):
        out = to_host(hd.apply_coarse(lat, Ab, hd.BF16C, to_dev(vv, torch.complex64)))
        err = np.abs(out - rr)
        assert np.all(err <= bb), float((err / bb).max())
    # one coarse CR iteration from x = 0: x1 = alpha b with alpha = Re<b, Ab>/|Ab|^2, the two sums
    # reduced in FP64 from the FP32 apply.  With e_i <= bound_i the apply's error, the sums move by
    # at most d1 = sum |b_i| bound_i and d2 = sum (2 |Ab_i| + bound_i) bound_i, so alpha by at most
    # |alpha| (d1 / |Re<b,Ab>| + d2 / |Ab|^2), plus one FP32 rounding of alpha and of alpha b_i.
    x, it = hd.coarse_solve(lat, Ab, hd.BF16C, to_dev(v[0], torch.complex64), maxiter=1, tol=0.0)
    assert it == 1
    b0, ab, e0 = v[0], ref[0], bound[0]
    rar, apap = np.vdot(b0, ab).real, np.vdot(ab, ab).real
    alpha = rar / apap
    d1 = float(np.sum(np.abs(b0) * e0))
    d2 = float(np.sum((2 * np.abs(ab) + e0) * e0))
    dalpha = abs(alpha) * (d1 / abs(rar) + d2 / apap + 2 * U24)
    err = np.abs(to_host(x) - alpha * b0)
    assert np.all(err <= dalpha * np.abs(b0) + abs(alpha) * U24 * np.abs(b0)), float(err.max())


@pytest.mark.parametrize("tune", [dict(restrict_rkg=32), dict(restrict_w=4), dict(restrict_w=2),
                                  dict(restrict_w=1, restrict_rkg=32), dict(restrict_w=8, restrict_rkg=32),
                                  dict(prolong_ni=4), dict(prolong_split=5), dict(prolong_ni=4, prolong_split=7)])
def test_restrict_prolong_shapes_bench_shape(space, tune):
    """Every restriction shape (32 vectors per workgroup: one group per chirality; 1, 2, 4 or 8
    s slots per work-item, 8 being the FP16 default), the four-index FP16 prolongation and the
    prolongation split over 5 and 7 workgroups per coarse site (ragged last parts) against the
    oracle at Nb = 64:
    FP64 at 1e-10, FP32 at 1e-5, FP16 basis within the derived bound."""
    torch = torch_dev()
    log(f"bench-shape restrict / prolong shape {tune}")
    lat, cs, basis, basis_ref = space["lat"].with_tune(**tune), space["cs"], space["basis"], space["basis_ref"]
    psi = hi.gaussian_fermion(L, LS, seed=27)
    v = hi.gaussian_coarse(cs.nc, cs.nb, seed=28)
    r_ref = oracle.restrict(basis_ref, psi, cs)
    pr_ref = oracle.prolong(basis_ref, v, cs)
    for dt, tol in ((torch.complex128, 1e-10), (torch.complex64, 1e-5)):
        r = to_host(hd.restrict(lat, basis, to_dev(hd.pack_fermion(psi), dt)))
        assert max_rel_elem(r, r_ref) <= tol, dt
        pr = hd.unpack_fermion(to_host(hd.prolong(lat, basis, to_dev(v, dt))), L, LS)
        assert max_rel_elem(pr, pr_ref) <= tol, dt
    bound_r = (2.0 ** -11 + 1e-5) * oracle.restrict(np.abs(basis_ref), np.abs(psi), cs).real
    bound_p = (2.0 ** -11 + 1e-5) * oracle.prolong(np.abs(basis_ref), np.abs(v), cs).real
    r = to_host(hd.restrict(lat, basis, to_dev(hd.pack_fermion(psi), torch.complex64), half_basis=True))
    assert np.all(np.abs(r - r_ref) <= bound_r)
    pr = hd.unpack_fermion(to_host(hd.prolong(lat, basis, to_dev(v, torch.complex64), half_basis=True)), L, LS)
    assert np.all(np.abs(pr - pr_ref) <= bound_p + 1e-300)
