"""GPU parity of the FP16-storage path against the FP64 oracle, through the C-ABI: the
parity-tile stencils reading and writing (fp16 re, fp16 im) fields (FP32 links and arithmetic),
the smoother whose recurrence fields are stored in FP16, and the two-level cycle and HDCR solve
with that smoother (inner_dtype F16C).

Bounds.
* One application of H on an FP16 field: the kernel computes in FP32 on the FP16 input and
  rounds each output component to nearest FP16 once, so against the oracle applied to the same
  FP16-rounded input, |got - ref| <= 2^-11 |ref| + e per real component, with e = 2e-5 max|ref|
  covering the FP32 arithmetic (the FP32 kernel's own parity bound is 1e-5) and FP16 subnormals.
* The smoother p(H^2) H x rounds to FP16 once at its input (after scaling to unit RMS, which the
  result undoes exactly up to FP32 rounding), once after each plain stencil pass and once per
  fused combination step, or twice when the combination is a separate pass (variant 6): at most
  3 order - 1 roundings in all.  With
  Clenshaw's recurrence bounded on the polynomial's interval, each rounding contributes at most
  2^-11 of the field's size to the result, so 2 (3 order - 1) 2^-11 max|ref| bounds the error:
  2.8e-2 at order 10.
* The cycle inherits the smoother's bound (its coarse correction is FP32); the solve is checked
  by its FP64 true residual."""
import numpy as np
import pytest

import hdcr_inputs as hi
import oracle
import paper_1611_06944_amd as hd
from tests.gpu_util import log, max_rel_elem, to_dev, to_host, torch_dev

pytestmark = pytest.mark.gpu

U16 = 2.0 ** -11


def _f16_round(psi):
    """The field as FP16 stores it: each real component rounded to nearest."""
    return psi.real.astype(np.float16).astype(np.float64) + 1j * psi.imag.astype(np.float16).astype(np.float64)


def _to_f16_dev(soa):
    torch = torch_dev()
    t = torch.from_numpy(np.ascontiguousarray(soa)).to("cuda:0")
    return torch.view_as_real(t.to(torch.complex64)).to(torch.float16).contiguous()


def _from_f16_dev(t):
    torch = torch_dev()
    return torch.view_as_complex(t.to(torch.float32).contiguous()).to("cpu").numpy().astype(np.complex128)


@pytest.mark.parametrize("L,bc", [((4, 4, 2, 6), (1, 1, 1, -1)), ((4, 6, 2, 8), (-1, 1, 1, -1)),
                                  ((8, 8, 8, 8), (1, 1, 1, -1))])
def test_apply_fine_f16_parity(L, bc):
    torch = torch_dev()
    Ls = 16
    log(f"apply f16 L={L} bc={bc}")
    p = oracle.Params(L, Ls, M5=1.8, mf=0.01, bc=bc)
    lat = hd.Lattice(L, Ls, M5=1.8, mf=0.01, bc=bc)
    U = hi.gauge_field(L, seed=3)
    psi = _f16_round(hi.gaussian_fermion(L, Ls, seed=4))
    ref = oracle.apply_h(U, psi, p)
    out = hd.apply_fine(lat, to_dev(hd.pack_gauge(U), torch.complex64), _to_f16_dev(hd.pack_fermion(psi)))
    assert out.dtype == torch.float16
    got = hd.unpack_fermion(_from_f16_dev(out), L, Ls)
    e = 2e-5 * np.abs(ref).max()
    for part in (np.real, np.imag):
        err = np.abs(part(got) - part(ref))
        assert np.all(err <= U16 * np.abs(part(ref)) + e), float((err - U16 * np.abs(part(ref))).max())
    log(f"  max rel elem {max_rel_elem(got, ref):.2e}")


@pytest.mark.parametrize("L,bc", [((4, 4, 2, 6), (1, 1, 1, -1)), ((6, 4, 8, 2), (-1, 1, -1, -1))])
def test_f16_kernels_agree(L, bc):
    """The two FP16-storage kernels (four slices per work-item, the default, and the paired
    kernel, variant 5) do the same operations in the same order per output: bitwise equal, for
    the plain apply and for the smoother, whose steps use the fused epilogues."""
    torch = torch_dev()
    Ls = 16
    log(f"f16 kernels agree L={L} bc={bc}")
    lat = hd.Lattice(L, Ls, M5=1.8, mf=0.01, bc=bc)
    U = to_dev(hd.pack_gauge(hi.gauge_field(L, seed=5)), torch.complex64)
    x = _to_f16_dev(hd.pack_fermion(hi.gaussian_fermion(L, Ls, seed=6)))
    outs, sm = [], []
    r = to_dev(hd.pack_fermion(hi.gaussian_fermion(L, Ls, seed=7)), torch.complex64)
    for v in (0, 5):
        lv = lat.with_tune(dslash_variant=v)
        outs.append(hd.apply_fine(lv, U, x))
        sm.append(hd.smooth(lv, U, r, order=4, f16=True))  # fused epilogues with 1, 2 and 3 fields
    assert torch.equal(outs[0].view(torch.int16), outs[1].view(torch.int16))
    assert torch.equal(sm[0], sm[1])


@pytest.mark.parametrize("order,variant", [(2, 0), (3, 0), (10, 0), (10, 6)])
def test_smoother_f16_parity(order, variant):
    """Variant 0: each Clenshaw step's combination fused into the second stencil pass (2 order
    roundings in all); variant 6: a plain pass, then an element-wise combination (3 order - 1)."""
    torch = torch_dev()
    L, Ls = (4, 4, 4, 6), 16
    log(f"smoother f16 order={order} variant={variant}")
    p = oracle.Params(L, Ls, M5=1.8, mf=0.01)
    lat = hd.Lattice(L, Ls, M5=1.8, mf=0.01).with_tune(dslash_variant=variant)
    U = hi.gauge_field(L)
    r = hi.gaussian_fermion(L, Ls, seed=4) * 1e-3   # the scaling to unit RMS makes the size irrelevant
    ref = oracle.smoother(lambda f: oracle.apply_h(U, f, p), r, order=order, lo=1.0, hi=64.0)
    out = hd.smooth(lat, to_dev(hd.pack_gauge(U), torch.complex64), to_dev(hd.pack_fermion(r), torch.complex64),
                    order=order, f16=True)
    got = hd.unpack_fermion(to_host(out), L, Ls)
    err = max_rel_elem(got, ref)
    bound = 2 * (3 * order - 1) * U16
    log(f"  max rel elem {err:.2e} (bound {bound:.2e})")
    assert err <= bound
    # accumulating form, through the cycle below; a zero input gives zero
    z = torch.zeros(12 * lat.N5, dtype=torch.complex64, device="cuda:0").reshape(12, lat.V4, Ls)
    out0 = hd.smooth(lat, to_dev(hd.pack_gauge(U), torch.complex64), z, order=order, f16=True)
    assert torch.count_nonzero(out0).item() == 0


def _two_level(L, Ls, block, nvec):
    p = oracle.Params(L, Ls, M5=1.8, mf=0.01)
    cs = oracle.Coarse(p, block, nvec)
    lat = hd.Lattice(L, Ls, M5=1.8, mf=0.01, block=block, nvec=nvec)
    U = hi.gauge_field(L)
    ap = lambda f: oracle.apply_h(U, f, p)
    lmax = oracle.power_max(ap, hi.gaussian_fermion(L, Ls, seed=99), iters=30) * 1.1
    vecs = [oracle.cheby_filter(ap, e, 12, 0.05 * lmax, lmax) for e in hi.subspace_noise(L, Ls, nvec)]
    return p, cs, lat, U, vecs


def test_vcycle_f16_parity():
    """One cycle with the FP16-storage smoother and 6 coarse CR iterations (C64 A) against the
    oracle's FP64 cycle; both smoother applications within the smoother bound."""
    torch = torch_dev()
    L, Ls, block, nvec = (4, 4, 4, 4), 16, (2, 2, 2, 2), 4
    log("vcycle f16")
    p, cs, lat, U, vecs = _two_level(L, Ls, block, nvec)
    basis_ref, _ = oracle.block_basis(vecs, cs)
    A_ref = oracle.coarse_build(U, basis_ref, cs)
    r = hi.gaussian_fermion(L, Ls, seed=5)
    ref = oracle.vcycle(lambda f: oracle.apply_h(U, f, p), A_ref, basis_ref, cs, r, order=10, lo=1.0, hi=64.0,
                        ctol=0.0, cmaxiter=6)
    Ud = to_dev(hd.pack_gauge(U))
    basis, A = hd.build_coarse(lat, Ud, to_dev(np.stack([hd.pack_fermion(v) for v in vecs])), hd.C64)
    prm = hd.default_params(inner_dtype=hd.F16C, coarse_dtype=hd.C64, coarse_tol=0.0, coarse_maxiter=6)
    e = hd.unpack_fermion(to_host(hd.vcycle(lat, Ud, basis, A, to_dev(hd.pack_fermion(r)), prm)), L, Ls)
    err = max_rel_elem(e, ref)
    log(f"  max rel elem {err:.2e}")
    assert err <= 2 * (3 * 10 - 1) * U16


@pytest.mark.parametrize("coarse", ["c64", "bf16"])
def test_hdcr_solve_f16_smoother(coarse):
    """The HDCR solve with the FP16-storage smoother reaches 1e-8 in FP64 (true residual from the
    oracle's operator), in at most two more outer iterations than with the FP32 smoother."""
    torch = torch_dev()
    L, Ls, block, nvec = (4, 4, 4, 8), 16, (2, 2, 2, 2), 4
    log(f"hdcr solve f16 smoother coarse={coarse}")
    p, cs, lat, U, vecs = _two_level(L, Ls, block, nvec)
    cdt = hd.C64 if coarse == "c64" else hd.BF16C
    Ud = to_dev(hd.pack_gauge(U))
    basis, A = hd.build_coarse(lat, Ud, to_dev(np.stack([hd.pack_fermion(v) for v in vecs])), cdt)
    b = to_dev(hd.pack_fermion(hi.gaussian_fermion(L, Ls, seed=11)))
    res = {}
    for inner in (hd.C64, hd.F16C):
        prm = hd.default_params(precond=hd.PRECOND_TWO_LEVEL, tol=1e-8, maxiter=200, inner_dtype=inner,
                                coarse_dtype=cdt, coarse_tol=0.05, coarse_maxiter=200, basis_dtype=hd.F16C)
        x, st, _ = hd.solve(lat, Ud, b, params=prm, basis=basis, A=A)
        assert st["status"] == 0, st
        res[inner] = (x, st)
    st32, st16 = res[hd.C64][1], res[hd.F16C][1]
    log(f"  outer iterations: FP32 smoother {st32['outer_iters']}, FP16 smoother {st16['outer_iters']}")
    assert st16["outer_iters"] <= st32["outer_iters"] + 2
    xh = hd.unpack_fermion(to_host(res[hd.F16C][0]), L, Ls)
    bh = hd.unpack_fermion(to_host(b), L, Ls)
    assert oracle.norm(bh - oracle.apply_h(U, xh, p)) <= 1.01e-8 * oracle.norm(bh)


@pytest.mark.parametrize("variant", [0, 6])
def test_subspace_filter_f16_parity(variant):
    """The subspace filter with FP16-stored recurrence fields (make_subspace with F16C, and several
    degrees per recurrence) against the oracle's FP64 filter.  Each step rounds three fields (two
    stencil passes and the combination) and each rescaling two more; the filter never amplifies an
    error injected at step j more than it amplifies the signal from step 0, so every rounding
    contributes at most 2^-11 of the result's scale: (3 d + 2 floor(d / 16)) 2^-11 bounds the
    element error of the normalised result relative to its largest entry.  Variant 0 fuses the
    combination into the second stencil pass (one rounding fewer per step), variant 6 does not."""
    torch = torch_dev()
    L, Ls = (4, 4, 4, 6), 16
    log(f"subspace filter f16 variant={variant}")
    p = oracle.Params(L, Ls, M5=1.8, mf=0.01)
    lat = hd.Lattice(L, Ls, M5=1.8, mf=0.01).with_tune(dslash_variant=variant)
    U = hi.gauge_field(L)
    ap = lambda f: oracle.apply_h(U, f, p)
    lam = oracle.power_max(ap, hi.gaussian_fermion(L, Ls, seed=99), iters=25)
    lo, hi_ = 0.02 * lam, 1.1 * lam
    noise = hi.subspace_noise(L, Ls, 2)
    Ud = to_dev(hd.pack_gauge(U))
    nd = to_dev(np.stack([hd.pack_fermion(e) for e in noise]))
    degrees = [0, 1, 16, 17, 40]
    many = to_host(hd.make_subspace_degrees(lat, Ud, nd, degrees, lo, hi_, dtype=hd.F16C))
    one = to_host(hd.make_subspace(lat, Ud, nd, 40, lo, hi_, dtype=hd.F16C))
    for k in range(2):
        for q, deg in enumerate(degrees):
            ref = oracle.cheby_filter(ap, noise[k], deg, lo, hi_)
            got = hd.unpack_fermion(many[k * len(degrees) + q], L, Ls)
            err = max_rel_elem(got, ref)
            bound = (3 * deg + 2 * (deg // 16) + 1) * U16
            log(f"  noise {k} degree {deg}: max rel elem {err:.2e} (bound {bound:.2e})")
            assert err <= bound
        assert max_rel_elem(hd.unpack_fermion(one[k], L, Ls), hd.unpack_fermion(many[k * len(degrees) + 4], L, Ls)) \
            <= 1e-12
