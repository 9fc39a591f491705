"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
function declared in include/hdcr.h, its structs match the ctypes mirror, and
argument validation rejects bad calls before any launch."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hdcr.h")


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hdcr_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1611_06944_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_1611_06944_amd import build
        build.build()
    return _abi.load()


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert "hdcr_apply_fine" in names and "hdcr_solve" in names
    out = subprocess.run(["nm", "-D", "--defined-only", os.path.join(ROOT, "paper_1611_06944_amd", "libhdcr.so")],
                         capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, f"declared but not exported: {missing}"
    for n in names:
        getattr(lib, n)


def test_ctypes_mirror_matches_c_layout(tmp_path):
    from paper_1611_06944_amd import _abi
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "hdcr.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(hdcr_fine_desc), sizeof(hdcr_coarse_desc), sizeof(hdcr_solve_params),
         sizeof(hdcr_solve_stats));
  printf("%zu %zu %zu %zu\n", offsetof(hdcr_fine_desc, M5), offsetof(hdcr_coarse_desc, nvec),
         offsetof(hdcr_solve_params, coarse_maxiter), offsetof(hdcr_solve_params, basis_dtype));
  printf("%zu %zu\n", offsetof(hdcr_solve_stats, true_rel_residual), offsetof(hdcr_solve_stats, history_len));
  printf("%zu %zu %zu %zu\n", offsetof(hdcr_fine_desc, cayley_b), offsetof(hdcr_fine_desc, tune),
         offsetof(hdcr_tuning, prolong_ni), offsetof(hdcr_solve_stats, coarse_breakdowns));
  printf("%zu %zu\n", offsetof(hdcr_tuning, wg_per_cu), offsetof(hdcr_tuning, prolong_split));
  printf("%zu %zu %zu %zu %zu\n", sizeof(hdcr_coarse_deflation), offsetof(hdcr_coarse_deflation, theta),
         offsetof(hdcr_coarse_deflation, W), sizeof(hdcr_deflation_params), offsetof(hdcr_deflation_params, cut));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"),
                    "-I/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    py = [ctypes.sizeof(_abi.FineDesc), ctypes.sizeof(_abi.CoarseDesc), ctypes.sizeof(_abi.SolveParams),
          ctypes.sizeof(_abi.SolveStats), _abi.FineDesc.M5.offset, _abi.CoarseDesc.nvec.offset,
          _abi.SolveParams.coarse_maxiter.offset, _abi.SolveParams.basis_dtype.offset,
          _abi.SolveStats.true_rel_residual.offset,
          _abi.SolveStats.history_len.offset, _abi.FineDesc.cayley_b.offset, _abi.FineDesc.tune.offset,
          _abi.Tuning.prolong_ni.offset, _abi.SolveStats.coarse_breakdowns.offset,
          _abi.Tuning.wg_per_cu.offset, _abi.Tuning.prolong_split.offset,
          ctypes.sizeof(_abi.CoarseDeflation), _abi.CoarseDeflation.theta.offset, _abi.CoarseDeflation.W.offset,
          ctypes.sizeof(_abi.DeflationParams), _abi.DeflationParams.cut.offset]
    assert vals == py


def test_argument_validation_before_launch(lib):
    from paper_1611_06944_amd import Lattice, _abi
    lat = Lattice((4, 4, 4, 4), 8)
    d = lat.fine_desc()
    fake = ctypes.c_void_p(4096)
    # null descriptor
    assert lib.hdcr_apply_fine(None, 0, fake, fake, ctypes.c_void_p(8192), None) == _abi.HDCR_EINVAL
    # bad dtype
    assert lib.hdcr_apply_fine(ctypes.byref(d), 2, fake, fake, ctypes.c_void_p(8192), None) == _abi.HDCR_EINVAL
    # null pointer
    assert lib.hdcr_apply_fine(ctypes.byref(d), 0, None, fake, ctypes.c_void_p(8192), None) == _abi.HDCR_EINVAL
    assert b"U" in lib.hdcr_last_error()
    # misaligned pointer
    assert lib.hdcr_apply_fine(ctypes.byref(d), 0, ctypes.c_void_p(4100), fake, ctypes.c_void_p(1 << 30),
                               None) == _abi.HDCR_EINVAL
    # aliased in/out
    assert lib.hdcr_apply_fine(ctypes.byref(d), 0, fake, fake, fake, None) == _abi.HDCR_EINVAL
    assert b"overlap" in lib.hdcr_last_error()
    # bad boundary condition and extent
    d.bc[3] = 0
    assert lib.hdcr_apply_fine(ctypes.byref(d), 0, fake, fake, ctypes.c_void_p(1 << 30), None) == _abi.HDCR_EINVAL
    d.bc[3] = -1
    d.L[0] = 0
    assert lib.hdcr_apply_fine(ctypes.byref(d), 0, fake, fake, ctypes.c_void_p(1 << 30), None) == _abi.HDCR_EINVAL
    # Cayley scale: negative is refused, 0 means the Shamir kernel (b = 1)
    d.L[0] = 4
    d.cayley_b = -0.5
    assert lib.hdcr_apply_fine(ctypes.byref(d), 0, fake, fake, ctypes.c_void_p(1 << 30), None) == _abi.HDCR_EINVAL
    assert b"cayley_b" in lib.hdcr_last_error()
    d.cayley_b = 0.0
    assert lib.hdcr_strerror(_abi.HDCR_ENOTCONV) == b"not converged within maxiter"


def test_force_argument_validation_before_launch(lib):
    from paper_1611_06944_amd import Lattice, _abi
    lat = Lattice((4, 4, 4, 4), 8)
    d = lat.fine_desc()
    U, chi, psi = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 24), ctypes.c_void_p(1 << 28)
    W, T = ctypes.c_void_p(1 << 32), ctypes.c_void_p(1 << 33)
    f = lib.hdcr_fermion_force
    assert f(None, 0, U, chi, psi, W, T, None) == _abi.HDCR_EINVAL
    assert f(ctypes.byref(d), 2, U, chi, psi, W, T, None) == _abi.HDCR_EINVAL       # coarse-only dtype
    assert f(ctypes.byref(d), 0, U, chi, psi, None, None, None) == _abi.HDCR_EINVAL  # nothing to write
    assert f(ctypes.byref(d), 0, U, None, psi, W, T, None) == _abi.HDCR_EINVAL
    assert b"chi" in lib.hdcr_last_error()
    assert f(ctypes.byref(d), 0, U, chi, psi, ctypes.c_void_p((1 << 32) + 8), T, None) == _abi.HDCR_EINVAL
    assert b"misaligned" in lib.hdcr_last_error()
    # W on top of psi, and W overlapping T
    assert f(ctypes.byref(d), 0, U, chi, psi, psi, T, None) == _abi.HDCR_EINVAL
    assert b"overlap" in lib.hdcr_last_error()
    assert f(ctypes.byref(d), 0, U, chi, psi, W, ctypes.c_void_p((1 << 32) + 4096), None) == _abi.HDCR_EINVAL
    assert b"overlap" in lib.hdcr_last_error()


def test_layout_roundtrip():
    import hdcr_inputs as hi
    from paper_1611_06944_amd import pack_fermion, pack_gauge, unpack_fermion
    L, Ls = (2, 3, 4, 5), 6
    psi = hi.gaussian_fermion(L, Ls, seed=1)
    soa = pack_fermion(psi)
    assert soa.shape == (12, 120, 6)
    # component c = spin*3 + col of site4 ((t*Lz+z)*Ly+y)*Lx+x, fifth coordinate s
    t, z, y, x, s, sp, col = 4, 3, 2, 1, 5, 2, 1
    assert soa[sp * 3 + col, ((t * 4 + z) * 3 + y) * 2 + x, s] == psi[t, z, y, x, s, sp, col]
    np.testing.assert_array_equal(unpack_fermion(soa, L, Ls), psi)
    U = hi.gauge_field(L, seed=2)
    g = pack_gauge(U)
    assert g.shape == (120, 4, 3, 3)
    assert g[((t * 4 + z) * 3 + y) * 2 + x, 3, 1, 2] == U[t, z, y, x, 3, 1, 2]


def test_two_level_param_validation(lib):
    """Invalid two-level parameters are rejected by the workspace query (host only)."""
    import paper_1611_06944_amd as hd
    lat = hd.Lattice((4, 4, 4, 4), 4, block=(2, 2, 2, 2), nvec=4)
    good = hd.default_params(precond=hd.PRECOND_TWO_LEVEL)
    assert hd.workspace_bytes(hd._abi.WS_SOLVE, lat, good) > 0
    # inner C64 needs C64 or BF16 coarse storage
    assert hd.workspace_bytes(hd._abi.WS_SOLVE, lat, hd.default_params(precond=hd.PRECOND_TWO_LEVEL,
                                                                       coarse_dtype=hd.C128)) == 0
    assert hd.workspace_bytes(hd._abi.WS_SOLVE, lat, hd.default_params(precond=hd.PRECOND_TWO_LEVEL,
                                                                       restart=99)) == 0
    # the FP16 basis copy serves the FP32 inner cycle only
    assert hd.workspace_bytes(hd._abi.WS_SOLVE, lat, hd.default_params(precond=hd.PRECOND_TWO_LEVEL,
                                                                       basis_dtype=hd.F16C)) > 0
    assert hd.workspace_bytes(hd._abi.WS_SOLVE, lat, hd.default_params(precond=hd.PRECOND_TWO_LEVEL,
                                                                       inner_dtype=hd.C128, coarse_dtype=hd.C128,
                                                                       basis_dtype=hd.F16C)) == 0
    assert hd.workspace_bytes(hd._abi.WS_SOLVE, lat, hd.default_params(precond=hd.PRECOND_TWO_LEVEL,
                                                                       cheb_lo=2.0, cheb_hi=1.0)) == 0
    # odd Ls or a block that does not divide the lattice: invalid coarse space
    assert hd.workspace_bytes(hd._abi.WS_SOLVE, hd.Lattice((4, 4, 4, 4), 5, block=(2, 2, 2, 2), nvec=4), good) == 0
    assert hd.workspace_bytes(hd._abi.WS_BUILD, hd.Lattice((4, 4, 4, 4), 4, block=(3, 2, 2, 2), nvec=4)) == 0
    assert hd.workspace_bytes(hd._abi.WS_BUILD, hd.Lattice((4, 4, 4, 4), 4, block=(2, 2, 2, 2), nvec=4)) > 0


def test_deflation_argument_validation_before_launch(lib):
    from paper_1611_06944_amd import Lattice, _abi
    lat = Lattice((8, 8, 8, 8), 8, block=(4, 4, 4, 4), nvec=4)
    cd = lat.coarse_desc()
    n = lat.nc * lat.nb
    A, v0, th = ctypes.c_void_p(1 << 32), ctypes.c_void_p(1 << 33), ctypes.c_void_p(1 << 34)
    V, W, work = ctypes.c_void_p(1 << 35), ctypes.c_void_p(1 << 36), ctypes.c_void_p(1 << 37)
    p = _abi.DeflationParams(4, 8, 10, 2, 10, 0, 0.05)
    ws = lib.hdcr_deflation_workspace_bytes(ctypes.byref(cd), _abi.C128, ctypes.byref(p))
    assert ws > 0
    b = lib.hdcr_build_deflation

    def call(dt=_abi.C128, prm=p, V_=V, W_=W, nbytes=ws):
        return b(ctypes.byref(cd), dt, A, ctypes.byref(prm), v0, th, V_, W_, None, None, work, nbytes, None)

    for bad in [_abi.DeflationParams(9, 8, 10, 2, 10, 0, 0.05),   # k > m
                _abi.DeflationParams(4, 65, 10, 2, 10, 0, 0.05),  # m above the maximum
                _abi.DeflationParams(4, 8, 0, 2, 10, 0, 0.05),    # degree
                _abi.DeflationParams(4, 8, 10, 0, 10, 0, 0.05),   # iters
                _abi.DeflationParams(4, 8, 10, 2, 10, 0, 1.0)]:   # cut
        assert call(prm=bad) == _abi.HDCR_EINVAL
        assert lib.hdcr_deflation_workspace_bytes(ctypes.byref(cd), _abi.C128, ctypes.byref(bad)) == 0
    assert call(dt=_abi.F16C) == _abi.HDCR_EINVAL
    assert call(W_=ctypes.c_void_p((1 << 35) + 16 * n)) == _abi.HDCR_EINVAL   # V and W overlap
    assert b"overlap" in lib.hdcr_last_error()
    assert call(nbytes=ws - 1) == _abi.HDCR_ENOMEM
    # the FP32 build needs less scratch than the FP64 one
    assert 0 < lib.hdcr_deflation_workspace_bytes(ctypes.byref(cd), _abi.BF16C, ctypes.byref(p)) < ws

    cs = lib.hdcr_coarse_solve
    bb, xx = ctypes.c_void_p(1 << 38), ctypes.c_void_p(1 << 39)
    prm = _abi.SolveParams()
    prm.coarse_dtype = _abi.C64
    cws = lib.hdcr_workspace_bytes(_abi.WS_COARSE, ctypes.byref(cd), ctypes.byref(prm))
    assert cws > 0
    d = _abi.CoarseDeflation(4, _abi.C64, th.value, V.value, W.value)
    it = ctypes.c_int32(0)
    assert cs(ctypes.byref(cd), _abi.C64, A, ctypes.byref(d), bb, bb, 10, 0.0, ctypes.byref(it), work, cws,
              None) == _abi.HDCR_EINVAL                                                    # b and x overlap
    d.dtype = _abi.C128
    assert cs(ctypes.byref(cd), _abi.C64, A, ctypes.byref(d), bb, xx, 10, 0.0, ctypes.byref(it), work, cws,
              None) == _abi.HDCR_EINVAL                                                    # vector precision
    d.dtype, d.k = _abi.C64, 0
    assert cs(ctypes.byref(cd), _abi.C64, A, ctypes.byref(d), bb, xx, 10, 0.0, ctypes.byref(it), work, cws,
              None) == _abi.HDCR_EINVAL
    assert b"deflation" in lib.hdcr_last_error()
    d.k = 4
    assert cs(ctypes.byref(cd), _abi.C64, A, ctypes.byref(d), bb, xx, -1, 0.0, ctypes.byref(it), work, cws,
              None) == _abi.HDCR_EINVAL
    assert cs(ctypes.byref(cd), _abi.C64, A, ctypes.byref(d), bb, xx, 10, 0.0, ctypes.byref(it), work, cws - 1,
              None) == _abi.HDCR_ENOMEM


def test_f16_storage_validation_before_launch(lib):
    from paper_1611_06944_amd import Lattice, _abi
    U, x, y, work = (ctypes.c_void_p(1 << 32), ctypes.c_void_p(1 << 33), ctypes.c_void_p(1 << 34),
                     ctypes.c_void_p(1 << 35))
    # FP16 fields need Ls = 16 and even extents
    d8 = Lattice((4, 4, 4, 4), 8).fine_desc()
    assert lib.hdcr_apply_fine(ctypes.byref(d8), _abi.F16C, U, x, y, None) == _abi.HDCR_EINVAL
    assert b"F16C" in lib.hdcr_last_error()
    dodd = Lattice((4, 4, 3, 4), 16).fine_desc()
    assert lib.hdcr_apply_fine(ctypes.byref(dodd), _abi.F16C, U, x, y, None) == _abi.HDCR_EINVAL
    d16 = Lattice((4, 4, 4, 4), 16).fine_desc()
    # F16C takes C64 links: an 8-byte-aligned U is accepted, a misaligned one is not
    assert lib.hdcr_apply_fine(ctypes.byref(d16), _abi.F16C, ctypes.c_void_p((1 << 32) + 4), x, y,
                               None) == _abi.HDCR_EINVAL
    # the FP16 smoother needs at least two Chebyshev terms
    assert lib.hdcr_smooth(ctypes.byref(d16), _abi.F16C, U, 1, 1.0, 64.0, x, y, work, 1 << 30,
                           None) == _abi.HDCR_EINVAL
    assert lib.hdcr_smooth(ctypes.byref(d8), _abi.F16C, U, 10, 1.0, 64.0, x, y, work, 1 << 30,
                           None) == _abi.HDCR_EINVAL
    # solve parameters: inner F16C needs an FP32 coarse operator and order >= 2
    cd = Lattice((8, 8, 8, 8), 16, block=(4, 4, 4, 4), nvec=4).coarse_desc()
    p = _abi.SolveParams()
    p.tol, p.maxiter, p.restart, p.precond = 1e-8, 10, 4, _abi.PRECOND_TWO_LEVEL
    p.cheb_order, p.cheb_lo, p.cheb_hi = 10, 1.0, 64.0
    p.inner_dtype, p.coarse_dtype, p.basis_dtype = _abi.F16C, _abi.BF16C, _abi.F16C
    assert lib.hdcr_workspace_bytes(_abi.WS_SOLVE, ctypes.byref(cd), ctypes.byref(p)) > 0
    p.cheb_order = 1
    assert lib.hdcr_workspace_bytes(_abi.WS_SOLVE, ctypes.byref(cd), ctypes.byref(p)) == 0
    p.cheb_order, p.coarse_dtype = 10, _abi.C128
    assert lib.hdcr_workspace_bytes(_abi.WS_SOLVE, ctypes.byref(cd), ctypes.byref(p)) == 0
    # ... and a lattice the FP16 stencil takes (Ls = 16, even extents)
    p.coarse_dtype = _abi.C64
    cd8 = Lattice((8, 8, 8, 8), 8, block=(4, 4, 4, 4), nvec=4).coarse_desc()
    assert lib.hdcr_vcycle(ctypes.byref(cd8), ctypes.byref(p), U, x, y, None, x, y, work, 1 << 30,
                           None) == _abi.HDCR_EINVAL
    assert b"F16C" in lib.hdcr_last_error()


def test_tuning_travels_in_the_descriptor():
    """Kernel-shape choices are per call (hdcr_fine_desc.tune), set through Lattice.with_tune;
    the library reads no environment variable."""
    from paper_1611_06944_amd import Lattice
    lat = Lattice((4, 4, 4, 4), 8)
    d = lat.with_tune(dslash_variant=5, xsplit=3, force_sum=2, restrict_rkg=32).fine_desc()
    assert (d.tune.dslash_variant, d.tune.xsplit, d.tune.force_sum, d.tune.restrict_rkg) == (5, 3, 2, 32)
    z = lat.fine_desc()
    assert all(getattr(z.tune, k) == 0 for k, _ in z.tune._fields_)
    with pytest.raises(ValueError):
        lat.with_tune(no_such_knob=1)
    src = os.path.join(ROOT, "paper_1611_06944_amd", "csrc")
    for fn in os.listdir(src):
        assert "getenv" not in open(os.path.join(src, fn)).read(), fn
