"""The allocation-free coarse solve (hdcr_coarse_solve_static, static device scratch) against
hdcr_coarse_solve with a caller workspace, through the C-ABI: same kernels, so the same bits,
iteration count and status, on two calls in a row, the second on a smaller coarse space (the
scratch keeps the first call's contents); and a coarse space too large for the static scratch
is refused before any launch."""
import numpy as np
import pytest

import hdcr_inputs as hi
import paper_1611_06944_amd as hd
from tests.gpu_util import log, to_dev, torch_dev

pytestmark = pytest.mark.gpu


def _space(L, Ls, block, nvec, dt):
    lat = hd.Lattice(L, Ls, M5=1.8, mf=0.03, block=block, nvec=nvec)
    U = to_dev(hd.pack_gauge(hi.gauge_field(L, seed=1)))
    vecs = to_dev(np.stack([hd.pack_fermion(hi.gaussian_fermion(L, Ls, seed=100 + k)) for k in range(nvec)]))
    _, A = hd.build_coarse(lat, U, vecs, hd.C128)
    if dt != hd.C128:
        A = hd.convert_coarse(lat, A, dt)
    return lat, A


@pytest.mark.parametrize("dt", [hd.C128, hd.C64, hd.BF16C])
def test_coarse_solve_static_matches_workspace_entry(dt):
    torch = torch_dev()
    # the larger space first, then a smaller one that reuses the scratch the first call left behind
    for L, Ls, block, nvec, seed in (((8, 8, 8, 8), 8, (2, 2, 2, 2), 8, 41), ((4, 4, 4, 4), 4, (2, 2, 2, 2), 4, 42)):
        log(f"coarse_solve_static L={L} block={block} nvec={nvec} dtype={dt}")
        lat, A = _space(L, Ls, block, nvec, dt)
        vdt = torch.complex128 if dt == hd.C128 else torch.complex64
        b = to_dev(hi.gaussian_coarse(lat.nc, lat.nb, seed=seed), vdt)
        for tol, maxiter in ((1e-3, 300), (0.0, 7)):
            x_ws, it_ws, st_ws = hd.coarse_solve(lat, A, dt, b, maxiter=maxiter, tol=tol, return_status=True)
            x_st, it_st, st_st = hd.coarse_solve_static(lat, A, dt, b, maxiter=maxiter, tol=tol, return_status=True)
            torch.cuda.synchronize()
            assert (it_st, st_st) == (it_ws, st_ws), (tol, it_st, it_ws, st_st, st_ws)
            assert it_st > 0
            assert torch.equal(x_st, x_ws), tol


def test_coarse_solve_static_refuses_oversized_space():
    torch = torch_dev()
    # coarse 8^4 with Nb = 64 in FP64: four coarse vectors alone take 16.8 MB > 8 MiB
    lat = hd.Lattice((16, 16, 16, 16), 4, block=(2, 2, 2, 2), nvec=32)
    log("coarse_solve_static oversized space")
    need = hd.workspace_bytes(hd._abi.WS_COARSE, lat, hd.default_params(coarse_dtype=hd.C128))
    assert need > hd._abi.COARSE_STATIC_BYTES
    A = torch.empty(hd.coarse_bytes(lat, hd.C128), dtype=torch.uint8, device="cuda:0")
    b = torch.zeros((lat.nc, lat.nb), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(hd.HDCRError) as ei:
        hd.coarse_solve_static(lat, A, hd.C128, b, maxiter=5, tol=1e-2)
    assert ei.value.code == hd._abi.HDCR_ENOMEM
    assert b"static" in hd.load().hdcr_last_error()
