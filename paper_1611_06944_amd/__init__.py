"""MI355X (gfx950) hot path of the Hierarchically Deflated Conjugate Residual
solver (Yamaguchi & Boyle, Lattice 2016): thin Python binding over the HIP
C-ABI library ``libhdcr.so`` (declared in ``include/hdcr.h``).

Every function here only marshals arguments: torch device tensors supply the
pointers and the HIP stream, the work runs in the library's kernels.  There
is no CPU fallback: without the built library every call raises.

Device layouts (see ``include/hdcr.h``):
  fine field   [12, V4, Ls]  complex128 / complex64   (component c = spin*3 + colour)
  gauge field  [V4, 4, 3, 3] complex128 / complex64   (mu, row, col)
  coarse vec   [nrhs, Nc, Nb] or [Nc, Nb]
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, replace

import numpy as np

from . import _abi
from ._abi import (BF16C, C64, C128, F16C, HDCRError, PRECOND_NONE, PRECOND_TWO_LEVEL, CoarseDesc, FineDesc,  # noqa: F401
                   SolveParams, SolveStats)

__all__ = ["Lattice", "apply_fine", "apply_cf", "fermion_force", "vec_dot", "solve", "pack_fermion", "unpack_fermion", "pack_gauge",
           "build_coarse", "convert_coarse", "export_coarse", "export_basis", "restrict", "prolong", "apply_coarse",
           "apply_coarse_batched", "tune_coarse_batched", "smooth", "vcycle", "make_subspace", "power_max", "load",
           "HDCRError", "stream_copy", "Deflation", "build_deflation", "coarse_solve", "coarse_solve_static", "make_subspace_degrees"]

load = _abi.load


@dataclass(frozen=True)
class Lattice:
    """Fine lattice L = (Lx, Ly, Lz, Lt), Ls, M5, mf, bc, Cayley scale b of the 4d part
    (b = 1: Shamir); optional coarse blocking; tune: kernel-shape choices of the calls
    made with this lattice, as (name, value) pairs of ``hdcr_tuning`` fields (empty: the
    library's choices; see ``with_tune``)."""
    L: tuple
    Ls: int
    M5: float = 1.8
    mf: float = 0.01
    bc: tuple = (1, 1, 1, -1)
    block: tuple = (1, 1, 1, 1)
    nvec: int = 0
    b: float = 1.0
    tune: tuple = ()

    def with_tune(self, **kw) -> "Lattice":
        """A copy whose calls use the given ``hdcr_tuning`` choices, e.g.
        ``lat.with_tune(dslash_variant=5)`` or ``lat.with_tune(xsplit=3, tslab=2)``."""
        for k in kw:
            if k not in _abi.TUNE_FIELDS:
                raise ValueError(f"unknown tuning field {k!r}")
        return replace(self, tune=tuple(sorted(kw.items())))

    @property
    def V4(self):
        return int(np.prod(self.L))

    @property
    def N5(self):
        return self.V4 * self.Ls

    @property
    def fshape(self):
        return (12, self.V4, self.Ls)

    @property
    def cdims(self):
        return tuple(int(l) // int(b) for l, b in zip(self.L, self.block))

    @property
    def nc(self):
        return int(np.prod(self.cdims))

    @property
    def nb(self):
        return 2 * self.nvec

    def fine_desc(self) -> FineDesc:
        d = FineDesc()
        d.L[:] = [int(v) for v in self.L]
        d.Ls = int(self.Ls)
        d.bc[:] = [int(v) for v in self.bc]
        d.M5 = float(self.M5)
        d.mf = float(self.mf)
        d.cayley_b = float(self.b)
        for k, v in self.tune:
            setattr(d.tune, k, int(v))
        return d

    def coarse_desc(self) -> CoarseDesc:
        c = CoarseDesc()
        c.fine = self.fine_desc()
        c.block[:] = [int(v) for v in self.block]
        c.nvec = int(self.nvec)
        return c


# ----------------------------------------------------------------------------
# layout conversion (host, numpy): canonical site-major <-> device SoA
# ----------------------------------------------------------------------------

def pack_fermion(psi_aos: np.ndarray) -> np.ndarray:
    """[t, z, y, x, s, spin, col] -> [12, V4, Ls]."""
    sh = psi_aos.shape
    V4 = sh[0] * sh[1] * sh[2] * sh[3]
    return np.ascontiguousarray(psi_aos.reshape(V4, sh[4], 12).transpose(2, 0, 1))


def unpack_fermion(psi_soa: np.ndarray, L, Ls: int) -> np.ndarray:
    """[12, V4, Ls] -> [t, z, y, x, s, spin, col]."""
    Lx, Ly, Lz, Lt = L
    return np.ascontiguousarray(np.asarray(psi_soa).transpose(1, 2, 0)).reshape(Lt, Lz, Ly, Lx, Ls, 4, 3)


def pack_gauge(U_aos: np.ndarray) -> np.ndarray:
    """[t, z, y, x, mu, row, col] -> [V4, mu, row, col] (site-major: the 36
    link entries of a site are contiguous)."""
    sh = U_aos.shape
    V4 = sh[0] * sh[1] * sh[2] * sh[3]
    return np.ascontiguousarray(U_aos.reshape(V4, 4, 3, 3))


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.complex128:
        return C128
    if t.dtype == torch.complex64:
        return C64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on a HIP device")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _check_fields(lat: Lattice, U, *fields):
    """The kernels read whole fields: a tensor of the wrong size or dtype would
    be read past its end, so sizes and dtypes are checked before any launch."""
    if U.numel() != 36 * lat.V4:
        raise ValueError(f"gauge field has {U.numel()} entries, expected 36*V4 = {36 * lat.V4}")
    for f in fields:
        if f.numel() != 12 * lat.N5:
            raise ValueError(f"fine field has {f.numel()} entries, expected 12*V4*Ls = {12 * lat.N5}")
        if f.dtype != U.dtype:
            raise TypeError(f"field dtype {f.dtype} differs from the gauge field's {U.dtype}")


# ----------------------------------------------------------------------------
# entry points
# ----------------------------------------------------------------------------

def apply_fine(lat: Lattice, U, psi, out=None, stream=None):
    """out = H psi, H = Gamma5 D_dwf (one HIP kernel launch).

    psi may also be an FP16-stored field: a float16 tensor [12, V4, Ls, 2] of (re, im)
    pairs, with complex64 links (FP32 arithmetic; Ls = 16 and even extents)."""
    torch = _torch()
    lib = load()
    if psi.dtype == torch.float16:
        if U.dtype != torch.complex64 or U.numel() != 36 * lat.V4:
            raise TypeError("FP16 fields take complex64 links of 36*V4 entries")
        if out is None:
            out = torch.empty_like(psi)
        for f in (psi, out):
            if f.dtype != torch.float16 or f.numel() != 24 * lat.N5:
                raise ValueError(f"FP16 field must be float16 with 24*V4*Ls = {24 * lat.N5} entries")
        code = F16C
    else:
        _check_fields(lat, U, psi)
        if out is None:
            out = torch.empty_like(psi)
        _check_fields(lat, U, out)
        code = _dtype_code(psi)
    d = lat.fine_desc()
    _abi.check(lib.hdcr_apply_fine(ctypes.byref(d), code, _ptr(U), _ptr(psi), _ptr(out), _stream(stream)),
               "hdcr_apply_fine")
    return out


def apply_cf(lat: Lattice, U, psi, beta, R: float, out=None, stream=None):
    """out = A psi for the continued-fraction form of the overlap operator (Sec. 3): lat.Ls = m + 1
    slices with m = len(beta) pole slices, H_W = gamma5 D_W(-lat.M5), caller coefficients beta
    (m positive values) and R (one HIP kernel launch; see hdcr_apply_cf)."""
    lib = load()
    beta = np.ascontiguousarray(np.asarray(beta, dtype=np.float64))
    if beta.ndim != 1 or len(beta) != lat.Ls - 1:
        raise ValueError(f"beta must hold Ls - 1 = {lat.Ls - 1} values")
    _check_fields(lat, U, psi)
    if out is None:
        out = _torch().empty_like(psi)
    _check_fields(lat, U, out)
    d = lat.fine_desc()
    _abi.check(lib.hdcr_apply_cf(ctypes.byref(d), _dtype_code(psi), beta.ctypes.data_as(_abi._dbl_p), float(R),
                                 _ptr(U), _ptr(psi), _ptr(out), _stream(stream)), "hdcr_apply_cf")
    return out


def fermion_force(lat: Lattice, U, chi, psi, W=None, T=None, want_w=True, want_t=True, stream=None):
    """Gauge-link gradient W = dL/dRe U + i dL/dIm U and su(3) force
    T = P_TA(U W^dag) of L = Re <chi, H psi> (one HIP kernel launch).
    Returns (W, T), each [V4, 4, 3, 3] like U, or None where not wanted."""
    torch = _torch()
    lib = load()
    _check_fields(lat, U, chi, psi)
    if want_w and W is None:
        W = torch.empty_like(U)
    if want_t and T is None:
        T = torch.empty_like(U)
    W = W if want_w else None
    T = T if want_t else None
    d = lat.fine_desc()
    _abi.check(lib.hdcr_fermion_force(ctypes.byref(d), _dtype_code(psi), _ptr(U), _ptr(chi), _ptr(psi), _ptr(W), _ptr(T),
                                      _stream(stream)), "hdcr_fermion_force")
    return W, T


def vec_dot(x, y, stream=None, work=None) -> complex:
    """<x, y> with FP64 accumulation (synchronous)."""
    lib = load()
    if work is None:
        work = _workspace(_abi.DOT_WORK_BYTES, x.device)
    out = (ctypes.c_double * 2)()
    _abi.check(lib.hdcr_vec_dot(_dtype_code(x), x.numel(), _ptr(x), _ptr(y), out, _ptr(work), work.numel(),
                                _stream(stream)), "hdcr_vec_dot")
    return complex(out[0], out[1])


def stream_copy(src, dst, stream=None):
    """dst = src with the library's plain streaming copy kernel (bandwidth calibration)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    _abi.check(load().hdcr_stream_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream)), "hdcr_stream_copy")
    return dst


def default_params(**kw) -> SolveParams:
    p = SolveParams()
    p.tol = 1e-8
    p.maxiter = 100000
    p.restart = 8
    p.precond = PRECOND_NONE
    p.cheb_order = 10
    p.cheb_lo = 1.0
    p.cheb_hi = 64.0
    p.coarse_tol = 1e-2
    p.coarse_maxiter = 500
    p.inner_dtype = C64
    p.coarse_dtype = C64
    p.basis_dtype = C64
    p.verbose = 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def workspace_bytes(which: int, lat: Lattice, params: SolveParams | None = None) -> int:
    lib = load()
    cd = lat.coarse_desc()
    return int(lib.hdcr_workspace_bytes(which, ctypes.byref(cd), ctypes.byref(params) if params is not None else None))


def solve(lat: Lattice, U, b, x=None, params: SolveParams | None = None, basis=None, A=None, work=None,
          history_cap: int = 100000, stream=None, defl: "Deflation | None" = None):
    """Solve H x = b (synchronous).  Returns (x, stats dict, relative-residual history).
    defl: coarse deflation space (``build_deflation``) used by every coarse solve."""
    torch = _torch()
    lib = load()
    params = params or default_params()
    if x is None:
        x = torch.zeros_like(b)
    cd = lat.coarse_desc()
    if work is None:
        work = _workspace(workspace_bytes(_abi.WS_SOLVE, lat, params), b.device)
    st = SolveStats()
    hist = (ctypes.c_double * max(1, history_cap))()
    ds = _defl_struct(defl)
    code = lib.hdcr_solve(ctypes.byref(cd), ctypes.byref(params), _ptr(U), _ptr(basis), _ptr(A),
                          ctypes.byref(ds) if ds is not None else None, _ptr(b), _ptr(x), ctypes.byref(st), hist,
                          history_cap, _ptr(work), work.numel(), _stream(stream))
    _abi.check(code, "hdcr_solve")
    return x, st.as_dict(), list(hist[:st.history_len])


# ----------------------------------------------------------------------------
# coarse space
# ----------------------------------------------------------------------------

def basis_bytes(lat: Lattice) -> int:
    cd = lat.coarse_desc()
    n = int(load().hdcr_basis_bytes(ctypes.byref(cd)))
    if n == 0:
        raise ValueError(f"invalid coarse description {lat}")
    return n


def coarse_bytes(lat: Lattice, dtype: int) -> int:
    cd = lat.coarse_desc()
    n = int(load().hdcr_coarse_bytes(ctypes.byref(cd), int(dtype)))
    if n == 0:
        raise ValueError(f"invalid coarse description {lat}")
    return n


def build_coarse(lat: Lattice, U, vecs, A_dtype: int = C128, work=None, stream=None):
    """Chirally split block-orthonormal basis and little Dirac operator (synchronous).

    vecs: complex128 tensor [nvec, 12, V4, Ls].  Returns (basis, A) opaque uint8 tensors.
    """
    torch = _torch()
    lib = load()
    dev = U.device
    basis = torch.empty(basis_bytes(lat), dtype=torch.uint8, device=dev)
    A = torch.empty(coarse_bytes(lat, A_dtype), dtype=torch.uint8, device=dev)
    if work is None:
        work = _workspace(workspace_bytes(_abi.WS_BUILD, lat), dev)
    cd = lat.coarse_desc()
    _abi.check(lib.hdcr_build_coarse(ctypes.byref(cd), _ptr(U), _ptr(vecs), _ptr(basis), _ptr(A), int(A_dtype),
                                     _ptr(work), work.numel(), _stream(stream)), "hdcr_build_coarse")
    return basis, A


def build_coarse_status(lat: Lattice, U, vecs, A_dtype: int = C128):
    """As build_coarse but returns the status code instead of raising on rank deficiency."""
    torch = _torch()
    lib = load()
    dev = U.device
    basis = torch.empty(basis_bytes(lat), dtype=torch.uint8, device=dev)
    A = torch.empty(coarse_bytes(lat, A_dtype), dtype=torch.uint8, device=dev)
    work = _workspace(workspace_bytes(_abi.WS_BUILD, lat), dev)
    cd = lat.coarse_desc()
    code = lib.hdcr_build_coarse(ctypes.byref(cd), _ptr(U), _ptr(vecs), _ptr(basis), _ptr(A), int(A_dtype),
                                 _ptr(work), work.numel(), _stream(None))
    _abi.check(code, "hdcr_build_coarse")
    return code


def convert_coarse(lat: Lattice, A128, dtype: int, stream=None):
    torch = _torch()
    out = torch.empty(coarse_bytes(lat, dtype), dtype=torch.uint8, device=A128.device)
    cd = lat.coarse_desc()
    _abi.check(load().hdcr_convert_coarse(ctypes.byref(cd), _ptr(A128), int(dtype), _ptr(out), _stream(stream)),
               "hdcr_convert_coarse")
    return out


def export_coarse(lat: Lattice, A, dtype: int, stream=None):
    """Logical A[a, d, j, k] (complex128) from any storage."""
    torch = _torch()
    out = torch.empty((lat.nc, 9, lat.nb, lat.nb), dtype=torch.complex128, device=A.device)
    cd = lat.coarse_desc()
    _abi.check(load().hdcr_export_coarse(ctypes.byref(cd), int(dtype), _ptr(A), _ptr(out), _stream(stream)),
               "hdcr_export_coarse")
    return out


def export_basis(lat: Lattice, basis, stream=None):
    """The basis as Nb full fine fields [Nb, 12, V4, Ls] (complex128)."""
    torch = _torch()
    out = torch.empty((lat.nb, 12, lat.V4, lat.Ls), dtype=torch.complex128, device=basis.device)
    cd = lat.coarse_desc()
    _abi.check(load().hdcr_export_basis(ctypes.byref(cd), _ptr(basis), _ptr(out), _stream(stream)),
               "hdcr_export_basis")
    return out


def restrict(lat: Lattice, basis, psi, out=None, stream=None, half_basis=False):
    """v = P^dag psi in the precision of psi; half_basis: complex64 psi with the FP16 basis copy."""
    torch = _torch()
    if out is None:
        out = torch.empty((lat.nc, lat.nb), dtype=psi.dtype, device=psi.device)
    cd = lat.coarse_desc()
    code = F16C if half_basis else _dtype_code(psi)
    _abi.check(load().hdcr_restrict(ctypes.byref(cd), code, _ptr(basis), _ptr(psi), _ptr(out),
                                    _stream(stream)), "hdcr_restrict")
    return out


def prolong(lat: Lattice, basis, v, out=None, stream=None, half_basis=False):
    """psi = P v in the precision of v; half_basis: complex64 v with the FP16 basis copy."""
    torch = _torch()
    if out is None:
        out = torch.empty(lat.fshape, dtype=v.dtype, device=v.device)
    cd = lat.coarse_desc()
    code = F16C if half_basis else _dtype_code(v)
    _abi.check(load().hdcr_prolong(ctypes.byref(cd), code, _ptr(basis), _ptr(v), _ptr(out),
                                   _stream(stream)), "hdcr_prolong")
    return out


def apply_coarse(lat: Lattice, A, A_dtype: int, v, out=None, stream=None):
    """out[r] = A v[r]; v: [nrhs, Nc, Nb] or [Nc, Nb] (complex128 for C128 storage, complex64 otherwise)."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(v)
    nrhs = 1 if v.dim() == 2 else v.shape[0]
    cd = lat.coarse_desc()
    _abi.check(load().hdcr_apply_coarse(ctypes.byref(cd), int(A_dtype), _ptr(A), _ptr(v), _ptr(out), nrhs,
                                        _stream(stream)), "hdcr_apply_coarse")
    return out


def apply_coarse_batched(lat: Lattice, A, v, out=None, variant: int = 0, terms: int = 1, stream=None):
    """out[r] = A v[r] on the matrix cores: A in BF16C storage, v complex64 [nrhs, Nc, Nb],
    FP32 accumulation.  terms: bf16 terms per FP32 component of v (1: v rounded to bf16;
    3: v exact, so the result is the complex64 apply of the stored A).  variant 0: the
    autotuned tile shape."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(v)
    nrhs = 1 if v.dim() == 2 else v.shape[0]
    cd = lat.coarse_desc()
    _abi.check(load().hdcr_apply_coarse_batched(ctypes.byref(cd), _ptr(A), _ptr(v), _ptr(out), nrhs, int(variant),
                                                int(terms), _stream(stream)), "hdcr_apply_coarse_batched")
    return out


def tune_coarse_batched(lat: Lattice, A, v, out=None, terms: int = 1, stream=None):
    """Times every tile shape of the batched apply that takes ``terms``; returns
    (best variant, [median ms per variant, -1 where it does not apply])."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(v)
    nrhs = 1 if v.dim() == 2 else v.shape[0]
    cd = lat.coarse_desc()
    best = ctypes.c_int32(0)
    ms = (ctypes.c_double * _abi.MFMA_VARIANTS)()
    _abi.check(load().hdcr_tune_coarse_batched(ctypes.byref(cd), _ptr(A), _ptr(v), _ptr(out), nrhs, int(terms),
                                               ctypes.byref(best), ms, _stream(stream)), "hdcr_tune_coarse_batched")
    return int(best.value), [float(x) for x in ms]


# ----------------------------------------------------------------------------
# smoother, two-level cycle, subspace filter
# ----------------------------------------------------------------------------

def smooth(lat: Lattice, U, x, order=10, lo=1.0, hi=64.0, out=None, work=None, stream=None, f16: bool = False):
    """out = p(H^2) H x (Chebyshev smoother); precision of x (U in the same precision).
    f16: complex64 x, U and out, with the smoother's own fields stored in FP16."""
    torch = _torch()
    _check_fields(lat, U, x)
    if out is None:
        out = torch.empty_like(x)
    _check_fields(lat, U, out)
    if work is None:
        work = _workspace(workspace_bytes(_abi.WS_SMOOTH, lat), x.device)
    code = _dtype_code(x)
    if f16:
        if code != C64:
            raise TypeError("the FP16-storage smoother takes complex64 fields")
        code = F16C
    d = lat.fine_desc()
    _abi.check(load().hdcr_smooth(ctypes.byref(d), code, _ptr(U), int(order), float(lo), float(hi), _ptr(x),
                                  _ptr(out), _ptr(work), work.numel(), _stream(stream)), "hdcr_smooth")
    return out


def vcycle(lat: Lattice, U, basis, A, r, params: SolveParams, out=None, work=None, stream=None,
           defl: "Deflation | None" = None):
    """One application of the two-level cycle to r (complex128); defl deflates its coarse solve."""
    torch = _torch()
    if out is None:
        out = torch.empty_like(r)
    if work is None:
        work = _workspace(workspace_bytes(_abi.WS_VCYCLE, lat, params), r.device)
    cd = lat.coarse_desc()
    ds = _defl_struct(defl)
    _abi.check(load().hdcr_vcycle(ctypes.byref(cd), ctypes.byref(params), _ptr(U), _ptr(basis), _ptr(A),
                                  ctypes.byref(ds) if ds is not None else None, _ptr(r), _ptr(out), _ptr(work),
                                  work.numel(), _stream(stream)), "hdcr_vcycle")
    return out


def make_subspace(lat: Lattice, U, noise, degree, lo, hi, dtype=C64, work=None, stream=None):
    """Chebyshev-filtered, normalised vectors T_d(yhat) noise[k] (noise: complex128 [nvec, 12, V4, Ls])."""
    torch = _torch()
    lib = load()
    d = lat.fine_desc()
    out = torch.empty_like(noise)
    if work is None:
        work = _workspace(lib.hdcr_subspace_workspace_bytes(ctypes.byref(d), int(dtype)), noise.device)
    _abi.check(lib.hdcr_make_subspace(ctypes.byref(d), int(dtype), int(noise.shape[0]), int(degree), float(lo),
                                      float(hi), _ptr(U), _ptr(noise), _ptr(out), _ptr(work), work.numel(),
                                      _stream(stream)), "hdcr_make_subspace")
    return out


def make_subspace_degrees(lat: Lattice, U, noise, degrees, lo, hi, dtype=C64, work=None, stream=None):
    """Normalised T_d(yhat) noise[k] for every d in degrees (ascending) from one recurrence per
    noise field; noise: complex128 [nnoise, 12, V4, Ls].  Returns [nnoise * len(degrees), 12, V4, Ls],
    field k * len(degrees) + q holding degree degrees[q] of noise k."""
    torch = _torch()
    lib = load()
    d = lat.fine_desc()
    degs = [int(x) for x in degrees]
    nn = int(noise.shape[0])
    out = torch.empty((nn * len(degs),) + tuple(noise.shape[1:]), dtype=noise.dtype, device=noise.device)
    if work is None:
        work = _workspace(lib.hdcr_subspace_workspace_bytes(ctypes.byref(d), int(dtype)), noise.device)
    arr = (ctypes.c_int32 * len(degs))(*degs)
    _abi.check(lib.hdcr_make_subspace_degrees(ctypes.byref(d), int(dtype), nn, len(degs), arr, float(lo), float(hi),
                                              _ptr(U), _ptr(noise), _ptr(out), _ptr(work), work.numel(),
                                              _stream(stream)), "hdcr_make_subspace_degrees")
    return out


def power_max(lat: Lattice, U, v0, iters=30, work=None, stream=None) -> float:
    """Rayleigh-quotient estimate of the largest eigenvalue of H^2 by power iteration."""
    lib = load()
    d = lat.fine_desc()
    if work is None:
        work = _workspace(lib.hdcr_subspace_workspace_bytes(ctypes.byref(d), C128), v0.device)
    lam = ctypes.c_double(0.0)
    _abi.check(lib.hdcr_power_max(ctypes.byref(d), _ptr(U), _ptr(v0), int(iters), ctypes.byref(lam), _ptr(work),
                                  work.numel(), _stream(stream)), "hdcr_power_max")
    return lam.value


# ----------------------------------------------------------------------------
# coarse-space eigenvector deflation
# ----------------------------------------------------------------------------

@dataclass
class Deflation:
    """Deflation space of the coarse solve: Ritz values theta [k] (float64) and the
    vectors V, W = A V [k, Nc, Nb] (complex128 for an FP64 coarse solve, complex64
    for FP32), all device tensors; theta_host: the same Ritz values on the host."""
    theta: object
    V: object
    W: object
    theta_host: list

    @property
    def k(self) -> int:
        return int(self.theta.numel())


def _defl_struct(defl):
    if defl is None:
        return None
    return _abi.CoarseDeflation(defl.k, _dtype_code(defl.V), _ptr(defl.theta).value, _ptr(defl.V).value,
                                _ptr(defl.W).value)


def _coarse_vec_dtype(A_dtype: int):
    torch = _torch()
    return torch.complex128 if int(A_dtype) == C128 else torch.complex64


def _check_coarse_operator(lat: Lattice, A, A_dtype: int):
    need = coarse_bytes(lat, A_dtype)
    if A.numel() * A.element_size() < need:
        raise ValueError(f"A holds {A.numel() * A.element_size()} bytes, {need} needed for dtype {A_dtype}")


def build_deflation(lat: Lattice, A, A_dtype: int, v0, k: int, degree: int = 40, iters: int = 4, cut: float = 0.05,
                    power_iters: int = 30, work=None, stream=None) -> Deflation:
    """The k eigenpairs of smallest |lambda| of the little Dirac operator A by Chebyshev-filtered
    subspace iteration in A^2 from the m start vectors v0 (complex128 [m, Nc, Nb]); synchronous."""
    torch = _torch()
    lib = load()
    _check_coarse_operator(lat, A, A_dtype)
    if v0.dtype != torch.complex128 or v0.dim() != 3 or tuple(v0.shape[1:]) != (lat.nc, lat.nb):
        raise ValueError(f"v0 must be complex128 [m, {lat.nc}, {lat.nb}], got {v0.dtype} {tuple(v0.shape)}")
    m = int(v0.shape[0])
    cd = lat.coarse_desc()
    prm = _abi.DeflationParams(int(k), m, int(degree), int(iters), int(power_iters), 0, float(cut))
    if work is None:
        nbytes = int(lib.hdcr_deflation_workspace_bytes(ctypes.byref(cd), int(A_dtype), ctypes.byref(prm)))
        if nbytes == 0:
            raise ValueError(f"invalid deflation parameters k={k} m={m} degree={degree} iters={iters} cut={cut}")
        work = _workspace(nbytes, v0.device)
    vdt = _coarse_vec_dtype(A_dtype)
    theta = torch.empty(int(k), dtype=torch.float64, device=v0.device)
    V = torch.empty((int(k), lat.nc, lat.nb), dtype=vdt, device=v0.device)
    W = torch.empty_like(V)
    th = (ctypes.c_double * int(k))()
    kf = ctypes.c_int32(0)
    code = lib.hdcr_build_deflation(ctypes.byref(cd), int(A_dtype), _ptr(A), ctypes.byref(prm), _ptr(v0), _ptr(theta),
                                    _ptr(V), _ptr(W), th, ctypes.byref(kf), _ptr(work), work.numel(), _stream(stream))
    if code != 0:
        raise _abi.HDCRError(code, "hdcr_build_deflation")
    n = int(kf.value)
    return Deflation(theta[:n], V[:n], W[:n], [float(t) for t in th[:n]])


def coarse_solve(lat: Lattice, A, A_dtype: int, b, maxiter: int = 500, tol: float = 1e-2, defl: Deflation | None = None,
                 x=None, work=None, stream=None, return_status: bool = False):
    """x = CR_A(b) on the coarse lattice (from 0, or from the Galerkin start of defl); tol <= 0:
    exactly maxiter iterations.  b: [Nc, Nb] complex128 for C128 storage, complex64 otherwise.
    Synchronous; returns (x, iterations), or (x, iterations, status) with return_status
    (0, or HDCR_EBREAKDOWN / HDCR_ENAN when the iteration stopped at a near-breakdown)."""
    torch = _torch()
    lib = load()
    _check_coarse_operator(lat, A, A_dtype)
    if b.dtype != _coarse_vec_dtype(A_dtype) or b.numel() != lat.nc * lat.nb:
        raise ValueError(f"b must be {_coarse_vec_dtype(A_dtype)} with {lat.nc * lat.nb} entries")
    if x is None:
        x = torch.empty_like(b)
    cd = lat.coarse_desc()
    if work is None:
        prm = default_params(coarse_dtype=int(A_dtype))
        work = _workspace(workspace_bytes(_abi.WS_COARSE, lat, prm), b.device)
    ds = _defl_struct(defl)
    it = ctypes.c_int32(0)
    code = _abi.check(lib.hdcr_coarse_solve(ctypes.byref(cd), int(A_dtype), _ptr(A),
                                            ctypes.byref(ds) if ds is not None else None, _ptr(b), _ptr(x), int(maxiter),
                                            float(tol), ctypes.byref(it), _ptr(work), work.numel(), _stream(stream)),
                      "hdcr_coarse_solve")
    if return_status:
        return x, int(it.value), int(code)
    return x, int(it.value)


def coarse_solve_static(lat: Lattice, A, A_dtype: int, b, maxiter: int = 500, tol: float = 1e-2,
                        defl: Deflation | None = None, x=None, stream=None, return_status: bool = False):
    """coarse_solve without a workspace: the library's static device scratch
    (``hdcr_coarse_solve_static``; at most COARSE_STATIC_BYTES of scratch, calls on one GPU must
    not overlap).  Returns as coarse_solve."""
    torch = _torch()
    lib = load()
    _check_coarse_operator(lat, A, A_dtype)
    if b.dtype != _coarse_vec_dtype(A_dtype) or b.numel() != lat.nc * lat.nb:
        raise ValueError(f"b must be {_coarse_vec_dtype(A_dtype)} with {lat.nc * lat.nb} entries")
    if x is None:
        x = torch.empty_like(b)
    cd = lat.coarse_desc()
    ds = _defl_struct(defl)
    it = ctypes.c_int32(0)
    code = _abi.check(lib.hdcr_coarse_solve_static(ctypes.byref(cd), int(A_dtype), _ptr(A),
                                                   ctypes.byref(ds) if ds is not None else None, _ptr(b), _ptr(x),
                                                   int(maxiter), float(tol), ctypes.byref(it), _stream(stream)),
                      "hdcr_coarse_solve_static")
    if return_status:
        return x, int(it.value), int(code)
    return x, int(it.value)
