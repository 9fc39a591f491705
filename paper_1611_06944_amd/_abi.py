"""ctypes view of the C ABI declared in include/hdcr.h (marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhdcr.so")

HDCR_OK = 0
HDCR_EINVAL = -1
HDCR_EHIP = -2
HDCR_ENOMEM = -3
HDCR_ENOTCONV = 1
HDCR_EBREAKDOWN = 2
HDCR_ENAN = 3
HDCR_ERANK = 4

C128, C64, BF16C, F16C = 0, 1, 2, 3
MFMA_VARIANTS = 9  # tile shapes of the batched coarse apply
PRECOND_NONE, PRECOND_TWO_LEVEL = 0, 1
WS_SOLVE, WS_BUILD, WS_SUBSPACE, WS_SMOOTH, WS_VCYCLE, WS_COARSE = 0, 1, 2, 3, 4, 5
DEFL_MAX = 64
DOT_WORK_BYTES = 32768
COARSE_STATIC_BYTES = 8 << 20


TUNE_FIELDS = ("dslash_variant", "tslab", "ysplit", "xsplit", "force_r", "force_ms", "force_p", "force_sum",
               "restrict_w", "restrict_rkg", "prolong_ni", "wg_per_cu", "prolong_split")


class Tuning(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in TUNE_FIELDS]


class FineDesc(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32 * 4), ("Ls", ctypes.c_int32), ("bc", ctypes.c_int32 * 4),
                ("reserved", ctypes.c_int32), ("M5", ctypes.c_double), ("mf", ctypes.c_double),
                ("cayley_b", ctypes.c_double), ("tune", Tuning)]


class CoarseDesc(ctypes.Structure):
    _fields_ = [("fine", FineDesc), ("block", ctypes.c_int32 * 4), ("nvec", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class SolveParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("cheb_order", ctypes.c_int32), ("cheb_lo", ctypes.c_double),
                ("cheb_hi", ctypes.c_double), ("coarse_tol", ctypes.c_double), ("coarse_maxiter", ctypes.c_int32),
                ("inner_dtype", ctypes.c_int32), ("coarse_dtype", ctypes.c_int32), ("basis_dtype", ctypes.c_int32),
                ("verbose", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer_iters", ctypes.c_int32), ("coarse_iters", ctypes.c_int64),
                ("fine_applies_f64", ctypes.c_int64), ("fine_applies_inner", ctypes.c_int64),
                ("coarse_applies", ctypes.c_int64), ("true_rel_residual", ctypes.c_double),
                ("seconds_total", ctypes.c_double), ("seconds_fine", ctypes.c_double),
                ("seconds_coarse", ctypes.c_double), ("seconds_outer", ctypes.c_double),
                ("history_len", ctypes.c_int32), ("coarse_breakdowns", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class CoarseDeflation(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("dtype", ctypes.c_int32), ("theta", ctypes.c_void_p),
                ("V", ctypes.c_void_p), ("W", ctypes.c_void_p)]


class DeflationParams(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("m", ctypes.c_int32), ("degree", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("power_iters", ctypes.c_int32), ("reserved", ctypes.c_int32), ("cut", ctypes.c_double)]


_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dbl_p = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes)
PROTOTYPES = {
    "hdcr_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "hdcr_last_error": (ctypes.c_char_p, []),
    "hdcr_apply_fine": (ctypes.c_int, [ctypes.POINTER(FineDesc), _i32, _vp, _vp, _vp, _vp]),
    "hdcr_apply_cf": (ctypes.c_int, [ctypes.POINTER(FineDesc), _i32, _dbl_p, ctypes.c_double, _vp, _vp, _vp, _vp]),
    "hdcr_fermion_force": (ctypes.c_int, [ctypes.POINTER(FineDesc), _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "hdcr_vec_dot": (ctypes.c_int, [_i32, _i64, _vp, _vp, _dbl_p, _vp, _sz, _vp]),
    "hdcr_stream_copy": (ctypes.c_int, [_vp, _vp, _sz, _vp]),
    "hdcr_workspace_bytes": (_sz, [ctypes.c_int, ctypes.POINTER(CoarseDesc), ctypes.POINTER(SolveParams)]),
    "hdcr_solve": (ctypes.c_int, [ctypes.POINTER(CoarseDesc), ctypes.POINTER(SolveParams), _vp, _vp, _vp,
                                  ctypes.POINTER(CoarseDeflation), _vp, _vp, ctypes.POINTER(SolveStats), _dbl_p, _i32,
                                  _vp, _sz, _vp]),
    "hdcr_coarse_solve": (ctypes.c_int, [ctypes.POINTER(CoarseDesc), _i32, _vp, ctypes.POINTER(CoarseDeflation), _vp,
                                         _vp, _i32, ctypes.c_double, ctypes.POINTER(ctypes.c_int32), _vp, _sz, _vp]),
    "hdcr_coarse_solve_static": (ctypes.c_int, [ctypes.POINTER(CoarseDesc), _i32, _vp, ctypes.POINTER(CoarseDeflation),
                                                _vp, _vp, _i32, ctypes.c_double, ctypes.POINTER(ctypes.c_int32), _vp]),
    "hdcr_deflation_workspace_bytes": (_sz, [ctypes.POINTER(CoarseDesc), _i32, ctypes.POINTER(DeflationParams)]),
    "hdcr_build_deflation": (ctypes.c_int, [ctypes.POINTER(CoarseDesc), _i32, _vp, ctypes.POINTER(DeflationParams),
                                            _vp, _vp, _vp, _vp, _dbl_p, ctypes.POINTER(ctypes.c_int32), _vp, _sz, _vp]),
    "hdcr_basis_bytes": (_sz, [ctypes.POINTER(CoarseDesc)]),
    "hdcr_coarse_bytes": (_sz, [ctypes.POINTER(CoarseDesc), _i32]),
    "hdcr_build_coarse": (ctypes.c_int, [ctypes.POINTER(CoarseDesc), _vp, _vp, _vp, _vp, _i32, _vp, _sz, _vp]),
    "hdcr_convert_coarse": (ctypes.c_int, [ctypes.POINTER(CoarseDesc), _vp, _i32, _vp, _vp]),
    "hdcr_export_coarse": (ctypes.c_int, [ctypes.POINTER(CoarseDesc), _i32, _vp, _vp, _vp]),
    "hdcr_export_basis": (ctypes.c_int, [ctypes.POINTER(CoarseDesc), _vp, _vp, _vp]),
    "hdcr_restrict": (ctypes.c_int, [ctypes.POINTER(CoarseDesc), _i32, _vp, _vp, _vp, _vp]),
    "hdcr_prolong": (ctypes.c_int, [ctypes.POINTER(CoarseDesc), _i32, _vp, _vp, _vp, _vp]),
    "hdcr_apply_coarse": (ctypes.c_int, [ctypes.POINTER(CoarseDesc), _i32, _vp, _vp, _vp, _i32, _vp]),
    "hdcr_apply_coarse_batched": (ctypes.c_int, [ctypes.POINTER(CoarseDesc), _vp, _vp, _vp, _i32, _i32, _i32, _vp]),
    "hdcr_tune_coarse_batched": (ctypes.c_int, [ctypes.POINTER(CoarseDesc), _vp, _vp, _vp, _i32, _i32,
                                                 ctypes.POINTER(ctypes.c_int32), _dbl_p, _vp]),
    "hdcr_smooth": (ctypes.c_int, [ctypes.POINTER(FineDesc), _i32, _vp, _i32, ctypes.c_double, ctypes.c_double, _vp,
                                   _vp, _vp, _sz, _vp]),
    "hdcr_vcycle": (ctypes.c_int, [ctypes.POINTER(CoarseDesc), ctypes.POINTER(SolveParams), _vp, _vp, _vp,
                                   ctypes.POINTER(CoarseDeflation), _vp, _vp, _vp, _sz, _vp]),
    "hdcr_subspace_workspace_bytes": (_sz, [ctypes.POINTER(FineDesc), _i32]),
    "hdcr_make_subspace": (ctypes.c_int, [ctypes.POINTER(FineDesc), _i32, _i32, _i32, ctypes.c_double,
                                          ctypes.c_double, _vp, _vp, _vp, _vp, _sz, _vp]),
    "hdcr_make_subspace_degrees": (ctypes.c_int, [ctypes.POINTER(FineDesc), _i32, _i32, _i32,
                                                  ctypes.POINTER(ctypes.c_int32), ctypes.c_double, ctypes.c_double,
                                                  _vp, _vp, _vp, _vp, _sz, _vp]),
    "hdcr_power_max": (ctypes.c_int, [ctypes.POINTER(FineDesc), _vp, _vp, _i32, _dbl_p, _vp, _sz, _vp]),
}

_lib = None


def load():
    """Load libhdcr.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1611_06944_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class HDCRError(RuntimeError):
    def __init__(self, code, where):
        lib = load()
        msg = lib.hdcr_last_error().decode() or lib.hdcr_strerror(code).decode()
        super().__init__(f"{where}: {lib.hdcr_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def check(code, where):
    if code < 0:
        raise HDCRError(code, where)
    return code
