"""ctypes declarations of the C ABI in ``include/skrylov.h`` (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# SKR_LIBRARY selects another build of the library (the host-sanitizer build, for instance)
LIB_PATH = os.environ.get("SKR_LIBRARY") or os.path.join(_HERE, "libskrylov.so")

SKR_OK, SKR_NOT_CONVERGED, SKR_BREAKDOWN = 0, 1, 2
SKR_EINVAL, SKR_EHIP, SKR_ENOMEM, SKR_ENOTSUP, SKR_EPROJ = -1, -2, -3, -4, -5
SKR_FP64, SKR_MIXED = 0, 1
SKR_SKETCH_SPARSE_SIGN, SKR_SKETCH_SRHT, SKR_SKETCH_NONE = 0, 1, 2
SKR_RECOVER_STORED, SKR_RECOVER_TWO_PASS = 0, 1
SKR_ORTH_EUCLIDEAN, SKR_ORTH_SKETCHED = 0, 1

STATUS_NAMES = {SKR_OK: "converged", SKR_NOT_CONVERGED: "maxit", SKR_BREAKDOWN: "breakdown"}


class Params(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32),
        ("maxit", ctypes.c_int32),
        ("p", ctypes.c_int32),
        ("zeta", ctypes.c_int32),
        ("s", ctypes.c_int64),
        ("tol", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("precision", ctypes.c_int32),
        ("sketch", ctypes.c_int32),
        ("recover", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("trunc_tol", ctypes.c_double),
        ("orth", ctypes.c_int32),
    ]


class SkrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"skrylov error {code}: {msg}")
        self.code = code


_vp = ctypes.c_void_p
_i32, _i64, _f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_pi32, _pi64, _pf64 = ctypes.POINTER(_i32), ctypes.POINTER(_i64), ctypes.POINTER(_f64)

# name -> (restype, argtypes); every symbol of include/skrylov.h
SIGNATURES = {
    "skr_params_default": (_i32, [ctypes.POINTER(Params)]),
    "skr_op_create_csr": (_i32, [_i64, _i64, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "skr_op_set_diag": (_i32, [_vp, _vp, _vp]),
    "skr_op_size": (_i32, [_vp, _pi64, _pi64]),
    "skr_op_destroy": (_i32, [_vp]),
    "skr_solve": (_i32, [_vp, _vp, _vp, _vp, _i64, ctypes.POINTER(Params), _vp, ctypes.POINTER(_vp)]),
    "skr_adjoint_solve": (_i32, [_vp, _vp, _vp, _vp, _i64, ctypes.POINTER(Params), _vp, ctypes.POINTER(_vp)]),
    "skr_result_info": (_i32, [_vp, _pi64, _pi32, _pf64, _pi32]),
    "skr_result_history": (_i32, [_vp, _pi32, _pf64, _i32, _pi32]),
    "skr_result_copy_factors": (_i32, [_vp, _vp, _vp, _vp]),
    "skr_result_timing": (_i32, [_vp, _pf64, _pf64, _pf64]),
    "skr_result_kernel_stats": (_i32, [_vp, _i32, _pi32, ctypes.POINTER(ctypes.c_char_p), _pi64, _pf64]),
    "skr_result_proj_stats": (_i32, [_vp, _pi32, _pi32, _pi32, _pf64]),
    "skr_result_failed_checks": (_i32, [_vp, _pi32]),
    "skr_result_destroy": (_i32, [_vp]),
    "skr_true_residual": (_i32, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _pf64]),
    "skr_true_residual_adjoint": (_i32, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _pf64]),
    "skr_pairing_grads": (_i32, [_i64, _i64, _i64, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _vp,
                                 _pf64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "skr_pairing_grads_noalloc": (_i32, [_i64, _i64, _i64, _i64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp,
                                         _vp, _pf64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "skr_lyap_solve": (_i32, [_vp, _vp, _i64, ctypes.POINTER(Params), _vp, ctypes.POINTER(_vp)]),
    "skr_release_cached_memory": (_i32, []),
    "skr_last_error": (ctypes.c_char_p, []),
    "skr_version": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises ImportError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} not found: build the HIP library first (python -m paper_2311_16019_amd.build)")
    # Load PyTorch's HIP runtime first: the library then binds to the same runtime instance
    # (same soname), so torch streams and device pointers are valid inside it.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int) -> int:
    """Raise SkrError for a negative return code; pass statuses through."""
    if code < 0:
        msg = load().skr_last_error()
        raise SkrError(code, msg.decode() if msg else "")
    return code
