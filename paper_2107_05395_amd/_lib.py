"""ctypes loader for libbandbatch.so (the C ABI of include/bandbatch.h).

Argument marshalling only.  The library must have been built in tree
(``python -m paper_2107_05395_amd.build``); there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbandbatch.so")

STATUS = {
    0: "BB_OK", -1: "BB_ERR_ARG", -2: "BB_ERR_ZERO_PIVOT", -3: "BB_ERR_SINGULAR_CAPACITANCE",
    -4: "BB_ERR_HIP", -5: "BB_ERR_OOM", -6: "BB_ERR_UNSUPPORTED",
}
PRECISION = {"f64": 0, "f32r": 1, "f32": 2, "f32rhs": 3, "f32rhs_f64": 4}

# every function the header declares, with its ctypes signature
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64
_S = ctypes.c_int
_FACTOR = ctypes.c_void_p
SIGNATURES = {
    "bb_factor_shared_tri": (_S, [_D, _D, _D, _I64, ctypes.POINTER(_FACTOR)]),
    "bb_factor_shared_tri_cyclic": (_S, [_D, _D, _D, _I64, ctypes.POINTER(_FACTOR)]),
    "bb_factor_shared_penta": (_S, [_D, _D, _D, _D, _D, _I64, ctypes.POINTER(_FACTOR)]),
    "bb_factor_shared_penta_cyclic": (_S, [_D, _D, _D, _D, _D, _I64, ctypes.POINTER(_FACTOR)]),
    "bb_factor_destroy": (_S, [_FACTOR]),
    "bb_factor_upload": (_S, [_FACTOR, _P]),
    "bb_factor_info": (_S, [_FACTOR, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_int32),
                            ctypes.POINTER(ctypes.c_int32)]),
    "bb_max_n": (_I64, []),
    "bb_plan": (_S, [_FACTOR, _I64, ctypes.c_int32, _S, ctypes.POINTER(ctypes.c_int32),
                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                     ctypes.POINTER(ctypes.c_int32)]),
    "bb_solve_batch_tri": (_S, [_FACTOR, _P, _P, _I64, _I64, _S, _P]),
    "bb_solve_batch_penta": (_S, [_FACTOR, _P, _P, _I64, _I64, _S, _P]),
    "bb_solve_batch_tri_cyclic": (_S, [_FACTOR, _P, _P, _I64, _I64, _S, _P]),
    "bb_solve_batch_penta_cyclic": (_S, [_FACTOR, _P, _P, _I64, _I64, _S, _P]),
    "bb_solve_batch_tri_adjoint": (_S, [_FACTOR, _P, _P, _I64, _I64, _S, _P]),
    "bb_solve_batch_penta_adjoint": (_S, [_FACTOR, _P, _P, _I64, _I64, _S, _P]),
    "bb_solve_batch_tri_thread_per_system": (_S, [_FACTOR, _P, _P, _I64, _I64, _P]),
    "bb_band_grad_workspace_bytes": (ctypes.c_size_t, [_FACTOR, _I64]),
    "bb_band_grad": (_S, [_FACTOR, _P, _P, _I64, _I64, _P, _P, ctypes.c_size_t, _P]),
    "bb_band_grad_noalloc": (_S, [_FACTOR, _P, _P, _I64, _I64, _P, _P]),
    "bb_band_grad_scratch_bytes": (_I64, []),
    "bb_ch_step": (_S, [_FACTOR, _P, _P, _I64, _I64, ctypes.c_double, _I64, _P]),
    "bb_cn_step": (_S, [_FACTOR, _P, _P, _P, _I64, _I64, _I64, _P]),
    "bb_cn_trajectory": (_S, [_FACTOR, _P, _P, _P, _I64, _I64, _I64, _P]),
    "bb_adjoint_trajectory": (_S, [_FACTOR, _P, _P, _I64, _I64, _I64, _P]),
    "bb_adjoint_band_grad": (_S, [_FACTOR, _P, _P, _P, _I64, _I64, _I64, _P, _P, ctypes.c_size_t,
                                  _P]),
    "bb_adjoint_band_grad_workspace_bytes": (ctypes.c_size_t, [_FACTOR, _I64, _I64]),
    "bb_adjoint_band_grad_fused": (ctypes.c_int32, [_FACTOR, _I64]),
    "bb_copy_tiles": (_S, [_P, _P, _I64, _P]),
    "bb_copy_rows": (_S, [_P, _P, _I64, _I64, _I64, _P]),
    "bb_ch_stats_workspace_bytes": (ctypes.c_size_t, [_FACTOR, _I64, _I64]),
    "bb_ch_forced_step": (_S, [_FACTOR, _P, _P, _I64, _I64, ctypes.c_double, ctypes.c_double,
                               _P, _P, _P, _I64, _P]),
    "bb_factor_ch": (_S, [_I64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                          ctypes.POINTER(_FACTOR), _D, _D]),
    "bb_ch_step_stats": (_S, [_FACTOR, _P, _P, _I64, _I64, ctypes.c_double, _I64, _I64, _P, _P,
                              ctypes.c_size_t, _P]),
    "bb_mse_workspace_bytes": (ctypes.c_size_t, [_I64, _I64]),
    "bb_mse_loss_grad": (_S, [_P, _P, _P, _P, _I64, _I64, _I64, _P, ctypes.c_size_t, _P]),
    "bb_set_tuning": (_S, [ctypes.c_char_p, _I64]),
    "bb_get_tuning": (_I64, [ctypes.c_char_p]),
    "bb_status_string": (ctypes.c_char_p, [_S]),
    "bb_last_error_message": (ctypes.c_char_p, []),
}


class BandBatchError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libbandbatch.so is not built (expected at %s); run "
                               "`python -m paper_2107_05395_amd.build`" % LIB_PATH)
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status: int) -> None:
    if status != 0:
        msg = lib().bb_last_error_message().decode()
        raise BandBatchError(status, msg)


def dptr(arr) -> _D:
    """ctypes double* for a C-contiguous float64 numpy array."""
    return arr.ctypes.data_as(_D)
