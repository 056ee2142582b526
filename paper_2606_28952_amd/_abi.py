"""ctypes declarations of the C ABI in include/pbs.h (argument marshalling only).

The shared library is loaded from the package directory.  If it is missing
the import of any GPU entry point fails with an error: there is no CPU
fallback.
"""

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_uint8, c_uint32, c_uint64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpbs.so")

PBS_OK = 0
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_RANGE", 3: "ERR_ALLOC", 4: "ERR_DEVICE", 5: "ERR_UNSUPPORTED"}
PBS_C128 = 0
PBS_C64 = 1

_vp = c_void_p
# name -> (restype, argtypes); the order follows include/pbs.h
SIGNATURES = {
    "pbs_last_error": (c_char_p, []),
    "pbs_abi_version": (c_int32, []),
    "pbs_pauli_mul": (c_int32, [c_uint32, c_uint64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pbs_sum_create": (c_int32, [c_uint32, c_uint64, _vp, _vp, _vp, _vp, POINTER(_vp)]),
    "pbs_sum_info": (c_int32, [_vp, POINTER(c_uint32), POINTER(c_uint64), POINTER(c_int32)]),
    "pbs_sum_read": (c_int32, [_vp, _vp, _vp, _vp, _vp]),
    "pbs_sum_view": (c_int32, [_vp, POINTER(c_uint32), POINTER(c_uint64), POINTER(_vp), POINTER(_vp),
                               POINTER(_vp)]),
    "pbs_sum_destroy": (None, [_vp]),
    "pbs_pauli_canonicalize": (c_int32, [_vp, c_double, _vp]),
    "pbs_pauli_sum_mul": (c_int32, [_vp, _vp, c_double, _vp, POINTER(_vp)]),
    "pbs_jw_transform": (c_int32, [c_uint32, _vp, _vp, c_double, c_double, c_double, _vp, POINTER(_vp)]),
    "pbs_group_by_xmask": (c_int32, [_vp, _vp, POINTER(_vp)]),
    "pbs_grouped_info": (c_int32, [_vp, POINTER(c_uint32), POINTER(c_uint64), POINTER(c_uint64)]),
    "pbs_grouped_read": (c_int32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "pbs_grouped_destroy": (None, [_vp]),
    "pbs_space_full": (c_int32, [c_uint32, POINTER(_vp)]),
    "pbs_space_sector": (c_int32, [c_uint32, c_uint32, c_uint32, _vp, POINTER(_vp)]),
    "pbs_space_dim": (c_int32, [_vp, POINTER(c_uint64)]),
    "pbs_space_shape": (c_int32, [_vp, POINTER(c_uint32), POINTER(c_uint32), POINTER(c_uint32),
                                  POINTER(c_uint64), POINTER(c_uint64)]),
    "pbs_space_rank": (c_int32, [_vp, c_uint64, _vp, _vp, _vp]),
    "pbs_space_unrank": (c_int32, [_vp, c_uint64, _vp, _vp, _vp]),
    "pbs_space_destroy": (None, [_vp]),
    "pbs_apply_pauli_sum": (c_int32, [_vp, _vp, c_int32, _vp, _vp, _vp]),
    "pbs_expval_workspace_bytes": (c_int32, [_vp, POINTER(c_uint64)]),
    "pbs_expval": (c_int32, [_vp, _vp, c_int32, _vp, _vp, _vp, _vp, c_uint64, _vp]),
    "pbs_expval_noalloc": (c_int32, [_vp, _vp, c_int32, _vp, _vp, _vp, _vp]),
    "pbs_apply_pauli_sum_rows": (c_int32, [_vp, _vp, c_int32, _vp, _vp, c_uint64, c_uint64, _vp]),
    "pbs_expval_rows": (c_int32, [_vp, _vp, c_int32, _vp, _vp, c_uint64, c_uint64, _vp, _vp, c_uint64, _vp]),
    "pbs_grouped_factor": (c_int32, [_vp, _vp, _vp]),
    "pbs_grouped_set_factored": (c_int32, [_vp, c_int32]),
    "pbs_grouped_factor_info": (c_int32, [_vp, _vp]),
    "pbs_batch_create": (c_int32, [c_uint32, _vp, _vp, c_int32, _vp, _vp, POINTER(_vp)]),
    "pbs_batch_run": (c_int32, [_vp, _vp, _vp]),
    "pbs_batch_set_config": (c_int32, [_vp, c_uint32]),
    "pbs_batch_tune": (c_int32, [_vp, c_uint32, _vp, POINTER(c_uint32), POINTER(c_double)]),
    "pbs_batch_info": (c_int32, [_vp, POINTER(c_uint32), POINTER(c_double), POINTER(c_uint32)]),
    "pbs_batch_destroy": (None, [_vp]),
    "pbs_krylov_workspace_bytes": (c_int32, [_vp, c_int32, c_uint32, POINTER(c_uint64)]),
    "pbs_krylov_step": (c_int32, [_vp, _vp, c_int32, _vp, c_double, c_uint32, _vp, c_uint64, _vp, _vp]),
    "pbs_vqe_create": (c_int32, [_vp, c_uint32, c_uint32, _vp, _vp, c_uint64, c_int32, _vp, POINTER(_vp)]),
    "pbs_vqe_energy_grad": (c_int32, [_vp, _vp, _vp, _vp, _vp]),
    "pbs_vqe_state": (c_int32, [_vp, _vp, _vp]),
    "pbs_vqe_minimize": (c_int32, [_vp, _vp, c_uint32, c_double, c_double, _vp, POINTER(c_double),
                                   POINTER(c_uint32), POINTER(c_uint32), POINTER(c_int32)]),
    "pbs_vqe_tune": (c_int32, [_vp, c_uint32, _vp, POINTER(c_uint32), POINTER(c_double)]),
    "pbs_vqe_set_config": (c_int32, [_vp, c_uint32]),
    "pbs_vqe_set_groups": (c_int32, [_vp, c_uint32, c_uint32]),
    "pbs_vqe_info": (c_int32, [_vp, POINTER(c_uint32), POINTER(c_uint32)]),
    "pbs_vqe_destroy": (None, [_vp]),
    "pbs_lbfgs_minimize": (c_int32, [c_uint32, _vp, _vp, _vp, c_uint32, c_uint32, c_double, c_double,
                                     POINTER(c_double), POINTER(c_uint32), POINTER(c_uint32), POINTER(c_int32)]),
    "pbs_mlp_param_count": (c_int32, [c_uint32, c_uint32, POINTER(c_uint64)]),
    "pbs_mlp_create": (c_int32, [c_uint32, c_uint32, c_uint32, _vp, _vp, POINTER(_vp)]),
    "pbs_mlp_set_params": (c_int32, [_vp, _vp, _vp]),
    "pbs_mlp_get_params": (c_int32, [_vp, _vp, _vp]),
    "pbs_mlp_forward": (c_int32, [_vp, c_uint32, _vp, _vp, _vp]),
    "pbs_mlp_loss_grad": (c_int32, [_vp, c_uint32, _vp, _vp, _vp, _vp, _vp]),
    "pbs_mlp_train": (c_int32, [_vp, c_uint32, _vp, _vp, c_uint32, c_float, _vp, _vp]),
    "pbs_mlp_destroy": (None, [_vp]),
}

_LIB = None


class PbsError(RuntimeError):
    def __init__(self, func, status, message):
        super().__init__(f"{func} failed with {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.func = func


def lib():
    """The loaded library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = handle
    return _LIB


def call(name, *args):
    """Calls a status-returning entry point and raises PbsError on failure."""
    fn = getattr(lib(), name)
    status = fn(*args)
    if status != PBS_OK:
        msg = lib().pbs_last_error().decode(errors="replace")
        raise PbsError(name, status, msg)
    return status
