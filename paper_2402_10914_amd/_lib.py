"""ctypes binding of the C ABI declared in ``include/dfweno.h`` (argument marshalling only).

The shared library ``libdfweno.so`` is built in-tree by ``paper_2402_10914_amd.build``; every step
of the method runs in its HIP kernels.  There is no fallback: if the library is missing the import
of the entry points raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdfweno.so")

DFW_OK, DFW_EINVAL, DFW_EDTYPE, DFW_EWORKSPACE, DFW_EHIP, DFW_ENONPHYS = range(6)
DFW_FLUX_LF, DFW_FLUX_GKS = 0, 1
DFW_TIME_S2O4, DFW_TIME_SSPRK3 = 0, 1
DFW_BC_PERIODIC, DFW_BC_TRANSMISSIVE = 0, 1
DFW_F64, DFW_F32 = 0, 1
KERNEL_KINDS = ["faces1", "update1", "faces2", "update2", "speed", "graph", "adj_faces1", "adj_faces2",
                "adj_gather", "rk_faces", "rk_update"]
DFW_ORDER_GRID, DFW_ORDER_LARGEST_FIRST, DFW_ORDER_INTERLEAVED = 0, 1, 2
DFW_NOALLOC_SCRATCH_BYTES = 64 << 20


class dfw_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32)]


class dfw_params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("dt_fixed", ctypes.c_double),
                ("alpha_thres", ctypes.c_double), ("d_h", ctypes.c_double), ("d_l", ctypes.c_double),
                ("eps_weno", ctypes.c_double), ("c1", ctypes.c_double), ("c2", ctypes.c_double),
                ("flux", ctypes.c_int32), ("tile", ctypes.c_int32), ("time_limiter", ctypes.c_int32),
                ("time_scheme", ctypes.c_int32), ("t_end", ctypes.c_double),
                ("switch_rule", ctypes.c_int32), ("componentwise", ctypes.c_int32), ("df_stage", ctypes.c_int32)]


class DFWError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dfweno status {status}: {msg}")
        self.status = status


_lib = None

_VP = ctypes.c_void_p
_GP = ctypes.POINTER(dfw_grid)
_PP = ctypes.POINTER(dfw_params)
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int32)

# name -> (restype, argtypes); kept in the order of include/dfweno.h
SIGNATURES = {
    "dfw_workspace_bytes": (ctypes.c_size_t, [_GP, ctypes.c_int32]),
    "dfw_run": (ctypes.c_int32, [_VP, _VP, _GP, _PP, ctypes.c_int32, ctypes.c_int32, _VP, ctypes.c_size_t,
                                 _VP, _DP, _IP, _VP]),
    "dfw_run_noalloc": (ctypes.c_int32, [_VP, _VP, _GP, _PP, ctypes.c_int32, ctypes.c_int32, _VP, _DP, _IP, _VP]),
    "dfw_max_speed": (ctypes.c_int32, [_VP, _GP, _PP, ctypes.c_int32, _VP, ctypes.c_size_t, _DP, _IP, _VP]),
    "dfw_rhs": (ctypes.c_int32, [_VP, _VP, _GP, _PP, ctypes.c_int32, ctypes.c_double, _VP, _VP, _VP, _VP,
                                 ctypes.c_size_t, _VP]),
    "dfw_batch_plan": (ctypes.c_int32, [_GP, ctypes.c_int32, _PP, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "dfw_batch_layout": (ctypes.c_int32, [_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                          ctypes.POINTER(ctypes.c_size_t)]),
    "dfw_batch_run": (ctypes.c_int32, [_VP, _VP, _VP, ctypes.c_int32, _VP, ctypes.c_size_t, ctypes.c_int32, _VP,
                                       _DP, _IP, _VP]),
    "dfw_batch_free": (None, [_VP]),
    "dfw_checkpoint_bytes": (ctypes.c_size_t, [_GP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "dfw_run_ckpt": (ctypes.c_int32, [_VP, _VP, _GP, _PP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP,
                                      ctypes.c_size_t, _VP, ctypes.c_size_t, _VP, _DP, _IP, _VP]),
    "dfw_adjoint_workspace_bytes": (ctypes.c_size_t, [_GP, ctypes.c_int32, ctypes.c_int32]),
    "dfw_adjoint": (ctypes.c_int32, [_GP, _PP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP, ctypes.c_size_t,
                                     _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "dfw_num_tiles": (ctypes.c_int32, []),
    "dfw_tile_shape": (ctypes.c_int32, [ctypes.c_int32, _IP, _IP]),
    "dfw_profile": (ctypes.c_int32, [ctypes.c_int32]),
    "dfw_profile_read": (ctypes.c_int32, [_DP, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
    "dfw_last_error": (ctypes.c_char_p, []),
}


def load(path: str = LIB_PATH):
    """Load libdfweno.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with paper_2402_10914_amd.build.build() "
                              "(the HIP path has no fallback)")
        L = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != DFW_OK:
        raise DFWError(status, load().dfw_last_error().decode())
