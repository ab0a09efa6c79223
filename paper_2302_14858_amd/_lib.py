"""ctypes declarations of the C ABI in include/cfd.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcfd_mi355x.so")

CFD_OK, CFD_EINVAL, CFD_EGHOST, CFD_ESHAPE, CFD_ESINGULAR, CFD_ENOMEM, CFD_EDEVICE, CFD_EUNSUPPORTED = range(8)
STATUS_NAMES = ["CFD_OK", "CFD_EINVAL", "CFD_EGHOST", "CFD_ESHAPE", "CFD_ESINGULAR", "CFD_ENOMEM", "CFD_EDEVICE",
                "CFD_EUNSUPPORTED"]
CFD_F64, CFD_F32, CFD_MIXED_BF16 = 0, 1, 2
CFD_BOUNDARY_CLOSURE, CFD_BOUNDARY_PERIODIC = 0, 1
CFD_SCHED_PERSISTENT, CFD_SCHED_SPLIT_X, CFD_SCHED_XCD, CFD_SCHED_CONCURRENT = 1, 2, 4, 8


class cfd_block(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("ng", ctypes.c_int), ("h", ctypes.c_double * 3),
                ("boundary", ctypes.c_int * 3), ("in_offset", ctypes.c_longlong), ("out_offset", ctypes.c_longlong)]


class cfd_op(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_void_p), ("dir", ctypes.c_int), ("field", ctypes.c_int),
                ("vel_field", ctypes.c_int), ("dir2", ctypes.c_int), ("aux_field", ctypes.c_int)]


class cfd_plan_desc(ctypes.Structure):
    _fields_ = [("nblocks", ctypes.c_int), ("blocks", ctypes.POINTER(cfd_block)), ("nfields", ctypes.c_int),
                ("nops", ctypes.c_int), ("ops", ctypes.POINTER(cfd_op)), ("dtype", ctypes.c_int),
                ("device", ctypes.c_int), ("flags", ctypes.c_int)]


_vp = ctypes.c_void_p
_ip = ctypes.POINTER(ctypes.c_int)
_dp = ctypes.POINTER(ctypes.c_double)
_llp = ctypes.POINTER(ctypes.c_longlong)
_pp = ctypes.POINTER(ctypes.c_void_p)
_i, _d, _ll, _s = ctypes.c_int, ctypes.c_double, ctypes.c_longlong, ctypes.c_char_p

SIGNATURES = {
    "cfd_abi_version": (_i, []),
    "cfd_last_error": (_s, []),
    "cfd_scheme_named": (_i, [_s, _pp]),
    "cfd_scheme_design": (_i, [_i, _i, _i, _i, _d, _i, _i, _pp]),
    "cfd_scheme_create": (_i, [_i, _i, _i, _dp, _i, _dp, _i, _i, _dp, _pp]),
    "cfd_scheme_get": (_i, [_vp, _ip, _ip, _ip, _ip, _ip, _ip, _dp, _dp, _dp]),
    "cfd_scheme_design_biased": (_i, [ctypes.c_char, _i, _d, _i, _pp]),
    "cfd_scheme_get_biased": (_i, [_vp, _ip, _ip, _dp, _dp, _dp]),
    "cfd_scheme_get_embedded": (_i, [_vp, _dp, _ip]),
    "cfd_scheme_dissipation": (_i, [_i, _d, _pp]),
    "cfd_taylor_scheme": (_i, [_i, _i, _i, _i, _ip, _ip, _ip, _dp, _i, _ip]),
    "cfd_scheme_required_ghosts": (_i, [_vp, _i, _ip]),
    "cfd_scheme_destroy": (None, [_vp]),
    "cfd_plan_create": (_i, [ctypes.POINTER(cfd_plan_desc), _pp]),
    "cfd_plan_sizes": (_i, [_vp, _llp, _llp]),
    "cfd_plan_offsets": (_i, [_vp, _llp, _llp]),
    "cfd_plan_stats": (_i, [_vp, _ip, _llp]),
    "cfd_apply": (_i, [_vp, _vp, _vp, _vp]),
    "cfd_plan_capture_graph": (_i, [_vp, _vp, _vp, _vp]),
    "cfd_plan_launch_graph": (_i, [_vp, _vp]),
    "cfd_plan_autotune": (_i, [_vp, _vp, _vp, _vp, _s]),
    "cfd_plan_set_schedule": (_i, [_vp, _i, _i, _i, _i]),
    "cfd_plan_get_schedule": (_i, [_vp, _ip, _ip, _ip, _ip, _ip, _ip, _i]),
    "cfd_plan_get_flags": (_i, [_vp, _ip]),
    "cfd_plan_destroy": (None, [_vp]),
    "cfd_halo_exchange": (_i, [_vp, _vp, _i, _i, _i, _vp]),
    "cfd_plan_set_neighbors": (_i, [_vp, _vp]),
    "cfd_halo_exchange_table": (_i, [_vp, _vp, _vp]),
    "cfd_plan_set_neighbors_vc": (_i, [_vp, _vp]),
    "cfd_shared_node_average": (_i, [_vp, _vp, _i, _vp]),
    "cfd_axpby": (_i, [_i, _ll, _d, _vp, _d, _vp, _vp]),
    "cfd_xpcy": (_i, [_i, _ll, _vp, _d, _vp, _vp, _vp]),
    "cfd_wave_rk_stage": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _d, _d, _vp]),
    "cfd_wave_rk_stage_halo": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _d, _d, _i, _i, _i, _vp]),
    "cfd_wave_rk_stage_fused": (_i, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _d, _d, _i, _i, _i, _vp]),
    "cfd_debug_fail_alloc": (None, [_ll]),
    "cfd_debug_fail_capture": (None, [_i]),
    "cfd_plan_graph_status": (_i, [_vp, _ip]),
    "cfd_plan_count_nonfinite": (_i, [_vp, _vp, _vp, _llp]),
    "cfd_plan_set_iteration": (_i, [_vp, _i, _i, _i, _i]),
    "cfd_apply_block_noalloc": (_i, [_vp, ctypes.POINTER(cfd_block), _i, _i, _i, _i, _vp, _vp, _vp]),
}

_lib = None


class CfdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2302_14858_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != CFD_OK:
        raise CfdError(status, lib().cfd_last_error().decode())
