"""ctypes binding of ``libbtdf.so`` (the C ABI of include/btdf.h).

Argument marshalling only: every call forwards to the library of the same
name. The library must be built (``python -m paper_1806_09403_amd.build``);
there is no fallback of any kind when it is missing.

torch is imported before the library is loaded so that the process has a
single HIP runtime (torch ships one with the same soname).
"""
import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# BTDF_LIBRARY may name another build of the same library (the host
# sanitizer build of the tests); by default the in-tree libbtdf.so
LIB_PATH = os.environ.get("BTDF_LIBRARY") or os.path.join(PKG, "libbtdf.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EUNSTABLE = 0, -1, -2, -3, -4, -5
PERIODIC, VELOCITY_INLET, ZERO_GRADIENT_OUTLET, BOUNCEBACK_WALL = 0, 1, 2, 3
FREE_SLIP_WALL, CONVECTIVE_OUTLET = 4, 5
LINEAR2, ROMA3, PESKIN4, COS4 = 2, 3, 4, 5
OPT_LBM_VARIANT, OPT_NUM_VARIANTS, OPT_GRAPH_CHUNK, OPT_XCD_REMAP, OPT_TILE_X, OPT_TILE_Y = 1, 2, 3, 4, 5, 6
OPT_ROW_PAD, OPT_PLANE_PAD, OPT_INTERIOR_PATH, OPT_FORCED_TILES = 7, 8, 9, 11
OPT_MASK_UNSTABLE = 12
OPT_ROW_ALIGN = 13
OPT_FORCING_PASSES = 14
OPT_FORCING_METHOD = 15
OPT_TEMPORAL_BLOCKING, OPT_FUSED_TILES, OPT_STEPS_PER_PASS = 16, 17, 18
OPT_EDGE_TILES, OPT_EDGE_FUSED_TILES, OPT_FUSED_NODES = 20, 21, 22
NOALLOC_MAX_MARKERS = 262144
FORCING_DIRECT, FORCING_IMPLICIT, FORCING_RKPM = 0, 1, 2

_NAMES = {OK: "BTDF_OK", EINVAL: "BTDF_EINVAL", ENOMEM: "BTDF_ENOMEM", EDEVICE: "BTDF_EDEVICE",
          ESTATE: "BTDF_ESTATE", EUNSTABLE: "BTDF_EUNSTABLE"}


class BtdfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_NAMES.get(code, str(code)), msg))
        self.code = code


class BtdfUnstable(BtdfError):
    pass


class btdf_grid(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("bc_west", ctypes.c_int32), ("bc_east", ctypes.c_int32),
        ("bc_south", ctypes.c_int32), ("bc_north", ctypes.c_int32),
        ("inflow_ux", ctypes.c_double), ("inflow_uy", ctypes.c_double),
        ("body_force_x", ctypes.c_double), ("body_force_y", ctypes.c_double),
        ("rho0", ctypes.c_double), ("ux0", ctypes.c_double), ("uy0", ctypes.c_double),
        ("precision", ctypes.c_int32), ("history_capacity", ctypes.c_int32),
        ("hip_stream", ctypes.c_void_p), ("flags", ctypes.c_uint64),
    ]


_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64

# name -> (restype, argtypes)
class btdf_gradients(ctypes.Structure):
    _fields_ = [("populations", ctypes.POINTER(ctypes.c_double)), ("inflow", ctypes.POINTER(ctypes.c_double)),
                ("body_force", ctypes.POINTER(ctypes.c_double)), ("marker_xy", ctypes.POINTER(ctypes.c_double)),
                ("marker_uv", ctypes.POINTER(ctypes.c_double)), ("centres", ctypes.POINTER(ctypes.c_double))]


SIGNATURES = {
    "btdf_last_error": (ctypes.c_char_p, []),
    "btdf_create": (ctypes.c_int, [ctypes.POINTER(btdf_grid), ctypes.c_double, ctypes.c_int,
                                   ctypes.c_double, ctypes.POINTER(_vp)]),
    "btdf_destroy": (ctypes.c_int, [_vp]),
    "btdf_workspace_bytes": (ctypes.c_size_t, [_vp]),
    "btdf_bind_workspace": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "btdf_set_stream": (ctypes.c_int, [_vp, _vp]),
    "btdf_add_body": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.POINTER(ctypes.c_int)]),
    "btdf_set_marker_velocity": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "btdf_step": (ctypes.c_int, [_vp, _i64]),
    "btdf_step_timed": (ctypes.c_int, [_vp, _i64, _dp, _dp]),
    "btdf_forces": (ctypes.c_int, [_vp, _dp, ctypes.c_int]),
    "btdf_force_history": (ctypes.c_int, [_vp, _dp, _i64, ctypes.POINTER(_i64)]),
    "btdf_init_equilibrium": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "btdf_get_macroscopic": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
    "btdf_get_populations": (ctypes.c_int, [_vp, _dp]),
    "btdf_set_populations": (ctypes.c_int, [_vp, _dp]),
    "btdf_get_populations_to": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "btdf_set_populations_from": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "btdf_get_marker_data": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp, _dp]),
    "btdf_marker_velocity": (ctypes.c_int, [_vp, _dp, _dp]),
    "btdf_marker_velocity_noalloc": (ctypes.c_int, [_vp, _dp, _dp]),
    "btdf_step_timed_split": (ctypes.c_int, [_vp, _i64, _dp]),
    "btdf_step_timed_pass": (ctypes.c_int, [_vp, _i64, _dp]),
    "btdf_set_body_motion": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "btdf_get_body_state": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "btdf_get_marker_positions": (ctypes.c_int, [_vp, _dp]),
    "btdf_state_bytes": (ctypes.c_size_t, [_vp]),
    "btdf_save": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "btdf_load": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "btdf_counts": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                   ctypes.POINTER(_i64)]),
    "btdf_set_option": (ctypes.c_int, [_vp, ctypes.c_int, _i64]),
    "btdf_get_option": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(_i64)]),
    "btdf_calibrate_thickening": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp, _dp]),
    "btdf_calibrate_thickening_markers": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double,
                                                         _dp, _dp]),
    "btdf_autotune": (ctypes.c_int, [_vp, _i64, ctypes.POINTER(ctypes.c_int)]),
    "btdf_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(btdf_grid), _dp,
                                         ctypes.POINTER(ctypes.c_int), _dp, ctypes.POINTER(_vp)]),
    "btdf_batch_destroy": (ctypes.c_int, [_vp]),
    "btdf_batch_case": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(_vp)]),
    "btdf_batch_add_body": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_int)]),
    "btdf_batch_workspace_bytes": (ctypes.c_size_t, [_vp]),
    "btdf_batch_bind_workspace": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "btdf_batch_set_stream": (ctypes.c_int, [_vp, _vp]),
    "btdf_batch_step": (ctypes.c_int, [_vp, _i64]),
    "btdf_batch_step_timed": (ctypes.c_int, [_vp, _i64, _dp, _dp]),
    "btdf_batch_status": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_i64)]),
    "btdf_batch_set_option": (ctypes.c_int, [_vp, ctypes.c_int, _i64]),
    "btdf_batch_get_option": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(_i64)]),
    "btdf_batch_autotune": (ctypes.c_int, [_vp, _i64, ctypes.POINTER(ctypes.c_int)]),
    "btdf_adjoint_workspace_bytes": (ctypes.c_size_t, [_vp, _i64, _i64]),
    "btdf_adjoint": (ctypes.c_int, [_vp, _i64, _i64, _dp, ctypes.POINTER(btdf_gradients), _vp, ctypes.c_size_t,
                                    _dp]),
}

_lib = None


def load():
    """Load libbtdf.so (after torch). Raises if the library has not been built."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  -- one HIP runtime per process: torch's
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbtdf.so is not built; run `python -m paper_1806_09403_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error():
    return load().btdf_last_error().decode(errors="replace")


def check(code):
    if code != OK:
        cls = BtdfUnstable if code == EUNSTABLE else BtdfError
        raise cls(code, last_error())
    return code


def dptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a
