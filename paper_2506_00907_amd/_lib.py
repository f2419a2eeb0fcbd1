"""ctypes declarations of include/lbm.h and loading of the in-tree liblbm.so.

Argument marshalling only: every step of the sweep runs in the HIP library.
Importing this module never falls back to anything else; if the library is
missing it raises.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; LBM_LIBRARY names another build of the same sources
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(_PKG, "liblbm.so")

LBM_NBUF = 8
STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ESIZE", -3: "LBM_EDEVICE", -4: "LBM_EUNSTABLE",
          -5: "LBM_ESTATE"}
LBM_F64, LBM_F32, LBM_F16, LBM_BF16 = 1, 2, 3, 4
LBM_REDUCE_STATIC_MAX_BLOCKS = 131072  # lbm_reduce_static: 256-node blocks its scratch holds


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class lbm_params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("periodic", C.c_int32 * 3),
                ("fluid", C.c_int32), ("scalar", C.c_int32), ("magnetic", C.c_int32),
                ("mag_ncomp", C.c_int32), ("mag_comp", C.c_int32 * 3), ("storage", C.c_int32),
                ("scalar_ncomp", C.c_int32), ("tau_f", C.c_double), ("tau_c", C.c_double),
                ("tau_m", C.c_double), ("rho0", C.c_double), ("C0", C.c_double), ("mu", C.c_double),
                ("B_ext", C.c_double * 3), ("accel", C.c_double * 3), ("store_scale", C.c_double * 3),
                ("wall_omega", C.c_double), ("tau_cs", C.c_double * 2)]


class lbm_link(C.Structure):
    _fields_ = [("node", C.c_uint32), ("enode", C.c_uint32), ("field", C.c_uint8), ("dir", C.c_uint8),
                ("kind", C.c_uint8), ("comp", C.c_uint8), ("flags", C.c_uint8),
                ("cross_comp", C.c_uint8 * 2), ("pad", C.c_uint8), ("d", C.c_double), ("value", C.c_double), ("a1", C.c_double),
                ("a3", C.c_double), ("weight", C.c_double), ("u_w", C.c_double * 3), ("quad", C.c_double),
                ("cross", C.c_double)]


class lbm_bc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("u_given", C.c_int32), ("profile_axis", C.c_int32),
                ("profile_len", C.c_int32), ("alt", C.c_int32), ("law", C.c_int32),
                ("value", C.c_double), ("a1", C.c_double), ("a3", C.c_double), ("quad", C.c_double),
                ("profile", C.POINTER(C.c_double)), ("k", C.c_double), ("phi_eq", C.c_double),
                ("c_w", C.c_double), ("H", C.c_double), ("cross_comp", C.c_int32 * 2),
                ("cross", C.c_double)]


class lbm_boundary(C.Structure):
    _fields_ = [("type", C.c_int32), ("axis", C.c_int32), ("side", C.c_int32), ("is_open", C.c_int32),
                ("q", C.c_double), ("center", C.c_double * 3), ("radius", C.c_double),
                ("u_w", C.c_double * 3), ("f", lbm_bc), ("h", lbm_bc), ("g", lbm_bc * 3),
                ("u_osc", C.c_int32), ("reserved", C.c_int32), ("d_scheme", C.c_double),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("h_more", lbm_bc * 2)]


class lbm_batch_config(C.Structure):
    _fields_ = [("mode", C.c_int32), ("block", C.c_int32), ("steps_per_launch", C.c_int32),
                ("graph_steps", C.c_int32)]


class lbm_nn_desc(C.Structure):
    _fields_ = [("batch", C.c_int32), ("size", C.c_int32), ("in_ch", C.c_int32), ("out_ch", C.c_int32),
                ("width", C.c_int32), ("precision", C.c_int32)]


LBM_BATCH_TILED, LBM_BATCH_RESIDENT = 1, 2
# lbm_flux_law
LAWS = {"coef": 0, "robin": 1, "reaction": 2, "shercliff": 3}
ITEM_STATUS = {0: "active", 1: "steady", 2: "nonfinite", 3: "disabled"}

# every entry point declared in include/lbm.h: name -> (restype, argtypes)
_VP = C.c_void_p
SIGNATURES = {
    "lbm_version": (C.c_char_p, []),
    "lbm_lattice_table": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), _VP, _VP, C.POINTER(C.c_double), _VP]),
    "lbm_build_links": (C.c_int, [C.POINTER(lbm_params), C.POINTER(lbm_boundary), C.c_int32, _VP, _VP,
                                  C.c_size_t, C.POINTER(C.c_size_t)]),
    "lbm_required_bytes": (C.c_size_t, [C.POINTER(lbm_params), C.c_size_t, C.POINTER(C.c_size_t)]),
    "lbm_create": (C.c_int, [C.POINTER(lbm_params), C.c_size_t, C.POINTER(_VP), _VP, C.POINTER(_VP)]),
    "lbm_set_geometry": (C.c_int, [_VP, _VP]),
    "lbm_set_links": (C.c_int, [_VP, _VP, C.c_size_t]),
    "lbm_init": (C.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "lbm_step": (C.c_int, [_VP, C.c_int64]),
    "lbm_step_prepare": (C.c_int, [_VP, C.c_int64]),
    "lbm_step_stats": (C.c_int, [_VP, C.POINTER(C.c_int64)]),
    "lbm_set_step_overlap": (C.c_int, [_VP, C.c_int32]),
    "lbm_timing_scratch_bytes": (C.c_size_t, [_VP]),
    "lbm_step_timed": (C.c_int, [_VP, C.c_int64, _VP, C.c_size_t, C.POINTER(C.c_float)]),
    "lbm_read_moments": (C.c_int, [_VP, _VP, C.c_int32]),
    "lbm_read_populations": (C.c_int, [_VP, C.c_int32, _VP]),
    "lbm_reduce": (C.c_int, [_VP, C.POINTER(C.c_double)]),
    "lbm_reduce_static": (C.c_int, [_VP, C.POINTER(C.c_double)]),
    "lbm_boundary_flux": (C.c_int, [_VP, C.POINTER(C.c_double)]),
    "lbm_boundary_flux_scalar": (C.c_int, [_VP, C.POINTER(C.c_double)]),
    "lbm_read_normalised": (C.c_int, [_VP, C.c_int32, C.c_double, _VP]),
    "lbm_state_bytes": (C.c_size_t, [_VP]),
    "lbm_save": (C.c_int, [_VP, _VP]),
    "lbm_load": (C.c_int, [_VP, _VP]),
    "lbm_stream_bandwidth": (C.c_int, [C.c_int32, _VP, _VP, C.c_size_t, C.c_int32, C.c_int32, _VP,
                                       C.POINTER(C.c_float)]),
    "lbm_time": (C.c_int64, [_VP]),
    "lbm_set_stream": (C.c_int, [_VP, _VP]),
    "lbm_last_error": (C.c_char_p, [_VP]),
    "lbm_destroy": (None, [_VP]),
    "lbm_batch_required_bytes": (C.c_size_t, [C.c_int32, C.POINTER(lbm_params), C.POINTER(C.c_size_t),
                                              C.POINTER(C.c_size_t)]),
    "lbm_batch_create": (C.c_int, [C.c_int32, C.POINTER(lbm_params), C.POINTER(C.c_size_t), C.POINTER(_VP), _VP,
                                   C.POINTER(_VP)]),
    "lbm_batch_item": (_VP, [_VP, C.c_int32]),
    "lbm_batch_set_active": (C.c_int, [_VP, _VP]),
    "lbm_batch_configure": (C.c_int, [_VP, C.POINTER(lbm_batch_config)]),
    "lbm_batch_get_config": (C.c_int, [_VP, C.POINTER(lbm_batch_config)]),
    "lbm_batch_step": (C.c_int, [_VP, C.c_int64]),
    "lbm_batch_run": (C.c_int, [_VP, C.c_double, C.c_int32, C.c_int64, C.POINTER(C.c_int64),
                                C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "lbm_batch_tune": (C.c_int, [_VP, C.c_int64, C.POINTER(lbm_batch_config), C.POINTER(lbm_batch_config),
                                 C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32)]),
    "lbm_batch_last_error": (C.c_char_p, [_VP]),
    "lbm_batch_destroy": (None, [_VP]),
    "lbm_nn_required_bytes": (C.c_size_t, [C.POINTER(lbm_nn_desc), C.POINTER(C.c_size_t)]),
    "lbm_nn_create": (C.c_int, [C.POINTER(lbm_nn_desc), C.POINTER(_VP), _VP, C.POINTER(_VP)]),
    "lbm_nn_num_params": (C.c_int64, [_VP]),
    "lbm_nn_set_params": (C.c_int, [_VP, _VP]),
    "lbm_nn_get_params": (C.c_int, [_VP, _VP]),
    "lbm_nn_forward": (C.c_int, [_VP, C.c_int32, _VP, _VP]),
    "lbm_nn_backward": (C.c_int, [_VP, _VP, _VP, C.POINTER(C.c_double)]),
    "lbm_nn_get_grads": (C.c_int, [_VP, _VP]),
    "lbm_nn_adam_step": (C.c_int, [_VP, C.c_float, C.c_float, C.c_float, C.c_float]),
    "lbm_nn_last_error": (C.c_char_p, [_VP]),
    "lbm_nn_destroy": (None, [_VP]),
}

_lib = None


def lib() -> C.CDLL:
    """The loaded liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2506_00907_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code: int, ctx=None, what: str = ""):
    if code != 0:
        msg = lib().lbm_last_error(ctx).decode() if ctx else what
        raise LbmError(code, msg or what)
