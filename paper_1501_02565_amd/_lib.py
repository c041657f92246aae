"""ctypes declarations of the C ABI in ``include/epic.h``.

Loading fails loudly when ``libepic.so`` has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libepic.so")

# epic_status
OK, ERR_ARG, ERR_WORKSPACE, ERR_NO_MATCHES, ERR_HIP, ERR_BUDGET, ERR_CAPACITY, \
    ERR_CONVERGENCE, ERR_COST, ERR_INVARIANT = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
NW, LA = 0, 1

SYMBOLS = ["epic_create", "epic_destroy", "epic_workspace_bytes", "epic_interp",
           "epic_interp_batch", "epic_get_stats", "epic_debug_stages",
           "epic_strerror", "epic_last_error", "epic_validate", "epic_profile",
           "epic_stage_times", "epic_stage_name", "epic_graph_capture",
           "epic_graph_launch", "epic_graph_destroy", "epic_prune", "epic_image_cost",
           "epic_interp_image", "epic_interp_noalloc", "epic_interp_exact",
           "epic_refine_defaults", "epic_refine_bytes", "epic_refine", "epic_pass_visits"]


class Options(ctypes.Structure):
    _fields_ = [("connectivity", ctypes.c_int),
                ("la_weight_power", ctypes.c_int),
                ("precision", ctypes.c_int),
                ("fp64_route", ctypes.c_float),
                ("degenerate_tau", ctypes.c_double),
                ("tile_w", ctypes.c_int),
                ("tile_h", ctypes.c_int),
                ("geo_passes", ctypes.c_int),
                ("geo_threads", ctypes.c_int),
                ("debug_validate", ctypes.c_int),
                ("prune_px", ctypes.c_float)]


class Request(ctypes.Structure):
    _fields_ = [("cost", ctypes.c_void_p),
                ("H", ctypes.c_int), ("W", ctypes.c_int),
                ("matches", ctypes.c_void_p),
                ("N", ctypes.c_int), ("K", ctypes.c_int),
                ("a", ctypes.c_float), ("mode", ctypes.c_int),
                ("flow", ctypes.c_void_p)]


class Image(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p),
                ("H", ctypes.c_int), ("W", ctypes.c_int), ("channels", ctypes.c_int),
                ("cost", ctypes.c_void_p)]


class RefineParams(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_float), ("delta", ctypes.c_float),
                ("gamma", ctypes.c_float), ("kappa", ctypes.c_float),
                ("eps", ctypes.c_float), ("zeta", ctypes.c_float),
                ("omega", ctypes.c_float), ("fixed_point", ctypes.c_int),
                ("sor", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("n_used", ctypes.c_int),
                ("n_outside", ctypes.c_int), ("n_duplicate", ctypes.c_int),
                ("n_edges", ctypes.c_int), ("n_degenerate", ctypes.c_int),
                ("n_fp64_fits", ctypes.c_int), ("tile_visits", ctypes.c_int),
                ("n_bad_cost", ctypes.c_int), ("n_pruned", ctypes.c_int),
                ("n_invariant", ctypes.c_int)]


_lib = None


def load():
    """Loads libepic.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    # torch first: the library then binds the HIP runtime torch already
    # loaded (it shares torch's device memory and streams); loaded first, it
    # would bring in a second runtime that does not see torch's device
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P, i32, f32, f64, sz = (ctypes.c_void_p, ctypes.c_int, ctypes.c_float,
                            ctypes.c_double, ctypes.c_size_t)
    L.epic_create.argtypes = [i32, sz, ctypes.POINTER(Options)]
    L.epic_create.restype = P
    L.epic_destroy.argtypes = [P]
    L.epic_destroy.restype = None
    L.epic_workspace_bytes.argtypes = [i32, i32, i32, i32, i32, i32]
    L.epic_workspace_bytes.restype = sz
    L.epic_interp.argtypes = [P, P, i32, i32, P, i32, i32, f32, i32, P, P]
    L.epic_interp.restype = i32
    L.epic_interp_batch.argtypes = [P, ctypes.POINTER(Request), i32, P]
    L.epic_interp_batch.restype = i32
    L.epic_get_stats.argtypes = [P, i32, ctypes.POINTER(Stats)]
    L.epic_get_stats.restype = i32
    L.epic_debug_stages.argtypes = [P, P, i32, i32, P, i32, i32, f32, i32,
                                    P, P, P, P, P, i32, P, P, P, P, P, P]
    L.epic_debug_stages.restype = i32
    L.epic_prune.argtypes = [P, P, i32, i32, P, i32, i32, f32, f32, P, P, P]
    L.epic_prune.restype = i32
    L.epic_image_cost.argtypes = [ctypes.POINTER(Image), i32, f32, P]
    L.epic_image_cost.restype = i32
    L.epic_interp_image.argtypes = [P, P, i32, i32, i32, f32, P, i32, i32, f32, i32, P, P]
    L.epic_interp_image.restype = i32
    L.epic_interp_noalloc.argtypes = [P, i32, i32, P, i32, i32, f32, i32, P, P]
    L.epic_interp_noalloc.restype = i32
    L.epic_interp_exact.argtypes = [P, P, i32, i32, P, i32, i32, f32, i32, P, P]
    L.epic_interp_exact.restype = i32
    L.epic_pass_visits.argtypes = [P, ctypes.POINTER(ctypes.c_int), i32]
    L.epic_pass_visits.restype = i32
    L.epic_refine_defaults.argtypes = [ctypes.POINTER(RefineParams)]
    L.epic_refine_defaults.restype = None
    L.epic_refine_bytes.argtypes = [i32, i32, i32]
    L.epic_refine_bytes.restype = sz
    L.epic_refine.argtypes = [P, P, P, i32, i32, i32, P, P, ctypes.POINTER(RefineParams), P]
    L.epic_refine.restype = i32
    L.epic_strerror.argtypes = [i32]
    L.epic_strerror.restype = ctypes.c_char_p
    L.epic_last_error.argtypes = []
    L.epic_last_error.restype = ctypes.c_char_p
    L.epic_validate.argtypes = [P, i32, i32, P, i32, i32, f32, i32, P]
    L.epic_validate.restype = i32
    L.epic_profile.argtypes = [P, i32]
    L.epic_profile.restype = i32
    L.epic_stage_times.argtypes = [P, ctypes.POINTER(ctypes.c_float), i32, i32]
    L.epic_stage_times.restype = i32
    L.epic_stage_name.argtypes = [i32]
    L.epic_stage_name.restype = ctypes.c_char_p
    L.epic_graph_capture.argtypes = [P, ctypes.POINTER(Request), i32]
    L.epic_graph_capture.restype = P
    L.epic_graph_launch.argtypes = [P, P]
    L.epic_graph_launch.restype = i32
    L.epic_graph_destroy.argtypes = [P]
    L.epic_graph_destroy.restype = None
    _lib = L
    return L


def strerror(status: int) -> str:
    return load().epic_strerror(int(status)).decode()


class EpicError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        super().__init__(f"{where}: {strerror(status)} ({status})")
