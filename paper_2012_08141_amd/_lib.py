"""ctypes binding of libatsparse.so (the C ABI declared in include/atsparse.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built --
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

from . import build as _build

c_int32, c_int64, c_uint32, c_float, c_void_p, c_size_t, c_double = (
    ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t,
    ctypes.c_double)

# ---- constants (mirrors include/atsparse.h; tests/test_capi.py checks them)
AT_OK, AT_E_INVALID, AT_E_CAPACITY, AT_E_HIP, AT_E_UNSUPPORTED, AT_E_STATE = 0, -1, -2, -3, -4, -5
AT_ROOT_BITMASK, AT_ROOT_POINTER = 0, 1
AT_COORD_VOXEL, AT_COORD_BLOCK = 0, 1
AT_OP_LAP_UPDATE, AT_OP_AXPY, AT_OP_JACOBI, AT_OP_COPY, AT_OP_FILL, AT_OP_INC = 1, 2, 3, 4, 5, 6
AT_OP_DIFFUSE, AT_OP_DIFFUSE_ADJ, AT_OP_NORMALISE = 7, 8, 9
AT_OP_ADVECT = 10
AT_OP_MACCORMACK = 11
AT_OP_MPM_GRID = 12
AT_ACT_PER_NODE, AT_ACT_PER_BLOCK, AT_ACT_NONE = 0, 1, 2
AT_TASK_ACTIVATE, AT_TASK_LISTGEN, AT_TASK_STENCIL, AT_TASK_ADVECT, AT_TASK_P2G, AT_TASK_G2P = 1, 2, 3, 4, 5, 6
AT_TASK_RESTRICT, AT_TASK_PROLONG = 7, 8
AT_TASK_P2G_MLS, AT_TASK_G2P_APIC = 9, 10
AT_TASKF_LOOP_UNIQUE = 1
AT_OPT_LGR, AT_OPT_AD, AT_OPT_FUSE, AT_OPT_DSE, AT_OPT_ALL = 1, 2, 4, 8, 15
AT_PLAN_MAX_MEMBERS = 16
AT_OPTION_MAX_FUSE_PER_TASK, AT_OPTION_FLUSH_PERIOD, AT_OPTION_OPT_FLAGS, AT_OPTION_PLAN_CACHE = 1, 2, 3, 4
AT_OPTION_STRUCT_FOR_WORKGROUPS = 5
AT_OPTION_STRUCT_FOR_KERNEL = 6
AT_OPTION_BATCH_WAVES = 7
AT_OPTION_G2P_BINS = 8
AT_OPTION_BIN_REUSE = 9
AT_OPTION_FUSE_BATCH = 10
AT_OPTION_GRAPHS = 11
AT_OPTION_GRAPHS_CACHED = 12
AT_OPTION_ASYNC = 13
AT_OPTION_VARIANTS = 14
AT_OPTION_VARIANTS_LOADED = 15
AT_OPTION_VERIFY_DEMOTED = 16
AT_STATIC_MAX_PARTICLES, AT_STATIC_MAX_CELLS = 1048576, 262144


class AtGridDesc(ctypes.Structure):
    _fields_ = [("n", c_int32 * 3), ("root_kind", c_int32), ("channels", c_int32), ("capacity_blocks", c_int32),
                ("particle_capacity", c_int32)]


class AtTimingEntry(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("op", c_int32), ("members", c_int32), ("reserved", c_int32),
                ("launches", c_int64), ("total_us", ctypes.c_double)]


class AtGridInfo(ctypes.Structure):
    _fields_ = [("n", c_int32), ("R", c_int32), ("root_kind", c_int32), ("channels", c_int32),
                ("capacity_blocks", c_int32), ("list_capacity", c_int32), ("ncells", c_int64),
                ("bytes", c_size_t)]


class AtTask(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("op", c_int32), ("flags", c_uint32), ("reserved", c_int32),
                ("grid", c_void_p), ("grid2", c_void_p), ("ch", c_int32 * 8), ("param", c_float * 8),
                ("ext", c_void_p * 4), ("n", c_int64)]


class AtStats(ctypes.Structure):
    _fields_ = [("tasks_in", c_int64), ("tasks_launched", c_int64), ("dispatches", c_int64),
                ("listgens_removed", c_int64), ("activations_demoted", c_int64), ("fusions", c_int64),
                ("stores_eliminated", c_int64), ("plan_cache_hits", c_int64), ("optimizer_us", c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class AtBatchDesc(ctypes.Structure):
    _fields_ = [("n", c_int32), ("max_grids", c_int32), ("pool_blocks", c_int32), ("reserved", c_int32)]


class AtBatchViews(ctypes.Structure):
    _fields_ = [("clock", c_void_p), ("count", c_void_p), ("window", c_void_p), ("roots", c_void_p),
                ("work", c_void_p), ("x", c_void_p), ("xn", c_void_p), ("b", c_void_p)]


class AtBatchAdmit(ctypes.Structure):
    _fields_ = [("cells", c_void_p), ("b", c_void_p), ("slots", c_void_p), ("gid", c_int32), ("nblocks", c_int32),
                ("iters", c_int32), ("reserved", c_int32)]


class AtBatchRetire(ctypes.Structure):
    _fields_ = [("gid", c_int32), ("reserved", c_int32), ("x_out", c_void_p)]


class AtPlanEntry(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("nmembers", c_int32), ("members", c_int32 * AT_PLAN_MAX_MEMBERS),
                ("check_activation", c_int32), ("activation_mode", c_int32), ("dropped", c_uint32),
                ("keep", c_uint32 * AT_PLAN_MAX_MEMBERS)]


_P = c_void_p
_SIGS = {
    "at_grid_footprint": (c_int32, [ctypes.POINTER(AtGridDesc), ctypes.POINTER(c_size_t)]),
    "at_grid_create": (c_int32, [ctypes.POINTER(AtGridDesc), _P, c_size_t, _P, ctypes.POINTER(_P)]),
    "at_grid_destroy": (c_int32, [_P]),
    "at_grid_views": (c_int32, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    "at_grid_get_info": (c_int32, [_P, ctypes.POINTER(AtGridInfo)]),
    "at_grid_clear": (c_int32, [_P, _P]),
    "at_device_status": (c_int32, [_P, _P, c_int32, ctypes.POINTER(c_int32)]),
    "at_active_count": (c_int32, [_P, _P, ctypes.POINTER(c_int64)]),
    "at_activate": (c_int32, [_P, _P, c_int64, c_int32, _P]),
    "at_listgen": (c_int32, [_P, _P]),
    "at_run_stencil": (c_int32, [_P, c_int32, ctypes.POINTER(c_int32), ctypes.POINTER(c_float), c_int32, _P]),
    "at_advect": (c_int32, [_P, _P, c_int64, c_float, _P]),
    "at_p2g": (c_int32, [_P, _P, _P, _P, c_int64, c_float, ctypes.POINTER(c_int32), c_int32, _P]),
    "at_p2g_static": (c_int32, [_P, _P, _P, _P, c_int64, c_float, ctypes.POINTER(c_int32), c_int32, _P]),
    "at_p2g_mls": (c_int32, [_P, _P, _P, _P, _P, c_int64, c_float, c_float, c_float, c_float, c_float, c_float,
                             ctypes.POINTER(c_int32), c_int32, _P]),
    "at_g2p_apic": (c_int32, [_P, _P, _P, _P, c_int64, c_float, ctypes.POINTER(c_int32), _P]),
    "at_g2p": (c_int32, [_P, _P, _P, c_int64, c_float, ctypes.POINTER(c_int32), _P]),
    "at_scatter_blocks": (c_int32, [_P, c_int32, _P, _P, c_int64, _P]),
    "at_gather_blocks": (c_int32, [_P, c_int32, _P, _P, c_int64, _P]),
    "at_run_sequence": (c_int32, [ctypes.POINTER(AtTask), c_int32, c_uint32, ctypes.POINTER(AtStats), _P]),
    "at_plan_sequence": (c_int32, [ctypes.POINTER(AtTask), c_int32, c_uint32, ctypes.POINTER(AtPlanEntry), c_int32,
                                   ctypes.POINTER(c_int32), ctypes.POINTER(AtStats)]),
    "at_enqueue": (c_int32, [ctypes.POINTER(AtTask), _P]),
    "at_flush": (c_int32, [ctypes.POINTER(AtStats), _P]),
    "at_set_option": (c_int32, [c_int32, c_int64]),
    "at_timing_enable": (c_int32, [c_int32]),
    "at_timing_collect": (c_int32, [ctypes.POINTER(AtTimingEntry), c_int32, ctypes.POINTER(c_int32)]),
    "at_get_option": (c_int32, [c_int32, ctypes.POINTER(c_int64)]),
    "at_engine_reset": (c_int32, []),
    "at_engine_sync": (c_int32, [ctypes.POINTER(AtStats)]),
    "at_variant_prepare": (c_int32, [ctypes.POINTER(AtTask), c_int32, ctypes.c_char_p, c_size_t,
                                     ctypes.POINTER(c_size_t)]),
    "at_ext_modified": (c_int32, [_P]),
    "at_batch_footprint": (c_int32, [ctypes.POINTER(AtBatchDesc), ctypes.POINTER(c_size_t)]),
    "at_batch_create": (c_int32, [ctypes.POINTER(AtBatchDesc), _P, c_size_t, _P, ctypes.POINTER(_P)]),
    "at_batch_destroy": (c_int32, [_P]),
    "at_batch_get_views": (c_int32, [_P, ctypes.POINTER(AtBatchViews)]),
    "at_batch_jacobi": (c_int32, [_P, c_int32, c_int32, _P]),
    "at_batch_update": (c_int32, [_P, ctypes.POINTER(AtBatchRetire), c_int32, ctypes.POINTER(AtBatchAdmit), c_int32,
                                  _P]),
    "at_dispatch_count": (c_int64, []),
    "at_last_error": (ctypes.c_char_p, []),
    "at_version": (ctypes.c_char_p, []),
}

_LIB = None


class AtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("atsparse error %d: %s" % (code, msg))
        self.code = code


def lib() -> ctypes.CDLL:
    """The loaded library.  Raises if it was never built (no fallback)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            raise RuntimeError("libatsparse.so is missing (%s); build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`" % _build.LIB)
        L = ctypes.CDLL(_build.LIB)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(code: int) -> int:
    if code != AT_OK:
        raise AtError(code, lib().at_last_error().decode())
    return code


def declared_symbols(header_path: str) -> list:
    """Names of the functions include/atsparse.h declares."""
    import re
    txt = open(header_path).read()
    return sorted(set(re.findall(r"\b(at_[a-z0-9_]+)\s*\(", txt)) - {"at_status"})
