"""The C ABI: the library loads, exports every function include/atsparse.h
declares, its constants match the Python binding, and argument validation
rejects bad calls without touching a device (host only)."""
import ctypes
import os
import re

import pytest

from paper_2012_08141_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "atsparse.h")


def test_exports_every_declared_symbol():
    lib = L.lib()
    names = L.declared_symbols(HEADER)
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_constants_match_header():
    txt = open(HEADER).read()
    defs = dict(re.findall(r"#define\s+(AT_[A-Z0-9_]+)\s+(-?\d+)u?\b", txt))
    assert len(defs) > 30
    for name, val in defs.items():
        assert hasattr(L, name), name
        assert getattr(L, name) == int(val), name


def test_struct_layouts():
    # at_task: 4 int32, 2 pointers, 8 int32, 8 float, 4 pointers, int64
    assert ctypes.sizeof(L.AtTask) == 16 + 16 + 32 + 32 + 32 + 8
    assert ctypes.sizeof(L.AtStats) == 8 * 9
    assert ctypes.sizeof(L.AtGridDesc) == 28
    assert ctypes.sizeof(L.AtPlanEntry) == 4 * (2 + L.AT_PLAN_MAX_MEMBERS + 3 + L.AT_PLAN_MAX_MEMBERS)


def _desc(n, kind=L.AT_ROOT_BITMASK, ch=2, cap=0):
    return L.AtGridDesc((n, n, n), kind, ch, cap, 0)


def test_footprint_layout_and_validation():
    lib = L.lib()
    b = ctypes.c_size_t()
    d = _desc(64)
    assert lib.at_grid_footprint(ctypes.byref(d), ctypes.byref(b)) == L.AT_OK
    # header 256 + scan flags 8 KiB + bits 256 + list 512 records * 32 B + 2 channels * 512 blocks * 2 KiB
    assert b.value == 256 + 8192 + 256 + 512 * 32 + 2 * 512 * 2048
    d = _desc(64, L.AT_ROOT_POINTER, 3, 100)
    assert lib.at_grid_footprint(ctypes.byref(d), ctypes.byref(b)) == L.AT_OK
    assert b.value == 256 + 8192 + 256 + 2048 + 3328 + 3 * 100 * 2048   # list: 100 records, 256-aligned
    for bad in (_desc(60), _desc(0), _desc(64, 7), _desc(64, L.AT_ROOT_BITMASK, 0),
                _desc(64, L.AT_ROOT_POINTER, 1, 0), _desc(64, L.AT_ROOT_POINTER, 1, 513)):
        assert lib.at_grid_footprint(ctypes.byref(bad), ctypes.byref(b)) == L.AT_E_INVALID
        assert lib.at_last_error()
    nc = L.AtGridDesc((64, 64, 32), 0, 1, 0, 0)
    assert lib.at_grid_footprint(ctypes.byref(nc), ctypes.byref(b)) == L.AT_E_UNSUPPORTED
    # particle binning workspace: 3 cell arrays (count, first, bins of 16 B) + 44 B per particle
    # (key and rank 8 B, record 32 B, outlier list 4 B)
    d = L.AtGridDesc((64, 64, 64), L.AT_ROOT_POINTER, 3, 100, 1000)
    assert lib.at_grid_footprint(ctypes.byref(d), ctypes.byref(b)) == L.AT_OK
    assert b.value == (256 + 8192 + 256 + 2048 + 3328 + 2048 + 2048 + 8192 + 8192 + 32000 + 4096
                       + 3 * 100 * 2048)
    d = L.AtGridDesc((64, 64, 64), L.AT_ROOT_POINTER, 3, 100, -1)
    assert lib.at_grid_footprint(ctypes.byref(d), ctypes.byref(b)) == L.AT_E_INVALID


def test_planning_handle_rejects_device_calls():
    lib = L.lib()
    d = _desc(32)
    h = ctypes.c_void_p()
    assert lib.at_grid_create(ctypes.byref(d), None, 0, None, ctypes.byref(h)) == L.AT_OK
    assert lib.at_listgen(h, None) == L.AT_E_STATE
    assert lib.at_grid_views(h, None, None, None, None) == L.AT_E_STATE
    bits = ctypes.c_int32()
    assert lib.at_device_status(h, None, 0, ctypes.byref(bits)) == L.AT_E_STATE
    assert lib.at_grid_destroy(h) == L.AT_OK
    assert lib.at_grid_destroy(None) == L.AT_E_INVALID


def test_create_rejects_small_or_misaligned_buffers():
    lib = L.lib()
    d = _desc(32)
    h = ctypes.c_void_p()
    assert lib.at_grid_create(ctypes.byref(d), ctypes.c_void_p(0x100000), 16, None, ctypes.byref(h)) == L.AT_E_INVALID
    assert lib.at_grid_create(ctypes.byref(d), ctypes.c_void_p(0x100010), 1 << 30, None, ctypes.byref(h)) == L.AT_E_INVALID


def test_task_validation_enqueues_nothing():
    lib = L.lib()
    d = _desc(32, L.AT_ROOT_BITMASK, 2)
    h = ctypes.c_void_p()
    assert lib.at_grid_create(ctypes.byref(d), None, 0, None, ctypes.byref(h)) == L.AT_OK
    before = lib.at_dispatch_count()
    t = L.AtTask()
    t.kind, t.op, t.grid = L.AT_TASK_STENCIL, 99, h.value
    for q in range(8):
        t.ch[q] = -1
    st = L.AtStats()
    assert lib.at_run_sequence(ctypes.byref(t), 1, L.AT_OPT_ALL, ctypes.byref(st), None) == L.AT_E_INVALID
    t.op = L.AT_OP_JACOBI
    t.ch[0], t.ch[1], t.ch[2] = 0, 1, 5          # channel out of range
    assert lib.at_run_sequence(ctypes.byref(t), 1, L.AT_OPT_ALL, ctypes.byref(st), None) == L.AT_E_INVALID
    t.ch[2] = 0                                   # output aliases the stencil input
    assert lib.at_run_sequence(ctypes.byref(t), 1, 0, ctypes.byref(st), None) == L.AT_E_INVALID
    assert lib.at_run_sequence(ctypes.byref(t), 1, 1 << 7, ctypes.byref(st), None) == L.AT_E_INVALID
    t.reserved = 1
    assert lib.at_run_sequence(ctypes.byref(t), 1, 0, ctypes.byref(st), None) == L.AT_E_INVALID
    assert lib.at_dispatch_count() == before
    assert lib.at_grid_destroy(h) == L.AT_OK


def test_normalise_rejects_overlapping_channels():
    """v = mv / m per component: v may replace mv in place, but velocity
    channels overlapping the mass or only part of the momentum would make a
    component read another component's result (the single-op kernel loads all
    inputs first, the fused one per component), so they are rejected."""
    lib = L.lib()
    d = _desc(32, L.AT_ROOT_BITMASK, 8)
    h = ctypes.c_void_p()
    assert lib.at_grid_create(ctypes.byref(d), None, 0, None, ctypes.byref(h)) == L.AT_OK
    st = L.AtStats()
    t = L.AtTask()
    t.kind, t.op, t.grid = L.AT_TASK_STENCIL, L.AT_OP_NORMALISE, h.value
    for q in range(8):
        t.ch[q] = -1
    for (m, mv, v), ok in (((0, 1, 4), True), ((0, 1, 1), True), ((0, 1, 2), False), ((0, 1, 3), False),
                           ((0, 2, 1), False), ((3, 0, 2), False), ((4, 1, 5), True)):
        t.ch[0], t.ch[1], t.ch[2] = m, mv, v
        r = lib.at_run_sequence(ctypes.byref(t), 1, 0, ctypes.byref(st), None)
        assert (r == L.AT_OK) == ok, (m, mv, v, r)
    assert lib.at_grid_destroy(h) == L.AT_OK


def test_options_roundtrip():
    lib = L.lib()
    v = ctypes.c_int64()
    assert lib.at_set_option(L.AT_OPTION_MAX_FUSE_PER_TASK, 2) == L.AT_OK
    assert lib.at_get_option(L.AT_OPTION_MAX_FUSE_PER_TASK, ctypes.byref(v)) == L.AT_OK and v.value == 2
    assert lib.at_set_option(L.AT_OPTION_MAX_FUSE_PER_TASK, 1) == L.AT_OK
    assert lib.at_set_option(L.AT_OPTION_MAX_FUSE_PER_TASK, 0) == L.AT_E_INVALID
    assert lib.at_set_option(999, 0) == L.AT_E_INVALID
    for opt, good, bad in ((L.AT_OPTION_G2P_BINS, (0, 1), (2, -1)), (L.AT_OPTION_BIN_REUSE, (0, 3, 8), (-1, 1025)),
                           (L.AT_OPTION_GRAPHS, (0, 1), (2, -1))):
        assert lib.at_get_option(opt, ctypes.byref(v)) == L.AT_OK
        default = v.value
        for x in good:
            assert lib.at_set_option(opt, x) == L.AT_OK
            assert lib.at_get_option(opt, ctypes.byref(v)) == L.AT_OK and v.value == x
        for x in bad:
            assert lib.at_set_option(opt, x) == L.AT_E_INVALID
        assert lib.at_set_option(opt, default) == L.AT_OK
    assert lib.at_get_option(L.AT_OPTION_GRAPHS_CACHED, ctypes.byref(v)) == L.AT_OK and v.value >= 0
    assert lib.at_set_option(L.AT_OPTION_GRAPHS_CACHED, 0) == L.AT_E_INVALID
    assert lib.at_version().startswith(b"atsparse")


def test_timing_collect_without_device_work():
    """Planning handles launch nothing, so a timed window records no events;
    bad arguments are rejected."""
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd.grid import SparseGrid
    lib = L.lib()
    g = SparseGrid(32, 2, "bitmask", device=None)
    E.reset()
    E.timing_enable(True)
    try:
        E.run_sequence([E.listgen(g), E.inc(g, 0, 1.0)], E.OPT_ALL, stream=0)
        assert E.timing_collect() == []
    finally:
        E.timing_enable(False)
    n = ctypes.c_int32()
    assert lib.at_timing_collect(None, 1, ctypes.byref(n)) == L.AT_E_INVALID
    assert lib.at_timing_collect(None, 0, None) == L.AT_E_INVALID
    assert lib.at_timing_collect(None, 0, ctypes.byref(n)) == L.AT_OK and n.value == 0
    E.reset()


def test_planning_window_launches_nothing_and_mixing_is_rejected():
    """A window on planning handles records state only, also for its tasks
    without a grid (advection over placeholder arrays); a window mixing
    planning handles and device grids is rejected before anything runs."""
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd.grid import SparseGrid

    class Fake:
        def __init__(self, shape, p):
            self.shape, self._p = shape, p

        def data_ptr(self):
            return self._p

    g = SparseGrid(64, 7, "pointer", 512, device=None)
    x, v, m = Fake((3, 100), 0x1000000), Fake((3, 100), 0x2000000), Fake((100,), 0x3000000)
    E.reset()
    before = L.lib().at_dispatch_count()
    st = E.run_sequence([E.listgen(g), E.advect(x, v, 1e-3), E.p2g(g, x, v, m, 1 / 64, 0, 1)], 0, stream=0)
    assert st["dispatches"] == 0 and L.lib().at_dispatch_count() == before
    E.reset()


def test_static_scatter_validates_on_the_host():
    lib = L.lib()
    ch = (ctypes.c_int32 * 2)(0, 1)
    assert lib.at_p2g_static(None, None, None, None, 0, 1.0, ch, 0, None) == L.AT_E_INVALID
    d = _desc(32, L.AT_ROOT_POINTER, 4, 64)
    h = ctypes.c_void_p()
    assert lib.at_grid_create(ctypes.byref(d), None, 0, None, ctypes.byref(h)) == L.AT_OK
    assert lib.at_p2g_static(h, None, None, None, 0, 1.0, ch, 0, None) == L.AT_E_STATE
    assert lib.at_grid_destroy(h) == L.AT_OK
