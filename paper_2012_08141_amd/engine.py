"""Task descriptors and the execution engine (paper Sections 4-7).

Builders return ``Task`` objects (a ctypes ``at_task`` plus references that
keep external torch arrays alive); ``run_sequence`` hands a window of them
to the library, which builds the state-flow graph, runs the selected passes
and launches the result on torch's current stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

from . import _lib as L
from .grid import SparseGrid, current_stream

OPT_NONE = 0
OPT_LGR, OPT_AD, OPT_FUSE, OPT_DSE, OPT_ALL = L.AT_OPT_LGR, L.AT_OPT_AD, L.AT_OPT_FUSE, L.AT_OPT_DSE, L.AT_OPT_ALL

KIND_NAMES = {L.AT_TASK_ACTIVATE: "activate", L.AT_TASK_LISTGEN: "listgen", L.AT_TASK_STENCIL: "struct_for",
              L.AT_TASK_ADVECT: "advect", L.AT_TASK_P2G: "p2g", L.AT_TASK_G2P: "g2p",
              L.AT_TASK_RESTRICT: "restrict", L.AT_TASK_PROLONG: "prolong", L.AT_TASK_P2G_MLS: "p2g_mls",
              L.AT_TASK_G2P_APIC: "g2p_apic"}
OP_NAMES = {L.AT_OP_LAP_UPDATE: "lap_update", L.AT_OP_AXPY: "axpy", L.AT_OP_JACOBI: "jacobi",
            L.AT_OP_COPY: "copy", L.AT_OP_FILL: "fill", L.AT_OP_INC: "inc", L.AT_OP_DIFFUSE: "diffuse",
            L.AT_OP_DIFFUSE_ADJ: "diffuse_adj", L.AT_OP_NORMALISE: "normalise", L.AT_OP_ADVECT: "advect_sl",
            L.AT_OP_MACCORMACK: "maccormack", L.AT_OP_MPM_GRID: "mpm_grid"}


@dataclass
class Task:
    c: L.AtTask
    keep: list = field(default_factory=list)   # objects whose memory the task points at

    @property
    def name(self) -> str:
        k = self.c.kind
        return OP_NAMES.get(self.c.op, "?") if k == L.AT_TASK_STENCIL else KIND_NAMES.get(k, "?")


def _task(kind: int, grid: SparseGrid | None, op: int = 0) -> Task:
    t = L.AtTask()
    t.kind, t.op, t.flags, t.reserved = kind, op, 0, 0
    t.grid = grid.handle.value if grid is not None else None
    t.grid2 = None
    for q in range(8):
        t.ch[q] = -1
    return Task(t, [grid])


def _ptr(x) -> int:
    return x.data_ptr() if x is not None else 0


# ---- grid tasks --------------------------------------------------------------
def activate(grid, coords, kind=L.AT_COORD_BLOCK) -> Task:
    """Range-for activation of the blocks containing ``coords`` (device int32
    [n, 3]).  The array must not be modified outside the engine afterwards
    (or call ``ext_modified``), since identical activations are demoted."""
    T = _task(L.AT_TASK_ACTIVATE, grid, kind)
    T.c.ext[0] = _ptr(coords)
    T.c.n = coords.shape[0] if coords is not None else 0
    T.keep.append(coords)
    return T


def listgen(grid) -> Task:
    return _task(L.AT_TASK_LISTGEN, grid)


def struct_for(grid, op: int, ch, param: float = 0.0) -> Task:
    T = _task(L.AT_TASK_STENCIL, grid, op)
    for q, c in enumerate(ch):
        T.c.ch[q] = c
    T.c.param[0] = param
    return T


def lap_update(grid, a, out, coef=0.1):
    return struct_for(grid, L.AT_OP_LAP_UPDATE, [a, out], coef)


def axpy(grid, y, x, alpha):
    return struct_for(grid, L.AT_OP_AXPY, [y, x], alpha)


def jacobi(grid, x, b, xn):
    return struct_for(grid, L.AT_OP_JACOBI, [x, b, xn])


def copy(grid, dst, src):
    return struct_for(grid, L.AT_OP_COPY, [dst, src])


def fill(grid, chans, value=0.0):
    return struct_for(grid, L.AT_OP_FILL, list(chans), value)


def inc(grid, x, value):
    return struct_for(grid, L.AT_OP_INC, [x], value)


def diffuse(grid, a, k, out, dt):
    return struct_for(grid, L.AT_OP_DIFFUSE, [a, k, out], dt)


def diffuse_adj(grid, a, k, lamn, lam, gk, dt):
    return struct_for(grid, L.AT_OP_DIFFUSE_ADJ, [a, k, lamn, lam, gk], dt)


def normalise(grid, m, mv0, v0):
    return struct_for(grid, L.AT_OP_NORMALISE, [m, mv0, v0])


def advect_sl(grid, q, v0, out, dt, rk3=False):
    """Semi-Lagrangian advection: out = q at the back-traced point of I (one
    Euler step, or the RK3 back-trace), trilinear (v on channels v0 .. v0 + 2)."""
    T = struct_for(grid, L.AT_OP_ADVECT, [q, v0, out], dt)
    T.c.param[1] = 1.0 if rk3 else 0.0
    return T


def maccormack(grid, q, v0, fwd, bwd, out, dt, rk3=False):
    """MacCormack correction: out = fwd + 0.5 (q - bwd), clamped to the range
    of q around the forward back-traced point (Euler or RK3)."""
    T = struct_for(grid, L.AT_OP_MACCORMACK, [q, v0, fwd, bwd, out], dt)
    T.c.param[1] = 1.0 if rk3 else 0.0
    return T


def mpm_grid(grid, m, mv0, v0, dt, gravity, bound):
    """MLS-MPM grid update: v = mv / m where m > 0, gravity along -z, walls
    ``bound`` nodes thick."""
    T = struct_for(grid, L.AT_OP_MPM_GRID, [m, mv0, v0], dt)
    T.c.param[1] = gravity
    T.c.param[2] = float(bound)
    return T


# ---- two-level transfers (struct-fors over the fine grid) ----------------------
def restrict(fine, coarse, src, dst, weight) -> Task:
    """coarse[dst][I/2] += weight * fine[src][I] over the fine grid's list,
    activating the coarse blocks written (coarse: half the domain edge)."""
    T = _task(L.AT_TASK_RESTRICT, fine)
    T.c.grid2 = coarse.handle.value
    T.c.ch[0], T.c.ch[1] = src, dst
    T.c.param[0] = weight
    T.keep.append(coarse)
    return T


def prolong(coarse, fine, src, dst) -> Task:
    """fine[dst][I] += coarse[src][I/2] over the fine grid's list."""
    T = _task(L.AT_TASK_PROLONG, fine)
    T.c.grid2 = coarse.handle.value
    T.c.ch[0], T.c.ch[1] = src, dst
    T.keep.append(coarse)
    return T


# ---- particle tasks ------------------------------------------------------------
def advect(x, v, dt, unique=True) -> Task:
    T = _task(L.AT_TASK_ADVECT, None)
    T.c.ext[0], T.c.ext[1] = _ptr(x), _ptr(v)
    T.c.n = x.shape[-1]
    T.c.param[0] = dt
    T.c.flags = L.AT_TASKF_LOOP_UNIQUE if unique else 0
    T.keep += [x, v]
    return T


def p2g(grid, x, v, m, dx, ch_m, ch_mv, activation=L.AT_ACT_PER_NODE, unique=True) -> Task:
    T = _task(L.AT_TASK_P2G, grid, activation)
    T.c.ext[0], T.c.ext[1], T.c.ext[2] = _ptr(x), _ptr(v), _ptr(m)
    T.c.n = x.shape[-1]
    T.c.param[0] = dx
    T.c.ch[0], T.c.ch[1] = ch_m, ch_mv
    T.c.flags = L.AT_TASKF_LOOP_UNIQUE if unique else 0
    T.keep += [x, v, m]
    return T


def g2p(grid, x, v, dx, ch_v, unique=True) -> Task:
    T = _task(L.AT_TASK_G2P, grid)
    T.c.ext[0], T.c.ext[1] = _ptr(x), _ptr(v)
    T.c.n = x.shape[-1]
    T.c.param[0] = dx
    T.c.ch[0] = ch_v
    T.c.flags = L.AT_TASKF_LOOP_UNIQUE if unique else 0
    T.keep += [x, v]
    return T


def p2g_mls(grid, x, v, C, F, dx, dt, mass, vol, mu, lam, ch_m, ch_mv, activation=L.AT_ACT_PER_NODE,
            unique=True) -> Task:
    """MLS-MPM scatter: F <- (I + dt C) F, fixed-corotated stress, mass and
    APIC momentum onto the grid (activating)."""
    T = _task(L.AT_TASK_P2G_MLS, grid, activation)
    T.c.ext[0], T.c.ext[1], T.c.ext[2], T.c.ext[3] = _ptr(x), _ptr(v), _ptr(C), _ptr(F)
    T.c.n = x.shape[-1]
    for q, val in enumerate((dx, dt, mass, vol, mu, lam)):
        T.c.param[q] = val
    T.c.ch[0], T.c.ch[1] = ch_m, ch_mv
    T.c.flags = L.AT_TASKF_LOOP_UNIQUE if unique else 0
    T.keep += [x, v, C, F]
    return T


def g2p_apic(grid, x, v, C, dx, ch_v, unique=True) -> Task:
    """MLS-MPM gather of v and the APIC affine matrix C."""
    T = _task(L.AT_TASK_G2P_APIC, grid)
    T.c.ext[0], T.c.ext[1], T.c.ext[2] = _ptr(x), _ptr(v), _ptr(C)
    T.c.n = x.shape[-1]
    T.c.param[0] = dx
    T.c.ch[0] = ch_v
    T.c.flags = L.AT_TASKF_LOOP_UNIQUE if unique else 0
    T.keep += [x, v, C]
    return T


# ---- engine --------------------------------------------------------------------
def _array(tasks):
    arr = (L.AtTask * max(1, len(tasks)))()
    for i, t in enumerate(tasks):
        arr[i] = t.c
    return arr


class Prepared:
    """A window's task descriptors packed once, for windows that run the same
    tasks again (the arrays and grids they point at stay alive with it)."""

    def __init__(self, tasks):
        self.arr = _array(tasks)
        self.n = len(tasks)
        self.keep = [t.keep for t in tasks]


def prepare(tasks) -> Prepared:
    return Prepared(tasks)


def run_sequence(tasks, opt_flags: int = OPT_ALL, stream=None) -> dict:
    """Plan and launch a window of tasks (a list, or a Prepared window);
    returns the window's counters."""
    if isinstance(tasks, Prepared):
        arr, n = tasks.arr, tasks.n
    else:
        arr, n = _array(tasks), len(tasks)
    st = L.AtStats()
    L.check(L.lib().at_run_sequence(arr, n, opt_flags, ctypes.byref(st),
                                    stream if stream is not None else current_stream()))
    return st.as_dict()


def plan_sequence(tasks, opt_flags: int = OPT_ALL):
    """The optimized plan of a window, without running it or changing the
    engine's state: (entries, counters).  Each entry lists the input task
    indices it runs, in order."""
    arr = _array(tasks)
    cap = max(1, len(tasks))
    out = (L.AtPlanEntry * cap)()
    n = ctypes.c_int32()
    st = L.AtStats()
    L.check(L.lib().at_plan_sequence(arr, len(tasks), opt_flags, out, cap, ctypes.byref(n), ctypes.byref(st)))
    entries = []
    for i in range(n.value):
        e = out[i]
        entries.append({"kind": e.kind, "members": [e.members[m] for m in range(e.nmembers)],
                        "check_activation": bool(e.check_activation), "activation_mode": e.activation_mode,
                        "dropped": e.dropped, "keep": [e.keep[m] for m in range(e.nmembers)],
                        "fill_channels": e.keep[0]})
    return entries, st.as_dict()


def enqueue(task: Task, stream=None):
    L.check(L.lib().at_enqueue(ctypes.byref(task.c), stream if stream is not None else current_stream()))


def flush(stream=None) -> dict:
    st = L.AtStats()
    L.check(L.lib().at_flush(ctypes.byref(st), stream if stream is not None else current_stream()))
    return st.as_dict()


def sync() -> dict:
    """Wait until every window flushed asynchronously (AT_OPTION_ASYNC) has
    been launched; returns their counters summed since the last sync, and
    raises the first failure of such a window.  Call it before a device
    synchronisation or before reading results."""
    st = L.AtStats()
    L.check(L.lib().at_engine_sync(ctypes.byref(st)))
    return st.as_dict()


def set_async(on: bool = True):
    """Hand flushed windows to the optimizer and launcher threads (True) or
    plan and launch them inside each call (False, the default)."""
    set_option(L.AT_OPTION_ASYNC, 1 if on else 0)


def set_option(option: int, value: int):
    L.check(L.lib().at_set_option(option, value))


def get_option(option: int) -> int:
    v = ctypes.c_int64()
    L.check(L.lib().at_get_option(option, ctypes.byref(v)))
    return int(v.value)


def reset():
    L.check(L.lib().at_engine_reset())


def ext_modified(x):
    L.check(L.lib().at_ext_modified(ctypes.c_void_p(_ptr(x))))


def dispatch_count() -> int:
    return int(L.lib().at_dispatch_count())


def paper_task_count(entries) -> int:
    """Tasks counted the paper's way (Section 6.1, Fig. 7): a list generation is a clear
    task plus a listgen task; this library folds the clear into one dispatch."""
    return sum(2 if e["kind"] == L.AT_TASK_LISTGEN else 1 for e in entries)


def timing_enable(on: bool = True):
    """Bracket every launched task of later windows with HIP events."""
    L.check(L.lib().at_timing_enable(1 if on else 0))


def timing_collect() -> list:
    """Wait for the recorded events; per launched kind (task kind, op,
    fused members): launches and mean event-measured microseconds."""
    cap = 64
    out = (L.AtTimingEntry * cap)()
    n = ctypes.c_int32()
    L.check(L.lib().at_timing_collect(out, cap, ctypes.byref(n)))
    res = []
    for i in range(n.value):
        e = out[i]
        name = OP_NAMES.get(e.op, "?") if e.kind == L.AT_TASK_STENCIL else KIND_NAMES.get(e.kind, "?")
        res.append({"name": name, "kind": e.kind, "op": e.op, "members": e.members, "launches": e.launches,
                    "mean_us": e.total_us / max(1, e.launches)})
    return res
