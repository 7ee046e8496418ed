"""The asynchronous engine (Section 7: the optimizer and the launcher run
beside the program) on planning handles (host only).

With AT_OPTION_ASYNC on, flushed windows go to an optimizer thread, which
plans them in flush order, and from it to a launcher thread.  The engine
state they leave must be the synchronous engine's: the same counters summed
over the windows and the same plan for the window after them; periodic
flushes and explicit flushes behave alike; invalid windows are refused at
the call; every other engine call waits for the pipeline first."""
import pytest

from paper_2012_08141_amd import _lib as L
from paper_2012_08141_amd import engine as E
from paper_2012_08141_amd import programs as PR
from paper_2012_08141_amd.autodiff import DiffusionTasks
from paper_2012_08141_amd.grid import SparseGrid

from test_optimizer_programs import FakeArray

PARAMS = dict(dt=1e-4, dx=1 / 64, mass=1e-3, vol=1e-6, mu=1.0, lam=1.0, gravity=9.8, bound=2)


@pytest.fixture(autouse=True)
def fresh_engine():
    E.reset()
    yield
    E.set_async(False)
    E.reset()


def _mpm_windows():
    grids = [SparseGrid(64, 7, "bitmask", device=None) for _ in range(2)]
    arrays = FakeArray((3, 1000)), FakeArray((3, 1000)), FakeArray((9, 1000)), FakeArray((9, 1000))
    wins = [sum((PR.mpm_step(grids, t, *arrays, PARAMS) for t in range(k, k + 2)), []) for k in range(0, 12, 2)]
    nxt = sum((PR.mpm_step(grids, t, *arrays, PARAMS) for t in range(12, 16)), [])
    return wins, nxt


def _diffusion_windows():
    g = SparseGrid(128, DiffusionTasks.channels(20, 5), "pointer", 2048, device=None)
    t = DiffusionTasks(g, 0.1, 20, 5)
    return [[E.listgen(g)], t.fwd, t.bwd_init] + t.bwd + [t.fwd], t.bwd_init


SUMMED = ("tasks_in", "tasks_launched", "dispatches", "listgens_removed", "activations_demoted", "fusions",
          "stores_eliminated", "plan_cache_hits")


def _run(make, async_on, flags=E.OPT_ALL):
    E.reset()
    wins, nxt = make()
    E.set_async(async_on)
    sums = dict.fromkeys(SUMMED, 0)
    for w in wins:
        st = E.run_sequence(w, flags)
        if not async_on:
            for k in SUMMED:
                sums[k] += st[k]
    if async_on:
        st = E.sync()
        sums = {k: st[k] for k in SUMMED}
    plan, _ = E.plan_sequence(nxt, flags)
    E.set_async(False)
    return sums, [(e["members"], e["keep"], e["check_activation"]) for e in plan]


@pytest.mark.parametrize("make", [_mpm_windows, _diffusion_windows])
@pytest.mark.parametrize("flags", [0, E.OPT_ALL, E.OPT_ALL & ~E.OPT_FUSE])
def test_async_windows_leave_the_synchronous_state(make, flags):
    sync_sums, sync_plan = _run(make, False, flags)
    async_sums, async_plan = _run(make, True, flags)
    assert async_sums == sync_sums
    assert async_plan == sync_plan
    assert sync_sums["tasks_in"] > 0


def test_async_enqueue_with_periodic_flush():
    """Tasks enqueued one by one with a flush period of 7 give the windows
    (and counters) of the synchronous engine with the same period."""
    res = []
    for async_on in (False, True):
        E.reset()
        wins, nxt = _mpm_windows()
        E.set_option(L.AT_OPTION_FLUSH_PERIOD, 7)
        E.set_async(async_on)
        tot = dict.fromkeys(SUMMED, 0)
        for w in wins:
            for t in w:
                E.enqueue(t)
        st = E.flush()
        if async_on:
            assert st["tasks_launched"] == 0     # only queued
            st = E.sync()
            tot = {k: st[k] for k in SUMMED}
        plan, _ = E.plan_sequence(nxt, E.OPT_ALL)
        E.set_async(False)
        E.set_option(L.AT_OPTION_FLUSH_PERIOD, 0)
        res.append(([e["members"] for e in plan], tot if async_on else None))
    assert res[0][0] == res[1][0]
    assert res[1][1]["tasks_in"] == sum(len(w) for w in _mpm_windows()[0])


def test_async_refuses_invalid_windows_at_the_call():
    g = SparseGrid(64, 3, "bitmask", device=None)
    E.set_async(True)
    bad = E.copy(g, 0, 9)                      # channel out of range
    with pytest.raises(L.AtError):
        E.run_sequence([bad], E.OPT_ALL)
    ok = E.run_sequence([E.listgen(g), E.copy(g, 0, 1)], E.OPT_ALL)
    assert ok["tasks_in"] == 2
    st = E.sync()
    assert st["tasks_in"] == 2 and st["tasks_launched"] == 2
    assert E.sync()["tasks_in"] == 0         # counters restart after a sync
    assert E.get_option(L.AT_OPTION_ASYNC) == 1
