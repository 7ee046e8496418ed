"""The asynchronous engine on the GPU (MI355X only): windows flushed to the
optimizer and launcher threads give the same device results, bit for bit,
and the same counters as the synchronous engine -- on the narrow-band
Jacobi (one window per iteration), the multigrid V-cycle (activating
restrictions across levels) and the MacCormack step (fused sampling nodes,
interpreted or compiled), all deterministic."""
import numpy as np
import pytest

from paper_2012_08141_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(autouse=True)
def engine():
    from paper_2012_08141_amd import engine as E
    E.reset()
    yield
    from paper_2012_08141_amd import _lib as L
    E.set_async(False)
    E.set_option(L.AT_OPTION_VARIANTS, 0)
    E.reset()


def _run(kind, async_on):
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd import programs as PR
    from paper_2012_08141_amd import _lib as L
    E.reset()
    # the compiled form: the fused sampling nodes run their compiled tile
    # programs, compiled and loaded on the launching thread
    E.set_option(L.AT_OPTION_VARIANTS, 2 if kind == "maccormack-compiled" else 0)
    E.set_async(async_on)
    tot = {"dispatches": 0, "tasks_launched": 0}
    if kind == "jacobi":
        w = I.band(1, n=128)
        g = PR.load_workload(w, {"b": PR.JACOBI["b"]}, 3)
        steps = [PR.jacobi_step(g) for _ in range(30)]
        outs = lambda: [g.channel(PR.JACOBI["x"])]
    elif kind == "multigrid":
        w = I.band(2, n=128)
        lv = PR.mg_levels(w, 3)
        steps = [PR.mg_vcycle(lv) for _ in range(6)]
        outs = lambda: [l.channel(PR.MG["x"]) for l in lv] + [l.channel(PR.MG["t"]) for l in lv]
    else:
        w = I.tube(3, n=64)
        g = PR.load_workload(w, {"q0": 0, "q1": 1, "q2": 2, "v0": 3, "v1": 4, "v2": 5}, 15)
        steps = [PR.maccormack_step(g, w.params["dt"], rk3=True) for _ in range(8)]
        outs = lambda: [g.channel(c) for c in range(3)]
    for s in steps:
        st = E.run_sequence(s, E.OPT_ALL)
        if not async_on:
            for k in tot:
                tot[k] += st[k]
    if async_on:
        st = E.sync()
        tot = {k: st[k] for k in tot}
    torch.cuda.synchronize()
    res = [o.clone() for o in outs()]
    E.set_async(False)
    E.set_option(L.AT_OPTION_VARIANTS, 0)
    return res, tot


@pytest.mark.parametrize("kind", ["jacobi", "multigrid", "maccormack", "maccormack-compiled"])
def test_async_equals_sync(kind):
    say("async", kind)
    a, ta = _run(kind, True)
    s, ts = _run(kind, False)
    assert ta == ts and ts["dispatches"] > 0
    for x, y in zip(a, s):
        assert torch.equal(x, y)
