"""Batching and serving on the GPU (MI355X only).

Each request's result must be the same alone and in any batch or mix:
Jacobi has no atomics, so the bar is bit-exact -- against the single-grid
engine path run alone, and (within the 1e-6 stencil bar, expected exact)
against the oracle's in-order Jacobi program."""
import numpy as np
import pytest

from oracle import programs as OP
from paper_2012_08141_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


def _requests(count, lo=32, hi=600, iters=12, seed=3):
    from paper_2012_08141_amd.serving import Request
    reqs = []
    for i in range(count):
        w = I.batch_request(seed, i, n=128, lo=lo, hi=hi)
        reqs.append(Request(i, 0.0, w.cells, w.channels["b"], iters))
    return reqs


def test_batch_alone_equals_mix_and_oracle():
    """Requests admitted at different global iterations, advanced together by
    a captured graph, retired when done; every result equals the request run
    alone through the single-grid engine and the oracle."""
    from paper_2012_08141_amd.batching import BatchArena
    from paper_2012_08141_amd.serving import solve_alone
    say("batch mix")
    reqs = _requests(10)
    arena = BatchArena(128, max_grids=8, pool_blocks=4096)
    graph = arena.capture(5)
    results = {}
    pending = list(reqs)
    live = {}
    steps = 0
    while pending or live:
        # admit at most two per replay boundary, so grids overlap at offsets
        for _ in range(2):
            if pending and arena.fits(pending[0].nblocks):
                r = pending.pop(0)
                r.gid = arena.admit(r.cells, r.b, r.iters)
                r.end_clock = arena.clock_host + r.iters
                live[r.rid] = r
        for r in [r for r in live.values() if r.end_clock <= arena.clock_host]:
            results[r.rid] = arena.retire(r.gid)
            del live[r.rid]
        if live:
            graph.replay()
            steps += 1
    torch.cuda.synchronize()
    assert steps > 3
    for r in reqs:
        alone = solve_alone(r, 128, 0)
        got = results[r.rid].cpu().numpy()
        assert np.array_equal(got, alone.cpu().numpy()), r.rid
        ref = OP.jacobi_program(128, I.cells_to_blocks(r.cells, 16), r.b, r.iters)
        order = np.argsort(r.cells)          # cells are ascending already
        assert np.array_equal(ref["cells"], r.cells[order])
        exp = ref["x"]
        tol = 1e-6 * np.maximum(np.abs(exp), 1e-3 * np.abs(exp).max())
        assert np.all(np.abs(got - exp) <= tol), r.rid


def test_serving_continuous_batching():
    """A request stream through the server with a footprint budget that
    forces admission to wait: all requests finish, several are resident at
    once, and each result equals the request solved alone."""
    from paper_2012_08141_amd.serving import JacobiServer, solve_alone
    say("serving")
    reqs = _requests(12, lo=64, hi=1500, iters=20, seed=5)
    need = max(r.nblocks for r in reqs)
    budget = int(2.5 * need * (3 * 2048 + 4))
    srv = JacobiServer(128, budget_bytes=budget, max_grids=8, iters_per_replay=5)
    st = srv.serve(reqs, realtime=False)
    summ = st.summary()
    say("  ", summ)
    assert summ["requests"] == len(reqs)
    assert st.max_resident >= 2
    for r in reqs:
        assert r.completed >= 0 and r.result is not None
        assert np.array_equal(r.result.cpu().numpy(), solve_alone(r, 128, 0).cpu().numpy()), r.rid


def test_batch_graph_replays_match_eager_launches():
    """The captured graph gives the same state after every replay as direct
    launches (a HIP graph replayed several times, with host work between)."""
    from paper_2012_08141_amd.batching import BatchArena
    say("graph replays")
    reqs = _requests(4, iters=40)
    a1 = BatchArena(128, 4, 4096)
    a2 = BatchArena(128, 4, 4096)
    for r in reqs:
        a1.admit(r.cells, r.b, r.iters)
        a2.admit(r.cells, r.b, r.iters)
    g = a1.capture(4)
    for _ in range(6):
        g.replay()
        a2.step(4)
        torch.cuda.synchronize()
        assert torch.equal(a1.x, a2.x) and torch.equal(a1.xn, a2.xn)
