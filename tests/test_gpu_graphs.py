"""HIP-graph replay of repeated optimized windows (AT_OPTION_GRAPHS).

A window whose plan comes from the plan cache and holds only struct-fors
and two-level transfers is captured into a HIP graph once and replayed
afterwards.  Every replay must equal direct launches of the same plan bit
for bit, also with other device work and synchronisations between replays,
and a graph must never outlive the grids it uses."""
import numpy as np
import pytest

from paper_2012_08141_amd import _lib as L
from paper_2012_08141_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(autouse=True)
def graphs_default():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2012_08141_amd import engine as E
    E.reset()
    yield
    E.set_option(L.AT_OPTION_GRAPHS, 0)
    E.reset()
    torch.cuda.synchronize()


def test_jacobi_windows_replayed_equal_direct():
    from paper_2012_08141_amd import engine as E, programs as PR
    say("graph replay: band128 jacobi windows")
    w = I.band(1, n=128)
    ga = PR.load_workload(w, PR.JACOBI, 3)
    gb = PR.load_workload(w, PR.JACOBI, 3)
    wa = E.prepare(sum((PR.jacobi_step(ga) for _ in range(10)), []))
    wb = E.prepare(sum((PR.jacobi_step(gb) for _ in range(10)), []))
    scratch = torch.zeros(1 << 20, device="cuda")
    for rep in range(6):
        E.set_option(L.AT_OPTION_GRAPHS, 1)
        sa = E.run_sequence(wa, E.OPT_ALL)
        if rep >= 2:                                     # window 1 makes the list; window 2 plans the steady state
            assert E.get_option(L.AT_OPTION_GRAPHS_CACHED) >= 1
        scratch.mul_(0.5).add_(1.0)                      # other device work between replays
        E.set_option(L.AT_OPTION_GRAPHS, 0)
        sb = E.run_sequence(wb, E.OPT_ALL)
        torch.cuda.synchronize()
        assert sa["dispatches"] == sb["dispatches"], rep
        assert torch.equal(ga.channel(0), gb.channel(0)), rep
        assert torch.equal(ga.channel(1), gb.channel(1)), rep


def test_vcycle_windows_replayed_equal_direct():
    from paper_2012_08141_amd import engine as E, programs as PR
    say("graph replay: multigrid V-cycles")
    w = I.band(2, n=128)
    la, lb = PR.mg_levels(w, 3), PR.mg_levels(w, 3)
    wa = E.prepare(PR.mg_vcycle(la))
    wb = E.prepare(PR.mg_vcycle(lb))
    for rep in range(5):
        E.set_option(L.AT_OPTION_GRAPHS, 1)
        E.run_sequence(wa, E.OPT_ALL)
        if rep >= 2:                                     # plans change until the hierarchy is built
            assert E.get_option(L.AT_OPTION_GRAPHS_CACHED) >= 1
        E.set_option(L.AT_OPTION_GRAPHS, 0)
        E.run_sequence(wb, E.OPT_ALL)
        torch.cuda.synchronize()
        for l in range(3):
            assert torch.equal(la[l].channel(0), lb[l].channel(0)), (rep, l)
            assert np.array_equal(la[l].active_cells(), lb[l].active_cells()), (rep, l)


def test_graph_dropped_with_its_grid():
    """A replacement grid of the same shape never runs an old grid's graph."""
    from paper_2012_08141_amd import engine as E, programs as PR
    say("graph replay: grid destroyed and replaced")
    w = I.band(4, n=64)
    E.set_option(L.AT_OPTION_GRAPHS, 1)
    results = []
    for trial in range(2):
        g = PR.load_workload(w, PR.JACOBI, 3)
        win = E.prepare(sum((PR.jacobi_step(g) for _ in range(10)), []))
        for _ in range(3):
            E.run_sequence(win, E.OPT_ALL)
        torch.cuda.synchronize()
        assert E.get_option(L.AT_OPTION_GRAPHS_CACHED) == 1
        results.append(g.read_blocks(0, w.cells))
        del win, g
        import gc
        gc.collect()
        assert E.get_option(L.AT_OPTION_GRAPHS_CACHED) == 0     # dropped with its grid
    assert np.array_equal(results[0], results[1])
