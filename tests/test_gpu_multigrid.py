"""Multigrid transfers and V-cycles on the device against the oracle.

The restriction (y[I/2] += w x[I], activating coarse blocks) and the
injection prolongation (x[I] += y[I/2]) of the multigrid solver (paper
Section 8.4, Fig. 12; the downsample pattern of Section 6.3) add each
coarse voxel's children in a fixed order, so they match the oracle bit for
bit, on every pairing of root kinds and with the activation check kept or
demoted.  V-cycle programs match within the stencil tolerance, eager and
optimized, with the optimized form demoting the restrictions' activation
from the second cycle on."""
import numpy as np
import pytest

import oracle
from oracle import programs as OP
from paper_2012_08141_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2012_08141_amd import engine as E
    E.reset()
    yield
    torch.cuda.synchronize()


def close_stencil(got, exp, what=""):
    exp = np.asarray(exp, np.float64)
    got = np.asarray(got, np.float64)
    scale = np.abs(exp).max() if exp.size else 0.0
    tol = 1e-6 * np.maximum(np.abs(exp), 1e-3 * scale)
    bad = np.abs(got - exp) > tol
    assert not bad.any(), "%s: %d of %d beyond 1e-6 rel (max abs diff %g)" % (
        what, int(bad.sum()), bad.size, float(np.abs(got - exp).max()))
    return int(np.sum(got != exp))


def device_and_oracle(w, names, nch=3):
    from paper_2012_08141_amd.grid import SparseGrid
    cap = w.R ** 3 if w.root_kind == "pointer" else 0
    g = SparseGrid(w.n, nch, w.root_kind, cap)
    o = oracle.OracleGrid(w.n, nch)
    for name, vals in w.channels.items():
        g.load_blocks(names[name], w.cells, vals)
    o.load(w.blocks, w.channels, names)
    return g, o


@pytest.mark.parametrize("fine_root,coarse_root", [("bitmask", "bitmask"), ("pointer", "pointer"),
                                                   ("bitmask", "pointer"), ("pointer", "bitmask")])
def test_transfers_match_oracle(fine_root, coarse_root):
    from paper_2012_08141_amd import engine as E
    say("transfers", fine_root, coarse_root)
    n = 64
    names = {"c0": 0, "c1": 1, "c2": 2}
    wf = I.random_blocks(21, n, 0.3, fine_root, channels=("c0", "c1", "c2"))
    wc = I.random_blocks(22, n // 2, 0.3, coarse_root, channels=("c0", "c1", "c2"))
    f, of = device_and_oracle(wf, names)
    c, oc = device_and_oracle(wc, names)
    E.reset()
    E.run_sequence([E.listgen(f)], 0)
    of.listgen()
    extra = I.random_blocks(23, n, 0.1, fine_root).blocks      # active, not listed
    f.activate(extra); of.activate(extra)
    # window 1: the restriction activates coarse parents (check kept)
    st = E.run_sequence([E.restrict(f, c, 0, 1, 0.375)], E.OPT_ALL)
    assert st["activations_demoted"] == 0
    of.restrict_to(oc, 0, 1, 0.375)
    torch.cuda.synchronize()
    cells = oc.active_cells()
    assert np.array_equal(c.active_cells(), cells)
    for q in range(3):
        assert np.array_equal(c.read_blocks(q, cells), oc.read_blocks(q, cells)), q
    # window 2: the same list restricted again: activation demoted, slots looked up
    st = E.run_sequence([E.restrict(f, c, 2, 2, -1.25)], E.OPT_ALL)
    assert st["activations_demoted"] == 1
    of.restrict_to(oc, 2, 2, -1.25)
    # window 3: prolongation back into the fine grid (inactive coarse blocks read 0)
    E.run_sequence([E.prolong(c, f, 1, 2)], E.OPT_ALL)
    of.prolong_from(oc, 1, 2)
    torch.cuda.synchronize()
    assert np.array_equal(c.active_cells(), oc.active_cells())
    for q in range(3):
        assert np.array_equal(c.read_blocks(q, cells), oc.read_blocks(q, cells)), q
    fc = of.active_cells()
    assert np.array_equal(f.active_cells(), fc)
    for q in range(3):
        assert np.array_equal(f.read_blocks(q, fc), of.read_blocks(q, fc)), q
    E.reset()


def test_restrict_into_empty_pointer_grid_fills_its_pool():
    """Coarse blocks allocated by the restriction take pool slots in any order;
    the values land by root cell, and a coarse pool that is too small is
    reported, not overrun."""
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd.grid import SparseGrid
    say("restrict into empty pointer grid")
    n = 64
    wf = I.random_blocks(31, n, 0.5, "pointer", channels=("c0",))
    f, of = device_and_oracle(wf, {"c0": 0}, 1)
    parents = np.unique(np.asarray(wf.blocks) // 2, axis=0)
    c = SparseGrid(n // 2, 1, "pointer", len(parents))
    oc = oracle.OracleGrid(n // 2, 1)
    E.reset()
    E.run_sequence([E.listgen(f), E.restrict(f, c, 0, 0, 0.125)], E.OPT_ALL)
    of.listgen(); of.restrict_to(oc, 0, 0, 0.125)
    torch.cuda.synchronize()
    cells = oc.active_cells()
    assert len(cells) == len(parents)
    assert np.array_equal(c.active_cells(), cells)
    assert np.array_equal(c.read_blocks(0, cells), oc.read_blocks(0, cells))
    small = SparseGrid(n // 2, 1, "pointer", max(1, len(parents) - 3))
    E.run_sequence([E.restrict(f, small, 0, 0, 0.125)], 0)
    torch.cuda.synchronize()
    assert small.device_status() & 1          # pool capacity exceeded
    E.reset()


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
@pytest.mark.parametrize("opt", [0, 15])
def test_vcycle_program(opt, root):
    """Two 3-level V-cycles on a 64^3 narrow band, eager and optimized, on both
    root kinds, against the oracle's V-cycle program; the optimized window
    launches far fewer tasks and demotes the second cycle's restrictions."""
    from paper_2012_08141_amd import engine as E, programs as PR
    say("vcycle opt", opt, root)
    w = I.band(3, n=64, root_kind=root)
    E.reset()
    levels = PR.mg_levels(w, 3)
    tasks = PR.mg_vcycle(levels) + PR.mg_vcycle(levels)
    st = E.run_sequence(tasks, opt)
    ref = OP.multigrid_program(w.n, w.blocks, w.channels["b"], 2, levels=3)
    torch.cuda.synchronize()
    if opt == 0:
        assert st["dispatches"] == len(tasks)
    else:
        assert st["dispatches"] < len(tasks) // 2
        assert st["activations_demoted"] >= 2
    for l in range(3):
        assert np.array_equal(levels[l].active_cells(), ref["level_cells"][l]), l
    exact = close_stencil(levels[0].read_blocks(0, ref["cells"]), ref["x"], "x")
    say("  values not bit-identical:", exact)
    E.reset()


def test_vcycle_full_size():
    """The multigrid workload at its benchmark size (256^3 band, 4 levels): one
    optimized V-cycle against the oracle, then three more cycles eager ==
    optimized bit for bit."""
    from paper_2012_08141_amd import engine as E, programs as PR
    say("vcycle 256 full")
    w = I.band(0, n=256)
    E.reset()
    lv = PR.mg_levels(w, 4)
    E.run_sequence(PR.mg_vcycle(lv), E.OPT_ALL)
    ref = OP.multigrid_program(w.n, w.blocks, w.channels["b"], 1, levels=4)
    torch.cuda.synchronize()
    for l in range(4):
        assert np.array_equal(lv[l].active_cells(), ref["level_cells"][l]), l
    close_stencil(lv[0].read_blocks(0, ref["cells"]), ref["x"], "x")
    E.reset()
    le, lo = PR.mg_levels(w, 4), PR.mg_levels(w, 4)
    E.run_sequence(sum((PR.mg_vcycle(le) for _ in range(3)), []), 0)
    E.reset()
    E.run_sequence(sum((PR.mg_vcycle(lo) for _ in range(3)), []), E.OPT_ALL)
    torch.cuda.synchronize()
    assert torch.equal(le[0].channel(0), lo[0].channel(0))
    E.reset()


def test_cleared_coarse_level_is_rebuilt():
    """Clearing a coarse level (a deactivating write) drops what the engine knew
    about restrictions into it: the next V-cycle activates its blocks again.
    Optimized equals eager bit for bit before and after the clear."""
    from paper_2012_08141_amd import engine as E, programs as PR
    say("vcycle with a cleared coarse level")
    w = I.band(5, n=64)
    E.reset()
    lo, le = PR.mg_levels(w, 3), PR.mg_levels(w, 3)
    for phase in range(2):
        E.run_sequence(PR.mg_vcycle(lo) + PR.mg_vcycle(lo), E.OPT_ALL)
        E.run_sequence(PR.mg_vcycle(le) + PR.mg_vcycle(le), 0)
        torch.cuda.synchronize()
        if phase == 1:
            # the cleared level got its blocks back from the restriction
            assert np.array_equal(lo[1].active_cells(), le[1].active_cells())
            assert len(lo[1].active_cells()) > 0
        for l in range(3):
            assert torch.equal(lo[l].channel(0), le[l].channel(0)), (phase, l)
        lo[1].clear(); le[1].clear()
    E.reset()
