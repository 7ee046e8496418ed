"""Runtime-compiled variants on the GPU (MI355X only): a fused element-wise
struct-for run through its compiled variant leaves every channel bit for bit
as the interpreter does -- the supplement's fill_array and chain_copy
microbenchmarks, the differentiation seed, and two normalisations each
fused with the clearing of its inputs (masses zero and nonzero), on both
roots; in background mode the interpreter runs until the variant is
loaded."""
import time

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
    E.set_option(L.AT_OPTION_VARIANTS, 0)
    E.reset()


def E_loaded():
    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd import engine as E
    return E.get_option(L.AT_OPTION_VARIANTS_LOADED)


def _program(name, g):
    from paper_2012_08141_amd import engine as E
    if name == "fill_array":
        return [E.fill(g, [0], 7.0) for _ in range(10)]
    if name == "chain_copy":
        return [E.copy(g, 1, 0), E.inc(g, 1, 1.0), E.copy(g, 2, 1), E.inc(g, 2, 4.0)]
    if name == "seed":
        return [E.fill(g, [3], 0.0), E.copy(g, 1, 0), E.axpy(g, 1, 0, 1.0), E.axpy(g, 1, 2, -2.0)]
    return [E.normalise(g, 0, 1, 4), E.fill(g, [0, 1, 2, 3], 0.0)] * 2


def _run(name, root, mode):
    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd.grid import SparseGrid
    E.reset()
    E.set_option(L.AT_OPTION_VARIANTS, mode)
    w = I.random_blocks(31, 64, 0.4, root, channels=tuple("c%d" % i for i in range(7)))
    g = SparseGrid(64, 7, root, len(w.cells) if root == "pointer" else 0)
    for i in range(7):
        v = w.channels["c%d" % i]
        if name == "normalise" and i == 0:
            v = np.where(v > 0, v, 0).astype(np.float32)     # masses: zero on about half the voxels
        g.load_blocks(i, w.cells, v)
    E.run_sequence([E.listgen(g)], E.OPT_ALL)
    loaded0 = E.get_option(L.AT_OPTION_VARIANTS_LOADED)
    # without dead store elimination, so fill_array's ten fills fuse rather
    # than shrink to one
    st = E.run_sequence([E.listgen(g)] + _program(name, g), E.OPT_ALL & ~E.OPT_DSE)
    torch.cuda.synchronize()
    used = E.get_option(L.AT_OPTION_VARIANTS_LOADED) - loaded0
    return [g.read_blocks(i, w.cells) for i in range(7)], st, used


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
@pytest.mark.parametrize("name", ["fill_array", "chain_copy", "seed", "normalise"])
def test_variant_equals_interpreter(name, root):
    say("variant", name, root)
    ref, st0, _ = _run(name, root, 0)
    got, st1, used = _run(name, root, 2)
    assert st0["dispatches"] == st1["dispatches"] == 1         # one fused launch
    assert used in (0, 1) and E_loaded() >= 1
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)


def test_background_compilation_switches_over():
    """Mode 1: the first runs use the interpreter while the variant compiles
    on the worker thread; once it is loaded the same window runs through it,
    with the same results."""
    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd.grid import SparseGrid
    say("variant background")
    E.set_option(L.AT_OPTION_VARIANTS, 1)
    w = I.random_blocks(32, 64, 0.4, "bitmask", channels=("a", "b", "c", "d"))
    g = SparseGrid(64, 4, "bitmask")
    for i, k in enumerate("abcd"):
        g.load_blocks(i, w.cells, w.channels[k])
    E.run_sequence([E.listgen(g)], E.OPT_ALL)
    prog = [E.copy(g, 1, 0), E.axpy(g, 1, 2, 0.5), E.inc(g, 3, 2.0), E.axpy(g, 3, 1, -1.0)]
    loaded0 = E.get_option(L.AT_OPTION_VARIANTS_LOADED)
    t0 = time.time()
    runs = 0
    while E.get_option(L.AT_OPTION_VARIANTS_LOADED) == loaded0 and time.time() - t0 < 60:
        E.run_sequence(prog, E.OPT_ALL)
        runs += 1
        time.sleep(0.02)
    torch.cuda.synchronize()
    assert E.get_option(L.AT_OPTION_VARIANTS_LOADED) == loaded0 + 1, "variant never loaded"
    # the same result as the interpreter, from the state the runs left: x1 =
    # c0 + 0.5 c2 every run; x3 grows by 2 - x1 per run
    a, c = w.channels["a"], w.channels["c"]
    x1 = (a + np.float32(0.5) * c).astype(np.float32)
    x3 = w.channels["d"].copy()
    for _ in range(runs):
        x3 = (x3 + np.float32(2.0)).astype(np.float32)
        x3 = (x3 + np.float32(-1.0) * x1).astype(np.float32)
    assert np.array_equal(g.read_blocks(1, w.cells), x1)
    assert np.array_equal(g.read_blocks(3, w.cells), x3)
