"""Semi-Lagrangian advection on the device against the oracle.

The advection op (the building block of the paper's MacCormack benchmark,
Section 8.2) samples q trilinearly at the back-traced point of every voxel,
in a fixed corner order, so it matches the oracle bit for bit: alone, with
and without the activation check, on both root kinds, with back-traced
points in other, inactive or absent blocks; and as the three-field program,
whose optimized form fuses the three advections and the three copies into
two launches per step."""
import numpy as np
import pytest

import oracle
from oracle import programs as OP
from paper_2012_08141_amd import _lib as L
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


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
@pytest.mark.parametrize("check", [True, False])
@pytest.mark.parametrize("rk3", [False, True])
def test_advect_op(root, check, rk3):
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd.grid import SparseGrid
    say("advect op", root, check, "rk3" if rk3 else "euler")
    n = 64
    w = I.random_blocks(31, n, 0.3, root, channels=("q", "v0", "v1", "v2", "o"))
    for c in ("v0", "v1", "v2"):
        w.channels[c] = (w.channels[c] * 9.0).astype(np.float32)      # back-traces up to ~8 voxels
    names = {"q": 0, "v0": 1, "v1": 2, "v2": 3, "o": 4}
    g = SparseGrid(n, 5, root, w.R ** 3 if root == "pointer" else 0)
    o = oracle.OracleGrid(n, 5)
    for name, vals in w.channels.items():
        g.load_blocks(names[name], w.cells, vals)
    o.load(w.blocks, w.channels, names)
    g.listgen(); o.listgen()
    extra = I.random_blocks(32, n, 0.1, root).blocks
    g.activate(extra); o.activate(extra)
    if rk3:
        E.run_sequence([E.advect_sl(g, 0, 1, 4, 0.6, rk3=True)], 15 if not check else 0)
    else:
        g.run_stencil(L.AT_OP_ADVECT, [0, 1, 4], 0.6, check)
    o.advect_sl(0, 1, 4, 0.6, rk3)
    torch.cuda.synchronize()
    cells = o.active_cells()
    assert np.array_equal(g.active_cells(), cells)
    for q in range(5):
        assert np.array_equal(g.read_blocks(q, cells), o.read_blocks(q, cells)), q


@pytest.mark.parametrize("opt", [0, 15])
def test_advection_program(opt):
    """Three steps of the three-field program on a 64^3 tube, one window per
    step, eager and optimized, bit-exact against the oracle."""
    from paper_2012_08141_amd import engine as E, programs as PR
    say("advection program opt", opt)
    w = I.tube(1, n=64)
    dt = w.params["dt"]
    E.reset()
    g = PR.load_workload(w, {"q0": 0, "q1": 1, "q2": 2, "v0": 3, "v1": 4, "v2": 5}, 9)
    step = E.prepare(PR.advection_step(g, dt))
    disp = [E.run_sequence(step, opt)["dispatches"] for _ in range(3)]
    assert disp[-1] == (12 if opt == 0 else 2)
    ref = OP.advection_program(w.n, w.blocks, w.channels, dt, 3)
    torch.cuda.synchronize()
    for c in range(3):
        assert np.array_equal(g.read_blocks(c, ref["cells"]), ref["q"][c]), c
    E.reset()


def test_advection_full_size():
    """The advection workload at its benchmark size (256^3 tube, 10,112 blocks):
    one optimized step against the oracle."""
    from paper_2012_08141_amd import engine as E, programs as PR
    say("advection tube256 full")
    w = I.tube(0)
    dt = w.params["dt"]
    E.reset()
    g = PR.load_workload(w, {"q0": 0, "q1": 1, "q2": 2, "v0": 3, "v1": 4, "v2": 5}, 9)
    E.run_sequence(PR.advection_step(g, dt), E.OPT_ALL)
    ref = OP.advection_program(w.n, w.blocks, w.channels, dt, 1)
    torch.cuda.synchronize()
    for c in range(3):
        assert np.array_equal(g.read_blocks(c, ref["cells"]), ref["q"][c]), c
    E.reset()


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
def test_maccormack_op(root):
    """The MacCormack correction (forward and backward advection, then the
    clamped correction) bit-exact against the oracle."""
    from paper_2012_08141_amd.grid import SparseGrid
    say("maccormack op", root)
    n = 64
    w = I.random_blocks(33, n, 0.3, root, channels=("q", "v0", "v1", "v2"))
    for c in ("v0", "v1", "v2"):
        w.channels[c] = (w.channels[c] * 5.0).astype(np.float32)
    names = {"q": 0, "v0": 1, "v1": 2, "v2": 3}
    g = SparseGrid(n, 7, root, w.R ** 3 if root == "pointer" else 0)
    o = oracle.OracleGrid(n, 7)
    for name, vals in w.channels.items():
        g.load_blocks(names[name], w.cells, vals)
    o.load(w.blocks, w.channels, names)
    g.listgen(); o.listgen()
    g.run_stencil(L.AT_OP_ADVECT, [0, 1, 4], 0.8, False)
    g.run_stencil(L.AT_OP_ADVECT, [4, 1, 5], -0.8, False)
    g.run_stencil(L.AT_OP_MACCORMACK, [0, 1, 4, 5, 6], 0.8, False)
    o.advect_sl(0, 1, 4, 0.8); o.advect_sl(4, 1, 5, -0.8); o.maccormack(0, 1, 4, 5, 6, 0.8)
    torch.cuda.synchronize()
    cells = o.active_cells()
    for q in range(7):
        assert np.array_equal(g.read_blocks(q, cells), o.read_blocks(q, cells)), q


@pytest.mark.parametrize("opt", [0, 15])
@pytest.mark.parametrize("rk3", [False, True])
def test_maccormack_program(opt, rk3):
    """Two MacCormack steps of three fields on a 64^3 tube, eager and optimized
    (5 launches per step instead of 24), Euler and RK3 back-traces, bit-exact
    against the oracle."""
    from paper_2012_08141_amd import engine as E, programs as PR
    say("maccormack program opt", opt, "rk3" if rk3 else "euler")
    w = I.tube(2, n=64)
    dt = w.params["dt"]
    E.reset()
    g = PR.load_workload(w, {"q0": 0, "q1": 1, "q2": 2, "v0": 3, "v1": 4, "v2": 5}, 15)
    step = E.prepare(PR.maccormack_step(g, dt, rk3))
    disp = [E.run_sequence(step, opt)["dispatches"] for _ in range(2)]
    assert disp[-1] == (24 if opt == 0 else 5)
    ref = OP.maccormack_program(w.n, w.blocks, w.channels, dt, 2, rk3=rk3)
    torch.cuda.synchronize()
    for c in range(3):
        assert np.array_equal(g.read_blocks(c, ref["cells"]), ref["q"][c]), c
    E.reset()


# ---- the tile programs through their compiled variants (AT_OPTION_VARIANTS)

def _variants(mode):
    from paper_2012_08141_amd import engine as E
    E.set_option(L.AT_OPTION_VARIANTS, mode)


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
@pytest.mark.parametrize("rk3", [False, True])
def test_compiled_tile_program_far_traces(root, rk3):
    """A fused node of two semi-Lagrangian ops, a MacCormack correction and
    element-wise ops, compiled for its op sequence: back-traces up to ~8
    voxels leave the staged tile (sampled from the grid instead), reach
    inactive and absent blocks; bit-exact against the oracle run op by op."""
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd.grid import SparseGrid
    say("compiled tile program", root, "rk3" if rk3 else "euler")
    n = 64
    w = I.random_blocks(35, n, 0.3, root, channels=("q0", "q1", "v0", "v1", "v2", "f", "b"))
    for c in ("v0", "v1", "v2"):
        w.channels[c] = (w.channels[c] * 9.0).astype(np.float32)
    names = {"q0": 0, "q1": 1, "v0": 2, "v1": 3, "v2": 4, "f": 5, "b": 6}
    try:
        E.reset()
        _variants(2)
        g = SparseGrid(n, 10, root, w.R ** 3 if root == "pointer" else 0)
        o = oracle.OracleGrid(n, 10)
        for name, vals in w.channels.items():
            g.load_blocks(names[name], w.cells, vals)
        o.load(w.blocks, w.channels, names)
        extra = I.random_blocks(36, n, 0.1, root).blocks      # listed blocks holding zeros
        g.activate(extra)
        o.activate(extra); o.listgen()
        loaded = E.get_option(L.AT_OPTION_VARIANTS_LOADED)
        prog = [E.listgen(g), E.advect_sl(g, 0, 2, 7, 0.6, rk3), E.advect_sl(g, 1, 2, 8, 0.6, rk3),
                E.maccormack(g, 0, 2, 5, 6, 9, 0.6, rk3), E.copy(g, 5, 9), E.inc(g, 6, 0.25)]
        st = E.run_sequence(prog, E.OPT_ALL)
        assert st["dispatches"] == 2, st          # the list generation and one fused node
        assert E.get_option(L.AT_OPTION_VARIANTS_LOADED) > loaded
        o.advect_sl(0, 2, 7, 0.6, rk3); o.advect_sl(1, 2, 8, 0.6, rk3)
        o.maccormack(0, 2, 5, 6, 9, 0.6, rk3); o.copy(5, 9); o.inc(6, 0.25)
        torch.cuda.synchronize()
        cells = o.list()
        assert np.array_equal(np.sort(g.list_cells()), np.sort(cells))
        for q in range(10):
            assert np.array_equal(g.read_blocks(q, cells), o.read_blocks(q, cells)), q
    finally:
        _variants(0)
        E.reset()


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
@pytest.mark.parametrize("mac", [False, True])
def test_compiled_tile_programs_match_oracle(mac, root):
    """The three-field advection and RK3 MacCormack programs on a 64^3 tube,
    optimized, with their fused nodes compiled: bit-exact against the
    oracle, on both root kinds."""
    from paper_2012_08141_amd import engine as E, programs as PR
    say("compiled tube programs", "maccormack" if mac else "advection", root)
    w = I.tube(3, n=64, root_kind=root)
    dt = w.params["dt"]
    try:
        E.reset()
        _variants(2)
        loaded = E.get_option(L.AT_OPTION_VARIANTS_LOADED)
        g = PR.load_workload(w, {"q0": 0, "q1": 1, "q2": 2, "v0": 3, "v1": 4, "v2": 5}, 15 if mac else 9)
        step = E.prepare(PR.maccormack_step(g, dt, rk3=True) if mac else PR.advection_step(g, dt))
        for _ in range(2):
            E.run_sequence(step, E.OPT_ALL)
        assert E.get_option(L.AT_OPTION_VARIANTS_LOADED) > loaded
        ref = (OP.maccormack_program(w.n, w.blocks, w.channels, dt, 2, rk3=True) if mac else
               OP.advection_program(w.n, w.blocks, w.channels, dt, 2))
        torch.cuda.synchronize()
        for c in range(3):
            assert np.array_equal(g.read_blocks(c, ref["cells"]), ref["q"][c]), c
    finally:
        _variants(0)
        E.reset()


def test_compiled_tile_program_background():
    """Mode 1: the fused node runs the interpreted tile kernel while its
    variant compiles on the worker thread, then through the variant; both
    leave the oracle's result (the node rewrites its outputs from unchanged
    inputs, so every run gives the same values)."""
    import time
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd.grid import SparseGrid
    say("compiled tile program, background")
    n = 64
    w = I.random_blocks(37, n, 0.3, "bitmask", channels=("q0", "q1", "v0", "v1", "v2"))
    for c in ("v0", "v1", "v2"):
        w.channels[c] = (w.channels[c] * 3.0).astype(np.float32)
    names = {"q0": 0, "q1": 1, "v0": 2, "v1": 3, "v2": 4}
    try:
        E.reset()
        _variants(1)
        g = SparseGrid(n, 7, "bitmask")
        o = oracle.OracleGrid(n, 7)
        for name, vals in w.channels.items():
            g.load_blocks(names[name], w.cells, vals)
        o.load(w.blocks, w.channels, names)
        o.listgen()
        o.advect_sl(0, 2, 5, 0.45); o.advect_sl(1, 2, 6, 0.45)
        cells = o.list()
        prog = [E.listgen(g), E.advect_sl(g, 0, 2, 5, 0.45), E.advect_sl(g, 1, 2, 6, 0.45)]
        loaded0 = E.get_option(L.AT_OPTION_VARIANTS_LOADED)
        E.run_sequence(prog, E.OPT_ALL)
        torch.cuda.synchronize()
        for q in (5, 6):                                # the interpreted tile kernel's result
            assert np.array_equal(g.read_blocks(q, cells), o.read_blocks(q, cells)), q
        t0 = time.time()
        while E.get_option(L.AT_OPTION_VARIANTS_LOADED) == loaded0 and time.time() - t0 < 60:
            E.run_sequence(prog, E.OPT_ALL)
            time.sleep(0.02)
        assert E.get_option(L.AT_OPTION_VARIANTS_LOADED) == loaded0 + 1, "variant never loaded"
        g.load_blocks(5, w.cells, np.zeros((len(w.cells), 512), np.float32))
        E.run_sequence(prog, E.OPT_ALL)                 # through the variant
        torch.cuda.synchronize()
        for q in range(7):
            assert np.array_equal(g.read_blocks(q, cells), o.read_blocks(q, cells)), q
    finally:
        _variants(0)
        E.reset()


@pytest.mark.parametrize("case", ["empty", "corner-block", "ragged"])
def test_compiled_tile_program_edge_cases(case):
    """Compiled tile programs on an empty list (no block: nothing written),
    on one block at the domain's corner (most of its halo outside the
    domain), and on a 40^3-voxel domain (R = 5, not a multiple of the
    workgroup slicing); bit-exact against the oracle."""
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd.grid import SparseGrid
    say("compiled tile program edge case", case)
    n = 40 if case == "ragged" else 32
    if case == "empty":
        blocks = np.zeros((0, 3), np.int32)
    elif case == "corner-block":
        blocks = np.array([[0, 0, 0]], np.int32)
    else:
        blocks = I.random_blocks(38, n, 0.5, "bitmask").blocks
    rng = np.random.default_rng(7)
    nb = len(blocks)
    chans = {k: rng.uniform(-1, 1, (nb, 512)).astype(np.float32) for k in ("q0", "q1")}
    for k in ("v0", "v1", "v2"):
        chans[k] = rng.uniform(-4, 4, (nb, 512)).astype(np.float32)
    names = {"q0": 0, "q1": 1, "v0": 2, "v1": 3, "v2": 4}
    try:
        E.reset()
        _variants(2)
        g = SparseGrid(n, 8, "bitmask")
        o = oracle.OracleGrid(n, 8)
        if nb:
            g.activate(blocks)
            cells = ((blocks[:, 0].astype(np.int64) * (n // 8) + blocks[:, 1]) * (n // 8) + blocks[:, 2])
            for k, q in names.items():
                g.load_blocks(q, cells, chans[k])
            o.load(blocks, chans, names)
        o.listgen()
        prog = [E.listgen(g), E.advect_sl(g, 0, 2, 5, 0.7, True), E.advect_sl(g, 1, 2, 6, 0.7, True),
                E.maccormack(g, 0, 2, 5, 1, 7, 0.7, True)]
        st = E.run_sequence(prog, E.OPT_ALL)
        assert st["dispatches"] == 2, st
        o.advect_sl(0, 2, 5, 0.7, True); o.advect_sl(1, 2, 6, 0.7, True); o.maccormack(0, 2, 5, 1, 7, 0.7, True)
        torch.cuda.synchronize()
        cl = o.list()
        assert np.array_equal(np.sort(g.list_cells()), np.sort(cl))
        for q in range(8):
            assert np.array_equal(g.read_blocks(q, cl), o.read_blocks(q, cl)), q
        assert g.device_status() == 0
    finally:
        _variants(0)
        E.reset()
