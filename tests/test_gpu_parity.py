"""Parity of the HIP path against the CPU oracle, element by element, on the
same seeded inputs (MI355X only).

Bars: activation masks and lists bit-exact (lists compared in order, since
both sides emit ascending cells); fp32 stencil values within 1e-6 relative
(|g - o| <= 1e-6 * max(|o|, 1e-3 * max|o|)); the stencils are designed to
match bit for bit (same operation order, no contraction), which the tests
also report.
"""
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


def grid_pair(w, nch, names, cap=0):
    from paper_2012_08141_amd.grid import SparseGrid
    cap = cap or (w.R ** 3 if w.root_kind == "pointer" else 0)
    g = SparseGrid(w.n, nch, w.root_kind, cap)
    o = oracle.OracleGrid(w.n, nch)
    cells = w.cells
    for name, vals in w.channels.items():
        g.load_blocks(names[name], cells, vals)
    o.load(w.blocks, w.channels, names)
    return g, o


# ----------------------------------------------------------- activation/list
@pytest.mark.parametrize("root", ["bitmask", "pointer"])
@pytest.mark.parametrize("n,frac,seed", [(32, 0.5, 0), (64, 0.1, 1), (128, 0.03, 2), (72, 0.2, 3)])
def test_activate_and_listgen(root, n, frac, seed):
    from paper_2012_08141_amd.grid import SparseGrid
    say("activate/listgen", root, n, frac, seed)
    w = I.random_blocks(seed, n, frac, root)
    rng = np.random.default_rng(seed)
    # block coordinates with duplicates (concurrent activation of one cell)
    coords = np.concatenate([w.blocks, w.blocks[rng.integers(0, max(1, w.nblocks), w.nblocks)]])
    rng.shuffle(coords)
    # voxel coordinates, some outside the domain
    vox = rng.integers(-4, n + 4, (257, 3)).astype(np.int32)
    g = SparseGrid(n, 1, root, (n // 8) ** 3 if root == "pointer" else 0)
    o = oracle.OracleGrid(n, 1)
    g.activate(coords)
    g.activate(vox, kind=0)
    g.listgen()
    o.activate(coords)
    o.activate(vox, "voxel")
    o.listgen()
    torch.cuda.synchronize()
    assert np.array_equal(g.list_cells(), o.list())
    assert np.array_equal(g.active_cells(), o.active_cells())
    assert g.active_count() == len(o.active_cells())
    assert g.device_status() == 0
    # activating again changes nothing
    g.activate(coords)
    g.listgen()
    assert np.array_equal(g.list_cells(), o.list())


@pytest.mark.parametrize("root,n,frac", [("bitmask", 576, 0.05), ("pointer", 576, 0.05), ("pointer", 1024, 0.03),
                                         ("pointer", 1296, 0.01), ("pointer", 2048, 0.004)])
def test_listgen_look_back_on_large_roots(root, n, frac):
    """Roots of more than 262,144 cells take the single-pass look-back scan
    across workgroups (8 to 64 cells per thread, up to 1,024 workgroups).
    About frac of the blocks at random plus one dense run of 20,000
    consecutive cells (whole workgroups with every cell active); the list
    and count must equal the oracle's ascending scan bit for bit (Section 3.2)."""
    from paper_2012_08141_amd.grid import SparseGrid
    say("listgen look-back", root, n, frac)
    R = n // 8
    assert R ** 3 > 262144
    rng = np.random.default_rng([n, 17])
    cells = np.flatnonzero(rng.uniform(size=R ** 3) < frac)
    start = R ** 3 // 3
    cells = np.union1d(cells, np.arange(start, start + 20000))
    coords = np.stack(np.unravel_index(cells, (R, R, R)), axis=1).astype(np.int32)
    rng.shuffle(coords)
    g = SparseGrid(n, 1, root, len(cells) if root == "pointer" else 0)
    o = oracle.OracleGrid(n, 1)
    g.activate(coords)
    g.listgen()
    o.activate(coords)
    o.listgen()
    torch.cuda.synchronize()
    assert g.device_status() == 0
    assert g.list_count() == len(cells)
    assert np.array_equal(g.list_cells(), o.list())
    g.listgen()                          # a second generation (new epoch) over the same flags
    assert np.array_equal(g.list_cells(), o.list())
    assert g.device_status() == 0
    del g


def test_empty_grid_and_empty_activation():
    from paper_2012_08141_amd.grid import SparseGrid
    say("empty grids")
    for root in ("bitmask", "pointer"):
        g = SparseGrid(16, 3, root, 8 if root == "pointer" else 0)
        g.activate(np.zeros((0, 3), np.int32))
        g.listgen()
        g.run_stencil(3, [0, 1, 2], 0.0, True)
        g.run_stencil(1, [0, 1], 0.1, False)
        torch.cuda.synchronize()
        assert g.list_count() == 0 and len(g.active_cells()) == 0


def test_pointer_pool_overflow_is_reported():
    from paper_2012_08141_amd.grid import SparseGrid
    say("pool overflow")
    g = SparseGrid(64, 1, "pointer", 10)
    coords = np.array([[a, b, 0] for a in range(4) for b in range(4)], np.int32)   # 16 blocks > 10
    g.activate(coords)
    g.listgen()
    bits = g.device_status(clear=True)
    assert bits & 1
    assert len(g.active_cells()) == 10 and g.list_count() == 10
    assert g.device_status() == 0


# --------------------------------------------------------- struct-for ops
OPS = {
    "lap_update": (1, [0, 1], 0.1, [1]),
    "axpy": (2, [0, 1], 0.5, [0]),
    "jacobi": (3, [0, 2, 1], 0.0, [1]),
    "copy": (4, [3, 0], 0.0, [3]),
    "fill": (5, [1, 3], -2.5, [1, 3]),
    "inc": (6, [2], 0.25, [2]),
    "diffuse": (7, [0, 2, 3], 0.1, [3]),
    "diffuse_adj": (8, [0, 2, 1, 3, 4], 0.1, [3, 4]),
}


ORACLE_CALLS = {
    "lap_update": lambda o: o.lap_update(0, 1, 0.1),
    "axpy": lambda o: o.axpy(0, 1, 0.5),
    "jacobi": lambda o: o.jacobi(0, 2, 1),
    "copy": lambda o: o.copy(3, 0),
    "fill": lambda o: (o.fill(1, -2.5), o.fill(3, -2.5)),
    "inc": lambda o: o.inc(2, 0.25),
    "diffuse": lambda o: o.diffuse(0, 2, 3, 0.1),
    "diffuse_adj": lambda o: o.diffuse_adj(0, 2, 1, 3, 4, 0.1),
}


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
@pytest.mark.parametrize("check", [1, 0])
@pytest.mark.parametrize("opname", list(OPS))
def test_struct_for_op(opname, check, root):
    op, ch, p, outs = OPS[opname]
    say("struct-for", opname, "check", check, root)
    n = 64
    w = I.random_blocks(11, n, 0.3, root, channels=("c0", "c1", "c2", "c3", "c4"))
    w.channels["c2"] = np.abs(w.channels["c2"]) + 0.5       # a positive conductance
    names = {"c%d" % q: q for q in range(5)}
    g, o = grid_pair(w, 5, names)
    g.listgen()
    o.listgen()
    # blocks activated after the list was built are active but not listed
    extra = I.random_blocks(12, n, 0.15, root).blocks
    g.activate(extra)
    o.activate(extra)
    g.run_stencil(op, ch, p, bool(check))
    ORACLE_CALLS[opname](o)
    torch.cuda.synchronize()
    cells = o.active_cells()
    assert np.array_equal(g.active_cells(), cells)
    exact = 0
    for q in range(5):
        exact += close_stencil(g.read_blocks(q, cells), o.read_blocks(q, cells), "%s ch%d" % (opname, q))
    say("  values not bit-identical:", exact)


def test_normalise():
    say("normalise")
    n = 64
    w = I.random_blocks(13, n, 0.3, "pointer", channels=("m", "mv0", "mv1", "mv2"))
    w.channels["m"] = np.where(w.channels["m"] > 0, w.channels["m"], 0).astype(np.float32)
    names = {"m": 0, "mv0": 1, "mv1": 2, "mv2": 3}
    g, o = grid_pair(w, 7, names)
    g.listgen(); o.listgen()
    g.run_stencil(9, [0, 1, 4], 0.0, False)
    o.normalise(0, 1, 4)
    torch.cuda.synchronize()
    cells = o.active_cells()
    for q in range(7):
        assert np.array_equal(g.read_blocks(q, cells), o.read_blocks(q, cells)), q


# ------------------------------------------------------- workload programs
@pytest.mark.parametrize("opt", [0, 15])
def test_shell_program(opt):
    """The 64^3 shell workload at its full size, 10 steps, eager and optimized."""
    from paper_2012_08141_amd import engine as E, programs as PR
    say("shell program opt", opt)
    w = I.shell(0)
    g = PR.load_workload(w, PR.SHELL, 2)
    coords = torch.as_tensor(w.blocks, device="cuda")
    E.run_sequence(PR.shell_setup(g, coords), opt)
    st = E.run_sequence(sum((PR.shell_step(g, coords) for _ in range(10)), []), opt)
    assert st["dispatches"] == (50 if opt == 0 else 20)
    ref = OP.shell_program(w.n, w.blocks, w.channels["a"], 10)
    torch.cuda.synchronize()
    assert np.array_equal(g.active_cells(), ref["cells"])
    assert np.array_equal(g.list_cells(), ref["list"])
    close_stencil(g.read_blocks(0, ref["cells"]), ref["a"], "a")
    close_stencil(g.read_blocks(1, ref["cells"]), ref["out"], "out")


@pytest.mark.parametrize("opt", [0, 15])
def test_jacobi_band_reduced(opt):
    """The narrow-band recipe on a 128^3 domain, 100 iterations."""
    from paper_2012_08141_amd import engine as E, programs as PR
    say("jacobi band128 opt", opt)
    w = I.band(0, n=128)
    g = PR.load_workload(w, PR.JACOBI, 3)
    st = E.run_sequence(sum((PR.jacobi_step(g) for _ in range(100)), []), opt)
    assert st["dispatches"] == (300 if opt == 0 else 201)
    ref = OP.jacobi_program(w.n, w.blocks, w.channels["b"], 100)
    torch.cuda.synchronize()
    close_stencil(g.read_blocks(0, ref["cells"]), ref["x"], "x")
    close_stencil(g.read_blocks(1, ref["cells"]), ref["xn"], "xn")


def test_jacobi_band_full_size():
    """The narrow-band workload at its full size (512^3): 12 iterations against the oracle
    (x and xn, every voxel), then 100 iterations eager == optimized bit for bit."""
    from paper_2012_08141_amd import engine as E, programs as PR
    say("jacobi band512 full")
    w = I.band(0)
    ref = OP.jacobi_program(w.n, w.blocks, w.channels["b"], 12)
    g = PR.load_workload(w, PR.JACOBI, 3)
    E.run_sequence(sum((PR.jacobi_step(g) for _ in range(12)), []), E.OPT_ALL)
    torch.cuda.synchronize()
    close_stencil(g.read_blocks(0, ref["cells"]), ref["x"], "x")
    close_stencil(g.read_blocks(1, ref["cells"]), ref["xn"], "xn")
    ge = PR.load_workload(w, PR.JACOBI, 3)
    go = PR.load_workload(w, PR.JACOBI, 3)
    E.run_sequence(sum((PR.jacobi_step(ge) for _ in range(100)), []), 0)
    E.run_sequence(sum((PR.jacobi_step(go) for _ in range(100)), []), E.OPT_ALL)
    torch.cuda.synchronize()
    xe, xo = ge.channel(0), go.channel(0)
    assert torch.equal(xe, xo)
    del ge, go, g


def test_fused_elementwise_program():
    """Section 6.1's example on the device: listgen, x += 1, listgen, x += 2
    runs as listgen + one fused struct-for and equals the oracle."""
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd.grid import SparseGrid
    say("fused inc")
    w = I.random_blocks(5, 64, 0.2, "pointer", channels=("x",))
    g, o = grid_pair(w, 1, {"x": 0})
    tasks = [E.listgen(g), E.inc(g, 0, 1.0), E.listgen(g), E.inc(g, 0, 2.0)]
    st = E.run_sequence(tasks, E.OPT_ALL)
    assert st["dispatches"] == 2 and st["fusions"] == 1
    o.listgen(); o.inc(0, 1.0); o.listgen(); o.inc(0, 2.0)
    torch.cuda.synchronize()
    cells = o.active_cells()
    assert np.array_equal(g.read_blocks(0, cells), o.read_blocks(0, cells))


HEADS = {
    "jacobi": (lambda E, g: E.jacobi(g, 0, 1, 2), lambda o: o.jacobi(0, 1, 2)),
    "lap_update": (lambda E, g: E.lap_update(g, 0, 2, 0.1), lambda o: o.lap_update(0, 2, 0.1)),
    "diffuse": (lambda E, g: E.diffuse(g, 0, 1, 2, 0.1), lambda o: o.diffuse(0, 1, 2, 0.1)),
}


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
@pytest.mark.parametrize("head", list(HEADS))
def test_fused_stencil_with_elementwise_tail(root, head):
    """A single-output stencil fused with the element-wise tasks after it (the
    tail reads the stencil's output, its stencil input and other channels,
    and writes them) equals the oracle running the tasks one by one, bit for
    bit."""
    from paper_2012_08141_amd import engine as E
    say("fused stencil + tail", head, root)
    w = I.random_blocks(17, 64, 0.3, root, channels=("c0", "c1", "c2", "c3", "c4", "c5"))
    w.channels["c1"] = np.abs(w.channels["c1"]) + 0.5       # a positive conductance for diffuse
    names = {"c%d" % q: q for q in range(6)}
    g, o = grid_pair(w, 6, names)
    E.reset()
    E.run_sequence([E.listgen(g)], E.OPT_ALL)
    mk, ref = HEADS[head]
    tasks = [mk(E, g), E.axpy(g, 2, 0, -1.0), E.inc(g, 3, 0.5), E.copy(g, 4, 2),
             E.axpy(g, 3, 1, 2.0), E.fill(g, [5], 1.5), E.axpy(g, 2, 3, 0.25)]
    plan, _ = E.plan_sequence(tasks, E.OPT_ALL)
    assert len(plan) == 1 and len(plan[0]["members"]) == len(tasks)
    st = E.run_sequence(tasks, E.OPT_ALL)
    assert st["dispatches"] == 1
    o.listgen()
    ref(o); o.axpy(2, 0, -1.0); o.inc(3, 0.5); o.copy(4, 2); o.axpy(3, 1, 2.0); o.fill(5, 1.5)
    o.axpy(2, 3, 0.25)
    torch.cuda.synchronize()
    cells = o.active_cells()
    for q in range(6):
        assert np.array_equal(g.read_blocks(q, cells), o.read_blocks(q, cells)), q
    E.reset()
