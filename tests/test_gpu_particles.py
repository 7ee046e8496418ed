"""Particle transfers on the GPU against the oracle (MI355X only).

Bars: active sets bit-exact; one P2G within the summation bound
|g - o| <= 1e-5 * A (A = per node and channel sum of |term|, from the
oracle); the gather, which sums in a fixed order, within
1e-5 * max(|o|, 0.1 * max|o|); the particle state after many steps within
1e-5 * max(|o|, s) where s is 0.1 * max|x0| for positions and
0.1 * max|v0| for velocities: fp32 atomics reorder the momentum sums, whose
rounding error is set by the scattered terms (the initial particle speeds),
not by the much smaller grid-averaged velocity that comes back.
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


@pytest.fixture
def bin_reuse():
    from paper_2012_08141_amd import _lib as L, engine as E
    default = E.get_option(L.AT_OPTION_BIN_REUSE)
    yield lambda k: E.set_option(L.AT_OPTION_BIN_REUSE, k)
    E.set_option(L.AT_OPTION_BIN_REUSE, default)


def close_state(got, exp, what, scale=None):
    exp = np.asarray(exp, np.float64)
    got = np.asarray(got, np.float64)
    s = 0.1 * np.abs(exp).max() if scale is None else scale
    tol = 1e-5 * np.maximum(np.abs(exp), s)
    bad = np.abs(got - exp) > tol
    assert not bad.any(), "%s: %d of %d beyond tolerance (max diff %g)" % (
        what, int(bad.sum()), bad.size, float(np.abs(got - exp).max()))


@pytest.mark.parametrize("binned", [False, True])
@pytest.mark.parametrize("root", ["pointer", "bitmask"])
@pytest.mark.parametrize("act", [0, 1])
@pytest.mark.parametrize("n,np_,lo,hi", [(64, 20000, 0.1, 0.6), (128, 3001, 0.1, 0.6), (32, 5000, -0.03, 1.03)])
def test_p2g_matches_oracle_within_summation_bound(root, act, n, np_, lo, hi, binned):
    """Direct and binned scatter; the last case puts particles on and beyond
    the domain boundary (nodes outside skipped; centre nodes outside send a
    particle down the direct path inside the binned scatter)."""
    from paper_2012_08141_amd.grid import SparseGrid
    say("p2g", root, act, n, np_, lo, hi, "binned" if binned else "direct")
    p = I.random_particles(3, n, np_, lo, hi, root)
    ref = OP.p2g_once(n, None, p.x, p.v, p.m, "f32")
    g = SparseGrid(n, 8, root, (n // 8) ** 3 if root == "pointer" else 0, particle_capacity=np_ if binned else 0)
    x, v, m = (torch.as_tensor(a, device="cuda").contiguous() for a in (p.x, p.v, p.m))
    import ctypes
    from paper_2012_08141_amd import _lib as L
    ch = (ctypes.c_int32 * 2)(0, 1)
    L.check(L.lib().at_p2g(g.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                           ctypes.c_void_p(m.data_ptr()), np_, 1.0 / n, ch, act,
                           torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    cells = ref["cells"]
    assert np.array_equal(g.active_cells(), cells)
    assert g.device_status() == 0
    got = [g.read_blocks(0, cells)] + [g.read_blocks(1 + c, cells) for c in range(3)]
    exp = [ref["m"]] + ref["mv"]
    for q in range(4):
        A = ref["abs"][q].astype(np.float64)
        err = np.abs(got[q].astype(np.float64) - exp[q].astype(np.float64))
        assert np.all(err <= 1e-5 * A + 1e-30), ("channel", q, float((err / np.maximum(A, 1e-30)).max()))
    # total mass is the number of particles (weights partition unity) when
    # every node lies in the domain
    if lo > 0 and hi < 1:
        assert abs(got[0].astype(np.float64).sum() - np_) < 1e-3 * np_


def test_g2p_matches_oracle():
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd.grid import SparseGrid
    say("g2p")
    n = 64
    w = I.random_blocks(21, n, 0.6, "pointer", channels=("v0", "v1", "v2"))
    p = I.random_particles(4, n, 5000, 0.05, 0.95)
    g = SparseGrid(n, 3, "pointer", (n // 8) ** 3)
    o = oracle.OracleGrid(n, 3)
    for q in range(3):
        g.load_blocks(q, w.cells, w.channels["v%d" % q])
    o.load(w.blocks, w.channels, {"v0": 0, "v1": 1, "v2": 2})
    x = torch.as_tensor(p.x, device="cuda").contiguous()
    v = torch.zeros_like(x)
    E.run_sequence([E.g2p(g, x, v, 1.0 / n, 0)], 0)
    torch.cuda.synchronize()
    exp = o.g2p(0, p.x, float(n))
    got = v.cpu().numpy()
    close_state(got, exp, "g2p")
    say("  bit-identical:", bool(np.array_equal(got, exp)))


@pytest.mark.parametrize("root", ["pointer", "bitmask"])
@pytest.mark.parametrize("n,np_,lo,hi,shift", [(64, 20000, 0.1, 0.6, 0.0), (32, 5000, -0.03, 1.03, 0.0),
                                               (64, 20000, 0.1, 0.6, 0.02)])
def test_g2p_through_bins_is_bit_identical(root, n, np_, lo, hi, shift):
    """A gather after a binned scatter of as many particles goes through the
    scatter's bins: it must equal the per-particle gather bit for bit and
    meet the gather bar against the oracle, also with particles whose centre
    node lies outside the domain (listed apart by the scatter) and after the
    particles have moved (shift, in units of the domain: many leave their
    bin's tile and gather directly).  A gather of another particle count
    does not use the bins."""
    from paper_2012_08141_amd import _lib as L, engine as E
    from paper_2012_08141_amd.grid import SparseGrid
    say("g2p bins", root, n, np_, lo, hi, shift)
    p = I.random_particles(6, n, np_, lo, hi, root)
    g = SparseGrid(n, 7, root, (n // 8) ** 3 if root == "pointer" else 0, particle_capacity=np_)
    x, v, m = (torch.as_tensor(a, device="cuda").contiguous() for a in (p.x, p.v, p.m))
    E.run_sequence([E.p2g(g, x, v, m, 1.0 / n, 0, 1)], 0)
    if shift:
        E.run_sequence([E.advect(x, torch.full_like(x, shift), 1.0)], 0)
    cells = g.active_cells()
    rng = np.random.default_rng([7, n, np_])
    vals = [rng.uniform(-1, 1, (len(cells), 512)).astype(np.float32) for _ in range(3)]
    for q in range(3):
        g.load_blocks(4 + q, cells, vals[q])
    o = oracle.OracleGrid(n, 3)
    o.load(I.cells_to_blocks(cells, n // 8), {"v%d" % q: vals[q] for q in range(3)}, {"v0": 0, "v1": 1, "v2": 2})
    xs = x.cpu().numpy()
    exp = o.g2p(0, xs, float(n))
    got = {}
    try:
        for on in (1, 0):
            E.set_option(L.AT_OPTION_G2P_BINS, on)
            out = torch.zeros_like(x)
            E.run_sequence([E.g2p(g, x, out, 1.0 / n, 4)], 0)
            torch.cuda.synchronize()
            got[on] = out.cpu().numpy()
    finally:
        E.set_option(L.AT_OPTION_G2P_BINS, 1)
    assert np.array_equal(got[1], got[0])
    close_state(got[1], exp, "g2p through bins")
    half = x[:, : np_ // 2].contiguous()
    out = torch.zeros_like(half)
    E.run_sequence([E.g2p(g, half, out, 1.0 / n, 4)], 0)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), got[0][:, : np_ // 2])
    assert g.device_status() == 0


@pytest.mark.parametrize("root", ["pointer", "bitmask"])
@pytest.mark.parametrize("shift", [0.0, 0.02])
def test_g2p_through_bins_in_one_window(root, shift):
    """Scatter, (advection,) normalisation and gather in one window: without
    advection the gather takes positions from the scatter's records, after
    it from x (records stale).  Both must agree with the gather that does not
    use bins (the scatter's fp32 atomics make the node values differ in the
    last bits between runs, so the bar is the gather bar)."""
    from paper_2012_08141_amd import _lib as L, engine as E
    from paper_2012_08141_amd.grid import SparseGrid
    say("g2p bins one window", root, shift)
    n, np_ = 64, 20000
    p = I.random_particles(8, n, np_, 0.1, 0.6, root)
    got = {}
    try:
        for on in (1, 0):
            E.set_option(L.AT_OPTION_G2P_BINS, on)
            g = SparseGrid(n, 7, root, (n // 8) ** 3 if root == "pointer" else 0, particle_capacity=np_)
            x, v, m = (torch.as_tensor(a, device="cuda").contiguous() for a in (p.x, p.v, p.m))
            out = torch.zeros_like(x)
            tasks = [E.p2g(g, x, v, m, 1.0 / n, 0, 1)]
            if shift:
                tasks.append(E.advect(x, torch.full_like(x, shift), 1.0))
            tasks += [E.listgen(g), E.normalise(g, 0, 1, 4), E.g2p(g, x, out, 1.0 / n, 4)]
            E.run_sequence(tasks, 0)
            torch.cuda.synchronize()
            got[on] = out.cpu().numpy()
            assert g.device_status() == 0
    finally:
        E.set_option(L.AT_OPTION_G2P_BINS, 1)
    close_state(got[1], got[0], "g2p bins vs direct, one window")


def _binning_extra(steps, reuse):
    """Dispatches beyond one per node of the optimized particle program with
    a particle workspace.  Step 0 bins afresh: keys (with the advection),
    ranks, scan, place, tiles.  Each later step's fused gather-advect-scatter
    node gathers through the previous scatter's bins and then either scatters
    over the same bins (gather, advection, tiles) while they have been reused
    fewer than `reuse` times, or bins afresh (gather, advection with keys,
    ranks, scan, place, tiles)."""
    extra, age = 4, 0
    for _ in range(1, steps):
        if age < reuse:
            extra, age = extra + 2, age + 1
        else:
            extra, age = extra + 5, 0
    return extra


def _particle_run(p, steps, opt, binned=True):
    from paper_2012_08141_amd import engine as E, programs as PR
    from paper_2012_08141_amd.grid import SparseGrid
    n = p.n
    grids = [SparseGrid(n, 7, p.root_kind, (n // 8) ** 3 if p.root_kind == "pointer" else 0,
                        particle_capacity=p.nparticles if binned else 0) for _ in range(2)]
    x, v, m = PR.device_particles(p)
    tasks = sum((PR.particle_step(grids, t, x, v, m, p.params["dt"], 1.0 / n) for t in range(steps)), [])
    st = E.run_sequence(tasks, opt)
    torch.cuda.synchronize()
    return grids, x, v, st


@pytest.mark.parametrize("binned,reuse", [(False, 0), (True, 0), (True, 8)])
@pytest.mark.parametrize("opt", [0, 15])
def test_particle_program_reduced(opt, binned, reuse, bin_reuse):
    """The particle recipe (3 boxes, N(0, 0.1^2) velocities, dt = 1e-3) with
    100k particles in a 128^3 grid, 20 steps, eager and optimized, direct
    and binned scatter, binning every scatter or reusing bins."""
    say("particle program opt", opt, "binned" if binned else "direct", "reuse", reuse)
    bin_reuse(reuse)
    p = I.particles(0, n=128, nparticles=100_000)
    grids, x, v, st = _particle_run(p, 20, opt, binned)
    assert st["tasks_launched"] == (140 if opt == 0 else 65)
    if not binned:
        assert st["dispatches"] == st["tasks_launched"]
    elif opt == 0:
        # every scatter bins (5 dispatches); the separate gathers go through bins
        assert st["dispatches"] == st["tasks_launched"] + 4 * 20
    else:
        assert st["dispatches"] == st["tasks_launched"] + _binning_extra(20, reuse)
    ref = OP.particle_program(p.n, p.x, p.v, p.m, 20, p.params["dt"], "f32")
    # positions at 0.1 |o|_inf; velocities at the scale of the scattered
    # terms (the particles' own speeds), which sets the rounding of the
    # momentum sums that fp32 atomics add in a varying order
    sx, sv = 0.1 * np.abs(ref["x"]).max(), 0.1 * np.abs(p.v).max()
    close_state(x.cpu().numpy(), ref["x"], "x", sx)
    close_state(v.cpu().numpy(), ref["v"], "v", sv)
    for gi in (0, 1):
        assert np.array_equal(grids[gi].active_cells(), ref["cells%d" % gi]), gi
        assert grids[gi].device_status() == 0


@pytest.mark.parametrize("root", ["pointer", "bitmask"])
@pytest.mark.parametrize("reuse", [3, 8])
def test_particle_program_bin_reuse_with_drift(reuse, root, bin_reuse):
    """Velocities ten times the recipe's and dt = 2e-3 on a 128^3 grid move a
    particle about a quarter node per step, so bins reused for several steps
    hold particles that have moved one node past their block (still summed in
    the tile) and further (scattered directly).  The state after 12 steps
    against the oracle, and the same run binning every scatter."""
    import dataclasses
    say("particle program bin reuse with drift", reuse, root)
    p0 = I.particles(0, n=128, nparticles=100_000)
    p = dataclasses.replace(p0, v=(p0.v * 10).astype(np.float32), params=dict(p0.params, dt=2e-3), root_kind=root)
    steps = 12
    ref = OP.particle_program(p.n, p.x, p.v, p.m, steps, p.params["dt"], "f32")
    sx, sv = 0.1 * np.abs(ref["x"]).max(), 0.1 * np.abs(p.v).max()     # as in the reduced program
    out = {}
    for k in (reuse, 0):
        bin_reuse(k)
        grids, x, v, st = _particle_run(p, steps, 15)
        assert st["dispatches"] == st["tasks_launched"] + _binning_extra(steps, k)
        close_state(x.cpu().numpy(), ref["x"], "x", sx)
        close_state(v.cpu().numpy(), ref["v"], "v", sv)
        for gi in (0, 1):
            assert np.array_equal(grids[gi].active_cells(), ref["cells%d" % gi]), gi
            assert grids[gi].device_status() == 0
        out[k] = v.cpu().numpy()
    close_state(out[reuse], out[0], "v reuse / rebin", sv)


@pytest.mark.parametrize("how", ["clear", "destroy"])
def test_reused_bins_are_not_used_after_their_workspace_goes(how, bin_reuse):
    """Two steps of the particle program in one window: the second step's
    scatter into grid 1 reuses the bins held in grid 0's workspace.  Once
    grid 0 is cleared (its workspace generation moves on) or destroyed (it
    leaves the engine's registry), a gather from grid 1 must not use those
    bins: it equals the per-particle gather bit for bit."""
    import gc
    from paper_2012_08141_amd import _lib as L, engine as E, programs as PR
    from paper_2012_08141_amd.grid import SparseGrid
    say("reused bins after", how)
    bin_reuse(8)
    p = I.particles(0, n=128, nparticles=50_000)
    n = p.n
    grids = [SparseGrid(n, 7, "pointer", (n // 8) ** 3, particle_capacity=p.nparticles) for _ in range(2)]
    x, v, m = PR.device_particles(p)
    tasks = sum((PR.particle_step(grids, t, x, v, m, p.params["dt"], 1.0 / n) for t in range(2)), [])
    st = E.run_sequence(tasks, E.OPT_ALL)
    torch.cuda.synchronize()
    assert st["dispatches"] == st["tasks_launched"] + _binning_extra(2, 8)   # the second scatter reused
    g1 = grids[1]
    want = torch.zeros_like(x)
    try:
        E.set_option(L.AT_OPTION_G2P_BINS, 0)
        E.run_sequence([E.g2p(g1, x, want, 1.0 / n, PR.PART["v"])], 0)
    finally:
        E.set_option(L.AT_OPTION_G2P_BINS, 1)
    if how == "clear":
        grids[0].clear()
    else:
        grids[0] = None
        del tasks          # the tasks hold the grid too
        gc.collect()
    got = torch.zeros_like(x)
    E.run_sequence([E.g2p(g1, x, got, 1.0 / n, PR.PART["v"])], 0)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    assert g1.device_status() == 0


def test_particle_full_size_three_steps_and_eager_vs_optimized():
    """The particle workload at full size (2M particles, 256^3): three optimized steps
    against the oracle (the second and third scatter over reused bins); 20 steps
    optimized against eager."""
    say("particles full size")
    p = I.particles(0)
    ref = OP.particle_program(p.n, p.x, p.v, p.m, 3, p.params["dt"], "f32")
    # at 2M particles the reordered fp32 momentum sums differ by up to about
    # 1.3e-7 in v, above 1e-5 * 0.1 |o|_inf of the grid-averaged velocity:
    # the scale is that of the scattered terms, 0.1 max|v0|
    sx, sv = 0.1 * np.abs(ref["x"]).max(), 0.1 * np.abs(p.v).max()
    grids, x, v, st = _particle_run(p, 3, 15)
    assert st["dispatches"] == st["tasks_launched"] + _binning_extra(3, 8)
    close_state(x.cpu().numpy(), ref["x"], "x", sx)
    close_state(v.cpu().numpy(), ref["v"], "v", sv)
    for gi in (0, 1):
        assert np.array_equal(grids[gi].active_cells(), ref["cells%d" % gi]), gi
    del grids
    ge, xe, ve, _ = _particle_run(p, 20, 0)
    go, xo, vo, _ = _particle_run(p, 20, 15)
    close_state(xo.cpu().numpy(), xe.cpu().numpy(), "x eager/opt", sx)
    close_state(vo.cpu().numpy(), ve.cpu().numpy(), "v eager/opt", sv)
    for gi in (0, 1):
        assert np.array_equal(ge[gi].active_cells(), go[gi].active_cells())


@pytest.mark.parametrize("binned", [False, True])
def test_p2g_without_activation(binned):
    """AT_ACT_NONE: on a grid whose touched blocks are already active the
    scatter equals the activating one; on a fresh grid it activates nothing
    and writes nothing."""
    import ctypes
    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd.grid import SparseGrid
    say("p2g none", "binned" if binned else "direct")
    n, np_ = 64, 20000
    p = I.random_particles(5, n, np_, 0.1, 0.6, "pointer")
    ref = OP.p2g_once(n, None, p.x, p.v, p.m, "f32")
    x, v, m = (torch.as_tensor(a, device="cuda").contiguous() for a in (p.x, p.v, p.m))
    ch = (ctypes.c_int32 * 2)(0, 1)

    def scatter(g, act):
        L.check(L.lib().at_p2g(g.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                               ctypes.c_void_p(m.data_ptr()), np_, 1.0 / n, ch, act,
                               torch.cuda.current_stream().cuda_stream))

    cap = np_ if binned else 0
    fresh = SparseGrid(n, 4, "pointer", (n // 8) ** 3, particle_capacity=cap)
    scatter(fresh, L.AT_ACT_NONE)
    torch.cuda.synchronize()
    assert len(fresh.active_cells()) == 0 and float(fresh.channel(0).abs().sum()) == 0.0
    pre = SparseGrid(n, 4, "pointer", (n // 8) ** 3, particle_capacity=cap)
    pre.activate(I.cells_to_blocks(ref["cells"], n // 8))
    act = SparseGrid(n, 4, "pointer", (n // 8) ** 3, particle_capacity=cap)
    scatter(pre, L.AT_ACT_NONE)
    scatter(act, L.AT_ACT_PER_BLOCK)
    torch.cuda.synchronize()
    cells = ref["cells"]
    assert np.array_equal(pre.active_cells(), cells) and np.array_equal(act.active_cells(), cells)
    for q in range(4):
        A = ref["abs"][q].astype(np.float64)
        for g in (pre, act):
            err = np.abs(g.read_blocks(q, cells).astype(np.float64) - (ref["m"] if q == 0 else ref["mv"][q - 1]))
            assert np.all(err <= 1e-5 * A + 1e-30), q
