"""MLS-MPM transfers on the GPU against the oracle (MI355X only).

Bars (fp32 against the fp64 oracle):
* active sets bit-exact;
* the gather (v and C) bit-exact against the fp32 build of the oracle,
  which sums in the same order;
* one scatter: F within 1e-5 relative; every node and channel within
  1e-5 * S, S the oracle's error scale of the node's sum (the magnitudes
  of the products each term is made of: fp32 atomics reorder the sum, and
  the stress term cancels inside F - R);
* several substeps: x and F within 1e-5 * max(|o|, 0.1 max|o|); v within
  1e-5 * max(|o|, s_v) with s_v = 0.1 (max|v0| + max|C0| dx), the scale of
  the momentum terms a grid velocity averages; C within
  1e-5 * max(|o|, 4 s_v / dx), the scale of a velocity difference over one
  cell that C estimates.
"""
import ctypes

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


def _dev(*arrays):
    return [torch.as_tensor(np.ascontiguousarray(a), device="cuda").contiguous() for a in arrays]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def close(got, exp, scale, what):
    got = np.asarray(got, np.float64)
    exp = np.asarray(exp, np.float64)
    tol = 1e-5 * np.maximum(np.abs(exp), scale)
    err = np.abs(got - exp)
    assert np.all(err <= tol), "%s: %d of %d beyond tolerance (max err %g, scale %g)" % (
        what, int((err > tol).sum()), err.size, float(err.max()), float(scale))


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
@pytest.mark.parametrize("order", ["lattice", "shuffled", "domain_edge"])
def test_g2p_apic_bit_exact(root, order):
    """The gather through the chunk tile (lattice order) and per node
    (shuffled particles, tiles too large), also with nodes outside the
    domain, equals the fp32 oracle bit for bit."""
    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd.grid import SparseGrid
    n = 64
    say("g2p_apic", root, order)
    w = I.random_blocks(21, n, 0.6, root, channels=("v0", "v1", "v2"))
    if order == "domain_edge":
        x = np.random.default_rng(5).uniform(-0.01, 1.01, (3, 20000)).astype(np.float32)
    else:
        x = I.mpm_cube(5, n, side=0.3, z_bottom=0.3).x
        if order == "shuffled":
            x = x[:, np.random.default_rng(1).permutation(x.shape[1])]
    g = SparseGrid(n, 3, root, (n // 8) ** 3 if root == "pointer" else 0)
    for q in range(3):
        g.load_blocks(q, w.cells, w.channels["v%d" % q])
    o = oracle.OracleGrid(n, 3, "f32")
    o.load(w.blocks, w.channels, {"v0": 0, "v1": 1, "v2": 2})
    xd, = _dev(x)
    vd = torch.zeros_like(xd)
    Cd = torch.zeros(9, xd.shape[1], device="cuda")
    ch = (ctypes.c_int32 * 1)(0)
    L.check(L.lib().at_g2p_apic(g.handle, _ptr(xd), _ptr(vd), _ptr(Cd), xd.shape[1], 1.0 / n, ch,
                                torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    ve, Ce = o.mpm_g2p(0, x, float(n))
    assert np.array_equal(vd.cpu().numpy(), ve)
    assert np.array_equal(Cd.cpu().numpy(), Ce)


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
@pytest.mark.parametrize("order", ["lattice", "shuffled"])
@pytest.mark.parametrize("act", [0, 1])
def test_p2g_mls_matches_oracle(root, order, act):
    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd.grid import SparseGrid
    n = 64
    say("p2g_mls", root, order, act)
    mp = I.mpm_cube(6, n, side=0.3, z_bottom=0.3, v_sigma=0.5, c_sigma=2.0, f_sigma=0.05)
    perm = np.arange(mp.nparticles) if order == "lattice" else np.random.default_rng(2).permutation(mp.nparticles)
    x, v, C, F = (np.ascontiguousarray(a[:, perm]) for a in (mp.x, mp.v, mp.C, mp.F))
    p = mp.params
    o = oracle.OracleGrid(n, 8, "f64")
    Fo, bad = o.mpm_p2g(0, 1, x, v, C, F, float(n), p["dt"], p["mass"], p["vol"], p["mu"], p["lam"], ch_abs=4)
    assert bad == 0
    g = SparseGrid(n, 4, root, (n // 8) ** 3 if root == "pointer" else 0)
    xd, vd, Cd, Fd = _dev(x, v, C, F)
    chs = (ctypes.c_int32 * 2)(0, 1)
    L.check(L.lib().at_p2g_mls(g.handle, _ptr(xd), _ptr(vd), _ptr(Cd), _ptr(Fd), xd.shape[1], 1.0 / n, p["dt"],
                               p["mass"], p["vol"], p["mu"], p["lam"], chs, act,
                               torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    cells = o.active_cells()
    assert np.array_equal(g.active_cells(), cells)
    assert g.device_status() == 0
    close(Fd.cpu().numpy(), Fo, np.abs(Fo).max(), "F")
    for q in range(4):
        got = g.read_blocks(q, cells).astype(np.float64)
        exp = o.read_blocks(q, cells)
        S = o.read_blocks(4 + q, cells)
        err = np.abs(got - exp)
        assert np.all(err <= 1e-5 * S + 1e-30), ("channel", q, float((err / np.maximum(S, 1e-30)).max()))


def _program(mp, K, flags, root):
    from paper_2012_08141_amd import engine as E, programs as PR
    mp.root_kind = root
    grids = PR.mpm_grids(mp)
    x, v, C, F = PR.device_mpm(mp)
    tasks = sum((PR.mpm_step(grids, t, x, v, C, F, mp.params) for t in range(K)), [])
    st = E.run_sequence(tasks, flags)
    torch.cuda.synchronize()
    return grids, (x, v, C, F), st


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
@pytest.mark.parametrize("flags", [0, 15])
@pytest.mark.parametrize("case", ["stirred", "falling"])
def test_mpm_program_matches_oracle(root, flags, case):
    """Four substeps, eager (7 launches each) and optimized (G2P2G fused,
    the stores of v and C dropped inside the window): a block with random
    velocities, affine matrices and deformations near the floor, and the
    paper's cube at rest, falling."""
    n, K = 64, 4
    say("mpm program", root, flags, case)
    if case == "stirred":
        mp = I.mpm_cube(7, n, side=0.3, z_bottom=0.1, v_sigma=0.3, c_sigma=1.0, f_sigma=0.02)
    else:
        mp = I.mpm_cube(8, n, side=0.25)
    x0, v0, C0, F0 = mp.x.copy(), mp.v.copy(), mp.C.copy(), mp.F.copy()
    grids, (x, v, C, F), st = _program(mp, K, flags, root)
    assert st["dispatches"] == 7 * K if flags == 0 else st["dispatches"] < 4 * K + 2
    p = mp.params
    ref = OP.mpm_program(n, x0, v0, C0, F0, K, p["dt"], p["mass"], p["vol"], p["mu"], p["lam"], p["gravity"],
                         p["bound"], "f64")
    for gi in range(2):
        assert np.array_equal(grids[gi].active_cells(), ref["cells%d" % gi])
        assert grids[gi].device_status() == 0
    dx = p["dx"]
    sv = 0.1 * (np.abs(v0).max() + np.abs(C0).max() * dx + p["gravity"] * p["dt"] * K)
    close(x.cpu().numpy(), ref["x"], 0.1 * np.abs(ref["x"]).max(), "x")
    close(F.cpu().numpy(), ref["F"], 0.1 * np.abs(ref["F"]).max(), "F")
    close(v.cpu().numpy(), ref["v"], sv, "v")
    close(C.cpu().numpy(), ref["C"], 4 * sv / dx, "C")


def test_mpm_full_size_free_fall():
    """The paper's cube at full size (256^3 grid, 16,777,216 particles), one
    optimized substep from rest: every node with mass gets the velocity
    (0, 0, -g dt) exactly and the grid holds the total mass; every particle
    falls with v = (0, 0, -g dt) and C = 0 (the gather reproduces a uniform
    velocity up to rounding), moves by dt v and keeps F = I."""
    from paper_2012_08141_amd import programs as PR
    say("mpm full size")
    mp = I.mpm_cube(0, 256, side=0.5)
    p = mp.params
    x0 = mp.x.copy()
    grids, (x, v, C, F), st = _program(mp, 1, 15, "bitmask")
    gdt = p["gravity"] * p["dt"]
    vv = v.cpu().numpy()
    assert np.abs(vv[:2]).max() <= 1e-6 * gdt
    assert np.abs(vv[2] + gdt).max() <= 1e-6 * gdt
    assert np.abs(C.cpu().numpy()).max() <= 1e-4 * 4 * gdt / p["dx"]
    assert np.abs(x.cpu().numpy() - (x0 + np.float32(p["dt"]) * vv)).max() <= 1e-7
    assert torch.equal(F, torch.as_tensor(mp.F, device="cuda"))
    g = grids[0]
    m = g.channel(PR.MPM["m"])
    N = mp.nparticles
    assert abs(m.double().sum().item() - N * p["mass"]) <= 1e-5 * N * p["mass"]
    has = m > 0
    vz = g.channel(PR.MPM["v"] + 2)[has]
    assert torch.all(vz == -torch.tensor(np.float32(p["dt"]) * np.float32(p["gravity"]), device="cuda"))
    for c in range(2):
        assert torch.all(g.channel(PR.MPM["v"] + c)[has] == 0)
    assert g.device_status() == 0
