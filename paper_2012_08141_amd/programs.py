"""Task programs of the synthetic workloads, as windows of engine tasks.

Each builder returns the task list of one window; the same list runs either
eagerly (opt_flags = 0) or optimized (opt_flags = OPT_ALL), so the two
pipelines run exactly the same program.
"""
from __future__ import annotations

import numpy as np
import torch

from . import engine as E
from . import inputs
from .grid import SparseGrid

# channel assignment of each workload's grid
SHELL = {"a": 0, "out": 1}
JACOBI = {"x": 0, "xn": 1, "b": 2}
PART = {"m": 0, "mv": 1, "v": 4}           # m; mv0..2; v0..2  (7 channels)
DIFF = {"a": 0, "a2": 1, "k": 2}


def load_workload(w: inputs.SparseWorkload, channels: dict, nch: int, capacity_blocks: int = 0,
                  stream=None) -> SparseGrid:
    """A device grid holding the workload's active blocks and channel values."""
    cap = capacity_blocks or (w.nblocks if w.root_kind == "pointer" else 0)
    g = SparseGrid(w.n, nch, w.root_kind, cap, stream=stream)
    cells = w.cells
    for name, vals in w.channels.items():
        if name in channels:
            g.load_blocks(channels[name], cells, vals, stream=stream)
    if not w.channels:
        g.load_blocks(0, cells, np.zeros((len(cells), 512), np.float32), stream=stream)
    return g


# ------------------------------------------------------------ shell workload
def shell_setup(g: SparseGrid, coords):
    """Setup window: activation of the shell blocks and the first list."""
    return [E.activate(g, coords), E.listgen(g)]


def shell_step(g: SparseGrid, coords, coef=0.1, alpha=0.5):
    """activate -> listgen -> lap_update (out = a + coef lap a) -> listgen ->
    axpy (a += alpha out)."""
    return [E.activate(g, coords), E.listgen(g), E.lap_update(g, SHELL["a"], SHELL["out"], coef),
            E.listgen(g), E.axpy(g, SHELL["a"], SHELL["out"], alpha)]


# ------------------------------------------------------ narrow-band workload
def jacobi_step(g: SparseGrid):
    """listgen -> jacobi (xn = (sum nb x + b)/6) -> copy (x = xn)."""
    return [E.listgen(g), E.jacobi(g, JACOBI["x"], JACOBI["b"], JACOBI["xn"]),
            E.copy(g, JACOBI["x"], JACOBI["xn"])]


# --------------------------------------------------------- particle workload
def particle_step(grids, t: int, x, v, m, dt: float, dx: float):
    """Step t on grid G = grids[t % 2]: listgen(G) -> reset(G) -> advect ->
    p2g(G) -> listgen(G) -> normalise(G) -> g2p(G)."""
    G = grids[t % 2]
    return [E.listgen(G), E.fill(G, [PART["m"], PART["mv"], PART["mv"] + 1, PART["mv"] + 2,
                                     PART["v"], PART["v"] + 1, PART["v"] + 2], 0.0),
            E.advect(x, v, dt), E.p2g(G, x, v, m, dx, PART["m"], PART["mv"]),
            E.listgen(G), E.normalise(G, PART["m"], PART["mv"], PART["v"]),
            E.g2p(G, x, v, dx, PART["v"])]


# -------------------------------------------------------- diffusion workload
def diffusion_forward_tasks(g: SparseGrid, steps: int, dt: float, src: int = 0, dst: int = 1, k: int = 2):
    """listgen, then ``steps`` diffusion steps ping-ponging between channels
    src and dst.  Returns (tasks, channel holding the result)."""
    tasks = [E.listgen(g)]
    for _ in range(steps):
        tasks.append(E.diffuse(g, src, k, dst, dt))
        src, dst = dst, src
    return tasks, src


def device_particles(p: inputs.ParticleWorkload):
    x = torch.as_tensor(p.x, device="cuda").contiguous()
    v = torch.as_tensor(p.v, device="cuda").contiguous()
    m = torch.as_tensor(p.m, device="cuda").contiguous()
    return x, v, m


# ------------------------------------------------------- multigrid V-cycle
MG = {"x": 0, "b": 1, "t": 2}


def mg_smooth(g: SparseGrid, omega: float):
    """Damped Jacobi: t = J(x); t = t - x; x = x + omega t, each struct-for
    preceded by its list generation."""
    return [E.listgen(g), E.jacobi(g, MG["x"], MG["b"], MG["t"]),
            E.listgen(g), E.axpy(g, MG["t"], MG["x"], -1.0),
            E.listgen(g), E.axpy(g, MG["x"], MG["t"], omega)]


def mg_vcycle(levels, pre: int = 2, post: int = 2, coarse_iters: int = 8, omega: float = 0.75,
              w_restrict: float = 1.5):
    """One V-cycle over ``levels`` (finest first, each half the previous
    domain edge): pre-smoothing, the scaled residual t = J(x) - x restricted
    into the cleared coarse right-hand side (coarse[b][I/2] += w t[I]), the
    coarsest level smoothed, then injection prolongation x[I] += x_c[I/2] and
    post-smoothing on the way up.  The coarse levels' blocks come from the
    restriction's activation on write."""
    tasks = []
    L = len(levels)
    for l in range(L - 1):
        g, c = levels[l], levels[l + 1]
        for _ in range(pre):
            tasks += mg_smooth(g, omega)
        tasks += [E.listgen(g), E.jacobi(g, MG["x"], MG["b"], MG["t"]),
                  E.listgen(g), E.axpy(g, MG["t"], MG["x"], -1.0),
                  E.listgen(c), E.fill(c, [MG["x"]], 0.0),
                  E.listgen(c), E.fill(c, [MG["b"]], 0.0),
                  E.listgen(g), E.restrict(g, c, MG["t"], MG["b"], w_restrict)]
    for _ in range(coarse_iters):
        tasks += mg_smooth(levels[L - 1], omega)
    for l in range(L - 2, -1, -1):
        g, c = levels[l], levels[l + 1]
        tasks += [E.listgen(g), E.prolong(c, g, MG["x"], MG["x"])]
        for _ in range(post):
            tasks += mg_smooth(g, omega)
    return tasks


def mg_levels(w: inputs.SparseWorkload, nlevels: int, stream=None):
    """The level grids of a V-cycle solve: the finest holds the workload's
    blocks and right-hand side ``b``; coarser levels start empty with room for
    every ancestor block (pointer roots when the finest has one)."""
    fine = SparseGrid(w.n, 3, w.root_kind, w.nblocks if w.root_kind == "pointer" else 0, stream=stream)
    fine.load_blocks(MG["b"], w.cells, w.channels["b"], stream=stream)
    levels = [fine]
    blocks = np.asarray(w.blocks, dtype=np.int64)
    for l in range(1, nlevels):
        n = w.n >> l
        anc = np.unique(blocks >> l, axis=0)
        cap = len(anc) if w.root_kind == "pointer" else 0
        levels.append(SparseGrid(n, 3, w.root_kind, cap, stream=stream))
    return levels


# ---------------------------------------------------------- advection workload
ADV = {"q": 0, "v": 3, "tmp": 6}            # q0..q2; v0..v2; tmp0..tmp2  (9 channels)


def advection_step(g: SparseGrid, dt: float):
    """Per scalar field c, as separate kernels (the multi-kernel structure of
    the paper's advection benchmark): listgen -> advect (tmp_c = q_c at the
    back-traced point) -> listgen -> copy (q_c = tmp_c)."""
    tasks = []
    for c in range(3):
        tasks += [E.listgen(g), E.advect_sl(g, ADV["q"] + c, ADV["v"], ADV["tmp"] + c, dt),
                  E.listgen(g), E.copy(g, ADV["q"] + c, ADV["tmp"] + c)]
    return tasks


MAC = {"q": 0, "v": 3, "fwd": 6, "bwd": 9, "out": 12}   # 15 channels


def maccormack_step(g: SparseGrid, dt: float, rk3: bool = False):
    """Per scalar field c (the multi-kernel structure of the paper's MacCormack
    benchmark): fwd = advect(q, dt), bwd = advect(fwd, -dt), out = MacCormack
    correction of q with clamping, q = out; each struct-for preceded by its list
    generation; rk3 selects the RK3 back-trace (the paper's setup)."""
    tasks = []
    for c in range(3):
        q, f, b, o = MAC["q"] + c, MAC["fwd"] + c, MAC["bwd"] + c, MAC["out"] + c
        tasks += [E.listgen(g), E.advect_sl(g, q, MAC["v"], f, dt, rk3),
                  E.listgen(g), E.advect_sl(g, f, MAC["v"], b, -dt, rk3),
                  E.listgen(g), E.maccormack(g, q, MAC["v"], f, b, o, dt, rk3),
                  E.listgen(g), E.copy(g, q, o)]
    return tasks


# ----------------------------------------------------------- MLS-MPM workload
MPM = {"m": 0, "mv": 1, "v": 4}            # m; mv0..2; v0..2  (7 channels)


def mpm_grids(w: inputs.MpmWorkload, stream=None):
    """The two grids the substeps alternate between (Section 8.3: two grids,
    swapped before each substep), empty."""
    cap = (w.n // 8) ** 3 if w.root_kind == "pointer" else 0
    return [SparseGrid(w.n, 7, w.root_kind, cap, stream=stream) for _ in range(2)]


def device_mpm(w: inputs.MpmWorkload):
    """x, v, C, F as contiguous device arrays."""
    return tuple(torch.as_tensor(a, device="cuda").contiguous() for a in (w.x, w.v, w.C, w.F))


def mpm_step(grids, t: int, x, v, C, F, params: dict):
    """Substep t on grid G = grids[t % 2]: listgen(G) -> fill(G: m, mv = 0) ->
    p2g_mls(G) (F updated, activating) -> listgen(G) -> mpm_grid(G) (v,
    gravity, walls) -> g2p_apic(G) (v and C) -> advect (x += dt v)."""
    G = grids[t % 2]
    p = params
    dt, dx = p["dt"], p["dx"]
    return [E.listgen(G), E.fill(G, [MPM["m"], MPM["mv"], MPM["mv"] + 1, MPM["mv"] + 2], 0.0),
            E.p2g_mls(G, x, v, C, F, dx, dt, p["mass"], p["vol"], p["mu"], p["lam"], MPM["m"], MPM["mv"]),
            E.listgen(G), E.mpm_grid(G, MPM["m"], MPM["mv"], MPM["v"], dt, p["gravity"], p["bound"]),
            E.g2p_apic(G, x, v, C, dx, MPM["v"]), E.advect(x, v, dt)]
