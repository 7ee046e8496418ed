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
