"""The workloads' task programs, executed eagerly in program order on the
oracle -- TEST INFRASTRUCTURE ONLY.

The inter-kernel optimizations (list generation removal, activation
demotion, task fusion, dead store elimination; paper Section 6) never change
a program's result (order independency of the state-flow graph, Section 4),
so the plain in-order execution below is the reference for both the eager
and the optimized GPU pipelines.

Every function takes plain arrays (block coordinates and per-block values in
the ``[nb, 512]`` layout, particles as SoA ``[3, np]``) and returns arrays.
"""
from __future__ import annotations

import numpy as np

from . import OracleGrid, advect


def _cells(blocks, R):
    b = np.asarray(blocks, dtype=np.int64)
    return ((b[:, 0] * R + b[:, 1]) * R + b[:, 2]).astype(np.int32)


# ---------------------------------------------------------------------------
def shell_program(n, blocks, a0, steps=10, coef=0.1, alpha=0.5, precision="f32"):
    """Per step: activate(blocks) -> listgen -> lap_update (out = a + coef *
    lap a) -> listgen -> axpy (a += alpha * out).  Returns (a, out) on the
    active blocks (ascending cells) and the final list."""
    g = OracleGrid(n, 2, precision)
    g.load(blocks, {"a": a0}, {"a": 0})
    g.listgen()
    for _ in range(steps):
        g.activate(blocks, "block")
        g.listgen()
        g.lap_update(0, 1, coef)
        g.listgen()
        g.axpy(0, 1, alpha)
    cells = g.active_cells()
    return {"cells": cells, "a": g.read_blocks(0, cells), "out": g.read_blocks(1, cells),
            "list": g.list()}


# ---------------------------------------------------------------------------
def jacobi_program(n, blocks, b, iters, precision="f32", x0=None):
    """Per iteration: listgen -> jacobi (xn = (sum of 6 neighbours of x + b) / 6)
    -> copy (x = xn).  Returns x and xn on the active blocks."""
    g = OracleGrid(n, 3, precision)
    vals = {"b": b}
    if x0 is not None:
        vals["x"] = x0
    g.load(blocks, vals, {"x": 0, "xn": 1, "b": 2})
    for _ in range(iters):
        g.listgen()
        g.jacobi(0, 2, 1)
        g.copy(0, 1)
    cells = g.active_cells()
    return {"cells": cells, "x": g.read_blocks(0, cells), "xn": g.read_blocks(1, cells)}


# ---------------------------------------------------------------------------
# Particle workload: two grids used alternately, channels m, mv(3), v(3).
CH_M, CH_MV, CH_V, CH_ABS = 0, 1, 4, 7


def particle_program(n, x, v, m, steps, dt, precision="f32", with_abs=False,
                     record_masks=False):
    """Step t uses grid G = grids[t % 2]:
    listgen(G) -> reset(G) (m, mv, v = 0) -> advect (x += dt v) -> p2g(G)
    (activating) -> listgen(G) -> normalise(G) -> g2p(G) (v = gathered v).
    Returns final particle state, the two grids' cells and channels."""
    inv_dx = float(n)
    nch = 11 if with_abs else 7
    grids = [OracleGrid(n, nch, precision), OracleGrid(n, nch, precision)]
    d = np.float32 if precision == "f32" else np.float64
    x = np.ascontiguousarray(x, dtype=d).copy()
    v = np.ascontiguousarray(v, dtype=d).copy()
    m = np.ascontiguousarray(m, dtype=d)
    masks = []
    for t in range(steps):
        G = grids[t % 2]
        G.listgen()
        for ch in range(nch):
            G.fill(ch, 0.0)
        x = advect(x, v, dt, precision)
        bad = G.p2g(CH_M, CH_MV, x, v, m, inv_dx, CH_ABS if with_abs else -1)
        if bad:
            raise RuntimeError("particle left the domain")
        G.listgen()
        G.normalise(CH_M, CH_MV, CH_V)
        v = G.g2p(CH_V, x, inv_dx)
        if record_masks:
            masks.append((t % 2, G.active_cells()))
    out = {"x": x, "v": v, "masks": masks}
    for gi, G in enumerate(grids):
        cells = G.active_cells()
        out["cells%d" % gi] = cells
        out["grid%d" % gi] = {ch: G.read_blocks(ch, cells) for ch in range(nch)}
    return out


def p2g_once(n, blocks_active, x, v, m, precision="f32"):
    """One activating P2G onto a zeroed grid (optionally pre-activated
    blocks); returns cells, m, mv(3) and the per-node sums of |term|."""
    g = OracleGrid(n, 8, precision)
    if blocks_active is not None and len(blocks_active):
        g.activate(blocks_active, "block")
    bad = g.p2g(0, 1, x, v, m, float(n), ch_abs=4)
    cells = g.active_cells()
    return {"cells": cells, "bad": bad,
            "m": g.read_blocks(0, cells), "mv": [g.read_blocks(1 + c, cells) for c in range(3)],
            "abs": [g.read_blocks(4 + q, cells) for q in range(4)]}


# ---------------------------------------------------------------------------
def diffusion_forward(n, blocks, a0, k, dt, steps, precision="f64"):
    """a_{t+1} = diffuse(a_t; k).  Returns the list of a_t (t = 0..steps)."""
    g = OracleGrid(n, 3, precision)
    g.load(blocks, {"a": a0, "k": k}, {"a": 0, "k": 2})
    g.listgen()
    cells = _cells(blocks, n // 8)
    hist = [g.read_blocks(0, cells)]
    src, dst = 0, 1
    for _ in range(steps):
        g.diffuse(src, 2, dst, dt)
        hist.append(g.read_blocks(dst, cells))
        src, dst = dst, src
    return hist


def diffusion_loss(n, blocks, a0, k, target, dt, steps, precision="f64"):
    aT = diffusion_forward(n, blocks, a0, k, dt, steps, precision)[-1]
    r = aT.astype(np.float64) - target.astype(np.float64)
    return float(np.sum(r * r))


def diffusion_grad(n, blocks, a0, k, target, dt, steps, precision="f64"):
    """Loss sum((a_T - target)^2) and its gradients w.r.t. a0 and k via the
    reverse sweep: lam_T = 2 (a_T - target), then for t = T-1 .. 0 one
    adjoint step at a_t (accumulating grad_k).  All states are stored."""
    hist = diffusion_forward(n, blocks, a0, k, dt, steps, precision)
    d = np.float32 if precision == "f32" else np.float64
    aT = hist[-1]
    lam = (d(2) * (aT - target.astype(d))).astype(d)
    r = aT.astype(np.float64) - target.astype(np.float64)
    loss = float(np.sum(r * r))
    # channels: a, k, lam_next, lam, gk
    g = OracleGrid(n, 5, precision)
    g.load(blocks, {"k": k}, {"k": 1})
    g.listgen()
    cells = _cells(blocks, n // 8)
    for t in range(steps - 1, -1, -1):
        g.write_blocks(0, cells, hist[t])
        g.write_blocks(2, cells, lam)
        g.diffuse_adj(0, 1, 2, 3, 4, dt)
        lam = g.read_blocks(3, cells)
    return {"loss": loss, "grad_a0": lam, "grad_k": g.read_blocks(4, cells), "aT": aT}


# ---------------------------------------------------------------------------
# Multigrid V-cycle (the MGPCG pattern of Section 8.4 / Fig. 12: restriction,
# smoothing and prolongation over a sparse grid hierarchy).  Level l has domain
# edge n >> l and channels x, b, t; the coarse levels start empty and get their
# blocks from the restriction's activation on write.
MG_X, MG_B, MG_T = 0, 1, 2


def mg_smooth(g, omega):
    """Damped Jacobi: t = J(x); t = t - x; x = x + omega * t (each a struct-for
    preceded by a list generation, as written)."""
    g.listgen(); g.jacobi(MG_X, MG_B, MG_T)
    g.listgen(); g.axpy(MG_T, MG_X, -1.0)
    g.listgen(); g.axpy(MG_X, MG_T, omega)


def mg_vcycle(G, pre=2, post=2, coarse_iters=8, omega=0.75, w_restrict=1.5):
    """One V-cycle over the grids G (finest first).  The scaled residual
    t = J(x) - x (= r / 6) is restricted with y[I/2] += w * t[I] and the
    coarse correction is prolonged by injection, x[I] += x_c[I/2].  With
    injection P, the Galerkin coarse operator P^T A P is 4 times the 7-point
    operator on the coarse grid, so the coarse right-hand side is
    P^T r / 4 = (6 / 4) * sum of the children's t: w = 1.5."""
    L = len(G)
    for l in range(L - 1):
        g, c = G[l], G[l + 1]
        for _ in range(pre):
            mg_smooth(g, omega)
        g.listgen(); g.jacobi(MG_X, MG_B, MG_T)
        g.listgen(); g.axpy(MG_T, MG_X, -1.0)
        c.listgen(); c.fill(MG_X, 0.0)
        c.listgen(); c.fill(MG_B, 0.0)
        g.listgen(); g.restrict_to(c, MG_T, MG_B, w_restrict)
    for _ in range(coarse_iters):
        mg_smooth(G[L - 1], omega)
    for l in range(L - 2, -1, -1):
        g, c = G[l], G[l + 1]
        g.listgen(); g.prolong_from(c, MG_X, MG_X)
        for _ in range(post):
            mg_smooth(g, omega)


def multigrid_program(n, blocks, b, cycles, levels=3, precision="f32", **kw):
    """``cycles`` V-cycles on the Poisson system of ``jacobi_program``
    (6 x - sum of neighbours = b on the active voxels, x = 0 at start).
    Returns x on the finest level's blocks and every level's active cells."""
    G = [OracleGrid(n >> l, 3, precision) for l in range(levels)]
    G[0].load(blocks, {"b": b}, {"x": MG_X, "b": MG_B})
    for _ in range(cycles):
        mg_vcycle(G, **kw)
    cells = G[0].active_cells()
    return {"cells": cells, "x": G[0].read_blocks(MG_X, cells),
            "level_cells": [g.active_cells() for g in G], "grids": G}



# ---------------------------------------------------------------------------
def advection_program(n, blocks, channels, dt, steps, precision="f32"):
    """Per step and scalar field c: listgen -> advect_sl (tmp_c = q_c at
    I - dt v(I)) -> listgen -> copy (q_c = tmp_c).  Channels: q0..q2 = 0..2,
    v0..v2 = 3..5, tmp0..tmp2 = 6..8.  Returns the three fields."""
    g = OracleGrid(n, 9, precision)
    g.load(blocks, channels, {"q0": 0, "q1": 1, "q2": 2, "v0": 3, "v1": 4, "v2": 5})
    for _ in range(steps):
        for c in range(3):
            g.listgen()
            g.advect_sl(c, 3, 6 + c, dt)
            g.listgen()
            g.copy(c, 6 + c)
    cells = g.active_cells()
    return {"cells": cells, "q": [g.read_blocks(c, cells) for c in range(3)]}



def maccormack_program(n, blocks, channels, dt, steps, precision="f32", rk3=False):
    """Per step and field c: listgen, advect_sl (fwd), listgen, advect_sl (bwd,
    -dt), listgen, maccormack, listgen, copy.  Channels: q 0..2, v 3..5, fwd
    6..8, bwd 9..11, out 12..14.  Returns the three fields."""
    g = OracleGrid(n, 15, precision)
    g.load(blocks, channels, {"q0": 0, "q1": 1, "q2": 2, "v0": 3, "v1": 4, "v2": 5})
    for _ in range(steps):
        for c in range(3):
            g.listgen(); g.advect_sl(c, 3, 6 + c, dt, rk3)
            g.listgen(); g.advect_sl(6 + c, 3, 9 + c, -dt, rk3)
            g.listgen(); g.maccormack(c, 3, 6 + c, 9 + c, 12 + c, dt, rk3)
            g.listgen(); g.copy(c, 12 + c)
    cells = g.active_cells()
    return {"cells": cells, "q": [g.read_blocks(c, cells) for c in range(3)]}


# ---------------------------------------------------------------------------
# MLS-MPM (Section 8.3): substep t uses grid G = grids[t % 2] (the paper's two
# grids swapped before each substep); channels m, mv (3), v (3), and with
# with_abs the per-node sums of |term| (4) of the last scatter into G.
MPM_M, MPM_MV, MPM_V, MPM_ABS = 0, 1, 4, 7


def mpm_program(n, x, v, C, F, steps, dt, mass, vol, mu, lam, gravity, bound, precision="f64",
                with_abs=False):
    """Per substep: listgen(G) -> fill(G: m, mv = 0) -> mpm_p2g(G) (F updated,
    activating) -> listgen(G) -> mpm_grid(G) (v, gravity, walls) ->
    mpm_g2p(G) (v and C gathered) -> advect (x += dt v).  Returns the final
    particle state and both grids' cells and channels."""
    inv_dx = float(n)
    nch = 11 if with_abs else 7
    grids = [OracleGrid(n, nch, precision), OracleGrid(n, nch, precision)]
    d = np.float32 if precision == "f32" else np.float64
    x = np.ascontiguousarray(x, dtype=d).copy()
    v = np.ascontiguousarray(v, dtype=d).copy()
    C = np.ascontiguousarray(C, dtype=d).copy()
    F = np.ascontiguousarray(F, dtype=d).copy()
    for t in range(steps):
        G = grids[t % 2]
        G.listgen()
        for ch in range(MPM_MV + 3):
            G.fill(ch, 0.0)
        if with_abs:
            for ch in range(MPM_ABS, MPM_ABS + 4):
                G.fill(ch, 0.0)
        F, bad = G.mpm_p2g(MPM_M, MPM_MV, x, v, C, F, inv_dx, dt, mass, vol, mu, lam,
                           MPM_ABS if with_abs else -1)
        if bad:
            raise RuntimeError("particle left the domain")
        G.listgen()
        G.mpm_grid(MPM_M, MPM_MV, MPM_V, dt, gravity, bound)
        v, C = G.mpm_g2p(MPM_V, x, inv_dx)
        x = advect(x, v, dt, precision)
    out = {"x": x, "v": v, "C": C, "F": F}
    for gi, G in enumerate(grids):
        cells = G.active_cells()
        out["cells%d" % gi] = cells
        out["grid%d" % gi] = {ch: G.read_blocks(ch, cells) for ch in range(nch)}
    return out
