"""Differentiation of sparse diffusion through the hand-written adjoint.

Forward: a_{t+1} = a_t + dt * sum_faces kf (a_nb - a_t), kf = (k + k_nb)/2,
for t = 0 .. T-1 on the active blocks of one grid; loss
L = sum (a_T - target)^2.  Backward: lam_T = 2 (a_T - target); per step, in
reverse, the adjoint kernel (AT_OP_DIFFUSE_ADJ) maps lam_{t+1} to lam_t and
accumulates grad_k at state a_t.  States are checkpointed every
``checkpoint_every`` steps in the forward pass and recomputed inside each
segment during the backward pass, so memory holds T/checkpoint_every
checkpoints plus one segment.

The program is written as a compiler without inter-kernel optimization
emits it (Section 3.2): every struct-for over the sparse grid gets its own
list generation, so a step is (listgen, diffuse) and an adjoint step
(listgen, diffuse_adj).  The optimizer removes the repeated list
generations.  The seed lam_T = 2 (a_T - target) is three element-wise tasks
of the library (copy, then two axpys: 2 a_T exactly, then one rounding of
2 a_T - 2 target), which fuse into one launch; the adjoint is linear in the
seed, so the upstream gradient multiplies the results.  Torch provides the
device buffers and the loss value (a sum of squares over a_T - target),
which is the user's objective outside the sparse path.
"""
from __future__ import annotations

import numpy as np
import torch

from . import engine as E
from .grid import SparseGrid


class DiffusionTasks:
    """The engine windows of one forward and one backward pass, on any grid
    handle with ``channels(steps, every)`` channels (a planning handle too).

    Channels: ck[0..S-1] checkpoints a_0, a_c, a_2c, ...; seg[1..c] segment
    states; k; lamA, lamB (adjoint ping-pong); gk; target.

    Windows: ``fwd`` (every step, the last state of each segment into the
    next checkpoint), ``bwd_init`` (gk = 0 and the seed lam_T), then one
    window per segment in reverse (``bwd``): recompute its states from the
    checkpoint, then the adjoint steps back through them."""

    @staticmethod
    def channels(steps: int, every: int) -> int:
        nseg = (steps + every - 1) // every
        return nseg + every + 1 + 5

    def __init__(self, grid, dt: float, steps: int, every: int):
        assert steps > 0 and every > 0
        self.grid, self.dt, self.steps, self.every = grid, float(dt), steps, every
        self.nseg = (steps + every - 1) // every
        self.ck = list(range(self.nseg))
        self.seg = list(range(self.nseg, self.nseg + every + 1))   # seg[0] unused (= checkpoint)
        base = self.nseg + every + 1
        self.K, self.LA, self.LB, self.GK, self.TG = base, base + 1, base + 2, base + 3, base + 4
        g = grid
        self.fwd = []
        for s in range(self.nseg):
            nxt = self.ck[s + 1] if s + 1 < self.nseg else None
            t, self.last = self._segment_tasks(s, self.seg_len(s), nxt)
            self.fwd += t
        LA, aT = self.LA, self.last
        self.bwd_init = [E.listgen(g), E.fill(g, [self.GK], 0.0),
                         E.listgen(g), E.copy(g, LA, aT),
                         E.listgen(g), E.axpy(g, LA, aT, 1.0),
                         E.listgen(g), E.axpy(g, LA, self.TG, -2.0)]
        self.bwd = []
        lamn, lam = self.LA, self.LB
        for s in reversed(range(self.nseg)):
            L = self.seg_len(s)
            tasks, _ = self._segment_tasks(s, L - 1) if L > 1 else ([], None)
            states = [self.ck[s]] + [self.seg[i] for i in range(1, L)]
            for i in reversed(range(L)):
                tasks += [E.listgen(g), E.diffuse_adj(g, states[i], self.K, lamn, lam, self.GK, self.dt)]
                lamn, lam = lam, lamn
            self.bwd.append(tasks)
        self.lam_out = lamn

    def _segment_tasks(self, s: int, nsteps: int, last_into=None):
        """Tasks computing a_{s*c+1 .. s*c+nsteps} from checkpoint s into
        segment channels (the last one into ``last_into`` when given)."""
        g = self.grid
        tasks, cur = [], self.ck[s]
        for i in range(1, nsteps + 1):
            dst = last_into if (i == nsteps and last_into is not None) else self.seg[i]
            tasks += [E.listgen(g), E.diffuse(g, cur, self.K, dst, self.dt)]
            cur = dst
        return tasks, cur

    def seg_len(self, s: int) -> int:
        return min(self.every, self.steps - s * self.every)


class DiffusionProblem:
    """A device grid holding the differentiation of ``steps`` diffusion
    steps over the given active blocks (layout and windows: DiffusionTasks)."""

    def __init__(self, n: int, blocks: np.ndarray, dt: float, steps: int, checkpoint_every: int = 5,
                 root_kind: str = "bitmask", opt_flags: int = E.OPT_ALL):
        self.n, self.opt = n, opt_flags
        R = n // 8
        b = np.asarray(blocks, dtype=np.int64)
        self.cells_np = ((b[:, 0] * R + b[:, 1]) * R + b[:, 2]).astype(np.int32)
        self.cells = torch.as_tensor(self.cells_np, device="cuda")
        cap = len(self.cells_np) if root_kind == "pointer" else 0
        self.grid = SparseGrid(n, DiffusionTasks.channels(steps, checkpoint_every), root_kind, cap)
        z = torch.zeros((len(self.cells_np), 512), dtype=torch.float32, device="cuda")
        self.grid.load_blocks(0, self.cells, z)          # activates the blocks
        E.run_sequence([E.listgen(self.grid)], self.opt)
        self.windows = 0
        self.t = t = DiffusionTasks(self.grid, dt, steps, checkpoint_every)
        # the windows' tasks never change: pack them once
        self.fwd = E.prepare(t.fwd)
        self.bwd_init = E.prepare(t.bwd_init)
        self.bwd = [E.prepare(w) for w in t.bwd]
        self.ck, self.seg, self.K, self.LA, self.LB, self.GK, self.TG = t.ck, t.seg, t.K, t.LA, t.LB, t.GK, t.TG
        self.last, self.lam_out = t.last, t.lam_out

    # ---- helpers --------------------------------------------------------------
    def _put(self, ch: int, t: torch.Tensor):
        self.grid.load_blocks(ch, self.cells, t.detach().to(torch.float32).contiguous())

    def _get(self, ch: int) -> torch.Tensor:
        return self.grid.read_blocks_t(ch, self.cells)

    def _run(self, tasks):
        self.windows += 1
        return E.run_sequence(tasks, self.opt)

    # ---- forward / backward -------------------------------------------------
    def forward(self, a0: torch.Tensor, k: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
        """a_T on the active blocks ([nb, 512], a new tensor); stores the
        checkpoints and the target."""
        self._put(self.ck[0], a0)
        self._put(self.K, k)
        self._put(self.TG, target)
        self._run(self.fwd)
        return self._get(self.last)

    def backward(self):
        """(grad_a0, grad_k) of L = sum (a_T - target)^2 for the last forward
        pass (new tensors).  The seed lam_T = 2 (a_T - target) is formed on
        the grid; then per segment, in reverse: recompute its states from
        the checkpoint, then run the adjoint steps back through them."""
        self._run(self.bwd_init)
        for w in self.bwd:
            self._run(w)
        return self._get(self.lam_out), self._get(self.GK)


class DiffusionLoss(torch.autograd.Function):
    """loss = sum((a_T(a0, k) - target)^2) with the adjoint backward."""

    @staticmethod
    def forward(ctx, a0, k, target, problem: DiffusionProblem):
        aT = problem.forward(a0, k, target)
        r = (aT - target).double()
        ctx.problem = problem
        return (r * r).sum().to(a0.dtype)

    @staticmethod
    def backward(ctx, gout):
        ga0, gk = ctx.problem.backward()
        g = gout.to(ga0.dtype)
        return ga0 * g, gk * g, None, None


def diffusion_loss(a0, k, target, problem: DiffusionProblem):
    return DiffusionLoss.apply(a0, k, target, problem)
