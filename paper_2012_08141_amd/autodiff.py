"""Differentiation of sparse diffusion through the hand-written adjoint.

Forward: a_{t+1} = a_t + dt * sum_faces kf (a_nb - a_t), kf = (k + k_nb)/2,
for t = 0 .. T-1 on the active blocks of one grid; loss
L = sum (a_T - target)^2.  Backward: lam_T = 2 (a_T - target); per step, in
reverse, the adjoint kernel (AT_OP_DIFFUSE_ADJ) maps lam_{t+1} to lam_t and
accumulates grad_k at state a_t.  States are checkpointed every
``checkpoint_every`` steps in the forward pass and recomputed inside each
segment during the backward pass, so memory holds T/checkpoint_every
checkpoints plus one segment.

Every step runs as an engine window of HIP kernels (the optimizer removes the
repeated list generations); torch provides the device buffers and the loss
value (sum of squares), which sits outside the sparse path.
"""
from __future__ import annotations

import numpy as np
import torch

from . import engine as E
from .grid import SparseGrid


class DiffusionProblem:
    """Grid and channel layout for differentiating ``steps`` diffusion steps.

    Channels: ck[0..S-1] checkpoints a_0, a_c, a_2c, ...; seg[1..c] segment
    states; k; lamA, lamB (adjoint ping-pong); gk."""

    def __init__(self, n: int, blocks: np.ndarray, dt: float, steps: int, checkpoint_every: int = 5,
                 root_kind: str = "bitmask", opt_flags: int = E.OPT_ALL):
        assert steps > 0 and checkpoint_every > 0
        self.n, self.dt, self.steps, self.every = n, float(dt), steps, checkpoint_every
        self.opt = opt_flags
        self.nseg = (steps + checkpoint_every - 1) // checkpoint_every
        self.ck = list(range(self.nseg))
        self.seg = list(range(self.nseg, self.nseg + checkpoint_every + 1))   # seg[0] unused (= checkpoint)
        base = self.nseg + checkpoint_every + 1
        self.K, self.LA, self.LB, self.GK = base, base + 1, base + 2, base + 3
        self.nch = base + 4
        R = n // 8
        b = np.asarray(blocks, dtype=np.int64)
        self.cells_np = ((b[:, 0] * R + b[:, 1]) * R + b[:, 2]).astype(np.int32)
        self.cells = torch.as_tensor(self.cells_np, device="cuda")
        cap = len(self.cells_np) if root_kind == "pointer" else 0
        self.grid = SparseGrid(n, self.nch, root_kind, cap)
        z = torch.zeros((len(self.cells_np), 512), dtype=torch.float32, device="cuda")
        self.grid.load_blocks(0, self.cells, z)          # activates the blocks
        E.run_sequence([E.listgen(self.grid)], self.opt)
        self.windows = 0
        # the windows' tasks never change: pack them once
        fwd = []
        for s in range(self.nseg):
            nxt = self.ck[s + 1] if s + 1 < self.nseg else None
            t, self.last = self._segment_tasks(s, self.seg_len(s), nxt)
            fwd += t
        self.fwd = E.prepare(fwd)
        g = self.grid
        self.bwd_init = E.prepare([E.listgen(g), E.fill(g, [self.GK], 0.0)])
        self.bwd = []
        lamn, lam = self.LA, self.LB
        for s in reversed(range(self.nseg)):
            L = self.seg_len(s)
            tasks, _ = self._segment_tasks(s, L - 1) if L > 1 else ([E.listgen(g)], None)
            states = [self.ck[s]] + [self.seg[i] for i in range(1, L)]
            for i in reversed(range(L)):
                tasks.append(E.diffuse_adj(g, states[i], self.K, lamn, lam, self.GK, self.dt))
                lamn, lam = lam, lamn
            self.bwd.append(E.prepare(tasks))
        self.lam_out = lamn

    # ---- helpers --------------------------------------------------------------
    def _put(self, ch: int, t: torch.Tensor):
        self.grid.load_blocks(ch, self.cells, t.detach().to(torch.float32).contiguous())

    def _get(self, ch: int) -> torch.Tensor:
        return self.grid.read_blocks_t(ch, self.cells)

    def _run(self, tasks):
        self.windows += 1
        return E.run_sequence(tasks, self.opt)

    def _segment_tasks(self, s: int, nsteps: int, last_into=None):
        """Tasks computing a_{s*c+1 .. s*c+nsteps} from checkpoint s into
        segment channels (the last one into ``last_into`` when given)."""
        g = self.grid
        tasks, cur = [E.listgen(g)], self.ck[s]
        for i in range(1, nsteps + 1):
            dst = last_into if (i == nsteps and last_into is not None) else self.seg[i]
            tasks.append(E.diffuse(g, cur, self.K, dst, self.dt))
            cur = dst
        return tasks, cur

    def seg_len(self, s: int) -> int:
        return min(self.every, self.steps - s * self.every)

    # ---- forward / backward -------------------------------------------------
    def forward(self, a0: torch.Tensor, k: torch.Tensor) -> torch.Tensor:
        """a_T on the active blocks ([nb, 512], a new tensor); stores the
        checkpoints."""
        self._put(self.ck[0], a0)
        self._put(self.K, k)
        self._run(self.fwd)
        return self._get(self.last)

    def backward(self, lam_T: torch.Tensor):
        """(grad_a0, grad_k) for adjoint seed lam_T = dL/da_T (new tensors).
        Per segment, in reverse: recompute its states from the checkpoint,
        then run the adjoint steps back through them."""
        self._put(self.LA, lam_T)
        self._run(self.bwd_init)
        for w in self.bwd:
            self._run(w)
        return self._get(self.lam_out), self._get(self.GK)


class DiffusionLoss(torch.autograd.Function):
    """loss = sum((a_T(a0, k) - target)^2) with the adjoint backward."""

    @staticmethod
    def forward(ctx, a0, k, target, problem: DiffusionProblem):
        aT = problem.forward(a0, k)
        r = aT - target
        ctx.problem = problem
        ctx.save_for_backward(r)
        return (r.double() * r.double()).sum().to(a0.dtype)

    @staticmethod
    def backward(ctx, gout):
        (r,) = ctx.saved_tensors
        lam_T = (2.0 * r) * gout.to(r.dtype)
        ga0, gk = ctx.problem.backward(lam_T)
        return ga0, gk, None, None


def diffusion_loss(a0, k, target, problem: DiffusionProblem):
    return DiffusionLoss.apply(a0, k, target, problem)
