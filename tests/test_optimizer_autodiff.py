"""The differentiation program (Section 8.5's pattern on the sparse diffusion
of the differentiation workload) through the optimizer, on planning handles
(host only).

Written as a compiler without inter-kernel optimization emits it, every
struct-for gets its own list generation: a forward step is (listgen,
diffuse), an adjoint step (listgen, diffuse_adj), the seed
lam_T = 2 (a_T - target) three element-wise tasks (copy, axpy, axpy) beside
the clearing of grad_k.  Nothing activates after the set-up, so list
generation removal drops every listgen (one launch per step against two);
the clear and the seed are element-wise at the loop index over one list and
fuse into one launch; consecutive stencil steps never fuse (each reads the
previous one's output at neighbours).
"""
import pytest

from paper_2012_08141_amd import engine as E
from paper_2012_08141_amd.autodiff import DiffusionTasks
from paper_2012_08141_amd.grid import SparseGrid


@pytest.fixture(autouse=True)
def fresh_engine():
    E.reset()
    yield
    E.reset()


def _windows(flags, steps=20, every=5, root="bitmask"):
    E.reset()
    g = SparseGrid(128, DiffusionTasks.channels(steps, every), root, 2048 if root == "pointer" else 0, device=None)
    E.run_sequence([E.listgen(g)], E.OPT_ALL)
    t = DiffusionTasks(g, 0.1, steps, every)
    out = []
    for w in [t.fwd, t.bwd_init] + t.bwd:
        plan, st = E.plan_sequence(w, flags)
        E.run_sequence(w, flags)
        names = ["+".join(w[i].name for i in e["members"]) for e in plan]
        out.append((len(w), names, st))
    return t, out


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
@pytest.mark.parametrize("steps,every", [(20, 5), (7, 3), (4, 1)])
def test_diffusion_launches(steps, every, root):
    t, eager = _windows(0, steps, every, root)
    t, opt = _windows(E.OPT_ALL, steps, every, root)
    n_adj = steps
    n_recompute = sum(t.seg_len(s) - 1 for s in range(t.nseg))
    # eager: every task is a launch, two per step
    assert [len(n) for _, n, _ in eager] == [w for w, _, _ in eager]
    assert sum(w for w, _, _ in eager) == 2 * steps + 8 + 2 * (n_recompute + n_adj)
    # optimized: one launch per step, the clear and seed fused into one
    fwd, init, bwd = opt[0], opt[1], opt[2:]
    assert fwd[1] == ["diffuse"] * steps
    assert len(init[1]) == 1 and sorted(init[1][0].split("+")) == ["axpy", "axpy", "copy", "fill"]
    assert sum(len(n) for _, n, _ in bwd) == n_recompute + n_adj
    for _, names, _ in bwd:
        assert set(names) <= {"diffuse", "diffuse_adj"}
    removed = sum(st["listgens_removed"] for _, _, st in opt)
    assert removed == steps + 4 + n_recompute + n_adj


def test_diffusion_ablations():
    """Without list generation removal the listgens stay (two launches per
    step); without fusion the seed stays four launches."""
    _, no_lgr = _windows(E.OPT_ALL & ~E.OPT_LGR)
    assert no_lgr[0][1].count("listgen") == 20
    _, no_fuse = _windows(E.OPT_ALL & ~E.OPT_FUSE)
    assert no_fuse[1][1] == ["fill", "copy", "axpy", "axpy"]
