"""Launches per step of each workload's task program, eager vs optimized,
and the per-pass ablations (host-only planning handles).

Expected counts (L = 1 dispatch per list generation, the clear folded in):
  shell (activate, listgen, lap_update, listgen, axpy):   eager 3+2L, optimized 2
  Jacobi (listgen, jacobi, copy):                          eager 2+L,  optimized 2
  particles (listgen, reset, advect, p2g, listgen, normalise, g2p):
                                                           eager 5+2L, optimized 2+L
  diffusion (listgen once, then diffuse per step):         optimized 1 per step
The optimized counts follow from Section 6: activation demotion removes the
repeated activation and the loop-index checks, which leaves the masks
unmodified so list generation removal deletes the listgens; lap_update ->
axpy and jacobi -> copy are not fusible (criterion 3); G2P, advection and
P2G of consecutive substeps fuse (Section 8.3); and since list generation
removal gives a grid's reset two steps later the same list version as its
normalise, those two element-wise struct-fors fuse as well."""
import pytest

from paper_2012_08141_amd import _lib as L
from paper_2012_08141_amd import engine as E
from paper_2012_08141_amd import programs as PR
from paper_2012_08141_amd.grid import SparseGrid


class FakeArray:
    _next = 0x7000000

    def __init__(self, shape):
        self.shape = shape
        self._p = FakeArray._next
        FakeArray._next += 1 << 24

    def data_ptr(self):
        return self._p


@pytest.fixture(autouse=True)
def fresh_engine():
    E.reset()
    yield
    E.reset()


def run_plan(setup, steps, flags):
    if setup:
        E.run_sequence(setup, E.OPT_ALL)          # planning handles: records state only
    entries, st = E.plan_sequence(steps, flags)
    return entries, st


def test_shell_launches():
    g = SparseGrid(64, 2, "bitmask", device=None)
    coords = FakeArray((80, 3))
    steps = sum((PR.shell_step(g, coords) for _ in range(10)), [])
    setup = PR.shell_setup(g, coords)
    expect = {0: 50, E.OPT_ALL: 20, E.OPT_LGR: 50, E.OPT_AD: 40, E.OPT_AD | E.OPT_LGR: 20,
              E.OPT_ALL & ~E.OPT_FUSE: 20, E.OPT_ALL & ~E.OPT_DSE: 20}
    for flags, n in expect.items():
        E.reset()
        ents, st = run_plan(setup, steps, flags)
        assert len(ents) == n, (flags, len(ents), st)
    # the two surviving tasks per step are the two struct-fors, unfused
    kinds = [(e["kind"], len(e["members"])) for e in ents]
    assert kinds == [(L.AT_TASK_STENCIL, 1)] * 20
    # without the setup window the first step keeps its activation and listgen
    E.reset()
    ents, st = run_plan(None, steps, E.OPT_ALL)
    assert len(ents) == 22


def test_jacobi_launches():
    g = SparseGrid(512, 3, "bitmask", device=None)
    steps = sum((PR.jacobi_step(g) for _ in range(100)), [])
    for flags, n in {0: 300, E.OPT_ALL: 201, E.OPT_LGR: 300, E.OPT_AD | E.OPT_LGR: 201}.items():
        E.reset()
        ents, st = run_plan(None, steps, flags)
        assert len(ents) == n, (flags, len(ents))
    # with the setup listgen preserved from an earlier window (partial GC)
    E.reset()
    ents, st = run_plan([E.listgen(g)], steps, E.OPT_ALL)
    assert len(ents) == 200 and st["listgens_removed"] == 100 and st["fusions"] == 0


def test_particle_launches():
    G = [SparseGrid(256, 7, "pointer", 4096, device=None) for _ in range(2)]
    x, v, m = FakeArray((3, 2000)), FakeArray((3, 2000)), FakeArray((2000,))
    steps = sum((PR.particle_step(G, t, x, v, m, 1e-3, 1 / 256) for t in range(20)), [])
    ents, st = run_plan(None, steps, 0)
    assert len(ents) == 140
    E.reset()
    ents, st = run_plan(None, steps, E.OPT_ALL)
    # t=0 and t=1: listgen, reset, (g2p+)advect+p2g, listgen, normalise+reset(t+2);
    # t=2..17: g2p+advect+p2g, listgen, normalise+reset(t+2); t=18, 19: g2p+advect+p2g,
    # listgen, normalise; then the last g2p alone
    assert len(ents) == 5 + 5 + 16 * 3 + 3 + 3 + 1, [(e["kind"], e["members"]) for e in ents]
    nr = [e for e in ents if len(e["members"]) == 2 and e["kind"] == L.AT_TASK_STENCIL]
    assert len(nr) == 18 and all(e["members"][1] - e["members"][0] == 2 * 7 - 4 for e in nr)
    fused = [e for e in ents if len(e["members"]) == 3]
    assert len(fused) == 19
    assert all(e["activation_mode"] == L.AT_ACT_PER_BLOCK for e in fused)
    # dead store elimination: reset's v = 0 (overwritten by normalise) goes
    assert st["stores_eliminated"] == 3 * 20


def test_diffusion_launches():
    g = SparseGrid(128, 3, "bitmask", device=None)
    tasks, _ = PR.diffusion_forward_tasks(g, 20, 0.1)
    ents, st = run_plan(None, tasks, 0)
    assert len(ents) == 21
    E.reset()
    ents, st = run_plan([E.listgen(g)], tasks, E.OPT_ALL)
    assert len(ents) == 20


def test_plan_cache_hits_and_is_identical():
    g = SparseGrid(64, 3, "bitmask", device=None)
    E.run_sequence([E.listgen(g)], E.OPT_ALL)
    step = PR.jacobi_step(g)
    s1 = E.run_sequence(step, E.OPT_ALL)
    s2 = E.run_sequence(step, E.OPT_ALL)
    assert s1["plan_cache_hits"] == 0 and s2["plan_cache_hits"] == 1
    assert s1["tasks_launched"] == s2["tasks_launched"] == 2
    # a mask change between windows invalidates the cached decision
    coords = FakeArray((4, 3))
    E.run_sequence([E.activate(g, coords)], 0)
    s3 = E.run_sequence(step, E.OPT_ALL)
    assert s3["plan_cache_hits"] == 0 and s3["tasks_launched"] == 3


def test_enqueue_flush_period():
    g = SparseGrid(64, 3, "bitmask", device=None)
    E.set_option(L.AT_OPTION_FLUSH_PERIOD, 0)
    for t in sum((PR.jacobi_step(g) for _ in range(4)), []):
        E.enqueue(t)
    st = E.flush()
    assert st["tasks_in"] == 12 and st["tasks_launched"] == 9
    # flush period 1 turns asynchrony off: every task is its own window
    E.set_option(L.AT_OPTION_FLUSH_PERIOD, 1)
    for t in PR.jacobi_step(g):
        E.enqueue(t)
    st = E.flush()
    assert st["tasks_in"] == 0
    E.set_option(L.AT_OPTION_FLUSH_PERIOD, 0)


def test_scatter_without_activation_leaves_the_list_current():
    """A scatter that activates nothing (AT_ACT_NONE) does not write the
    mask, so the list generation after it is removable; one that activates
    (per node or per block) keeps it (Section 6.2)."""
    G = SparseGrid(256, 7, "pointer", 4096, device=None)
    x, v, m = FakeArray((3, 1000)), FakeArray((3, 1000)), FakeArray((1000,))
    for act, removed in ((L.AT_ACT_NONE, 1), (L.AT_ACT_PER_BLOCK, 0), (L.AT_ACT_PER_NODE, 0)):
        E.reset()
        tasks = [E.listgen(G), E.p2g(G, x, v, m, 1 / 256, 0, 1, activation=act), E.listgen(G)]
        _, st = E.plan_sequence(tasks, E.OPT_LGR)
        assert st["listgens_removed"] == removed, act
    E.reset()
