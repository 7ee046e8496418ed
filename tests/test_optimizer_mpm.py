"""The MLS-MPM program (Section 8.3) through the optimizer, on planning
handles (host only).

Per substep t (grid G = grids[t % 2]) the program is listgen(G), fill(G: m,
mv), p2g_mls(G), listgen(G), mpm_grid(G), g2p_apic(G), advect: 7 launches
eager.  After a window of two substeps has recorded the engine state, a
window of K substeps optimizes to 3K + 3 launches:

* list generation removal drops the first listgen of every substep (the
  list of G is current since the listgen after G's scatter two substeps
  before, and nothing has modified G's mask since);
* fusion joins the gather and advection of substep t with the scatter of
  substep t + 1 into one G2P2G task over the same particle arrays (the
  loop_unique hint of supplement Section 4.4), and the grid update of G with
  the fill of G two substeps later (both element-wise at the loop index over
  the same list version);
* dead store elimination then drops the stores of v and C of every G2P2G
  task: inside it they reach the scatter in registers, and the next access
  to each array is the next gather's complete overwrite.  The last gather of
  the window keeps both stores (the host may read them).

The ablations mirror the paper's Table 4: without DSE the launches are the
same but every store stays; without fusion nothing is eliminated either.
"""
import pytest

from paper_2012_08141_amd import _lib as L
from paper_2012_08141_amd import engine as E
from paper_2012_08141_amd import programs as PR
from paper_2012_08141_amd.grid import SparseGrid

from test_optimizer_programs import FakeArray

PARAMS = dict(dt=1e-4, dx=1 / 64, mass=1e-3, vol=1e-6, mu=1.0, lam=1.0, gravity=9.8, bound=2)


@pytest.fixture(autouse=True)
def fresh_engine():
    E.reset()
    yield
    E.reset()


def _window(K, flags, root="bitmask"):
    E.reset()
    grids = [SparseGrid(64, 7, root, 512 if root == "pointer" else 0, device=None) for _ in range(2)]
    arrays = FakeArray((3, 1000)), FakeArray((3, 1000)), FakeArray((9, 1000)), FakeArray((9, 1000))
    setup = sum((PR.mpm_step(grids, t, *arrays, PARAMS) for t in range(2)), [])
    E.run_sequence(setup, E.OPT_ALL)
    tasks = sum((PR.mpm_step(grids, t, *arrays, PARAMS) for t in range(2, 2 + K)), [])
    plan, st = E.plan_sequence(tasks, flags)
    names = ["+".join(tasks[i].name for i in e["members"]) for e in plan]
    return tasks, plan, names, st


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
@pytest.mark.parametrize("K", [4, 8, 16])
def test_mpm_launches_and_passes(K, root):
    tasks, plan, names, st = _window(K, 0, root)
    assert len(tasks) == 7 * K and len(plan) == 7 * K
    tasks, plan, names, st = _window(K, E.OPT_ALL, root)
    assert len(plan) == 3 * K + 3
    assert names.count("g2p_apic+advect+p2g_mls") == K - 1
    assert names.count("mpm_grid+fill") == K - 2
    assert names.count("listgen") == K
    assert st["listgens_removed"] == K
    assert st["stores_eliminated"] == 2 * (K - 1)
    # every G2P2G drops the stores of v and C; the window's last gather keeps both
    for e, nm in zip(plan, names):
        if nm == "g2p_apic+advect+p2g_mls":
            assert e["keep"][0] & 3 == 0
        if nm == "g2p_apic+advect":
            assert e["keep"][0] & 3 == 3
    # the G2P2G of substeps t, t + 1 takes the gather of t and the scatter of t + 1
    for e, nm in zip(plan, names):
        if nm == "g2p_apic+advect+p2g_mls":
            g, a, s = e["members"]
            assert a == g + 1 and s == g + 4 and tasks[s].c.grid != tasks[g].c.grid


def test_mpm_ablations():
    K = 8
    full = _window(K, E.OPT_ALL)[3]
    no_dse = _window(K, E.OPT_ALL & ~E.OPT_DSE)
    assert len(no_dse[1]) == 3 * K + 3 and no_dse[3]["stores_eliminated"] == 0
    assert full["stores_eliminated"] == 2 * (K - 1)
    no_fuse = _window(K, E.OPT_ALL & ~E.OPT_FUSE)
    assert len(no_fuse[1]) == 6 * K and no_fuse[3]["stores_eliminated"] == 0
    no_lgr = _window(K, E.OPT_ALL & ~E.OPT_LGR)
    assert len(no_lgr[1]) == 5 * K + 1 and no_lgr[3]["listgens_removed"] == 0


def test_mpm_tasks_validate():
    g = SparseGrid(64, 7, "bitmask", device=None)
    x, v, C, F = FakeArray((3, 10)), FakeArray((3, 10)), FakeArray((9, 10)), FakeArray((9, 10))
    bad = E.g2p_apic(g, x, v, v, PARAMS["dx"], 4)          # v and C alias
    with pytest.raises(L.AtError):
        E.plan_sequence([bad], 0)
    bad = E.mpm_grid(g, 0, 1, 2, 1e-4, 9.8, 2)             # v overlaps mv
    with pytest.raises(L.AtError):
        E.plan_sequence([bad], 0)
    bad = E.mpm_grid(g, 0, 1, 4, 1e-4, 9.8, 2.5)           # fractional wall
    with pytest.raises(L.AtError):
        E.plan_sequence([bad], 0)
    ok = [E.p2g_mls(g, x, v, C, F, PARAMS["dx"], 1e-4, 1.0, 1.0, 1.0, 1.0, 0, 1), E.mpm_grid(g, 0, 1, 4, 1e-4, 9.8, 2),
          E.g2p_apic(g, x, v, C, PARAMS["dx"], 4)]
    E.plan_sequence(ok, E.OPT_ALL)
