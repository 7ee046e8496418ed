"""The optimizer on multigrid V-cycles (paper Section 8.4, Fig. 12; the
downsample pattern of Section 6.3), on host-only planning handles.

A restriction y[I/2] += w x[I] activates the coarse parents of the fine
grid's listed blocks.  Once the same version of the fine list has been
restricted into a coarse grid, a later restriction of it adds no block:
activation demotion drops its check, the coarse mask stays unmodified and
list generation removal deletes the coarse levels' list generations.  So in
a solve whose hierarchy never changes, only the first cycle generates
lists."""
import ctypes

import pytest

from paper_2012_08141_amd import _lib as L
from paper_2012_08141_amd import engine as E
from paper_2012_08141_amd import programs as PR
from paper_2012_08141_amd.grid import SparseGrid


@pytest.fixture(autouse=True)
def fresh_engine():
    E.reset()
    yield
    E.reset()


def levels(n=64, nl=3, root="bitmask"):
    return [SparseGrid(n >> l, 3, root, (n >> l) ** 3 // 512 if root == "pointer" else 0, device=None)
            for l in range(nl)]


def kinds(entries, kind):
    return [e for e in entries if e["kind"] == kind]


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
def test_vcycle_plan_demotes_repeated_restrictions(root):
    lv = levels(root=root)
    one = len(PR.mg_vcycle(lv))
    tasks = PR.mg_vcycle(lv) + PR.mg_vcycle(lv)
    eager, st0 = E.plan_sequence(tasks, 0)
    assert len(eager) == st0["dispatches"] == 2 * one
    opt, st = E.plan_sequence(tasks, E.OPT_ALL)
    r = kinds(opt, L.AT_TASK_RESTRICT)
    assert [e["check_activation"] for e in r] == [True, True, False, False]
    # lists: the finest once, each coarse level before its first fill and after
    # the restriction that activated it; nothing in the second cycle
    assert len(kinds(opt, L.AT_TASK_LISTGEN)) == 1 + 2 * 2
    assert st["listgens_removed"] == len(kinds(eager, L.AT_TASK_LISTGEN)) - 5
    assert st["dispatches"] < 2 * one // 2
    # prolongations keep their place and never activate
    assert all(not e["check_activation"] for e in kinds(opt, L.AT_TASK_PROLONG))


def test_restriction_knowledge_persists_across_windows():
    """The coarse activation recorded by one window demotes the next
    window's restriction of the same fine list; a new fine list (after an
    activation and list generation) restores the check."""
    lv = levels()
    E.run_sequence(PR.mg_vcycle(lv), E.OPT_ALL)             # records state only
    opt, st = E.plan_sequence(PR.mg_vcycle(lv), E.OPT_ALL)
    assert [e["check_activation"] for e in kinds(opt, L.AT_TASK_RESTRICT)] == [False, False]
    assert kinds(opt, L.AT_TASK_LISTGEN) == []
    E.run_sequence(PR.mg_vcycle(lv), E.OPT_ALL)
    # the fine grid gains a block: its list changes, so the first restriction
    # must activate again (the second level's list is unchanged by that)

    class Coords:
        shape = (1, 3)

        def data_ptr(self):
            return 0x5000000

    tasks = [E.activate(lv[0], Coords())] + PR.mg_vcycle(lv)
    opt, _ = E.plan_sequence(tasks, E.OPT_ALL)
    checks = [e["check_activation"] for e in kinds(opt, L.AT_TASK_RESTRICT)]
    assert checks[0] is True


def test_plan_cache_separates_known_and_unknown_restrictions():
    """A cached plan is reused only when the restriction knowledge matches:
    the same window planned before and after the coarse activation is known
    gives different plans."""
    lv = levels()
    w = PR.mg_vcycle(lv)
    first, _ = E.plan_sequence(w, E.OPT_ALL)
    E.run_sequence(w, E.OPT_ALL)
    second, _ = E.plan_sequence(w, E.OPT_ALL)
    assert [e["check_activation"] for e in kinds(first, L.AT_TASK_RESTRICT)] == [True, True]
    assert [e["check_activation"] for e in kinds(second, L.AT_TASK_RESTRICT)] == [False, False]


def test_two_level_task_validation():
    lib = L.lib()
    f = SparseGrid(64, 3, "bitmask", device=None)
    c = SparseGrid(32, 2, "bitmask", device=None)
    wrong = SparseGrid(16, 3, "bitmask", device=None)
    st = L.AtStats()

    def status(t):
        return lib.at_run_sequence(ctypes.byref(t.c), 1, E.OPT_ALL, ctypes.byref(st), None)

    assert status(E.restrict(f, c, 0, 1, 0.5)) == L.AT_OK
    assert status(E.restrict(f, wrong, 0, 1, 0.5)) == L.AT_E_INVALID      # not half the edge
    assert status(E.restrict(f, f, 0, 1, 0.5)) == L.AT_E_INVALID          # same grid
    assert status(E.restrict(f, c, 0, 2, 0.5)) == L.AT_E_INVALID          # coarse has 2 channels
    assert status(E.prolong(c, f, 2, 0)) == L.AT_E_INVALID                # coarse channel 2
    assert status(E.prolong(c, f, 1, 3)) == L.AT_E_INVALID                # fine channel 3
    t = E.jacobi(f, 0, 1, 2)
    t.c.grid2 = c.handle.value                                             # grid2 only on transfers
    assert status(t) == L.AT_E_INVALID
    t = E.restrict(f, c, 0, 1, 0.5)
    t.c.grid2 = None
    assert status(t) == L.AT_E_INVALID


def test_plan_cache_tells_coarse_grids_apart():
    """Two windows that differ only in the coarse grid of a restriction get
    their own plans, even from start states that look alike to the cache:
    restricting into c1 modifies c1's mask, so the list generation of c1 after
    it stays; restricting into c2 leaves c1's list current and removes it."""
    f = SparseGrid(64, 3, "bitmask", device=None)
    c1 = SparseGrid(32, 3, "bitmask", device=None)
    c2 = SparseGrid(32, 3, "bitmask", device=None)
    fresh = [E.listgen(f), E.listgen(c1), E.listgen(c2)]

    def window(c):
        return [E.listgen(c1), E.listgen(c2), E.restrict(f, c, 0, 1, 0.5), E.listgen(c1), E.inc(c1, 0, 1.0)]

    E.run_sequence(fresh, E.OPT_ALL)
    st2 = E.run_sequence(window(c2), E.OPT_ALL)            # records state only
    assert st2["tasks_launched"] == 2 and st2["listgens_removed"] == 3
    E.run_sequence(fresh, E.OPT_ALL)
    st1 = E.run_sequence(window(c1), E.OPT_ALL)
    assert st1["plan_cache_hits"] == 0
    assert st1["tasks_launched"] == 3 and st1["listgens_removed"] == 2
