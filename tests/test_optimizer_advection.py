"""The optimizer on the three-field advection program (paper Section 8.2),
on host-only planning handles: per step and field, listgen -> advect ->
listgen -> copy.  List generation removal deletes the list generations, and
fusion joins the three advections (independent tasks over the same list that
share only the velocity they read) and the three copies: 12 launches become
2.  An advection and the copy into the field it reads at other voxels never
fuse (criterion 3)."""
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


def test_three_field_step_fuses_to_two_launches():
    g = SparseGrid(256, 9, "bitmask", device=None)
    E.run_sequence([E.listgen(g)], E.OPT_ALL)
    step = PR.advection_step(g, 1.0 / 256)
    eager, _ = E.plan_sequence(step, 0)
    assert len(eager) == 12 and E.paper_task_count(eager) == 18
    opt, st = E.plan_sequence(step, E.OPT_ALL)
    assert [e["members"] for e in opt] == [[1, 5, 9], [3, 7, 11]]
    assert st["listgens_removed"] == 6


def test_advection_and_copy_into_its_source_do_not_fuse():
    g = SparseGrid(64, 9, "bitmask", device=None)
    E.run_sequence([E.listgen(g)], E.OPT_ALL)
    opt, _ = E.plan_sequence([E.advect_sl(g, 0, 3, 6, 0.1), E.copy(g, 0, 6)], E.OPT_ALL)
    assert len(opt) == 2


def test_advect_validation():
    lib = L.lib()
    import ctypes
    g = SparseGrid(64, 6, "bitmask", device=None)
    st = L.AtStats()

    def status(t):
        return lib.at_run_sequence(ctypes.byref(t.c), 1, E.OPT_ALL, ctypes.byref(st), None)

    assert status(E.advect_sl(g, 0, 1, 4, 0.1)) == L.AT_OK
    assert status(E.advect_sl(g, 0, 1, 0, 0.1)) == L.AT_E_INVALID       # out aliases q
    assert status(E.advect_sl(g, 0, 1, 2, 0.1)) == L.AT_E_INVALID       # out aliases a velocity
    assert status(E.advect_sl(g, 0, 4, 1, 0.1)) == L.AT_E_INVALID       # velocity needs 3 channels


def test_maccormack_step_plan():
    """The three-field MacCormack step (per field: forward and backward
    advection, correction, copy back, each after a list generation) plans to 5
    launches instead of 24 (paper-style 36)."""
    g = SparseGrid(256, 15, "bitmask", device=None)
    E.run_sequence([E.listgen(g)], E.OPT_ALL)
    step = PR.maccormack_step(g, 1.0 / 256)
    eager, _ = E.plan_sequence(step, 0)
    assert len(eager) == 24 and E.paper_task_count(eager) == 36
    opt, _ = E.plan_sequence(step, E.OPT_ALL)
    assert len(opt) == 5
    assert sorted(m for e in opt for m in e["members"]) == [i for i in range(24) if i % 2 == 1]


def test_maccormack_ablations_follow_the_paper():
    """The paper's MacCormack ablation: fusion gives most of the cut, and
    disabling list generation removal transitively disables fusion (the
    kept list generations sit between the tasks); activation demotion is needed
    for list generation removal (the struct-fors' checks write the mask)."""
    g = SparseGrid(256, 15, "bitmask", device=None)
    E.run_sequence([E.listgen(g)], E.OPT_ALL)
    step = PR.maccormack_step(g, 1.0 / 256)
    E.run_sequence(step, E.OPT_ALL)
    count = {k: len(E.plan_sequence(step, fl)[0]) for k, fl in (
        ("all", E.OPT_ALL), ("no_lgr", E.OPT_ALL & ~E.OPT_LGR), ("no_ad", E.OPT_ALL & ~E.OPT_AD),
        ("no_fusion", E.OPT_ALL & ~E.OPT_FUSE), ("no_dse", E.OPT_ALL & ~E.OPT_DSE), ("eager", 0))}
    assert count == {"all": 5, "no_lgr": 24, "no_ad": 23, "no_fusion": 12, "no_dse": 5, "eager": 24}
