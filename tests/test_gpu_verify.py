"""The debug mode for activation demotion (AT_OPTION_VERIFY_DEMOTED).

With the mode on, every launched node whose activation check the optimizer
dropped (Section 6.3: a struct-for writing at its loop index, a restriction
whose list version was already restricted into the coarse grid) checks that
each block it writes is still active.  A correct plan never trips it: the
band Jacobi and multigrid V-cycle programs run with it on, leave bit 2 of
every grid's status clear and give the results of the mode switched off.
A block removed from a pointer root behind the engine's back (so list
generation removal keeps serving a list that still holds it) is caught by
the struct-for, the demoted restriction and the prolongation: the bit is
set and the block is left unwritten, where the mode switched off writes it
and reports nothing."""
import numpy as np
import pytest

from paper_2012_08141_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEMOTED = 4     # status bit of a demoted write that found its block inactive


def say(*a):
    print(*a, flush=True)


@pytest.fixture(autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2012_08141_amd import engine as E, _lib as L
    E.reset()
    yield
    torch.cuda.synchronize()
    E.set_option(L.AT_OPTION_VERIFY_DEMOTED, 0)
    E.reset()


def verify(on):
    from paper_2012_08141_amd import engine as E, _lib as L
    E.set_option(L.AT_OPTION_VERIFY_DEMOTED, 1 if on else 0)
    assert E.get_option(L.AT_OPTION_VERIFY_DEMOTED) == (1 if on else 0)


def close(got, exp, what):
    got, exp = np.asarray(got, np.float64), np.asarray(exp, np.float64)
    scale = np.abs(exp).max() if exp.size else 0.0
    bad = np.abs(got - exp) > 1e-6 * np.maximum(np.abs(exp), 1e-3 * scale)
    assert not bad.any(), "%s: %d of %d differ (max abs diff %g)" % (
        what, int(bad.sum()), bad.size, float(np.abs(got - exp).max()))


def root_view(g):
    """The pointer root as an int32 tensor on the device (cell -> slot)."""
    _, _, _, root = g._views()
    return g._slice(root, g.ncells * 4).view(torch.int32)


def test_option_values():
    from paper_2012_08141_amd import engine as E, _lib as L
    with pytest.raises(L.AtError):
        E.set_option(L.AT_OPTION_VERIFY_DEMOTED, 2)
    assert E.get_option(L.AT_OPTION_VERIFY_DEMOTED) == 0


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
def test_correct_plans_flag_nothing(root):
    """Band Jacobi (two windows, the second serving the cached list) and two
    multigrid V-cycles, optimized, with the mode on and off: no grid's bit 2
    is set and the results agree."""
    from paper_2012_08141_amd import engine as E, programs as PR
    say("verify: correct plans", root)
    w = I.band(0, n=128, root_kind=root)
    out = {}
    for on in (False, True):
        E.reset()
        verify(on)
        g = PR.load_workload(w, PR.JACOBI, 3)
        for _ in range(2):
            st = E.run_sequence(sum((PR.jacobi_step(g) for _ in range(3)), []), E.OPT_ALL)
            assert st["activations_demoted"] >= 1
        lv = PR.mg_levels(w, 3)
        for _ in range(2):
            E.run_sequence(PR.mg_vcycle(lv), E.OPT_ALL)
        torch.cuda.synchronize()
        assert g.device_status() == 0, on
        for l, c in enumerate(lv):
            assert c.device_status() == 0, (on, l)
        out[on] = (g.read_blocks(PR.JACOBI["x"], w.cells), lv[0].read_blocks(PR.MG["x"], w.cells),
                   [c.active_cells() for c in lv])
    close(out[True][0], out[False][0], "jacobi x")
    close(out[True][1], out[False][1], "multigrid x")
    for l in range(3):
        assert np.array_equal(out[True][2][l], out[False][2][l]), l


def test_struct_for_over_a_stale_list():
    """A listed block set inactive in the root without telling the engine:
    the second window's list generation is removed, and the demoted Jacobi
    over the stale list reaches the block."""
    from paper_2012_08141_amd import engine as E, programs as PR
    say("verify: stale struct-for list")
    w = I.random_blocks(5, 64, 0.3, "pointer", channels=("x", "b"))
    res = {}
    for on in (False, True):
        E.reset()
        verify(on)
        g = PR.load_workload(w, {"x": PR.JACOBI["x"], "b": PR.JACOBI["b"]}, 3)
        E.run_sequence(PR.jacobi_step(g), E.OPT_ALL)
        torch.cuda.synchronize()
        rec = g.list_records()
        cell, slot = int(rec[len(rec) // 2, 0]), int(rec[len(rec) // 2, 1])
        before = g.channel(PR.JACOBI["xn"])[slot].cpu().numpy().copy()
        root_view(g)[cell] = -1
        torch.cuda.synchronize()
        st = E.run_sequence(PR.jacobi_step(g), E.OPT_ALL)
        torch.cuda.synchronize()
        assert st["listgens_removed"] >= 1
        bits = g.device_status(clear=True)
        after = g.channel(PR.JACOBI["xn"])[slot].cpu().numpy()
        others = rec[rec[:, 0] != cell, 1]
        res[on] = (bits, np.array_equal(after, before), g.channel(PR.JACOBI["x"])[
                   torch.as_tensor(others, device="cuda").long()].cpu().numpy())
        root_view(g)[cell] = slot
        torch.cuda.synchronize()
    assert res[True][0] == DEMOTED and res[True][1], "verify on: flagged and the block left unwritten"
    assert res[False][0] == 0 and not res[False][1], "verify off: the stale block is written, nothing flagged"
    close(res[True][2], res[False][2], "the other blocks")


def test_demoted_transfers_check_their_blocks():
    """Multigrid transfers: a coarse parent cleared after the first
    restriction trips the demoted second restriction; a fine block cleared
    behind a removed list generation trips the prolongation."""
    from paper_2012_08141_amd import engine as E
    from paper_2012_08141_amd.grid import SparseGrid
    say("verify: demoted transfers")
    n = 64
    wf = I.random_blocks(7, n, 0.4, "pointer", channels=("a", "b"))
    for on in (False, True):
        E.reset()
        verify(on)
        f = SparseGrid(n, 3, "pointer", wf.nblocks)
        f.load_blocks(0, wf.cells, wf.channels["a"])
        f.load_blocks(1, wf.cells, wf.channels["b"])
        c = SparseGrid(n // 2, 3, "pointer", (n // 16) ** 3)
        E.run_sequence([E.listgen(f), E.restrict(f, c, 0, 1, 0.5)], E.OPT_ALL)
        torch.cuda.synchronize()
        ccells = c.active_cells()
        assert len(ccells) > 2
        cc = int(ccells[len(ccells) // 2])
        cslot = int(root_view(c)[cc].item())
        root_view(c)[cc] = -1
        torch.cuda.synchronize()
        st = E.run_sequence([E.listgen(f), E.restrict(f, c, 0, 1, 0.5)], E.OPT_ALL)
        torch.cuda.synchronize()
        assert st["activations_demoted"] >= 1
        bits = c.device_status(clear=True)
        if on:
            assert bits == DEMOTED, "the demoted restriction found an inactive parent"
        else:
            assert bits == 0
        root_view(c)[cc] = cslot
        # prolongation over a stale fine list
        rec = f.list_records()
        fc, fs = int(rec[1, 0]), int(rec[1, 1])
        before = f.channel(2)[fs].cpu().numpy().copy()
        root_view(f)[fc] = -1
        torch.cuda.synchronize()
        st = E.run_sequence([E.listgen(f), E.prolong(c, f, 1, 2)], E.OPT_ALL)
        torch.cuda.synchronize()
        assert st["listgens_removed"] >= 1
        bits = f.device_status(clear=True)
        unchanged = np.array_equal(f.channel(2)[fs].cpu().numpy(), before)
        if on:
            assert bits == DEMOTED and unchanged
        else:
            assert bits == 0
        root_view(f)[fc] = fs
        torch.cuda.synchronize()
