"""The scatter that allocates nothing (at_p2g_static), through the C ABI,
against the binned at_p2g on the same particles and against the oracle
(MI355X only).

Two calls in a row share the device's static workspace, the second with
fewer particles on a smaller domain (and no particle whose centre node lies
outside it, where the first had such outliers), so what the first call
leaves behind must not leak into the second.  Bars: active sets bit-exact;
mass and momentum within the scatter's summation bound
|g - o| <= 1e-5 * A (A = per node and channel sum of |term|, from the
oracle), against the oracle and against the binned at_p2g.
"""
import ctypes

import numpy as np
import pytest

from oracle import programs as OP
from paper_2012_08141_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2012_08141_amd import engine as E
    E.reset()
    yield
    torch.cuda.synchronize()


def _scatter(entry, g, x, v, m, np_, n, act):
    from paper_2012_08141_amd import _lib as L
    ch = (ctypes.c_int32 * 2)(0, 1)
    L.check(getattr(L.lib(), entry)(g.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                    ctypes.c_void_p(m.data_ptr()), np_, 1.0 / n, ch, act,
                                    torch.cuda.current_stream().cuda_stream))


def _channels(g, cells):
    return [g.read_blocks(q, cells).astype(np.float64) for q in range(4)]


@pytest.mark.parametrize("root", ["pointer", "bitmask"])
def test_static_scatter_matches_binned_scatter_twice(root):
    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd.grid import SparseGrid
    cases = [(64, 60000, -0.03, 1.03, 7, L.AT_ACT_PER_NODE), (32, 9000, 0.1, 0.8, 8, L.AT_ACT_PER_BLOCK)]
    for n, np_, lo, hi, seed, act in cases:
        say("p2g_static", root, n, np_, lo, hi, "act", act)
        p = I.random_particles(seed, n, np_, lo, hi, root)
        ref = OP.p2g_once(n, None, p.x, p.v, p.m, "f32")
        cap = (n // 8) ** 3 if root == "pointer" else 0
        # the static scatter bins even on a grid without a workspace of its own
        gs = SparseGrid(n, 4, root, cap, particle_capacity=0)
        gb = SparseGrid(n, 4, root, cap, particle_capacity=np_)
        x, v, m = (torch.as_tensor(a, device="cuda").contiguous() for a in (p.x, p.v, p.m))
        _scatter("at_p2g_static", gs, x, v, m, np_, n, act)
        _scatter("at_p2g", gb, x, v, m, np_, n, act)
        torch.cuda.synchronize()
        cells = ref["cells"]
        assert np.array_equal(gs.active_cells(), cells)
        assert np.array_equal(gb.active_cells(), cells)
        assert gs.device_status() == 0 and gb.device_status() == 0
        got, base = _channels(gs, cells), _channels(gb, cells)
        exp = [ref["m"]] + ref["mv"]
        for q in range(4):
            A = ref["abs"][q].astype(np.float64)
            e_or = np.abs(got[q] - exp[q])
            e_bn = np.abs(got[q] - base[q])
            assert np.all(e_or <= 1e-5 * A + 1e-30), ("oracle", q, float((e_or / np.maximum(A, 1e-30)).max()))
            assert np.all(e_bn <= 1e-5 * A + 1e-30), ("binned", q, float((e_bn / np.maximum(A, 1e-30)).max()))
        if lo > 0 and hi < 1:
            assert abs(got[0].sum() - np_) < 1e-3 * np_


def test_static_scatter_rejects_sizes_beyond_its_limits():
    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd.grid import SparseGrid
    say("p2g_static limits")
    ch = (ctypes.c_int32 * 2)(0, 1)
    lib = L.lib()
    s = torch.cuda.current_stream().cuda_stream
    g = SparseGrid(32, 4, "pointer", 64)
    x = torch.zeros(3, device="cuda")
    big = L.AT_STATIC_MAX_PARTICLES + 1
    assert lib.at_p2g_static(g.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                             ctypes.c_void_p(x.data_ptr()), big, 1.0 / 32, ch, 0, s) == L.AT_E_INVALID
    assert b"static workspace" in lib.at_last_error()
    wide = SparseGrid(1024, 1, "pointer", 8)   # 128^3 root cells, beyond the limit
    assert lib.at_p2g_static(wide.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                             ctypes.c_void_p(x.data_ptr()), 1, 1.0 / 1024, ch, 0, s) == L.AT_E_INVALID
    torch.cuda.synchronize()
    assert len(g.active_cells()) == 0 and len(wide.active_cells()) == 0
