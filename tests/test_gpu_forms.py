"""Every struct-for kernel form and launch shape against the oracle (MI355X
only).

The library has three struct-for kernel forms (pipelined with list
records, direct with list records, direct with neighbour lookups in the
root) and a persistent grid whose size can be overridden.  Each op runs on
a ragged grid (72^3: 9 root cells per axis) with the list current, so the
record forms are the ones that run, and with one wavefront handling many
blocks (8 workgroups) as well as the default shape.  Results must meet the
stencil bar against the oracle and be bit-identical across forms.
"""
import numpy as np
import pytest

import oracle
from paper_2012_08141_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OPS = {
    "lap_update": (1, [0, 1], 0.1, lambda o: o.lap_update(0, 1, 0.1)),
    "axpy": (2, [0, 1], 0.5, lambda o: o.axpy(0, 1, 0.5)),
    "jacobi": (3, [0, 2, 1], 0.0, lambda o: o.jacobi(0, 2, 1)),
    "copy": (4, [3, 0], 0.0, lambda o: o.copy(3, 0)),
    "fill": (5, [1, 3], -2.5, lambda o: (o.fill(1, -2.5), o.fill(3, -2.5))),
    "inc": (6, [2], 0.25, lambda o: o.inc(2, 0.25)),
    "diffuse": (7, [0, 2, 3], 0.1, lambda o: o.diffuse(0, 2, 3, 0.1)),
    "diffuse_adj": (8, [0, 2, 1, 3, 4], 0.1, lambda o: o.diffuse_adj(0, 2, 1, 3, 4, 0.1)),
}


def say(*a):
    print(*a, flush=True)


@pytest.fixture
def form_options():
    from paper_2012_08141_amd import _lib as L, engine as E
    yield lambda form, wgs: (E.set_option(L.AT_OPTION_STRUCT_FOR_KERNEL, form),
                             E.set_option(L.AT_OPTION_STRUCT_FOR_WORKGROUPS, wgs))
    E.set_option(L.AT_OPTION_STRUCT_FOR_KERNEL, 0)
    E.set_option(L.AT_OPTION_STRUCT_FOR_WORKGROUPS, 0)


def within(got, exp, what):
    exp = np.asarray(exp, np.float64)
    got = np.asarray(got, np.float64)
    scale = np.abs(exp).max() if exp.size else 0.0
    tol = 1e-6 * np.maximum(np.abs(exp), 1e-3 * scale)
    bad = np.abs(got - exp) > tol
    assert not bad.any(), "%s: %d beyond 1e-6 rel" % (what, int(bad.sum()))


def run_case(root, opname, check, frac=0.3, seed=21, first=None):
    from paper_2012_08141_amd.grid import SparseGrid
    op, ch, p, ocall = OPS[opname]
    n = 72
    w = I.random_blocks(seed, n, frac, root, channels=("c0", "c1", "c2", "c3", "c4"))
    if first is not None:       # keep only the first ``first`` blocks
        w = I.SparseWorkload(w.name, n, root, w.blocks[:first], {k: v[:first] for k, v in w.channels.items()},
                             w.params)
    w.channels["c2"] = np.abs(w.channels["c2"]) + 0.5
    names = {"c%d" % q: q for q in range(5)}
    g = SparseGrid(n, 5, root, (n // 8) ** 3 if root == "pointer" else 0)
    o = oracle.OracleGrid(n, 5)
    for name, vals in w.channels.items():
        g.load_blocks(names[name], w.cells, vals)
    o.load(w.blocks, w.channels, names)
    g.listgen()
    o.listgen()
    g.run_stencil(op, ch, p, bool(check))
    ocall(o)
    torch.cuda.synchronize()
    cells = o.active_cells()
    assert np.array_equal(g.active_cells(), cells)
    out = [g.read_blocks(q, cells) for q in range(5)]
    for q in range(5):
        within(out[q], o.read_blocks(q, cells), "%s ch%d" % (opname, q))
    return out


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
@pytest.mark.parametrize("wgs", [0, 8, 136])
@pytest.mark.parametrize("form", [0, 1, 2])
def test_every_op_every_form(form, wgs, root, form_options):
    say("forms: form", form, "workgroups", wgs, root)
    form_options(0, 0)
    base = {(k, c): run_case(root, k, c) for k in OPS for c in (0, 1)}
    form_options(form, wgs)
    for k in OPS:
        for c in (0, 1):
            got = run_case(root, k, c)
            for q in range(5):
                assert np.array_equal(got[q], base[(k, c)][q]), (k, c, q)


@pytest.mark.parametrize("form", [0, 1, 2])
def test_forms_on_empty_and_single_block(form, form_options):
    """An empty list (every kernel must exit at once) and a single block
    (every face neighbour absent)."""
    say("forms: empty and single, form", form)
    form_options(form, 0)
    for first in (0, 1):
        for k in OPS:
            run_case("pointer", k, 0, seed=22, first=first)
