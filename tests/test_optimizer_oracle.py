"""The optimizer never changes a program's result (Section 4: any
topological order of the state-flow graph behaves the same; Section 6: the
passes only remove redundant or dead work).

Random task programs over two grids are planned by the library's planner
(host only, planning handles), and the plan -- its surviving tasks in plan
order, dropped stores skipped -- is executed on the CPU oracle.  A fused
struct-for runs the way a fused kernel interleaves its members: block by
block (every member on one block, then the next block), once in ascending
and once in descending block order, so a fusion that lets one member see
another's writes across blocks changes the result.  The final state must
equal the program executed in order on the oracle, bit for bit, for every
subset of passes."""
import numpy as np
import pytest

import oracle
from paper_2012_08141_amd import engine as E
from paper_2012_08141_amd import inputs as I
from paper_2012_08141_amd.grid import SparseGrid

pytestmark = pytest.mark.usefixtures("oracle_built")

N, NCH = 32, 5


class FakeArray:
    _next = 0x9000000

    def __init__(self, n):
        self.shape = (n, 3)
        self._p = FakeArray._next
        FakeArray._next += 1 << 20

    def data_ptr(self):
        return self._p


def random_program(rng, grids, coord_sets, length):
    prog = []
    for _ in range(length):
        g = int(rng.integers(0, len(grids)))
        k = rng.choice(["listgen", "listgen", "fill", "inc", "axpy", "copy", "lap", "jacobi", "diffuse", "activate"])
        c = rng.permutation(NCH)
        if k == "fill":
            prog.append(("fill", g, sorted(c[:int(rng.integers(1, 3))].tolist()), float(rng.integers(-3, 4))))
        elif k == "inc":
            prog.append(("inc", g, int(c[0]), float(rng.integers(-2, 3)) * 0.5))
        elif k == "axpy":
            prog.append(("axpy", g, int(c[0]), int(c[1]), 0.5))
        elif k == "copy":
            prog.append(("copy", g, int(c[0]), int(c[1])))
        elif k == "lap":
            prog.append(("lap", g, int(c[0]), int(c[1]), 0.1))
        elif k == "jacobi":
            prog.append(("jacobi", g, int(c[0]), int(c[1]), int(c[2])))
        elif k == "diffuse":
            prog.append(("diffuse", g, int(c[0]), int(c[1]), int(c[2]), 0.1))
        elif k == "activate":
            prog.append(("activate", g, int(rng.integers(0, len(coord_sets)))))
        else:
            prog.append(("listgen", g))
    return prog


def to_tasks(prog, grids, fakes):
    out = []
    for t in prog:
        g = grids[t[1]]
        k = t[0]
        if k == "listgen":
            out.append(E.listgen(g))
        elif k == "fill":
            out.append(E.fill(g, t[2], t[3]))
        elif k == "inc":
            out.append(E.inc(g, t[2], t[3]))
        elif k == "axpy":
            out.append(E.axpy(g, t[2], t[3], t[4]))
        elif k == "copy":
            out.append(E.copy(g, t[2], t[3]))
        elif k == "lap":
            out.append(E.lap_update(g, t[2], t[3], t[4]))
        elif k == "jacobi":
            out.append(E.jacobi(g, t[2], t[3], t[4]))
        elif k == "diffuse":
            out.append(E.diffuse(g, t[2], t[3], t[4], t[5]))
        elif k == "activate":
            out.append(E.activate(g, fakes[t[2]]))
    return out


def run_plan(og, prog, coord_sets, entries, offset=0, reverse=False):
    """Run plan entries on oracle grids; fused struct-fors block by block."""
    for e in entries:
        pairs = [(offset + m, kp) for m, kp in zip(e["members"], e["keep"])]
        t0 = prog[pairs[0][0]]
        if len(pairs) > 1 and t0[0] not in ("listgen", "activate"):
            o = og[t0[1]]
            full = o.list()
            for cell in (full[::-1] if reverse else full):
                o.set_list([cell])
                execute(og, prog, coord_sets, pairs)
            o.set_list(full)
        else:
            execute(og, prog, coord_sets, pairs)


def execute(og, prog, coord_sets, order):
    """Run (task index, keep mask) pairs on oracle grids ``og``."""
    for ti, keep in order:
        t = prog[ti]
        o = og[t[1]]
        k = t[0]
        if k == "listgen":
            o.listgen()
        elif k == "fill":
            for q, ch in enumerate(t[2]):
                if (keep >> q) & 1:
                    o.fill(ch, t[3])
        elif k == "inc":
            o.inc(t[2], t[3])
        elif k == "axpy":
            o.axpy(t[2], t[3], t[4])
        elif k == "copy":
            o.copy(t[2], t[3])
        elif k == "lap":
            o.lap_update(t[2], t[3], t[4])
        elif k == "jacobi":
            o.jacobi(t[2], t[3], t[4])
        elif k == "diffuse":
            o.diffuse(t[2], t[3], t[4], t[5])
        elif k == "activate":
            o.activate(coord_sets[t[2]])


def fresh_oracles(w):
    og = []
    for wk in w:
        o = oracle.OracleGrid(N, NCH, "f32")
        o.load(wk.blocks, wk.channels, {"c%d" % q: q for q in range(NCH)})
        og.append(o)
    return og


def state(og):
    return [(o.active_cells(), [o.to_dense(q) for q in range(NCH)]) for o in og]


FLAGS = [E.OPT_ALL, E.OPT_LGR, E.OPT_AD, E.OPT_FUSE, E.OPT_DSE, E.OPT_AD | E.OPT_LGR,
         E.OPT_AD | E.OPT_DSE, E.OPT_AD | E.OPT_LGR | E.OPT_FUSE]


@pytest.mark.parametrize("seed", range(40))
def test_random_programs_plans_equal_in_order_execution(seed):
    rng = np.random.default_rng([77, seed])
    w = [I.random_blocks(seed, N, 0.35, "bitmask", channels=["c%d" % q for q in range(NCH)]),
         I.random_blocks(seed + 1000, N, 0.35, "pointer", channels=["c%d" % q for q in range(NCH)])]
    coord_sets = [I.random_blocks(seed + 2000 + j, N, 0.15).blocks for j in range(3)]
    fakes = [FakeArray(len(c)) for c in coord_sets]
    grids = [SparseGrid(N, NCH, "bitmask", device=None), SparseGrid(N, NCH, "pointer", (N // 8) ** 3, device=None)]
    prog = random_program(rng, grids, coord_sets, int(rng.integers(8, 40)))
    tasks = to_tasks(prog, grids, fakes)
    og = fresh_oracles(w)
    execute(og, prog, coord_sets, [(i, ~0) for i in range(len(prog))])
    ref = state(og)
    fused = 0
    for flags in FLAGS:
        E.reset()
        entries, st = E.plan_sequence(tasks, flags)
        fused += st["fusions"]
        for reverse in (False, True):
            og = fresh_oracles(w)
            run_plan(og, prog, coord_sets, entries, reverse=reverse)
            got = state(og)
            for gi in range(2):
                assert np.array_equal(got[gi][0], ref[gi][0]), (seed, flags, gi, "mask")
                for q in range(NCH):
                    assert np.array_equal(got[gi][1][q], ref[gi][1][q]), (seed, flags, reverse, gi, q, prog, entries)
    E.reset()


@pytest.mark.parametrize("seed", range(10))
def test_random_programs_with_preserved_owners(seed):
    """Windows after a setup window: list generation removal and activation
    demotion use the owners kept by partial garbage collection."""
    rng = np.random.default_rng([78, seed])
    w = [I.random_blocks(seed, N, 0.35, "bitmask", channels=["c%d" % q for q in range(NCH)]),
         I.random_blocks(seed + 1000, N, 0.35, "pointer", channels=["c%d" % q for q in range(NCH)])]
    coord_sets = [I.random_blocks(seed + 2000 + j, N, 0.15).blocks for j in range(3)]
    fakes = [FakeArray(len(c)) for c in coord_sets]
    grids = [SparseGrid(N, NCH, "bitmask", device=None), SparseGrid(N, NCH, "pointer", (N // 8) ** 3, device=None)]
    setup = random_program(rng, grids, coord_sets, 10) + [("listgen", 0), ("listgen", 1)]
    prog = random_program(rng, grids, coord_sets, 25)
    og = fresh_oracles(w)
    execute(og, setup + prog, coord_sets, [(i, ~0) for i in range(len(setup) + len(prog))])
    ref = state(og)
    E.reset()
    E.run_sequence(to_tasks(setup, grids, fakes), E.OPT_ALL)       # planning handles: state only
    entries, st = E.plan_sequence(to_tasks(prog, grids, fakes), E.OPT_ALL)
    # the setup window itself, as the engine planned it, then this plan
    E.reset()
    sent, _ = E.plan_sequence(to_tasks(setup, grids, fakes), E.OPT_ALL)
    og = fresh_oracles(w)
    run_plan(og, setup + prog, coord_sets, sent)
    run_plan(og, setup + prog, coord_sets, entries, offset=len(setup))
    got = state(og)
    for gi in range(2):
        assert np.array_equal(got[gi][0], ref[gi][0])
        for q in range(NCH):
            assert np.array_equal(got[gi][1][q], ref[gi][1][q]), (seed, gi, q)
    E.reset()
