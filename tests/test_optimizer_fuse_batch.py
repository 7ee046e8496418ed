"""The planner's batched fusion search gives exactly the plans of fusing one
pair at a time (Section 6.4's greedy order), on random two-grid programs and
on the workload programs, for every pass subset and with one and two
fusions per task and round (host-only planning handles)."""
import numpy as np
import pytest

from paper_2012_08141_amd import _lib as L
from paper_2012_08141_amd import engine as E
from paper_2012_08141_amd import inputs as I
from paper_2012_08141_amd import programs as PR
from paper_2012_08141_amd.grid import SparseGrid

import test_optimizer_oracle as T

FLAGS = [E.OPT_FUSE, E.OPT_ALL, E.OPT_AD | E.OPT_FUSE, E.OPT_LGR | E.OPT_FUSE | E.OPT_DSE]


class FakeParticles:
    _next = 0x5000000

    def __init__(self, shape):
        self.shape = shape
        self._p = FakeParticles._next
        FakeParticles._next += 1 << 24

    def data_ptr(self):
        return self._p


@pytest.fixture(autouse=True)
def options():
    yield
    E.set_option(L.AT_OPTION_FUSE_BATCH, 1)
    E.set_option(L.AT_OPTION_MAX_FUSE_PER_TASK, 1)
    E.set_option(L.AT_OPTION_PLAN_CACHE, 1)
    E.reset()


def plans(tasks, flags):
    out = []
    for batch in (1, 0):
        E.set_option(L.AT_OPTION_FUSE_BATCH, batch)
        E.reset()
        entries, st = E.plan_sequence(tasks, flags)
        out.append(([(e["kind"], e["members"], e["dropped"], e["keep"], e["check_activation"],
                      e["activation_mode"]) for e in entries], st["fusions"]))
    return out


@pytest.mark.parametrize("max_fuse", [1, 2])
def test_random_programs(max_fuse):
    E.set_option(L.AT_OPTION_PLAN_CACHE, 0)
    E.set_option(L.AT_OPTION_MAX_FUSE_PER_TASK, max_fuse)
    fused = 0
    for seed in range(60):
        rng = np.random.default_rng([93, seed])
        coord_sets = [I.random_blocks(seed + 3000 + j, T.N, 0.15).blocks for j in range(3)]
        fakes = [T.FakeArray(len(c)) for c in coord_sets]
        grids = [SparseGrid(T.N, T.NCH, "bitmask", device=None),
                 SparseGrid(T.N, T.NCH, "pointer", (T.N // 8) ** 3, device=None)]
        prog = T.random_program(rng, grids, coord_sets, int(rng.integers(8, 90)))
        tasks = T.to_tasks(prog, grids, fakes)
        for flags in FLAGS:
            batched, single = plans(tasks, flags)
            assert batched == single, (seed, flags)
            fused += batched[1]
    assert fused > 500


@pytest.mark.parametrize("max_fuse", [1, 2])
def test_workload_programs(max_fuse):
    E.set_option(L.AT_OPTION_PLAN_CACHE, 0)
    E.set_option(L.AT_OPTION_MAX_FUSE_PER_TASK, max_fuse)
    grids = [SparseGrid(256, 7, "pointer", 32768, device=None) for _ in range(2)]
    x, v, m = FakeParticles((3, 1000)), FakeParticles((3, 1000)), FakeParticles((1000,))
    part = sum((PR.particle_step(grids, t, x, v, m, 1e-3, 1 / 256) for t in range(30)), [])
    g = SparseGrid(512, 3, "bitmask", 0, device=None)
    band = sum((PR.jacobi_step(g) for _ in range(30)), [])
    for tasks in (part, band):
        for flags in FLAGS:
            batched, single = plans(tasks, flags)
            assert batched == single, flags
    assert plans(part, E.OPT_ALL)[0][1] >= 80
