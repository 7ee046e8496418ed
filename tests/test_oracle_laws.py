"""Law-based pins of the oracle's element-wise and particle-update functions.

The pins elsewhere check normalise, inc and the particle advection against the
dense implementation, which restates the same formulas.  These tests tie them
to facts that do not depend on how the formula is written:

* normalise (paper, Section 8.3, the PIC transfer: grid velocity is momentum
  over mass) -- with every particle carrying one velocity u, P2G followed by
  normalise gives v = u at every node holding mass, and the gather returns u;
  normalise inverts momentum formation exactly when m is a power of two;
* particle advection (x += dt v) -- exact displacements when dt v is a dyadic
  number, +dt then -dt restoring x, and a whole PIC program with one uniform
  velocity moving every particle by T dt u;
* inc (the x[i] += c task of Section 6.1) -- exact on integer-valued fields,
  +c then -c restoring them, only the listed blocks of the named channel touched.

Each pin is then run against copies of the oracle with a planted mistake
(swapped mass and momentum, a flipped sign, a wrong channel) and must fail.
"""
import numpy as np
import pytest

import oracle
from oracle import build as OB
from oracle import programs as P
from paper_2012_08141_amd import inputs as I

pytestmark = pytest.mark.usefixtures("oracle_built")

U = np.array([0.3125, -0.71875, 1.09375])      # a velocity with three distinct dyadic components


def _uniform_particles(seed, n, count):
    rng = np.random.default_rng([7001, seed, n])
    x = rng.uniform(0.25, 0.75, (3, count))
    v = np.repeat(U[:, None], count, axis=1)
    m = rng.uniform(0.5, 2.0, count)            # unequal masses: momentum must be mass-weighted
    return x, v, m


# ------------------------------------------------------------------- pins
def pin_uniform_velocity_p2g_normalise_g2p(prec="f64"):
    n = 32
    x, v, m = _uniform_particles(0, n, 2000)
    g = oracle.OracleGrid(n, 7, prec)
    g.p2g(0, 1, x, v, m, float(n))
    g.activate([[0, 0, 0]])                     # an active block that no particle reaches: m = 0
    g.listgen()
    g.normalise(0, 1, 4)
    mass = g.to_dense(0)
    tol = 1e-12 if prec == "f64" else 2e-6
    assert np.count_nonzero(mass > 0) > 1000
    for c in range(3):
        vc = g.to_dense(4 + c)
        assert np.max(np.abs(vc[mass > 0] - U[c])) <= tol * abs(U[c])
        assert np.all(vc[mass == 0] == 0)
    vp = g.g2p(4, x, float(n))
    assert np.max(np.abs(vp - U[:, None])) <= tol


def pin_normalise_inverts_momentum(prec="f64"):
    """With m = 2^e (e in -3..3) and mv = m * v, v is recovered exactly; m = 0
    gives 0; an active block that is not listed keeps its old v."""
    n = 24
    w = I.random_blocks(11, n, 0.5)
    rng = np.random.default_rng([7002, n])
    nb = w.blocks.shape[0]
    m = np.ldexp(1.0, rng.integers(-3, 4, (nb, 512)))
    m[rng.uniform(size=(nb, 512)) < 0.1] = 0.0
    v = rng.integers(-512, 513, (3, nb, 512)) / 64.0
    g = oracle.OracleGrid(n, 7, prec)
    g.load(w.blocks, {"m": m, "mv0": m * v[0], "mv1": m * v[1], "mv2": m * v[2]},
           {"m": 0, "mv0": 1, "mv1": 2, "mv2": 3})
    g.listgen()
    R = n // 8
    extra = [b for b in ([a, b, c] for a in range(R) for b in range(R) for c in range(R))
             if not g.is_active(*b)][:2]
    g.activate(extra)                                        # active after the list: not listed
    cells_x = np.array([(b[0] * R + b[1]) * R + b[2] for b in extra])
    for c in range(3):
        g.write_blocks(4 + c, cells_x, np.full((len(extra), 512), 7.0))
    g.normalise(0, 1, 4)
    cells = g.list()
    order = np.argsort(((w.blocks[:, 0] * R + w.blocks[:, 1]) * R + w.blocks[:, 2]))
    for c in range(3):
        got = g.read_blocks(4 + c, cells)
        exp = np.where(m > 0, v[c], 0.0)[order]
        assert np.array_equal(got, exp)
        assert np.all(g.read_blocks(4 + c, cells_x) == 7.0)


def pin_advect_exact_and_reversible(prec="f64"):
    rng = np.random.default_rng(7003)
    x = rng.integers(1024, 3072, (3, 5000)) / 4096.0          # 12 fractional bits
    v = rng.integers(-64, 65, (3, 5000)) / 64.0               # dt * v has 16 fractional bits
    v[0] += 0.25
    v[2] -= 0.5                                               # components differ on average
    dt = 2.0 ** -10
    fwd = oracle.advect(x, v, dt, prec)
    assert np.array_equal(fwd - x, dt * v)                    # exact: every value is dyadic
    back = oracle.advect(fwd, v, -dt, prec)
    assert np.array_equal(back, x)


def pin_uniform_velocity_program(prec="f64"):
    """A PIC program (advect, P2G, normalise, G2P over two alternating grids)
    whose particles all move with u keeps v = u and moves x by T dt u."""
    n = 32
    x, v, m = _uniform_particles(1, n, 1500)
    T, dt = 5, 2.0 ** -9
    r = P.particle_program(n, x, v, m, T, dt, prec)
    tol = 1e-12 if prec == "f64" else 2e-6
    assert np.max(np.abs(r["v"] - U[:, None])) <= tol
    assert np.max(np.abs(r["x"] - (x + T * dt * U[:, None]))) <= tol * T * dt + (1e-15 if prec == "f64" else 1e-6)


def pin_inc_exact_and_reversible(prec="f32"):
    n = 24
    w = I.random_blocks(12, n, 0.5)
    rng = np.random.default_rng([7004, n])
    nb = w.blocks.shape[0]
    f0 = rng.integers(-1000, 1001, (nb, 512)).astype(np.float64)
    f1 = rng.integers(-1000, 1001, (nb, 512)).astype(np.float64)
    g = oracle.OracleGrid(n, 2, prec)
    half = nb // 2
    g.load(w.blocks[:half], {"f0": f0[:half], "f1": f1[:half]}, {"f0": 0, "f1": 1})
    g.listgen()
    g.load(w.blocks[half:], {"f0": f0[half:], "f1": f1[half:]}, {"f0": 0, "f1": 1})   # active, not listed
    listed = g.list()
    allc = g.active_cells()
    before = {ch: g.read_blocks(ch, allc) for ch in (0, 1)}
    g.inc(1, 37.0)
    lmask = np.isin(allc, listed)
    after = {ch: g.read_blocks(ch, allc) for ch in (0, 1)}
    assert np.array_equal(after[0], before[0])
    assert np.array_equal(after[1][lmask], before[1][lmask] + 37.0)
    assert np.array_equal(after[1][~lmask], before[1][~lmask])
    g.inc(1, -37.0)
    assert np.array_equal(g.read_blocks(1, allc), before[1])


PINS = {
    "uniform_velocity": pin_uniform_velocity_p2g_normalise_g2p,
    "normalise_inverse": pin_normalise_inverts_momentum,
    "advect": pin_advect_exact_and_reversible,
    "program": pin_uniform_velocity_program,
    "inc": pin_inc_exact_and_reversible,
}


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("name", sorted(PINS))
def test_law(name, prec):
    PINS[name](prec)


# --------------------------------------------------------- planted mistakes
PLANTED = [
    ("normalise: mass over momentum",
     "rd(g, ch_mv + c, i, j, k) / mm", "mm / rd(g, ch_mv + c, i, j, k)",
     ["uniform_velocity", "normalise_inverse", "program"]),
    ("normalise: wrong output channel",
     "wr(g, ch_v + c, i, j, k, r);", "wr(g, ch_v + (c + 1) % 3, i, j, k, r);",
     ["uniform_velocity", "normalise_inverse", "program"]),
    ("p2g: mass and momentum channels swapped on store",
     "g->pool[ch][t] = (REAL)acc[q * len + t];", "g->pool[ch][t] = (REAL)acc[((q + 1) % 4) * len + t];",
     ["uniform_velocity", "program"]),
    ("p2g: momentum without the particle mass",
     "term[1 + c] = term[0] * vp[c];", "term[1 + c] = wt * vp[c];",
     ["uniform_velocity", "program"]),
    ("g2p: wrong velocity channel",
     "acc[c] = acc[c] + wt * rd(g, ch_v + c, i, j, k);", "acc[c] = acc[c] + wt * rd(g, ch_v + (c + 2) % 3, i, j, k);",
     ["uniform_velocity", "program"]),
    ("advect: sign flip",
     "x[c * np + p] + dt * v[c * np + p];", "x[c * np + p] - dt * v[c * np + p];",
     ["advect", "program"]),
    ("advect: wrong velocity component",
     "x[c * np + p] + dt * v[c * np + p];", "x[c * np + p] + dt * v[((c + 1) % 3) * np + p];",
     ["advect", "program"]),
    ("inc: sign flip",
     "rd(g, ch, i, j, k) + value", "rd(g, ch, i, j, k) - value",
     ["inc"]),
    ("inc: reads the wrong channel",
     "rd(g, ch, i, j, k) + value", "rd(g, 0, i, j, k) + value",
     ["inc"]),
]


@pytest.mark.parametrize("desc,old,new,pins", PLANTED, ids=[p[0] for p in PLANTED])
def test_pins_fail_on_planted_mistake(desc, old, new, pins, tmp_path):
    prec = "f64"
    path = OB.build_planted(old, new, str(tmp_path), prec)
    with oracle.substituted(path, prec):
        for name in pins:
            with pytest.raises(AssertionError):
                PINS[name](prec)
