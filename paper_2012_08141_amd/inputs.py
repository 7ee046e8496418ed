"""Seeded synthetic workload generators.

This module only *produces inputs*: which leaf blocks start active, the
initial channel values, particle sets, request streams.  It holds none of the
method's arithmetic (no activation, list generation, stencil or transfer), so
both the CPU oracle and the HIP path can take their inputs from it.

Conventions shared by every workload
------------------------------------
* The domain is ``n^3`` voxels, stored as a root of ``R^3`` cells (``R = n/8``)
  over dense ``8^3`` leaf blocks (the two-level pointer/bitmasked-over-dense
  layout of the paper's Section 3, "Data-oriented programming").
* A block is named by its root coordinate ``(bi, bj, bk)``; its linear root
  index is ``(bi*R + bj)*R + bk``.  Inside a block, voxel ``(i, j, k)`` (local
  coordinates 0..7) sits at offset ``i*64 + j*8 + k`` (k fastest).
* ``blocks`` arrays are int32 ``[nb, 3]`` sorted by linear root index, and
  every per-block channel array is float32 ``[nb, 512]`` in the same order.
* RNG: NumPy PCG64 via ``default_rng([workload_id, seed, ...])``; the order of
  draws inside each generator is fixed so that a (workload, seed) pair always
  yields the same bits.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BLOCK = 8
BLOCK_VOXELS = BLOCK ** 3


@dataclass
class SparseWorkload:
    """A sparse grid workload: active blocks plus per-block channel values."""
    name: str
    n: int                       # domain edge in voxels
    root_kind: str               # "bitmask" or "pointer"
    blocks: np.ndarray           # int32 [nb, 3], ascending linear root index
    channels: dict = field(default_factory=dict)   # name -> float32 [nb, 512]
    params: dict = field(default_factory=dict)     # scalar parameters

    @property
    def R(self) -> int:
        return self.n // BLOCK

    @property
    def nblocks(self) -> int:
        return int(self.blocks.shape[0])

    @property
    def cells(self) -> np.ndarray:
        """Linear root index of every active block (int32 [nb])."""
        return block_cells(self.blocks, self.R)

    @property
    def active_voxels(self) -> int:
        return self.nblocks * BLOCK_VOXELS


@dataclass
class ParticleWorkload:
    """Particles in a sparse grid (SoA float32 arrays)."""
    name: str
    n: int
    root_kind: str
    x: np.ndarray                # float32 [3, np]  positions in [0, 1)
    v: np.ndarray                # float32 [3, np]
    m: np.ndarray                # float32 [np]
    params: dict = field(default_factory=dict)

    @property
    def R(self) -> int:
        return self.n // BLOCK

    @property
    def nparticles(self) -> int:
        return int(self.m.shape[0])


def block_cells(blocks: np.ndarray, R: int) -> np.ndarray:
    b = np.asarray(blocks, dtype=np.int64)
    return ((b[:, 0] * R + b[:, 1]) * R + b[:, 2]).astype(np.int32)


def cells_to_blocks(cells: np.ndarray, R: int) -> np.ndarray:
    c = np.asarray(cells, dtype=np.int64)
    return np.stack([c // (R * R), (c // R) % R, c % R], axis=1).astype(np.int32)


def _block_centres(R: int) -> np.ndarray:
    """Unit-cube centres of all R^3 root cells, in linear-index order."""
    g = (np.arange(R, dtype=np.float64) + 0.5) / R
    bi, bj, bk = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([bi.ravel(), bj.ravel(), bk.ravel()], axis=1)


def _select(mask_flat: np.ndarray, R: int) -> np.ndarray:
    cells = np.nonzero(mask_flat)[0].astype(np.int32)
    return cells_to_blocks(cells, R)


# ---------------------------------------------------------------------------
# Shell workload: 64^3 spherical shell, activate/listgen/lap_update/listgen/axpy.
# ---------------------------------------------------------------------------
def shell(seed: int = 0, n: int = 64, r_in: float = 0.30, r_out: float = 0.40,
          root_kind: str = "bitmask") -> SparseWorkload:
    """Blocks whose centre lies at distance [r_in, r_out] from a jittered
    centre (radius 0.35, thickness 0.1 by default); ``a`` ~ U(-1, 1)."""
    rng = np.random.default_rng([1, seed])
    centre = 0.5 + rng.uniform(-0.05, 0.05, 3)
    R = n // BLOCK
    d = np.linalg.norm(_block_centres(R) - centre, axis=1)
    blocks = _select((d >= r_in) & (d <= r_out), R)
    a = rng.uniform(-1.0, 1.0, (blocks.shape[0], BLOCK_VOXELS)).astype(np.float32)
    return SparseWorkload("shell%d" % n, n, root_kind, blocks,
                          {"a": a, "out": np.zeros_like(a)},
                          {"centre": centre, "steps": 10, "lap_coef": 0.1,
                           "axpy_alpha": 0.5})


# ---------------------------------------------------------------------------
# Narrow-band workload: 512^3 band around 4 random spheres, Jacobi iterations.
# ---------------------------------------------------------------------------
def band(seed: int = 0, n: int = 512, nspheres: int = 4, band_blocks: float = 1.5,
         root_kind: str = "bitmask") -> SparseWorkload:
    """Blocks with |sdf(block centre)| <= 1.5 blocks, sdf = min over spheres of
    (|p - c_s| - r_s); c_s ~ U(0.25, 0.75)^3, r_s ~ U(0.10, 0.20).
    ``b`` ~ N(0, 1) on active voxels, ``x`` = 0."""
    rng = np.random.default_rng([2, seed])
    centres = rng.uniform(0.25, 0.75, (nspheres, 3))
    radii = rng.uniform(0.10, 0.20, nspheres)
    R = n // BLOCK
    p = _block_centres(R)
    sdf = np.full(p.shape[0], np.inf)
    for s in range(nspheres):
        sdf = np.minimum(sdf, np.linalg.norm(p - centres[s], axis=1) - radii[s])
    blocks = _select(np.abs(sdf) <= band_blocks / R, R)
    b = rng.standard_normal((blocks.shape[0], BLOCK_VOXELS)).astype(np.float32)
    z = np.zeros_like(b)
    return SparseWorkload("band%d" % n, n, root_kind, blocks,
                          {"x": z, "xn": z.copy(), "b": b},
                          {"iters": 100, "centres": centres, "radii": radii})


# ---------------------------------------------------------------------------
# Particle workload: 2M particles in 3 random boxes in a 256^3 grid.
# ---------------------------------------------------------------------------
def particles(seed: int = 0, n: int = 256, nparticles: int = 2_000_000,
              nboxes: int = 3, root_kind: str = "pointer") -> ParticleWorkload:
    """Box sides ~ U(0.10, 0.30)^3, lower corner ~ U(0.05, 0.95 - side);
    particles split over boxes multinomially by volume, uniform inside;
    mass 1, velocity ~ N(0, 0.1^2)^3, dt = 1e-3, dx = 1/n."""
    rng = np.random.default_rng([3, seed])
    side = rng.uniform(0.10, 0.30, (nboxes, 3))
    lo = rng.uniform(0.05, 0.95 - side)
    vol = side.prod(axis=1)
    counts = rng.multinomial(nparticles, vol / vol.sum())
    xs = []
    for bx in range(nboxes):
        xs.append(lo[bx] + side[bx] * rng.uniform(0.0, 1.0, (counts[bx], 3)))
    x = np.concatenate(xs, axis=0).astype(np.float32)
    v = rng.normal(0.0, 0.1, (nparticles, 3)).astype(np.float32)
    m = np.ones(nparticles, dtype=np.float32)
    return ParticleWorkload("particles%d" % n, n, root_kind,
                            np.ascontiguousarray(x.T), np.ascontiguousarray(v.T), m,
                            {"dt": 1e-3, "dx": 1.0 / n, "steps": 20,
                             "boxes_lo": lo, "boxes_side": side, "counts": counts})


# ---------------------------------------------------------------------------
# Request workload: a stream of independent 128^3 Jacobi requests.
# ---------------------------------------------------------------------------
def batch_request(seed: int, index: int, n: int = 128, lo: int = 32, hi: int = 4096,
                  root_kind: str = "pointer") -> SparseWorkload:
    """Request ``index`` of the stream: nb = round(exp(U(ln lo, ln hi))) blocks,
    the nb root cells closest to a sphere shell (| |c_b - c| - r |, ties by
    linear index), c ~ U(0.3, 0.7)^3, r ~ U(0.15, 0.35); ``b`` ~ N(0, 1)."""
    rng = np.random.default_rng([4, seed, index])
    R = n // BLOCK
    nb = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    nb = max(1, min(nb, R ** 3))
    c = rng.uniform(0.3, 0.7, 3)
    r = rng.uniform(0.15, 0.35)
    dist = np.abs(np.linalg.norm(_block_centres(R) - c, axis=1) - r)
    order = np.lexsort((np.arange(R ** 3), dist))   # by distance, then index
    cells = np.sort(order[:nb]).astype(np.int32)
    blocks = cells_to_blocks(cells, R)
    b = rng.standard_normal((nb, BLOCK_VOXELS)).astype(np.float32)
    z = np.zeros_like(b)
    return SparseWorkload("req%d" % index, n, root_kind, blocks,
                          {"x": z, "xn": z.copy(), "b": b}, {"iters": 50})


def poisson_arrivals(seed: int, count: int, rate_per_s: float) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson stream of ``count`` requests."""
    rng = np.random.default_rng([4, seed, 1 << 30])
    return np.cumsum(rng.exponential(1.0 / rate_per_s, count))


# ---------------------------------------------------------------------------
# Diffusion workload: 128^3 shell diffusion with a differentiable loss.
# ---------------------------------------------------------------------------
def diffusion(seed: int = 0, n: int = 128, r_in: float = 0.32, r_out: float = 0.38,
              root_kind: str = "bitmask") -> SparseWorkload:
    """Shell blocks (centre distance in [r_in, r_out] from a jittered centre);
    k ~ U(0.5, 1.5), a0 ~ N(0, 1), target ~ N(0, 1); dt = 0.1, 20 steps,
    checkpoints every 5 steps."""
    rng = np.random.default_rng([5, seed])
    centre = 0.5 + rng.uniform(-0.05, 0.05, 3)
    R = n // BLOCK
    d = np.linalg.norm(_block_centres(R) - centre, axis=1)
    blocks = _select((d >= r_in) & (d <= r_out), R)
    nb = blocks.shape[0]
    k = rng.uniform(0.5, 1.5, (nb, BLOCK_VOXELS)).astype(np.float32)
    a0 = rng.standard_normal((nb, BLOCK_VOXELS)).astype(np.float32)
    target = rng.standard_normal((nb, BLOCK_VOXELS)).astype(np.float32)
    return SparseWorkload("diffusion%d" % n, n, root_kind, blocks,
                          {"a": a0, "k": k, "target": target},
                          {"dt": 0.1, "steps": 20, "checkpoint_every": 5})


# ---------------------------------------------------------------------------
# Small random workloads for parity tests.
# ---------------------------------------------------------------------------
def random_blocks(seed: int, n: int, frac: float, root_kind: str = "bitmask",
                  channels=("a",), dist: str = "uniform") -> SparseWorkload:
    """Each root cell active with probability ``frac``; channel values
    U(-1, 1) (or N(0, 1) with ``dist='normal'``) on active blocks."""
    rng = np.random.default_rng([100, seed, n])
    R = n // BLOCK
    blocks = _select(rng.uniform(0.0, 1.0, R ** 3) < frac, R)
    ch = {}
    for name in channels:
        if dist == "normal":
            ch[name] = rng.standard_normal((blocks.shape[0], BLOCK_VOXELS)).astype(np.float32)
        else:
            ch[name] = rng.uniform(-1.0, 1.0, (blocks.shape[0], BLOCK_VOXELS)).astype(np.float32)
    return SparseWorkload("random%d" % n, n, root_kind, blocks, ch, {"frac": frac})


def random_particles(seed: int, n: int, nparticles: int, lo: float = 0.1, hi: float = 0.9,
                     root_kind: str = "pointer") -> ParticleWorkload:
    """Particles uniform in [lo, hi)^3 with N(0, 0.1^2) velocities and mass 1."""
    rng = np.random.default_rng([101, seed, n, nparticles])
    x = rng.uniform(lo, hi, (3, nparticles)).astype(np.float32)
    v = rng.normal(0.0, 0.1, (3, nparticles)).astype(np.float32)
    m = np.ones(nparticles, dtype=np.float32)
    return ParticleWorkload("randp%d" % n, n, root_kind, x, v, m,
                            {"dt": 1e-3, "dx": 1.0 / n, "steps": 4})


# ---------------------------------------------------------------------------
# Advection workload: a tube domain (the paper's MacCormack benchmark setup:
# 256^3 cells, tube of inner radius 0.32 and outer radius 0.45) carrying three
# scalar fields and a swirling velocity field.
# ---------------------------------------------------------------------------
def tube(seed: int = 0, n: int = 256, r_in: float = 0.32, r_out: float = 0.45,
         root_kind: str = "bitmask") -> SparseWorkload:
    """Blocks whose centre lies at a distance in [r_in, r_out] from the axis
    x = y = 0.5; scalar fields ``q0``, ``q1``, ``q2`` ~ U(0, 1); velocity (in
    voxels per unit time) v = s * (-(y - 0.5), x - 0.5, w) * n at voxel
    centres, with s ~ U(2, 4) and w ~ U(-0.5, 0.5) from the seed, so that a
    step of dt = 1 / n moves a voxel by at most about 2 voxels."""
    rng = np.random.default_rng([6, seed])
    R = n // BLOCK
    c = _block_centres(R)
    d = np.hypot(c[:, 0] - 0.5, c[:, 1] - 0.5)
    blocks = _select((d >= r_in) & (d <= r_out), R)
    s = rng.uniform(2.0, 4.0)
    wz = rng.uniform(-0.5, 0.5)
    ch = {}
    for name in ("q0", "q1", "q2"):
        ch[name] = rng.uniform(0.0, 1.0, (blocks.shape[0], BLOCK_VOXELS)).astype(np.float32)
    li, lj, _ = np.meshgrid(np.arange(BLOCK), np.arange(BLOCK), np.arange(BLOCK), indexing="ij")
    x = ((blocks[:, 0:1] * BLOCK + li.reshape(1, -1)) + 0.5) / n
    y = ((blocks[:, 1:2] * BLOCK + lj.reshape(1, -1)) + 0.5) / n
    ch["v0"] = (s * -(y - 0.5) * n).astype(np.float32)
    ch["v1"] = (s * (x - 0.5) * n).astype(np.float32)
    ch["v2"] = np.full_like(ch["v0"], s * wz * n)
    return SparseWorkload("tube%d" % n, n, root_kind, blocks, ch, {"dt": 1.0 / n, "speed": s, "axial": wz})


# ---------------------------------------------------------------------------
# MLS-MPM workload: the falling cube of the paper's Section 8.3 benchmark
# (supplement Section 4.3).
# ---------------------------------------------------------------------------
@dataclass
class MpmWorkload:
    """Particles with APIC affine velocity C and deformation gradient F
    (SoA float32: x, v [3, np]; C, F [9, np], row-major 3x3 per particle)."""
    name: str
    n: int
    root_kind: str
    x: np.ndarray
    v: np.ndarray
    C: np.ndarray
    F: np.ndarray
    params: dict = field(default_factory=dict)

    @property
    def nparticles(self) -> int:
        return int(self.x.shape[1])


def mpm_cube(seed: int = 0, n: int = 256, side: float = 0.5, z_bottom: float = 49.0 / 1024.0,
             jitter: float = 0.25, root_kind: str = "bitmask", E: float = 2e4, nu: float = 0.4,
             rho: float = 1e3, gravity: float = 9.8, dt: float = 1e-4, v_sigma: float = 0.0,
             c_sigma: float = 0.0, f_sigma: float = 0.0) -> MpmWorkload:
    """A cube of edge ``side`` filled with a lattice of particles two per cell
    per axis (spacing dx/2, dx = 1/n), centred in x and y, the lowest layer's
    centres at ``z_bottom`` (z, axis 2, is up).  Each particle stands for a
    cube of edge dx/2 of density ``rho``: volume (dx/2)^3, mass rho times
    that.  Material: Young's modulus E and Poisson ratio nu, given as the
    Lame parameters mu = E / (2 (1 + nu)), lambda = E nu / ((1 + nu)(1 - 2 nu)).
    Walls 1/32 of the domain from each side (``bound`` = n/32 nodes).

    Seeded: each lattice point moves by U(-jitter, jitter) of the spacing per
    axis (so the B-spline weights take generic values) and the cube centre by
    U(-0.5, 0.5) cells in x and y.  The paper's cube starts at rest with F = I
    and C = 0; ``v_sigma``, ``c_sigma``, ``f_sigma`` > 0 draw v ~ N(0, v_sigma^2),
    C ~ N(0, c_sigma^2) and F = I + N(0, f_sigma^2) per entry instead (test
    states that exercise every term).  Order: blocks of 8^3 lattice points in
    lexicographic block order, lexicographic inside a block."""
    rng = np.random.default_rng([11, seed, n])
    h = 0.5 / n
    P = int(round(side / h))
    centre = 0.5 + rng.uniform(-0.5, 0.5, 2) / n
    lo = np.array([centre[0] - 0.5 * side + 0.5 * h, centre[1] - 0.5 * side + 0.5 * h, z_bottom])
    idx = np.arange(P)
    bsz = 8
    nb = (P + bsz - 1) // bsz
    order = []
    for bi in range(nb):
        for bj in range(nb):
            for bk in range(nb):
                ii, jj, kk = np.meshgrid(idx[bi * bsz:(bi + 1) * bsz], idx[bj * bsz:(bj + 1) * bsz],
                                         idx[bk * bsz:(bk + 1) * bsz], indexing="ij")
                order.append(np.stack([ii.ravel(), jj.ravel(), kk.ravel()]))
    lat = np.concatenate(order, axis=1).astype(np.float64)
    npart = lat.shape[1]
    x = lo[:, None] + h * lat + h * rng.uniform(-jitter, jitter, (3, npart))
    v = rng.normal(0.0, v_sigma, (3, npart)) if v_sigma > 0 else np.zeros((3, npart))
    C = rng.normal(0.0, c_sigma, (9, npart)) if c_sigma > 0 else np.zeros((9, npart))
    F = np.zeros((9, npart))
    F[0] = F[4] = F[8] = 1.0
    if f_sigma > 0:
        F = F + rng.normal(0.0, f_sigma, (9, npart))
    vol = h ** 3
    params = {"dt": dt, "dx": 1.0 / n, "mass": rho * vol, "vol": vol,
              "mu": E / (2.0 * (1.0 + nu)), "lam": E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)),
              "gravity": gravity, "bound": max(1, n // 32), "side": side, "lattice": P}
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return MpmWorkload("mpm_cube%d" % n, n, root_kind, f32(x), f32(v), f32(C), f32(F), params)
