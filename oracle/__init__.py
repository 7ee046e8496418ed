"""CPU oracle for the sparse-grid hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  It never imports the product
package and the product never imports it.

Two independent implementations live here:

* ``OracleGrid`` -- ctypes wrapper over ``oracle.c``: a plain single-threaded
  C implementation of the sparse-grid semantics (root table + block pool,
  activation on write with zero fill, ascending list generation, struct-fors
  over the list, 7-point stencils, PIC particle transfers, the diffusion step
  and its hand-derived adjoint, MLS-MPM transfers with fixed-corotated
  stress), built for fp32 and for fp64.
* ``oracle.dense`` -- a NumPy dense-array implementation for tiny grids, used
  to pin the C oracle's sparse machinery.

What pins each function (tests/test_oracle_pins.py):

* activate, listgen -- brute-force mask scans, idempotence, the union
  invariant, whole-block activation (Fig. 3), the restriction pattern.
* lap_update, axpy, jacobi, copy, fill, inc, diffuse, diffuse_adj -- the
  dense implementation (bit-exact in fp32 and fp64), plus closed forms:
  inactive-neighbour counts, exactness on polynomials of degree <= 2,
  Jacobi eigenmodes, a direct Poisson solve, linear-field diffusion fluxes.
* diffuse_adj -- dot-product identities in a and k, and central finite
  differences of a multi-step loss.
* maccormack -- the dense implementation (bit-exact), zero velocity (q back),
  exactness on affine fields (no correction), and the clamp bounds.
* advect_sl -- the dense implementation (bit-exact), zero velocity (a copy),
  whole-voxel velocities (exact shifts with zeros entering), reproduction of
  linear fields, and one block's values carried into a neighbour block.
* restrict_to, prolong_from -- the dense implementation (bit-exact), the
  parent-block active set, constants, and the adjoint identity between the
  two transfers.
* p2g, normalise, g2p -- B-spline moment identities, mass and momentum
  conservation, the on-node (1/8, 3/4, 1/8) stencil, affine reproduction by
  the gather, and the dense implementation; with one uniform particle
  velocity u, normalise gives u wherever there is mass and the gather
  returns u; normalise inverts momentum formation exactly on powers of two
  (tests/test_oracle_laws.py).
* advect (particles) -- exact dyadic displacements, +dt then -dt restoring x,
  and a uniform-velocity PIC program moving every particle by T dt u.
* inc -- exact on integer fields, +c then -c restoring them, only the listed
  blocks of its channel touched.

* polar, fcr_stress, mpm_p2g, mpm_grid, mpm_g2p (MLS-MPM, Section 8.3) --
  rotations from the polar decomposition against numpy's SVD; stress zero on
  rotations, symmetric, frame indifferent and in closed form on uniform
  scalings; affine fields reproduced by the gather (v and C); mass, momentum
  and APIC angular momentum conserved by the scatter; free fall under
  gravity, the floor wall, and a uniformly stretched block at rest inside
  with its faces pulled inward (tests/test_oracle_mpm.py).

tests/test_oracle_laws.py and tests/test_oracle_mpm.py also compile copies
of oracle.c with planted mistakes and check that those pins fail on each.

Every function has at least one such pin; none is "parity unpinned".
"""
from __future__ import annotations

import contextlib
import ctypes
import os

import numpy as np

from . import build as _build

_LIBS = {}
_DTYPES = {"f32": np.float32, "f64": np.float64}
_CREAL = {"f32": ctypes.c_float, "f64": ctypes.c_double}


def _lib(prec: str):
    if prec in _LIBS:
        return _LIBS[prec]
    if not _build.built():
        _build.build()
    _LIBS[prec] = _load(_build.LIBS[prec], prec)
    return _LIBS[prec]


def _load(path: str, prec: str):
    """Open one build of oracle.c and declare its signatures."""
    L = ctypes.CDLL(path)
    R = _CREAL[prec]
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int, ctypes.c_int64
    sig = {
        "og_create": (P, [i32, i32]),
        "og_destroy": (None, [P]),
        "og_root_edge": (i32, [P]),
        "og_num_slots": (i64, [P]),
        "og_is_active": (i32, [P, i32, i32, i32]),
        "og_activate": (i64, [P, P, i64, i32]),
        "og_listgen": (i64, [P]),
        "og_active_cells": (i64, [P, P]),
        "og_get_list": (i64, [P, P]),
        "og_set_list": (None, [P, P, i64]),
        "og_read": (R, [P, i32, i32, i32, i32]),
        "og_read_block": (None, [P, i32, ctypes.c_int32, P]),
        "og_write_block": (None, [P, i32, ctypes.c_int32, P]),
        "og_lap_update": (None, [P, i32, i32, R]),
        "og_axpy": (None, [P, i32, i32, R]),
        "og_jacobi": (None, [P, i32, i32, i32]),
        "og_copy": (None, [P, i32, i32]),
        "og_fill": (None, [P, i32, R]),
        "og_inc": (None, [P, i32, R]),
        "og_diffuse": (None, [P, i32, i32, i32, R]),
        "og_diffuse_adj": (None, [P, i32, i32, i32, i32, i32, R]),
        "og_advect": (None, [P, P, i64, R]),
        "og_p2g": (i64, [P, i32, i32, i32, P, P, P, i64, R]),
        "og_normalise": (None, [P, i32, i32, i32]),
        "og_restrict": (None, [P, P, i32, i32, R]),
        "og_advect_sl": (None, [P, i32, i32, i32, R, i32]),
        "og_maccormack": (None, [P, i32, i32, i32, i32, i32, R, i32]),
        "og_prolong": (None, [P, P, i32, i32]),
        "og_g2p": (None, [P, i32, P, P, i64, R]),
        "og_bspline": (i32, [R, P]),
        "og_polar": (i32, [P, P]),
        "og_fcr_stress": (None, [P, R, R, P]),
        "og_mpm_p2g": (i64, [P, i32, i32, i32, P, P, P, P, i64, R, R, R, R, R, R]),
        "og_mpm_grid": (None, [P, i32, i32, i32, R, R, i32]),
        "og_mpm_g2p": (None, [P, i32, P, P, P, i64, R]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


@contextlib.contextmanager
def substituted(path: str, prec: str):
    """Within the block, grids and functions of precision ``prec`` use the
    oracle build at ``path`` (a copy of oracle.c with a planted mistake,
    compiled by a test, so the test can show that its pin catches it)."""
    prev = _lib(prec)
    _LIBS[prec] = _load(path, prec)
    try:
        yield
    finally:
        _LIBS[prec] = prev


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def bspline_weights(X: float, precision: str = "f32"):
    """(base, [w0, w1, w2]) of the quadratic B-spline at grid coordinate X."""
    dt = _DTYPES[precision]
    w = np.zeros(3, dtype=dt)
    base = _lib(precision).og_bspline(dt(X), _ptr(w))
    return base, w


def advect(x: np.ndarray, v: np.ndarray, dt: float, precision: str = "f32") -> np.ndarray:
    """Return x + dt * v (SoA [3, np]) computed by the oracle."""
    d = _DTYPES[precision]
    xo = np.ascontiguousarray(x, dtype=d).copy()
    vv = np.ascontiguousarray(v, dtype=d)
    _lib(precision).og_advect(_ptr(xo), _ptr(vv), xo.shape[1], d(dt))
    return xo


def polar(F, precision: str = "f64"):
    """(R, iterations) of the polar decomposition F = R S of one 3x3 matrix
    (iterations -1 when det F <= 0)."""
    d = _DTYPES[precision]
    f = np.ascontiguousarray(np.asarray(F, dtype=d).reshape(9))
    r = np.zeros(9, dtype=d)
    it = _lib(precision).og_polar(_ptr(f), _ptr(r))
    return r.reshape(3, 3), int(it)


def fcr_stress(F, mu: float, lam: float, precision: str = "f64"):
    """Kirchhoff stress of the fixed-corotated model at one 3x3 F."""
    d = _DTYPES[precision]
    f = np.ascontiguousarray(np.asarray(F, dtype=d).reshape(9))
    t = np.zeros(9, dtype=d)
    _lib(precision).og_fcr_stress(_ptr(f), d(mu), d(lam), _ptr(t))
    return t.reshape(3, 3)


class OracleGrid:
    """A sparse grid of ``n^3`` voxels (root of (n/8)^3 cells over 8^3 blocks)
    with ``channels`` value channels, in fp32 or fp64."""

    def __init__(self, n: int, channels: int, precision: str = "f32"):
        self.n, self.channels, self.precision = n, channels, precision
        self.R = n // 8
        self.dtype = _DTYPES[precision]
        self._L = _lib(precision)
        self._g = self._L.og_create(n, channels)
        if not self._g:
            raise ValueError("invalid oracle grid shape")

    def __del__(self):
        g, self._g = getattr(self, "_g", None), None
        if g:
            self._L.og_destroy(g)

    # -- activation, lists, masks -------------------------------------------
    def activate(self, coords, kind: str = "block") -> int:
        c = np.ascontiguousarray(np.asarray(coords, dtype=np.int32).reshape(-1, 3))
        return int(self._L.og_activate(self._g, _ptr(c), c.shape[0], 0 if kind == "voxel" else 1))

    def listgen(self) -> int:
        return int(self._L.og_listgen(self._g))

    def list(self) -> np.ndarray:
        out = np.zeros(self.R ** 3, dtype=np.int32)
        cnt = self._L.og_get_list(self._g, _ptr(out))
        return out[:cnt].copy()

    def set_list(self, cells) -> None:
        """Replace the list state (a struct-for then visits exactly these blocks)."""
        c = np.ascontiguousarray(np.asarray(cells, dtype=np.int32))
        self._L.og_set_list(self._g, _ptr(c), c.shape[0])

    def active_cells(self) -> np.ndarray:
        out = np.zeros(self.R ** 3, dtype=np.int32)
        cnt = self._L.og_active_cells(self._g, _ptr(out))
        return out[:cnt].copy()

    def is_active(self, bi: int, bj: int, bk: int) -> bool:
        return bool(self._L.og_is_active(self._g, bi, bj, bk))

    @property
    def num_slots(self) -> int:
        return int(self._L.og_num_slots(self._g))

    # -- values -----------------------------------------------------------------
    def read(self, ch: int, i: int, j: int, k: int) -> float:
        return float(self._L.og_read(self._g, ch, i, j, k))

    def read_blocks(self, ch: int, cells) -> np.ndarray:
        cells = np.asarray(cells, dtype=np.int32)
        out = np.zeros((cells.shape[0], 512), dtype=self.dtype)
        buf = np.zeros(512, dtype=self.dtype)
        for t, c in enumerate(cells):
            self._L.og_read_block(self._g, ch, int(c), _ptr(buf))
            out[t] = buf
        return out

    def write_blocks(self, ch: int, cells, values) -> None:
        cells = np.asarray(cells, dtype=np.int32)
        vals = np.ascontiguousarray(values, dtype=self.dtype).reshape(cells.shape[0], 512)
        for t, c in enumerate(cells):
            row = np.ascontiguousarray(vals[t])
            self._L.og_write_block(self._g, ch, int(c), _ptr(row))

    def to_dense(self, ch: int) -> np.ndarray:
        """Dense (n, n, n) copy of channel ``ch`` (zeros where inactive)."""
        out = np.zeros((self.n,) * 3, dtype=self.dtype)
        cells = self.active_cells()
        vals = self.read_blocks(ch, cells)
        R = self.R
        for t, c in enumerate(cells):
            bi, bj, bk = c // (R * R), (c // R) % R, c % R
            out[bi * 8:bi * 8 + 8, bj * 8:bj * 8 + 8, bk * 8:bk * 8 + 8] = vals[t].reshape(8, 8, 8)
        return out

    # -- struct-for tasks over the current list ------------------------------
    def lap_update(self, ch_a: int, ch_out: int, coef: float = 0.1):
        self._L.og_lap_update(self._g, ch_a, ch_out, self.dtype(coef))

    def axpy(self, ch_y: int, ch_x: int, alpha: float):
        self._L.og_axpy(self._g, ch_y, ch_x, self.dtype(alpha))

    def jacobi(self, ch_x: int, ch_b: int, ch_xn: int):
        self._L.og_jacobi(self._g, ch_x, ch_b, ch_xn)

    def copy(self, ch_dst: int, ch_src: int):
        self._L.og_copy(self._g, ch_dst, ch_src)

    def fill(self, ch: int, value: float):
        self._L.og_fill(self._g, ch, self.dtype(value))

    def inc(self, ch: int, value: float):
        self._L.og_inc(self._g, ch, self.dtype(value))

    def diffuse(self, ch_a: int, ch_k: int, ch_out: int, dt: float):
        self._L.og_diffuse(self._g, ch_a, ch_k, ch_out, self.dtype(dt))

    def diffuse_adj(self, ch_a: int, ch_k: int, ch_lamn: int, ch_lam: int, ch_gk: int, dt: float):
        self._L.og_diffuse_adj(self._g, ch_a, ch_k, ch_lamn, ch_lam, ch_gk, self.dtype(dt))

    def advect_sl(self, ch_q: int, ch_v: int, ch_out: int, dt: float, rk3: bool = False):
        """out[I] = q at the back-traced point of I (Euler, or RK3), trilinear
        (v in ch_v .. ch_v + 2)."""
        self._L.og_advect_sl(self._g, ch_q, ch_v, ch_out, self.dtype(dt), 1 if rk3 else 0)

    def maccormack(self, ch_q: int, ch_v: int, ch_fwd: int, ch_bwd: int, ch_out: int, dt: float,
                   rk3: bool = False):
        """out = clamp(fwd + 0.5 (q - bwd)) to q's corner range at the forward
        back-traced point (Euler, or RK3)."""
        self._L.og_maccormack(self._g, ch_q, ch_v, ch_fwd, ch_bwd, ch_out, self.dtype(dt), 1 if rk3 else 0)

    # -- two-level transfers (struct-fors over this, the fine grid) -----------
    def restrict_to(self, coarse: "OracleGrid", ch_x: int, ch_y: int, w: float = 0.125):
        """coarse.y[I/2] += w * x[I] over this grid's list, activating coarse blocks."""
        if coarse.n * 2 != self.n or coarse.precision != self.precision:
            raise ValueError("coarse grid must have half the domain edge and the same precision")
        self._L.og_restrict(self._g, coarse._g, ch_x, ch_y, self.dtype(w))

    def prolong_from(self, coarse: "OracleGrid", ch_y: int, ch_x: int):
        """x[I] += coarse.y[I/2] over this grid's list."""
        if coarse.n * 2 != self.n or coarse.precision != self.precision:
            raise ValueError("coarse grid must have half the domain edge and the same precision")
        self._L.og_prolong(coarse._g, self._g, ch_y, ch_x)

    # -- particles ------------------------------------------------------------
    def p2g(self, ch_m: int, ch_mv: int, x, v, m, inv_dx: float, ch_abs: int = -1) -> int:
        d = self.dtype
        xx = np.ascontiguousarray(x, dtype=d)
        vv = np.ascontiguousarray(v, dtype=d)
        mm = np.ascontiguousarray(m, dtype=d)
        return int(self._L.og_p2g(self._g, ch_m, ch_mv, ch_abs, _ptr(xx), _ptr(vv), _ptr(mm),
                                  mm.shape[0], d(inv_dx)))

    def normalise(self, ch_m: int, ch_mv: int, ch_v: int):
        self._L.og_normalise(self._g, ch_m, ch_mv, ch_v)

    def g2p(self, ch_v: int, x, inv_dx: float) -> np.ndarray:
        d = self.dtype
        xx = np.ascontiguousarray(x, dtype=d)
        out = np.zeros_like(xx)
        self._L.og_g2p(self._g, ch_v, _ptr(xx), _ptr(out), xx.shape[1], d(inv_dx))
        return out

    # -- MLS-MPM (Section 8.3) --------------------------------------------------
    def mpm_p2g(self, ch_m: int, ch_mv: int, x, v, C, F, inv_dx: float, dt: float, mass: float, vol: float,
                mu: float, lam: float, ch_abs: int = -1):
        """Scatter of mass and APIC momentum with the fixed-corotated stress;
        returns (updated F [9, np], node writes skipped outside the domain)."""
        d = self.dtype
        xx = np.ascontiguousarray(x, dtype=d)
        vv = np.ascontiguousarray(v, dtype=d)
        cc = np.ascontiguousarray(C, dtype=d)
        ff = np.ascontiguousarray(F, dtype=d).copy()
        bad = self._L.og_mpm_p2g(self._g, ch_m, ch_mv, ch_abs, _ptr(xx), _ptr(vv), _ptr(cc), _ptr(ff),
                                 xx.shape[1], d(inv_dx), d(dt), d(mass), d(vol), d(mu), d(lam))
        return ff, int(bad)

    def mpm_grid(self, ch_m: int, ch_mv: int, ch_v: int, dt: float, gravity: float, bound: int):
        self._L.og_mpm_grid(self._g, ch_m, ch_mv, ch_v, self.dtype(dt), self.dtype(gravity), bound)

    def mpm_g2p(self, ch_v: int, x, inv_dx: float):
        """(v [3, np], C [9, np]) gathered at the particles."""
        d = self.dtype
        xx = np.ascontiguousarray(x, dtype=d)
        v = np.zeros_like(xx)
        C = np.zeros((9, xx.shape[1]), dtype=d)
        self._L.og_mpm_g2p(self._g, ch_v, _ptr(xx), _ptr(v), _ptr(C), xx.shape[1], d(inv_dx))
        return v, C

    # -- convenience ----------------------------------------------------------
    def load(self, blocks, channel_values: dict, channel_index: dict) -> None:
        """Activate ``blocks`` (block coordinates, in order) and store the
        given per-block values into the named channels."""
        self.activate(blocks, "block")
        R = self.R
        b = np.asarray(blocks, dtype=np.int64)
        cells = ((b[:, 0] * R + b[:, 1]) * R + b[:, 2]).astype(np.int32)
        for name, vals in channel_values.items():
            self.write_blocks(channel_index[name], cells, vals)
