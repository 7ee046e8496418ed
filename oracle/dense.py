"""Dense NumPy implementation of the sparse-grid semantics, for tiny grids.

TEST INFRASTRUCTURE ONLY.  This is a second, independent implementation
used to pin the C oracle's sparse machinery (root lookups, block/voxel
indexing, inactive-reads-zero, activation, list order): it stores every
channel as a full (n, n, n) array plus an (R, R, R) block mask, and expresses
each struct-for as whole-array operations restricted to the listed blocks.

Floating-point expressions are evaluated in the same operation order as the
C oracle, elementwise in the grid's dtype, so fp32 results agree bit for bit.
"""
from __future__ import annotations

import numpy as np

_FACES = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))


class DenseGrid:
    def __init__(self, n: int, channels: int, dtype=np.float32):
        assert n % 8 == 0
        self.n, self.R, self.dtype = n, n // 8, np.dtype(dtype)
        self.mask = np.zeros((self.R,) * 3, dtype=bool)
        self.vals = np.zeros((channels, n, n, n), dtype=self.dtype)
        self.list = np.zeros(0, dtype=np.int64)

    # -- structure ---------------------------------------------------------------
    def _activate_block(self, bi, bj, bk):
        if not (0 <= bi < self.R and 0 <= bj < self.R and 0 <= bk < self.R):
            return False
        if not self.mask[bi, bj, bk]:
            self.mask[bi, bj, bk] = True
            self.vals[:, bi * 8:bi * 8 + 8, bj * 8:bj * 8 + 8, bk * 8:bk * 8 + 8] = 0
        return True

    def activate(self, coords, kind="block"):
        for c in np.asarray(coords, dtype=np.int64).reshape(-1, 3):
            if kind == "voxel":
                if np.any(c < 0) or np.any(c >= self.n):
                    continue
                c = c // 8
            self._activate_block(*c)

    def listgen(self) -> int:
        self.list = np.flatnonzero(self.mask.ravel())
        return int(self.list.shape[0])

    def active_voxels(self) -> np.ndarray:
        return np.repeat(np.repeat(np.repeat(self.mask, 8, 0), 8, 1), 8, 2)

    def listed_voxels(self) -> np.ndarray:
        m = np.zeros(self.R ** 3, dtype=bool)
        m[self.list] = True
        m = m.reshape((self.R,) * 3)
        return np.repeat(np.repeat(np.repeat(m, 8, 0), 8, 1), 8, 2)

    def active_cells(self) -> np.ndarray:
        return np.flatnonzero(self.mask.ravel()).astype(np.int32)

    # -- reads -------------------------------------------------------------------
    def _field(self, ch):
        """Channel with inactive voxels read as 0."""
        return np.where(self.active_voxels(), self.vals[ch], self.dtype.type(0))

    def _shift(self, f, di, dj, dk):
        """g[i, j, k] = f[i+di, j+dj, k+dk], 0 outside the domain."""
        n = self.n
        p = np.zeros((n + 2,) * 3, dtype=f.dtype)
        p[1:-1, 1:-1, 1:-1] = f
        return p[1 + di:1 + di + n, 1 + dj:1 + dj + n, 1 + dk:1 + dk + n]

    def _nbsum(self, f):
        s = self._shift(f, -1, 0, 0) + self._shift(f, 1, 0, 0)
        s = s + self._shift(f, 0, -1, 0)
        s = s + self._shift(f, 0, 1, 0)
        s = s + self._shift(f, 0, 0, -1)
        s = s + self._shift(f, 0, 0, 1)
        return s

    def _store(self, ch, new):
        lv = self.listed_voxels()
        self.vals[ch] = np.where(lv, new.astype(self.dtype), self.vals[ch])

    # -- struct-for tasks ----------------------------------------------------------
    def lap_update(self, ch_a, ch_out, coef=0.1):
        T = self.dtype.type
        a = self._field(ch_a)
        s = self._nbsum(a)
        self._store(ch_out, a + T(coef) * (s - T(6) * a))

    def axpy(self, ch_y, ch_x, alpha):
        T = self.dtype.type
        self._store(ch_y, self._field(ch_y) + T(alpha) * self._field(ch_x))

    def jacobi(self, ch_x, ch_b, ch_xn):
        T = self.dtype.type
        sixth = T(1.0 / 6.0)
        s = self._nbsum(self._field(ch_x))
        self._store(ch_xn, (s + self._field(ch_b)) * sixth)

    def copy(self, ch_dst, ch_src):
        self._store(ch_dst, self._field(ch_src))

    def fill(self, ch, value):
        self._store(ch, np.full((self.n,) * 3, value, dtype=self.dtype))

    def inc(self, ch, value):
        self._store(ch, self._field(ch) + self.dtype.type(value))

    def _sample(self, f, p):
        """Trilinear sample of field f (n^3, zero outside) at points p (3, n, n, n),
        fixed corner order, each step rounded to the grid's dtype."""
        T = self.dtype.type
        n = self.n
        pad = np.zeros((n + 6,) * 3, dtype=self.dtype)
        pad[3:n + 3, 3:n + 3, 3:n + 3] = f
        base, w = [], []
        for d in range(3):
            pd = np.minimum(np.maximum(p[d], T(-2)), T(n + 1)).astype(self.dtype)
            bd = np.floor(pd).astype(self.dtype)
            fd = (pd - bd).astype(self.dtype)
            base.append(bd.astype(np.int64) + 3)
            w.append(((T(1) - fd).astype(self.dtype), fd))
        s = np.zeros((n, n, n), dtype=self.dtype)
        for a in (0, 1):
            for b in (0, 1):
                for c in (0, 1):
                    wt = ((w[0][a] * w[1][b]).astype(self.dtype) * w[2][c]).astype(self.dtype)
                    s = (s + wt * pad[base[0] + a, base[1] + b, base[2] + c]).astype(self.dtype)
        return s, base

    def _backtrace(self, ch_v, dt, rk3):
        T = self.dtype.type
        n = self.n
        I = np.indices((n, n, n)).astype(self.dtype)
        v1 = [self._field(ch_v + d) for d in range(3)]
        if not rk3:
            return [(I[d] - T(dt) * v1[d]).astype(self.dtype) for d in range(3)]
        h1, h2 = T(0.5) * T(dt), T(0.75) * T(dt)
        p1 = np.stack([(I[d] - h1 * v1[d]).astype(self.dtype) for d in range(3)])
        v2 = [self._sample(self._field(ch_v + d), p1)[0] for d in range(3)]
        p2 = np.stack([(I[d] - h2 * v2[d]).astype(self.dtype) for d in range(3)])
        v3 = [self._sample(self._field(ch_v + d), p2)[0] for d in range(3)]
        c1, c2, c3 = T(2.0 / 9.0), T(1.0 / 3.0), T(4.0 / 9.0)
        out = []
        for d in range(3):
            sv = (c1 * v1[d]).astype(self.dtype)
            sv = (sv + c2 * v2[d]).astype(self.dtype)
            sv = (sv + c3 * v3[d]).astype(self.dtype)
            out.append((I[d] - T(dt) * sv).astype(self.dtype))
        return out

    def advect_sl(self, ch_q, ch_v, ch_out, dt, rk3=False):
        """out[I] = q at the back-traced point of I (Euler or RK3), trilinear,
        with whole-array gathers into a zero-padded copy of q."""
        p = np.stack(self._backtrace(ch_v, dt, rk3))
        self._store(ch_out, self._sample(self._field(ch_q), p)[0])

    def maccormack(self, ch_q, ch_v, ch_fwd, ch_bwd, ch_out, dt, rk3=False):
        """clamp(fwd + 0.5 (q - bwd)) to the range of q over the 8 corners of the
        forward back-traced point, whole-array."""
        T = self.dtype.type
        n = self.n
        q = self._field(ch_q)
        p = np.stack(self._backtrace(ch_v, dt, rk3))
        _, base = self._sample(q, p)
        pad = np.zeros((n + 6,) * 3, dtype=self.dtype)
        pad[3:n + 3, 3:n + 3, 3:n + 3] = q
        corners = [pad[base[0] + a, base[1] + b, base[2] + c] for a in (0, 1) for b in (0, 1) for c in (0, 1)]
        lo = np.min(np.stack(corners), axis=0)
        hi = np.max(np.stack(corners), axis=0)
        val = (self._field(ch_fwd) + (T(0.5) * (q - self._field(ch_bwd))).astype(self.dtype)).astype(self.dtype)
        self._store(ch_out, np.minimum(np.maximum(val, lo), hi))

    # -- two-level transfers (this grid is the fine one) ----------------------------
    def restrict_to(self, coarse, ch_x, ch_y, w):
        """coarse.y[I//2] += w * x[I] over this grid's listed blocks: the coarse
        parents of the listed blocks are activated (zero-filled if new), then
        each coarse voxel adds its 8 children one at a time in ascending order
        of their index inside the fine block."""
        T = self.dtype.type
        R = self.R
        listed = np.zeros(R ** 3, dtype=bool)
        listed[self.list] = True
        listed = listed.reshape((R,) * 3)
        for bi, bj, bk in np.argwhere(listed):
            coarse._activate_block(bi // 2, bj // 2, bk // 2)
        x = self._field(ch_x)
        under = np.repeat(np.repeat(np.repeat(listed, 4, 0), 4, 1), 4, 2)   # coarse voxels fed by a listed block
        y = coarse._field(ch_y)
        for a in (0, 1):
            for b in (0, 1):
                for c in (0, 1):
                    y = np.where(under, y + T(w) * x[a::2, b::2, c::2], y)
        coarse.vals[ch_y] = np.where(under, y, coarse.vals[ch_y])

    def prolong_from(self, coarse, ch_y, ch_x):
        """x[I] += coarse.y[I//2] over this grid's listed blocks."""
        y = coarse._field(ch_y)
        up = np.repeat(np.repeat(np.repeat(y, 2, 0), 2, 1), 2, 2)
        self._store(ch_x, self._field(ch_x) + up)

    def diffuse(self, ch_a, ch_k, ch_out, dt):
        T = self.dtype.type
        a, k = self._field(ch_a), self._field(ch_k)
        f = np.zeros_like(a)
        for d in _FACES:
            kf = T(0.5) * (k + self._shift(k, *d))
            f = f + kf * (self._shift(a, *d) - a)
        self._store(ch_out, a + T(dt) * f)

    def diffuse_adj(self, ch_a, ch_k, ch_lamn, ch_lam, ch_gk, dt):
        T = self.dtype.type
        a, k, l = self._field(ch_a), self._field(ch_k), self._field(ch_lamn)
        f = np.zeros_like(a)
        q = np.zeros_like(a)
        for d in _FACES:
            ln = self._shift(l, *d)
            kf = T(0.5) * (k + self._shift(k, *d))
            f = f + kf * (ln - l)
            q = q + (self._shift(a, *d) - a) * (l - ln)
        gk = self._field(ch_gk)
        self._store(ch_lam, l + T(dt) * f)
        self._store(ch_gk, gk + (T(dt) * T(0.5)) * q)

    # -- particles -----------------------------------------------------------------
    def _weights(self, x, inv_dx):
        T = self.dtype.type
        X = x.astype(self.dtype) * T(inv_dx)                       # [3, np]
        base = np.floor(X - T(0.5)).astype(np.int64)
        fx = X - base.astype(self.dtype)
        w = np.stack([T(0.5) * ((T(1.5) - fx) * (T(1.5) - fx)),
                      T(0.75) - (fx - T(1)) * (fx - T(1)),
                      T(0.5) * ((fx - T(0.5)) * (fx - T(0.5)))], axis=1)  # [3, 3, np]
        return base, w

    def p2g(self, ch_m, ch_mv, x, v, m, inv_dx, ch_abs=-1):
        base, w = self._weights(x, inv_dx)
        npart = x.shape[1]
        vv = v.astype(self.dtype)
        mm = m.astype(self.dtype)
        # activation, in write order
        for p in range(npart):
            for a in range(3):
                for b in range(3):
                    for c in range(3):
                        i, j, k = base[0, p] + a, base[1, p] + b, base[2, p] + c
                        if 0 <= i < self.n and 0 <= j < self.n and 0 <= k < self.n:
                            self._activate_block(i // 8, j // 8, k // 8)
        acc = [self.vals[ch_m].astype(np.float64)] + [self.vals[ch_mv + c].astype(np.float64) for c in range(3)]
        absacc = None
        if ch_abs >= 0:
            absacc = [self.vals[ch_abs + q].astype(np.float64) for q in range(4)]
        for a in range(3):
            for b in range(3):
                for c in range(3):
                    wt = (w[0, a] * w[1, b]) * w[2, c]
                    idx = (base[0] + a, base[1] + b, base[2] + c)
                    terms = [wt * mm] + [(wt * mm) * vv[q] for q in range(3)]
                    for q in range(4):
                        np.add.at(acc[q], idx, terms[q].astype(np.float64))
                        if absacc is not None:
                            np.add.at(absacc[q], idx, np.abs(terms[q].astype(np.float64)))
        self.vals[ch_m] = acc[0].astype(self.dtype)
        for q in range(3):
            self.vals[ch_mv + q] = acc[1 + q].astype(self.dtype)
        if absacc is not None:
            for q in range(4):
                self.vals[ch_abs + q] = absacc[q].astype(self.dtype)

    def normalise(self, ch_m, ch_mv, ch_v):
        T = self.dtype.type
        mm = self._field(ch_m)
        pos = mm > T(0)
        safe = np.where(pos, mm, T(1))
        for c in range(3):
            self._store(ch_v + c, np.where(pos, self._field(ch_mv + c) / safe, T(0)))

    def g2p(self, ch_v, x, inv_dx):
        base, w = self._weights(x, inv_dx)
        out = np.zeros((3, x.shape[1]), dtype=self.dtype)
        fields = [self._field(ch_v + c) for c in range(3)]
        n = self.n
        for a in range(3):
            for b in range(3):
                for c in range(3):
                    wt = (w[0, a] * w[1, b]) * w[2, c]
                    i, j, k = base[0] + a, base[1] + b, base[2] + c
                    ok = (i >= 0) & (j >= 0) & (k >= 0) & (i < n) & (j < n) & (k < n)
                    ii, jj, kk = np.clip(i, 0, n - 1), np.clip(j, 0, n - 1), np.clip(k, 0, n - 1)
                    for q in range(3):
                        val = np.where(ok, fields[q][ii, jj, kk], self.dtype.type(0))
                        out[q] = out[q] + wt * val
        return out

    # -- layout helpers ------------------------------------------------------------
    def load(self, blocks, channel_values: dict, channel_index: dict):
        self.activate(blocks, "block")
        for name, vals in channel_values.items():
            ch = channel_index[name]
            for t, (bi, bj, bk) in enumerate(np.asarray(blocks)):
                self.vals[ch, bi * 8:bi * 8 + 8, bj * 8:bj * 8 + 8, bk * 8:bk * 8 + 8] = \
                    np.asarray(vals[t], dtype=self.dtype).reshape(8, 8, 8)

    def to_dense(self, ch):
        return self._field(ch)
