"""Batched Jacobi over many independent sparse grids (one shared leaf pool).

``BatchArena`` owns one device buffer laid out by ``at_batch_create``: a
root row per resident grid (pool slot per root cell), a shared pool of
leaves for x, xn and b, a work list of (grid, cell) entries and, per grid,
the window of global iterations in which it is active.  Admission and
retirement go through ``at_batch_update``, which applies one replay
boundary's changes in two launches, in stream order, without host
synchronisation: the host keeps only ids and counts, and a request's cells
and right-hand side are already on the device.  The iterations themselves
are ``at_batch_jacobi`` launches -- the same Jacobi and copy arithmetic as
the single-grid kernels -- which can be captured once in a HIP graph and
replayed while grids come and go.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from .grid import current_stream


def _dev_i32(x, dev):
    t = x if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x, dtype=np.int32))
    return t.to(device=dev, dtype=torch.int32).contiguous()


def _dev_f32(x, dev, nb):
    t = x if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x, dtype=np.float32))
    return t.to(device=dev, dtype=torch.float32).reshape(nb, 512).contiguous()


class BatchArena:
    def __init__(self, n: int = 128, max_grids: int = 256, pool_blocks: int = 65536, device="cuda"):
        self.n, self.R = n, n // 8
        self.ncells = self.R ** 3
        self.max_grids, self.pool_blocks = max_grids, pool_blocks
        self._lib = L.lib()
        desc = L.AtBatchDesc(n, max_grids, pool_blocks, 0)
        nbytes = ctypes.c_size_t()
        L.check(self._lib.at_batch_footprint(ctypes.byref(desc), ctypes.byref(nbytes)))
        self.bytes = int(nbytes.value)
        self.buf = torch.empty(self.bytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        L.check(self._lib.at_batch_create(ctypes.byref(desc), ctypes.c_void_p(self.buf.data_ptr()), self.bytes,
                                          current_stream(), ctypes.byref(h)))
        self.handle = h
        v = L.AtBatchViews()
        L.check(self._lib.at_batch_get_views(h, ctypes.byref(v)))

        def view(ptr, nbytes, dtype, shape):
            off = ptr - self.buf.data_ptr()
            return self.buf[off:off + nbytes].view(dtype).view(*shape)

        self.clock = view(v.clock, 8, torch.int64, (1,))
        self.count = view(v.count, 4, torch.int32, (1,))
        self.window = view(v.window, max_grids * 16, torch.int64, (max_grids, 2))
        self.roots = view(v.roots, max_grids * self.ncells * 4, torch.int32, (max_grids, self.ncells))
        self.work = view(v.work, pool_blocks * 4, torch.int32, (pool_blocks,))
        self.x = view(v.x, pool_blocks * 2048, torch.float32, (pool_blocks, 512))
        self.xn = view(v.xn, pool_blocks * 2048, torch.float32, (pool_blocks, 512))
        self.b = view(v.b, pool_blocks * 2048, torch.float32, (pool_blocks, 512))
        # host bookkeeping: ids and counts only
        self.clock_host = 0
        self.nfree = pool_blocks
        self.free_gids = list(range(max_grids - 1, -1, -1))
        self.grids = {}            # gid -> (cells, slots, b: device tensors kept alive; window)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                self._lib.at_batch_destroy(h)
            except Exception:
                pass
            self.handle = None

    # ---- admission ------------------------------------------------------------
    @staticmethod
    def footprint(nblocks: int) -> int:
        """HBM bytes a request occupies: 3 leaf channels plus its work-list share."""
        return nblocks * (3 * 2048 + 4)

    def free_blocks(self) -> int:
        return self.nfree

    def fits(self, nblocks: int) -> bool:
        return bool(self.free_gids) and self.nfree >= nblocks

    def update(self, retire=(), admit=(), stream=None):
        """Apply one replay boundary's changes in stream order: retire the
        grids ``retire`` (ids), then admit ``admit`` -- (cells, b, iters)
        triples, cells ascending ([nb] int32) and b ([nb, 512] float32), on
        the device already for a host-free update.  Returns (x of each
        retired grid [nb, 512], valid in stream order; id of each admitted
        grid)."""
        dev = self.x.device
        rets, outs = [], []
        for gid in retire:
            cells, slots, _, _ = self.grids[gid]
            out = torch.empty((cells.numel(), 512), dtype=torch.float32, device=dev)
            rets.append(L.AtBatchRetire(gid, 0, out.data_ptr()))
            outs.append(out)
        freed = sum(self.grids[g][0].numel() for g in retire)
        need = 0
        adms, gids, keep = [], [], []
        free_gids = self.free_gids + list(retire)
        for cells, b, iters in admit:
            if not 0 <= int(iters) < (1 << 31):
                raise ValueError("iterations must lie in [0, 2^31)")
            cells_t = _dev_i32(cells, dev)
            nb = cells_t.numel()
            b_t = _dev_f32(b, dev, nb)
            slots_t = torch.empty(nb, dtype=torch.int32, device=dev)
            if not free_gids:
                raise RuntimeError("batch arena has no free grid slot")
            gid = free_gids.pop()
            adms.append(L.AtBatchAdmit(cells_t.data_ptr(), b_t.data_ptr(), slots_t.data_ptr(), gid, nb, int(iters), 0))
            gids.append(gid)
            keep.append((cells_t, slots_t, b_t, (self.clock_host, self.clock_host + int(iters))))
            need += nb
        if need > self.nfree + freed:
            raise RuntimeError("batch arena full")
        ra = (L.AtBatchRetire * max(1, len(rets)))(*rets)
        aa = (L.AtBatchAdmit * max(1, len(adms)))(*adms)
        L.check(self._lib.at_batch_update(self.handle, ra, len(rets), aa, len(adms),
                                          stream if stream is not None else current_stream()))
        for gid in retire:
            del self.grids[gid]
        self.free_gids = free_gids
        self.nfree += freed - need
        for gid, k in zip(gids, keep):
            self.grids[gid] = k
        return outs, gids

    def admit(self, cells, b, iters: int) -> int:
        """Make a grid with active root cells ``cells`` (ascending), right-hand
        side ``b`` ([nb, 512]) and x = 0 resident, active for the next
        ``iters`` global iterations.  Returns its grid id."""
        if not self.fits(len(cells)):
            raise RuntimeError("batch arena full")
        return self.update((), [(cells, b, iters)])[1][0]

    def done(self, gid: int) -> bool:
        return self.clock_host >= self.grids[gid][3][1]

    def retire(self, gid: int):
        """Remove a grid; returns its x values [nb, 512] (a device tensor,
        valid in stream order)."""
        return self.update([gid], ())[0][0]

    # ---- iterations -------------------------------------------------------------
    def launch(self, iters: int, workgroups: int = 0, stream=None):
        """iters x (jacobi, copy) over the work list, then clock += iters."""
        L.check(self._lib.at_batch_jacobi(self.handle, iters, workgroups,
                                          stream if stream is not None else current_stream()))

    def step(self, iters: int, workgroups: int = 0):
        self.launch(iters, workgroups)
        self.clock_host += iters

    def capture(self, iters: int, workgroups: int = 0, waves: int = 0):
        """A replayable graph of ``iters`` iterations (the launches read all
        per-iteration state from device memory).  ``waves``: wavefronts per
        workgroup of the captured launches (0: the library's current setting)."""
        return CapturedSteps(self, iters, workgroups, waves)


def _get_waves() -> int:
    v = ctypes.c_int64()
    L.check(L.lib().at_get_option(L.AT_OPTION_BATCH_WAVES, ctypes.byref(v)))
    return int(v.value)


def _set_waves(w: int):
    L.check(L.lib().at_set_option(L.AT_OPTION_BATCH_WAVES, w))


class CapturedSteps:
    def __init__(self, arena: BatchArena, iters: int, workgroups: int = 0, waves: int = 0):
        self.arena, self.iters = arena, iters
        prev = _get_waves()
        if waves:
            _set_waves(waves)
        try:
            self._capture(arena, iters, workgroups)
        finally:
            _set_waves(prev)

    def _capture(self, arena, iters, workgroups):
        self.graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            # warm the launch path once outside capture on the side stream;
            # it must not advance the clock, so run zero iterations
            arena.launch(0, workgroups, s.cuda_stream)
        torch.cuda.current_stream().wait_stream(s)
        with torch.cuda.graph(self.graph):
            arena.launch(iters, workgroups, torch.cuda.current_stream().cuda_stream)

    def replay(self):
        self.graph.replay()
        self.arena.clock_host += self.iters
