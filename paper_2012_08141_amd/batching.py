"""Batched Jacobi over many independent sparse grids (one shared leaf pool).

``BatchArena`` owns one device buffer laid out by ``at_batch_create``: a
root row per resident grid (pool slot per root cell), a shared pool of
leaves for x, xn and b, a work list of (grid, cell) entries and, per grid,
the window of global iterations in which it is active.  Admission and
retirement only edit those arrays (stream-ordered device copies); the
iterations themselves are ``at_batch_jacobi`` launches -- the same Jacobi
and copy arithmetic as the single-grid kernels -- which can be captured once
in a HIP graph and replayed while grids come and go.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from .grid import current_stream


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
        # host bookkeeping
        self.clock_host = 0
        self.free_slots = list(range(pool_blocks - 1, -1, -1))
        self.free_gids = list(range(max_grids - 1, -1, -1))
        self.grids = {}            # gid -> (slots tensor, cells np, window)
        self._dirty = False

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
        return len(self.free_slots)

    def fits(self, nblocks: int) -> bool:
        return bool(self.free_gids) and len(self.free_slots) >= nblocks

    def admit(self, cells: np.ndarray, b, iters: int) -> int:
        """Make a grid with active root cells ``cells`` (ascending), right-hand
        side ``b`` ([nb, 512]) and x = 0 resident, active for the next
        ``iters`` global iterations.  Returns its grid id."""
        nb = len(cells)
        if not self.fits(nb):
            raise RuntimeError("batch arena full")
        gid = self.free_gids.pop()
        slots = np.array([self.free_slots.pop() for _ in range(nb)], dtype=np.int64)
        dev = self.x.device
        slots_t = torch.as_tensor(slots, device=dev)
        cells_t = torch.as_tensor(np.asarray(cells, dtype=np.int64), device=dev)
        row = torch.full((self.ncells,), -1, dtype=torch.int32, device=dev)
        row[cells_t] = slots_t.to(torch.int32)
        self.roots[gid].copy_(row)
        bt = b if isinstance(b, torch.Tensor) else torch.as_tensor(np.asarray(b, np.float32))
        self.b.index_copy_(0, slots_t, bt.to(device=dev, dtype=torch.float32).reshape(nb, 512))
        z = torch.zeros((nb, 512), dtype=torch.float32, device=dev)
        self.x.index_copy_(0, slots_t, z)
        self.xn.index_copy_(0, slots_t, z)
        win = (self.clock_host, self.clock_host + iters)
        self.window[gid].copy_(torch.tensor(win, dtype=torch.int64))
        self.grids[gid] = (slots_t, np.asarray(cells, dtype=np.int32), win)
        self._dirty = True
        return gid

    def done(self, gid: int) -> bool:
        return self.clock_host >= self.grids[gid][2][1]

    def retire(self, gid: int):
        """Remove a grid; returns its x values [nb, 512] (a device tensor,
        valid in stream order)."""
        slots_t, cells, win = self.grids.pop(gid)
        out = self.x.index_select(0, slots_t)
        self.roots[gid].fill_(-1)
        self.window[gid].zero_()
        self.free_slots.extend(slots_t.cpu().tolist())
        self.free_gids.append(gid)
        self._dirty = True
        return out

    def sync_work_list(self):
        """Upload the work list (ascending grid, then cell) if it changed."""
        if not self._dirty:
            return
        parts = [gid * self.ncells + cells.astype(np.int64) for gid, (_, cells, _) in sorted(self.grids.items())]
        w = np.concatenate(parts).astype(np.int32) if parts else np.zeros(0, np.int32)
        if len(w):
            self.work[:len(w)].copy_(torch.as_tensor(w))
        self.count.copy_(torch.tensor([len(w)], dtype=torch.int32))
        self._dirty = False

    # ---- iterations -------------------------------------------------------------
    def launch(self, iters: int, workgroups: int = 0, stream=None):
        """iters x (jacobi, copy) over the work list, then clock += iters."""
        L.check(self._lib.at_batch_jacobi(self.handle, iters, workgroups,
                                          stream if stream is not None else current_stream()))

    def step(self, iters: int, workgroups: int = 0):
        self.sync_work_list()
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
        self.arena.sync_work_list()
        self.graph.replay()
        self.arena.clock_host += self.iters
