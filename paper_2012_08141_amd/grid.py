"""Sparse grid handle: a torch-allocated device buffer laid out and
initialised by the library (root, list, leaf pool; paper Section 3)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as L

try:
    import torch
except ImportError:      # planning handles work without torch
    torch = None


_HAS_DEVICE = None


def current_stream():
    """hipStream_t of torch's current stream (0 without a device)."""
    global _HAS_DEVICE
    if _HAS_DEVICE is None:
        _HAS_DEVICE = torch is not None and torch.cuda.is_available()
    return torch.cuda.current_stream().cuda_stream if _HAS_DEVICE else None


_KINDS = {"bitmask": L.AT_ROOT_BITMASK, "pointer": L.AT_ROOT_POINTER}


def footprint(n: int, channels: int, root_kind: str = "bitmask", capacity_blocks: int = 0,
              particle_capacity: int = 0) -> int:
    d = L.AtGridDesc((n, n, n), _KINDS[root_kind], channels, capacity_blocks, particle_capacity)
    b = ctypes.c_size_t()
    L.check(L.lib().at_grid_footprint(ctypes.byref(d), ctypes.byref(b)))
    return int(b.value)


class SparseGrid:
    """An ``n^3`` sparse grid with ``channels`` fp32 channels.

    ``device=None`` makes a planning handle (no device memory): it can be
    used in task sequences for planning only.  ``particle_capacity`` sizes
    the workspace that lets a particle scatter into this grid bin up to that
    many particles (0: scatters add straight into global memory)."""

    def __init__(self, n: int, channels: int, root_kind: str = "bitmask", capacity_blocks: int = 0,
                 device="cuda", stream=None, particle_capacity: int = 0):
        self.n, self.channels, self.root_kind = n, channels, root_kind
        self.R = n // 8
        self._lib = L.lib()
        desc = L.AtGridDesc((n, n, n), _KINDS[root_kind], channels, capacity_blocks, particle_capacity)
        self.bytes = footprint(n, channels, root_kind, capacity_blocks, particle_capacity)
        self.buf = None
        h = ctypes.c_void_p()
        if device is None:
            L.check(self._lib.at_grid_create(ctypes.byref(desc), None, 0, None, ctypes.byref(h)))
        else:
            self.buf = torch.empty(self.bytes, dtype=torch.uint8, device=device)
            if self.buf.data_ptr() % 256:
                raise RuntimeError("torch returned a buffer that is not 256-byte aligned")
            st = stream if stream is not None else current_stream()
            L.check(self._lib.at_grid_create(ctypes.byref(desc), ctypes.c_void_p(self.buf.data_ptr()),
                                             self.bytes, st, ctypes.byref(h)))
        self.handle = h
        info = L.AtGridInfo()
        L.check(self._lib.at_grid_get_info(h, ctypes.byref(info)))
        self.capacity = info.capacity_blocks
        self.list_capacity = info.list_capacity
        self.ncells = info.ncells

    @property
    def virtual(self) -> bool:
        return self.buf is None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                self._lib.at_grid_destroy(h)
            except Exception:
                pass
            self.handle = None

    # ---- device views ---------------------------------------------------------
    def _views(self):
        ch = (ctypes.c_void_p * self.channels)()
        lst, cnt, root = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        L.check(self._lib.at_grid_views(self.handle, ch, ctypes.byref(lst), ctypes.byref(cnt), ctypes.byref(root)))
        return ch, lst.value, cnt.value, root.value

    def _slice(self, ptr: int, nbytes: int):
        off = ptr - self.buf.data_ptr()
        return self.buf[off:off + nbytes]

    def channel(self, c: int):
        """Channel ``c`` as a float32 tensor [capacity, 512] (indexed by slot)."""
        ch, _, _, _ = self._views()
        return self._slice(ch[c], self.capacity * 512 * 4).view(torch.float32).view(self.capacity, 512)

    def list_count(self) -> int:
        _, _, cnt, _ = self._views()
        return int(self._slice(cnt, 4).view(torch.int32).item())

    def list_records(self) -> np.ndarray:
        """The list state: one record per entry, int32 [count, 8] =
        (cell, slot, slots of the 6 face neighbours)."""
        _, lst, cnt, _ = self._views()
        c = int(self._slice(cnt, 4).view(torch.int32).item())
        return self._slice(lst, self.list_capacity * 32).view(torch.int32).view(-1, 8)[:c].cpu().numpy()

    def list_cells(self) -> np.ndarray:
        """The list state's root cells, in list order."""
        return self.list_records()[:, 0].copy()

    def active_cells(self) -> np.ndarray:
        """Active root cells read from the mask, ascending."""
        _, _, _, root = self._views()
        if self.root_kind == "pointer":
            p = self._slice(root, self.ncells * 4).view(torch.int32).cpu().numpy()
            return np.nonzero(p >= 0)[0].astype(np.int32)
        words = (self.ncells + 31) // 32
        b = self._slice(root, words * 4).view(torch.int32).cpu().numpy().view(np.uint32)
        bits = np.unpackbits(b.view(np.uint8), bitorder="little")[:self.ncells]
        return np.nonzero(bits)[0].astype(np.int32)

    def slots(self, cells) -> np.ndarray:
        """Leaf slot of each root cell (-1 when inactive)."""
        cells = np.asarray(cells, dtype=np.int64)
        if self.root_kind == "bitmask":
            act = np.zeros(self.ncells, bool)
            act[self.active_cells()] = True
            return np.where(act[cells], cells, -1).astype(np.int32)
        _, _, _, root = self._views()
        p = self._slice(root, self.ncells * 4).view(torch.int32).cpu().numpy()
        return np.where(p[cells] >= 0, p[cells], -1).astype(np.int32)

    # ---- immediate tasks ------------------------------------------------------
    def activate(self, coords, kind: int = L.AT_COORD_BLOCK, stream=None):
        c = _as_dev_i32(coords).reshape(-1, 3).contiguous()
        L.check(self._lib.at_activate(self.handle, ctypes.c_void_p(c.data_ptr()), c.shape[0], kind,
                                      stream if stream is not None else current_stream()))
        return c

    def listgen(self, stream=None):
        L.check(self._lib.at_listgen(self.handle, stream if stream is not None else current_stream()))

    def run_stencil(self, op: int, ch, param: float = 0.0, check_activation: bool = True, stream=None):
        chs = list(ch) + [-1] * (8 - len(ch))
        carr = (ctypes.c_int32 * 8)(*chs)
        parr = (ctypes.c_float * 4)(param, 0, 0, 0)
        L.check(self._lib.at_run_stencil(self.handle, op, carr, parr, 1 if check_activation else 0,
                                         stream if stream is not None else current_stream()))

    def clear(self, stream=None):
        L.check(self._lib.at_grid_clear(self.handle, stream if stream is not None else current_stream()))

    def device_status(self, clear: bool = False, stream=None) -> int:
        b = ctypes.c_int32()
        L.check(self._lib.at_device_status(self.handle, stream if stream is not None else current_stream(),
                                           1 if clear else 0, ctypes.byref(b)))
        return int(b.value)

    def active_count(self, stream=None) -> int:
        c = ctypes.c_int64()
        L.check(self._lib.at_active_count(self.handle, stream if stream is not None else current_stream(),
                                          ctypes.byref(c)))
        return int(c.value)

    # ---- block transfer (setup / inspection) ---------------------------------
    def load_blocks(self, ch: int, cells, values, stream=None):
        """Activate ``cells`` (in order) and store per-block values [n, 512]."""
        cells_t = _as_dev_i32(cells).contiguous()
        vals = _as_dev_f32(values).reshape(-1, 512).contiguous()
        assert vals.shape[0] == cells_t.shape[0]
        L.check(self._lib.at_scatter_blocks(self.handle, ch, ctypes.c_void_p(cells_t.data_ptr()),
                                            ctypes.c_void_p(vals.data_ptr()), cells_t.shape[0],
                                            stream if stream is not None else current_stream()))
        return cells_t, vals

    def read_blocks(self, ch: int, cells, stream=None) -> np.ndarray:
        cells_t = _as_dev_i32(cells).contiguous()
        out = torch.empty((cells_t.shape[0], 512), dtype=torch.float32, device=self.buf.device)
        L.check(self._lib.at_gather_blocks(self.handle, ch, ctypes.c_void_p(cells_t.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), cells_t.shape[0],
                                           stream if stream is not None else current_stream()))
        return out.cpu().numpy()

    def read_blocks_t(self, ch: int, cells_t, out=None, stream=None):
        """Device version of read_blocks: returns a float32 tensor [n, 512]."""
        if out is None:
            out = torch.empty((cells_t.shape[0], 512), dtype=torch.float32, device=self.buf.device)
        L.check(self._lib.at_gather_blocks(self.handle, ch, ctypes.c_void_p(cells_t.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), cells_t.shape[0],
                                           stream if stream is not None else current_stream()))
        return out


def _as_dev_i32(x):
    if torch is not None and isinstance(x, torch.Tensor):
        return x.to(device="cuda", dtype=torch.int32)
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.int32), device="cuda")


def _as_dev_f32(x):
    if torch is not None and isinstance(x, torch.Tensor):
        return x.to(device="cuda", dtype=torch.float32)
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32), device="cuda")
