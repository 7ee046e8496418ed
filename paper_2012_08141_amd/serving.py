"""Continuous-batching server for sparse Jacobi solves.

Requests (a sparse grid plus right-hand side, wanting a fixed number of
Jacobi iterations) arrive over time.  The server keeps admitted grids
resident in one ``BatchArena`` and advances all of them together with one
captured graph of K iterations per replay.  At every replay boundary it
admits waiting requests in FIFO order while their HBM footprint fits the
budget and a grid slot is free -- so requests that arrive while others are
on the GPU join them -- and retires the requests whose iteration window has
ended, freeing their pool space.  Latency is completion minus arrival; the
completion time of a request is the device time at which the replay that ran
its last iteration finished.

The loop never waits for the device except to bound the replays in flight:
a boundary's retirements and admissions are one ``at_batch_update`` (two
launches, descriptors as kernel arguments), a request's cells and
right-hand side are on the device from its creation (inputs resident in
HBM), and completion times are read from events as they complete.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import engine as E
from . import inputs
from .batching import BatchArena
from .grid import SparseGrid


@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the stream
    cells: np.ndarray         # active root cells, ascending
    b: np.ndarray             # [nb, 512] float32
    iters: int = 50
    admitted: float = -1.0
    completed: float = -1.0
    result: torch.Tensor = None
    gid: int = -1
    end_clock: int = -1
    cells_dev: torch.Tensor = None    # the same on the device (uploaded at creation)
    b_dev: torch.Tensor = None

    @property
    def nblocks(self) -> int:
        return len(self.cells)

    @property
    def voxel_iters(self) -> int:
        return self.nblocks * 512 * self.iters


def make_requests(seed: int, count: int, arrivals: np.ndarray, n: int = 128, iters: int = 50, device="cuda"):
    """The seeded request stream; each request's cells and b are also put on
    ``device`` (None: host only)."""
    reqs = []
    for i in range(count):
        w = inputs.batch_request(seed, i, n=n)
        r = Request(i, float(arrivals[i]), w.cells, w.channels["b"], iters)
        if device is not None:
            r.cells_dev = torch.as_tensor(r.cells.astype(np.int32), device=device)
            r.b_dev = torch.as_tensor(np.ascontiguousarray(r.b, dtype=np.float32), device=device)
        reqs.append(r)
    return reqs


@dataclass
class ServeStats:
    latencies: list = field(default_factory=list)
    makespan: float = 0.0
    voxel_iters: int = 0
    replays: int = 0
    max_resident: int = 0

    def summary(self) -> dict:
        lat = np.asarray(self.latencies)
        return {"requests": len(lat), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
                "makespan_s": self.makespan, "voxel_steps_per_s": self.voxel_iters / self.makespan,
                "replays": self.replays, "max_resident": self.max_resident}


class JacobiServer:
    def __init__(self, n: int = 128, budget_bytes: int = 256 << 20, max_grids: int = 64,
                 iters_per_replay: int = 10, workgroups: int = 0, max_inflight: int = 8, waves: int = 0):
        pool = max(1, budget_bytes // BatchArena.footprint(1))
        self.arena = BatchArena(n, max_grids, pool)
        self.budget = budget_bytes
        self.K = iters_per_replay
        self.graph = self.arena.capture(self.K, workgroups, waves)
        self.max_inflight = max_inflight

    def serve(self, requests, realtime: bool = True) -> ServeStats:
        """Serve requests (sorted by arrival).  With realtime=False all
        requests count as arrived at time 0 (a closed batch)."""
        A = self.arena
        st = ServeStats()
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting = deque()
        resident = {}             # rid -> request whose grid is in the arena
        unfinished = {}           # rid -> request admitted but not yet known complete
        inflight = deque()        # (event, clock after the replay)
        start_ev = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        start_ev.record()

        def finish(ev, clock_after):
            t_done = start_ev.elapsed_time(ev) * 1e-3
            for r in [r for r in unfinished.values() if r.end_clock <= clock_after]:
                del unfinished[r.rid]
                r.completed = t_done
                st.latencies.append(t_done - (r.arrival if realtime else 0.0))

        def drain(block_until):
            # completed replays first, without waiting; then wait for the
            # oldest while more than block_until are in flight
            while inflight and inflight[0][0].query():
                finish(*inflight.popleft())
            while len(inflight) > block_until:
                inflight[0][0].synchronize()
                finish(*inflight.popleft())

        while pending or waiting or resident or unfinished:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                waiting.append(pending.popleft())
            # retire grids whose last iteration is already enqueued, admit
            # FIFO while the footprint fits: one update
            gone = [r for r in resident.values() if r.end_clock <= A.clock_host]
            free_blocks = A.free_blocks() + sum(r.nblocks for r in gone)
            free_ids = len(A.free_gids) + len(gone)
            new = []
            while waiting and free_ids > 0 and waiting[0].nblocks <= free_blocks:
                r = waiting.popleft()
                free_blocks -= r.nblocks
                free_ids -= 1
                new.append(r)
            if gone or new:
                outs, gids = A.update([r.gid for r in gone],
                                      [(r.cells_dev if r.cells_dev is not None else r.cells,
                                        r.b_dev if r.b_dev is not None else r.b, r.iters) for r in new])
                for r, x in zip(gone, outs):
                    r.result = x
                    del resident[r.rid]
                for r, gid in zip(new, gids):
                    r.gid = gid
                    r.end_clock = A.clock_host + r.iters
                    r.admitted = now
                    resident[r.rid] = r
                    unfinished[r.rid] = r
            st.max_resident = max(st.max_resident, len(resident))
            if resident:
                self.graph.replay()
                st.replays += 1
                ev = torch.cuda.Event(enable_timing=True)
                ev.record()
                inflight.append((ev, A.clock_host))
                drain(self.max_inflight)
            else:
                drain(0)
                if waiting:
                    raise RuntimeError("a request of %d blocks can never fit the arena" % waiting[0].nblocks)
                if pending and realtime:
                    time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
        torch.cuda.synchronize()
        st.makespan = time.perf_counter() - t0
        st.voxel_iters = sum(r.voxel_iters for r in requests)
        return st


def solve_alone(req: Request, n: int = 128, opt_flags: int = 0) -> torch.Tensor:
    """One request on its own grid through the single-grid engine path
    (iters x (listgen, jacobi, copy)); returns x [nb, 512]."""
    g = SparseGrid(n, 3, "pointer", req.nblocks)
    g.load_blocks(2, req.cells, req.b)
    E.run_sequence(sum(([E.listgen(g), E.jacobi(g, 0, 2, 1), E.copy(g, 0, 1)] for _ in range(req.iters)), []),
                   opt_flags)
    return g.read_blocks_t(0, torch.as_tensor(req.cells, device="cuda"))


def serve_eager_fifo(requests, n: int = 128, realtime: bool = True) -> ServeStats:
    """Baseline: the same stream served one request at a time, each as the
    eager single-grid pipeline."""
    st = ServeStats()
    reqs = sorted(requests, key=lambda r: r.arrival)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        now = time.perf_counter() - t0
        if realtime and r.arrival > now:
            time.sleep(r.arrival - now)
        r.result = solve_alone(r, n, 0)
        torch.cuda.synchronize()
        r.completed = time.perf_counter() - t0
        st.latencies.append(r.completed - (r.arrival if realtime else 0.0))
    st.makespan = time.perf_counter() - t0
    st.voxel_iters = sum(r.voxel_iters for r in requests)
    st.max_resident = 1
    return st
