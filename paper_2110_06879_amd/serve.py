"""Warm-start tracking service with continuous batching on one GPU.

The paper motivates fast tracking of the ACOPF optimum under load changes
(Sec. I, Sec. IV-C): each new load picture is solved warm from the previous
solution. This module serves a stream of such requests over several resident
grids. Every step of every solve runs in the HIP kernels of libacopf.so; this
file only schedules.

Layout: one acopf handle holds, for every resident grid j, 1 + k_j instances
of the same grid data. One of them is the grid's *home* (its last committed
ADMM state); the others are free slots that requests run in. The k_j are
chosen so that the device footprint of all instances fits the HBM budget,
which defaults to 90% of the device memory free when the server starts.

A request (grid j, new loads) is admitted between iteration chunks as soon as
a slot of grid j is free: the home state is copied into the slot on the
device (one launch), the loads are set, and a WARM start joins the running
batch, so its inner iterations overlap with those of every other request in
flight. When it finishes, its slot becomes the grid's home (the next request
for the grid warm-starts from it) and the previous home becomes a free slot:
a completion copies nothing. A grid whose budget allows no slot runs its
requests on its home instance, one at a time.

Because every grid of a handle is an independent problem whose arithmetic
does not depend on the other grids in the launch, a request's result is
bitwise the same alone and in the mix (tested).
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import acopf as A
from .gridgen import Grid


def instance_bytes(g: Grid) -> int:
    """Device footprint of one grid instance in the library's layout."""
    m = g.n_coupling
    nb, ng, nl = g.n_bus, g.n_gen, g.n_branch
    # coupling vectors; branch data, state and records; generators; buses
    doubles = 5 * m + 9 * nl + 8 * nl + 5 * nl + 16 * nl + 9 * ng + 6 * nb
    ints = 2 * nl + nl + 2 * nl + 2 * nl + ng + 3 * nb + 2
    return 8 * doubles + 4 * ints + 6 * 8 * (1 << 15)  # + residual history


def device_free_bytes(device: int = 0) -> float:
    """90% of the device memory free now, the default HBM budget."""
    free, _ = A.device_memory(device)
    return 0.9 * free


@dataclass
class Request:
    rid: int
    grid: int
    arrival: float          # seconds after the start of the stream
    pd: np.ndarray
    qd: np.ndarray
    admitted: float = math.nan
    finished: float = math.nan
    result: dict = field(default_factory=dict)
    slot: int = -1


class TrackingServer:
    """Continuous-batching warm-start server over resident grids."""

    def __init__(self, grids: list[Grid], params: A.Params | None = None,
                 hbm_budget_bytes: float | None = None, max_slots_per_grid: int = 4,
                 device: int = 0, cold_start: bool = True, chunk: int | None = None):
        self.grids = list(grids)
        n = len(self.grids)
        sizes = [instance_bytes(g) for g in self.grids]
        homes = sum(sizes)
        budget = hbm_budget_bytes if hbm_budget_bytes is not None else device_free_bytes(device)
        if homes > budget:
            raise ValueError(f"HBM budget {budget:.3g} B cannot hold the {n} resident grids "
                             f"({homes:.3g} B)")
        # slots: round robin, smallest grids first, while the budget allows
        slots = [0] * n
        left = budget - homes
        order = sorted(range(n), key=lambda j: sizes[j])
        grew = True
        while grew:
            grew = False
            for j in order:
                if slots[j] < max_slots_per_grid and sizes[j] <= left:
                    slots[j] += 1
                    left -= sizes[j]
                    grew = True
        self.slots_per_grid = slots
        self.bytes_used = budget - left
        # handle layout: homes 0..n-1, then the slots of each grid
        inst = list(self.grids)
        self.slot_ids: list[list[int]] = []
        for j in range(n):
            ids = []
            for _ in range(slots[j]):
                ids.append(len(inst))
                inst.append(self.grids[j])
            self.slot_ids.append(ids)
        self.solver = A.Solver(inst, params, device=device)
        if chunk is not None:  # iterations between admissions (graph replay length)
            self.solver.set_tuning(chunk=int(chunk))
        self.free = [deque(ids) for ids in self.slot_ids]
        self.home = list(range(n))   # the instance holding each grid's committed state
        self.home_busy = [False] * n
        self.queue: list[deque] = [deque() for _ in range(n)]
        self.cold = None
        if cold_start:
            for j in range(n):
                self.solver.start(j, A.COLD)
            while self.solver.run(1 << 16) > 0:
                pass
            self.cold = [self.solver.poll(j)[1] for j in range(n)]

    def close(self):
        self.solver.close()

    # ------------------------------------------------------------------
    def _admit(self, req: Request, now: float) -> bool:
        j = req.grid
        s = self.solver
        if self.slot_ids[j]:
            if not self.free[j]:
                return False
            slot = self.free[j].popleft()
            s.copy_grid(self.home[j], slot)
        else:
            if self.home_busy[j]:
                return False
            slot = self.home[j]
            self.home_busy[j] = True
        s.update_loads(slot, req.pd, req.qd)
        s.start(slot, A.WARM)
        req.slot = slot
        req.admitted = now
        return True

    def _complete(self, req: Request, now: float):
        j = req.grid
        s = self.solver
        _, res = s.poll(req.slot)
        req.result = res
        req.finished = now
        if self.slot_ids[j]:
            # commit: the finished slot is the new home, the old home is free
            self.free[j].append(self.home[j])
            self.home[j] = req.slot
        else:
            self.home_busy[j] = False

    def serve(self, requests: list[Request], chunk: int | None = None,
              realtime: bool = True) -> dict:
        """Replay a request stream; arrival times are honoured in wall-clock
        time when realtime, else every request is available at once."""
        s = self.solver
        chunk = chunk or s.tuning()["chunk"]
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        inflight: dict[int, Request] = {}
        done: list[Request] = []
        iters = 0
        t0 = time.perf_counter()
        while pending or inflight or any(self.queue):
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                r = pending.popleft()
                self.queue[r.grid].append(r)
            for j in range(len(self.grids)):
                while self.queue[j] and self._admit(self.queue[j][0], now):
                    r = self.queue[j].popleft()
                    inflight[r.slot] = r
            if inflight:
                s.run(chunk)
                iters += chunk
                now = time.perf_counter() - t0
                for slot in [k for k in inflight if not s.is_running(k)]:
                    r = inflight.pop(slot)
                    self._complete(r, now)
                    done.append(r)
            elif pending and realtime:
                time.sleep(max(0.0, min(pending[0].arrival - now, 0.002)))
        wall = time.perf_counter() - t0
        lat = np.array([r.finished - r.arrival for r in done]) * 1e3
        its = np.array([r.result["inner_iters"] for r in done])
        conv = sum(1 for r in done if r.result["status"] == A.CONVERGED)
        solves = sum(r.result["inner_iters"] * self.grids[r.grid].n_branch for r in done)
        worst = max((max(r.result["r_pri"], r.result["r_dual"], r.result["r_z"]) for r in done),
                    default=0.0)
        return {"requests": len(done), "wall_s": wall,
                "p50_ms": float(np.percentile(lat, 50)) if len(lat) else math.nan,
                "p99_ms": float(np.percentile(lat, 99)) if len(lat) else math.nan,
                "mean_iters": float(its.mean()) if len(its) else math.nan,
                "converged": conv, "requests_per_s": len(done) / wall,
                "branch_solves_per_s": solves / wall, "worst_residual": worst,
                "chunks": iters // max(chunk, 1), "done": done}


def poisson_requests(grids: list[Grid], rate: float, duration: float, seed: int = 5000,
                     lo: float = 0.01, hi: float = 0.03) -> list[Request]:
    """Poisson arrivals at `rate`/s over `duration` s; each request picks a
    grid uniformly and perturbs every bus load by d ~ U(-x, x), x ~ U(lo, hi)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        j = int(rng.integers(len(grids)))
        x = rng.uniform(lo, hi)
        d = rng.uniform(-x, x, grids[j].n_bus)
        g = grids[j]
        out.append(Request(len(out), j, t, g.pd * (1.0 + d), g.qd * (1.0 + d)))
    return out


def serve_one_at_a_time(grids: list[Grid], requests: list[Request],
                        params: A.Params | None = None, device: int = 0,
                        realtime: bool = True) -> dict:
    """Baseline: one handle per grid, one request on the GPU at a time (FIFO)."""
    solvers = [A.Solver(g, params, device=device) for g in grids]
    for s in solvers:
        s.solve(A.COLD)
    pending = deque(sorted(requests, key=lambda r: r.arrival))
    done = []
    t0 = time.perf_counter()
    while pending:
        now = time.perf_counter() - t0
        r = pending[0]
        if realtime and r.arrival > now:
            time.sleep(min(r.arrival - now, 0.002))
            continue
        pending.popleft()
        s = solvers[r.grid]
        s.update_loads(0, r.pd, r.qd)
        res = s.solve(A.WARM)[0]
        r.result = res
        r.finished = time.perf_counter() - t0
        done.append(r)
    wall = time.perf_counter() - t0
    for s in solvers:
        s.close()
    lat = np.array([r.finished - r.arrival for r in done]) * 1e3
    solves = sum(r.result["inner_iters"] * grids[r.grid].n_branch for r in done)
    return {"requests": len(done), "wall_s": wall,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "converged": sum(1 for r in done if r.result["status"] == A.CONVERGED),
            "requests_per_s": len(done) / wall, "branch_solves_per_s": solves / wall,
            "worst_residual": max(max(r.result["r_pri"], r.result["r_dual"], r.result["r_z"])
                                  for r in done)}
