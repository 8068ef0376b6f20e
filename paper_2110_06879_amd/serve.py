"""Warm-start tracking service with continuous batching on one GPU: the
Python side of the library's tracking server (acopf_server_* in acopf.h).

The paper motivates fast tracking of the ACOPF optimum under load changes
(Sec. I, Sec. IV-C): each new load picture is solved warm from the previous
solution. The server, native code in the library, keeps several grids
resident and serves a stream of such requests: per grid a home instance (its
last committed ADMM state) and slot instances within an HBM budget; a request
is admitted between iteration chunks into a free slot (a one-launch device
copy of the home state, its loads, a warm start) and joins the running
launches; a finished slot becomes the grid's home. This module only
marshals requests and results and replays a timed request stream; every step
of a solve runs in the HIP kernels of libacopf.so.

Because every grid of a handle is an independent problem whose arithmetic
does not depend on the other grids in the launch, a request's result is
bitwise the same alone and in the mix (tested).
"""
from __future__ import annotations

import ctypes as C
import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import acopf as A
from .gridgen import Grid


def serving_plan(grids: list[Grid], budget_bytes: float, max_slots_per_grid: int = 4):
    """Slots per grid and the planned footprint for a budget (the library's
    acopf_serving_plan; no device needed). Raises ValueError when the budget
    cannot hold the resident grids (ACOPF_EBUDGET)."""
    lib = A.load()
    cg, keep = A.grid_structs(grids)
    slots = (C.c_int32 * len(grids))()
    used = C.c_double(0.0)
    rc = lib.acopf_serving_plan(cg, len(grids), float(budget_bytes), int(max_slots_per_grid),
                                slots, C.byref(used))
    if rc == A.EBUDGET:
        raise ValueError(lib.acopf_last_error().decode())
    if rc != 0:
        raise A.AcopfError(f"acopf error {rc}: {lib.acopf_last_error().decode()}")
    return list(slots), used.value


def instance_bytes(g: Grid) -> float:
    """The library's estimate of one instance's device footprint."""
    return serving_plan([g], 1e30, 0)[1]


@dataclass
class Request:
    rid: int
    grid: int
    arrival: float          # seconds after the start of the stream
    pd: np.ndarray
    qd: np.ndarray
    submit_delay: float = 0.0   # from the scheduled arrival to the submission
    latency: float = math.nan   # seconds from arrival to the result being seen
    result: dict = field(default_factory=dict)
    slot: int = -1              # handle instance that ran it (its grid's new home)


class TrackingServer:
    """Continuous-batching warm-start server over resident grids (the
    library's acopf_server)."""

    def __init__(self, grids: list[Grid], params: A.Params | None = None,
                 hbm_budget_bytes: float | None = None, max_slots_per_grid: int = 4,
                 device: int = 0, chunk: int | None = None):
        self.lib = A.load()
        self.grids = list(grids)
        self.params = params or A.Params()
        cg, keep = A.grid_structs(self.grids)
        p = self.params.c()
        srv = C.c_void_p()
        rc = self.lib.acopf_server_create(cg, len(self.grids), C.byref(p),
                                          float(hbm_budget_bytes or 0.0),
                                          int(max_slots_per_grid), int(chunk or 0), device,
                                          C.byref(srv))
        if rc == A.EBUDGET:
            raise ValueError(self.lib.acopf_last_error().decode())
        if rc != 0:
            raise A.AcopfError(f"acopf error {rc}: {self.lib.acopf_last_error().decode()}")
        self.srv = srv
        n = len(self.grids)
        slots = (C.c_int32 * n)()
        cold = (A._Result * n)()
        used = C.c_double(0.0)
        h = C.c_void_p()
        self._check(self.lib.acopf_server_info(self.srv, slots, None, cold, C.byref(used),
                                               C.byref(h)))
        self.slots_per_grid = list(slots)
        self.bytes_used = used.value
        self.cold = [c.as_dict() for c in cold]
        # instances: the homes 0..n-1, then each grid's slots
        inst = list(self.grids)
        for j in range(n):
            inst += [self.grids[j]] * self.slots_per_grid[j]
        self.solver = A.Solver.view(h, inst, self.params)

    def _check(self, rc: int):
        if rc != 0:
            raise A.AcopfError(f"acopf error {rc}: {self.lib.acopf_last_error().decode()}")

    def close(self):
        if getattr(self, "srv", None):
            self.lib.acopf_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def home(self) -> list[int]:
        """The instance holding each grid's committed state."""
        out = (C.c_int32 * len(self.grids))()
        self._check(self.lib.acopf_server_info(self.srv, None, out, None, None, None))
        return list(out)

    def submit(self, req: Request):
        pd = np.ascontiguousarray(req.pd, dtype=np.float64)
        qd = np.ascontiguousarray(req.qd, dtype=np.float64)
        self._check(self.lib.acopf_server_submit(self.srv, req.grid, A._dp(pd), A._dp(qd),
                                                 req.rid))

    def step(self) -> tuple[int, int]:
        """Admit, run one chunk, retire; returns (in flight, queued)."""
        f, q = C.c_int32(), C.c_int32()
        self._check(self.lib.acopf_server_step(self.srv, C.byref(f), C.byref(q)))
        return f.value, q.value

    def finished(self) -> list:
        out = []
        buf = (A._Served * 64)()
        while True:
            n = C.c_int32()
            self._check(self.lib.acopf_server_poll(self.srv, buf, 64, C.byref(n)))
            out += [buf[k] for k in range(n.value)]
            if n.value < 64:
                return out

    def serve(self, requests: list[Request], realtime: bool = True) -> dict:
        """Replay a request stream; arrival times are honoured in wall-clock
        time when realtime, else every request is available at once."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        by_id = {r.rid: r for r in requests}
        done: list[Request] = []
        in_flight = queued = 0
        t0 = time.perf_counter()
        while pending or in_flight or queued:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                r = pending.popleft()
                r.submit_delay = max(0.0, now - r.arrival) if realtime else 0.0
                self.submit(r)
                queued += 1
            if in_flight or queued:
                in_flight, queued = self.step()
                for d in self.finished():
                    r = by_id[d.request_id]
                    r.result = d.result.as_dict()
                    r.slot = d.instance
                    r.latency = r.submit_delay + (d.finished - d.submitted)
                    done.append(r)
            elif pending and realtime:
                time.sleep(max(0.0, min(pending[0].arrival - now, 0.002)))
        wall = time.perf_counter() - t0
        lat = np.array([r.latency for r in done]) * 1e3
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
                "done": done}


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
        r.latency = time.perf_counter() - t0 - r.arrival
        done.append(r)
    wall = time.perf_counter() - t0
    for s in solvers:
        s.close()
    lat = np.array([r.latency for r in done]) * 1e3
    solves = sum(r.result["inner_iters"] * grids[r.grid].n_branch for r in done)
    return {"requests": len(done), "wall_s": wall,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "converged": sum(1 for r in done if r.result["status"] == A.CONVERGED),
            "requests_per_s": len(done) / wall, "branch_solves_per_s": solves / wall,
            "worst_residual": max(max(r.result["r_pri"], r.result["r_dual"], r.result["r_z"])
                                  for r in done)}
