"""Batched and served workloads on one GPU, each against the plain
one-grid-per-launch method on the same device and inputs.

  python -m paper_2110_06879_amd.bench_systems --batch   # 64 uneven grids, cold, to 1e-4
  python -m paper_2110_06879_amd.bench_systems --serve   # Poisson tracking requests
  python -m paper_2110_06879_amd.bench_systems --track   # 30-period horizon, ramp limits
  python -m paper_2110_06879_amd.bench_systems --lanes-multigrid  # launch lanes, 1-4 x 70k grids
  python -m paper_2110_06879_amd.bench_systems --grid-scaling     # 2k to 1.12M buses; 1-16 x 70k
  python -m paper_2110_06879_amd.bench_systems --lanes-trace      # 2 x 70k at two lanes (for a trace)

Prints one JSON line per experiment.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import acopf as A
from . import serve as S
from . import tracking as T
from .gridgen import batch_grids, config_grid, gridgen, serving_grids


def batch(n_grids: int, tune_iters: int) -> dict:
    grids = batch_grids(n_grids)
    sizes = [g.n_bus for g in grids]
    params = A.Params()
    # batched: every grid in one handle, one set of launches per iteration
    s = A.Solver(grids, params)
    tuning = s.autotune(tune_iters) if tune_iters > 0 else s.tuning()
    t0 = time.perf_counter()
    res = s.solve(A.COLD)
    tb = time.perf_counter() - t0
    s.close()
    conv_b = sum(1 for r in res if r["status"] == A.CONVERGED)
    solves_b = sum(r["inner_iters"] * g.n_branch for r, g in zip(res, grids))
    worst_b = max(max(r["r_pri"], r["r_dual"], r["r_z"]) for r in res)
    # plain: one handle and one launch sequence per grid, one grid at a time
    tp = 0.0
    solves_p = 0
    conv_p = 0
    worst_p = 0.0
    for g in grids:
        with A.Solver(g, params) as sp:
            t1 = time.perf_counter()
            r = sp.solve(A.COLD)[0]
            tp += time.perf_counter() - t1
            solves_p += r["inner_iters"] * g.n_branch
            conv_p += r["status"] == A.CONVERGED
            worst_p = max(worst_p, r["r_pri"], r["r_dual"], r["r_z"])
    return {"experiment": "batched", "grids": n_grids, "total_buses": int(sum(sizes)),
            "total_branches": int(sum(g.n_branch for g in grids)),
            "min_buses": int(min(sizes)), "max_buses": int(max(sizes)), "tuning": tuning,
            "batched": {"seconds": tb, "branch_solves_per_s": solves_b / tb,
                        "converged": conv_b, "worst_residual": worst_b,
                        "max_iters": int(max(r["inner_iters"] for r in res))},
            "one_grid_per_launch": {"seconds": tp, "branch_solves_per_s": solves_p / tp,
                                    "converged": conv_p, "worst_residual": worst_p},
            "speedup": tp / tb}


def serve(duration: float, rate: float, with_70k: bool, baseline: bool,
          chunk: int | None = None, lanes: int | None = None) -> dict:
    grids = serving_grids(with_70k=with_70k)
    reqs = S.poisson_requests(grids, rate, duration)
    srv = S.TrackingServer(grids, chunk=chunk)
    if lanes:
        srv.solver.set_tuning(lanes=lanes)
    tuning = srv.solver.tuning()
    out = srv.serve(reqs, realtime=True)
    slots = srv.slots_per_grid
    srv.close()
    out.pop("done")
    print(f"continuous batching: {len(reqs)} requests served", file=sys.stderr, flush=True)
    res = {"experiment": "served", "grids": len(grids),
           "buses": [g.n_bus for g in grids], "rate_per_s": rate, "duration_s": duration,
           "slots_per_grid": slots, "tuning": tuning, "continuous_batching": out}
    if baseline:
        reqs2 = S.poisson_requests(grids, rate, duration)
        b = S.serve_one_at_a_time(grids, reqs2, realtime=True)
        res["one_request_at_a_time"] = b
        print(f"one at a time: {len(reqs2)} requests served", file=sys.stderr, flush=True)
    return res


def lanes_multigrid(iters: int = 200) -> dict:
    """Launch lanes on handles of one to four copies of the 70k-bus grid
    (us per grid-iteration over `iters` iterations after a 20-iteration cold
    start, at one and two lanes), two one-grid handles run from two host
    threads on their own streams against one after the other, and the
    64-grid batch cold to 1e-4 at one and two lanes; every lane count's
    iterates are compared bitwise."""
    import hashlib
    import threading
    import torch
    g = config_grid("c3_70kbus")

    def digest(s, k):
        m = hashlib.sha256()
        for key in ("u", "v", "z", "y", "lam", "bx"):
            m.update(s.get(key, k).tobytes())
        return m.hexdigest()

    out = {"experiment": "lanes_multigrid", "iterations": iters, "us_per_grid_iteration": {}}
    same = True
    for n in (1, 2, 3, 4):
        ref = None
        for lanes in ((1, 2) if n > 1 else (1,)):
            with A.Solver([g] * n) as s:
                s.set_tuning(lanes=lanes)
                s.solve(A.COLD, 20)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.solve(A.CONTINUE, iters)
                t = time.perf_counter() - t0
                out["us_per_grid_iteration"][f"{n}x70k lanes={lanes}"] = t / (iters * n) * 1e6
                d = [digest(s, k) for k in range(n)]
                same = same and (ref is None or d == ref)
                ref = d
        print(f"{n} x 70k done", file=sys.stderr, flush=True)
    s1, s2 = A.Solver(g), A.Solver(g)
    for s in (s1, s2):
        s.solve(A.COLD, 20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s1.solve(A.CONTINUE, iters)
    s2.solve(A.CONTINUE, iters)
    seq = time.perf_counter() - t0
    for s in (s1, s2):
        s.solve(A.COLD, 20)
    ts = [threading.Thread(target=lambda s=s: s.solve(A.CONTINUE, iters)) for s in (s1, s2)]
    t0 = time.perf_counter()
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    conc = time.perf_counter() - t0
    same = same and digest(s1, 0) == digest(s2, 0)
    s1.close()
    s2.close()
    out["two_handles_us_per_grid_iteration"] = {"one_after_the_other": seq / (2 * iters) * 1e6,
                                                "two_threads": conc / (2 * iters) * 1e6}
    gs = batch_grids(64)
    out["batch64_seconds"] = {}
    for lanes in (1, 2):
        with A.Solver(gs) as s:
            s.set_tuning(lanes=lanes)
            t0 = time.perf_counter()
            r = s.solve(A.COLD)
            out["batch64_seconds"][f"lanes={lanes}"] = time.perf_counter() - t0
            out["batch64_converged"] = sum(1 for x in r if x["status"] == A.CONVERGED)
    out["bitwise_equal"] = same
    return out


def grid_scaling(iters: int = 100) -> dict:
    """Throughput against size: single grids of the 70k recipe's proportions
    (one generator per 7 buses, 1.257 branches per bus, 30% rated, load
    factor 0.2) from 2,000 to 1,120,000 buses, and handles of 1, 4 and 16
    copies of the 70k-bus grid at two launch lanes. Each point: a cold start
    of 20 iterations, then `iters` timed iterations between two device
    synchronizations; device memory held by the handle from the allocator's
    free-memory counter."""
    import torch
    from .gridgen import LOAD_FACTOR

    def point(grids, lanes):
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        with A.Solver(grids) as s:
            if lanes:
                s.set_tuning(lanes=lanes)
            s.solve(A.COLD, 20)
            torch.cuda.synchronize()
            held = free0 - torch.cuda.mem_get_info()[0]
            t0 = time.perf_counter()
            s.solve(A.CONTINUE, iters)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / iters
        nbr = sum(g.n_branch for g in grids)
        return {"buses": int(sum(g.n_bus for g in grids)), "branches": int(nbr),
                "us_per_iteration": t * 1e6, "branch_solves_per_s": nbr / t,
                "device_bytes": int(held)}

    out = {"experiment": "grid_scaling", "iterations": iters, "single": [], "copies_of_70k": []}
    for k, nb in enumerate((2000, 10000, 35000, 70000, 140000, 280000, 560000, 1120000)):
        g = gridgen(nb, nb // 7, int(round(nb * 88 / 70)), 0.3, 900 + k,
                    load_factor=LOAD_FACTOR)
        out["single"].append(point([g], None))
        print(f"single grid {nb} buses done", file=sys.stderr, flush=True)
    g = config_grid("c3_70kbus")
    for n in (1, 4, 16):
        out["copies_of_70k"].append({"grids": n, **point([g] * n, 2 if n > 1 else None)})
        print(f"{n} x 70k done", file=sys.stderr, flush=True)
    return out


def lanes_trace(iters: int = 64) -> dict:
    """Two copies of the 70k-bus grid in one handle at two launch lanes: a
    cold start of 20 iterations, then `iters` iterations, for a kernel trace
    of how the lanes' launches overlap."""
    import torch
    g = config_grid("c3_70kbus")
    with A.Solver([g, g]) as s:
        s.set_tuning(lanes=2)
        s.solve(A.COLD, 20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.solve(A.CONTINUE, iters)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
    return {"experiment": "lanes_trace", "grids": 2, "lanes": 2, "iterations": iters,
            "us_per_grid_iteration": t / (2 * iters) * 1e6}


def track(names, periods: int) -> dict:
    out = {"experiment": "tracking", "periods": periods, "drift": 0.05, "ramp": 0.02,
           "grids": {}}
    for name in names:
        g = config_grid(name)
        with A.Solver(g) as s:
            recs = T.track(s, g, 0, periods=periods)
        warm = recs[1:]
        secs = np.array([r["seconds"] for r in warm])
        out["grids"][name] = {
            "n_bus": g.n_bus, "cold_seconds": recs[0]["seconds"],
            "cold_iters": recs[0]["inner_iters"],
            "warm_seconds_p50": float(np.percentile(secs, 50)) if secs.size else None,
            "warm_seconds_max": float(secs.max()) if secs.size else None,
            "horizon_seconds": float(sum(r["seconds"] for r in recs)),
            "warm_iters_mean": float(np.mean([r["inner_iters"] for r in warm])) if warm else None,
            "converged": int(sum(1 for r in recs if r["status"] == A.CONVERGED)),
            "max_violation_max": float(max(r["max_violation"] for r in recs)),
            "ramp_ratio_max": float(max(r["ramp_ratio"] for r in recs)),
            "periods": recs}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--batch", action="store_true")
    ap.add_argument("--serve", action="store_true")
    ap.add_argument("--grids", type=int, default=64)
    ap.add_argument("--tune-iters", type=int, default=0,
                    help="batch: autotune the launch shape over this many iterations first "
                         "(0: the library's defaults)")
    ap.add_argument("--duration", type=float, default=10.0)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--no-70k", action="store_true")
    ap.add_argument("--no-baseline", action="store_true")
    ap.add_argument("--chunk", type=int, default=None,
                    help="serving: iterations between admissions (default: the tuned chunk)")
    ap.add_argument("--lanes", type=int, default=None,
                    help="serving: launch lanes of the server's handle (default: the library's)")
    ap.add_argument("--track", action="store_true")
    ap.add_argument("--periods", type=int, default=30)
    ap.add_argument("--lanes-multigrid", action="store_true")
    ap.add_argument("--grid-scaling", action="store_true")
    ap.add_argument("--lanes-trace", action="store_true")
    args = ap.parse_args()
    if args.batch:
        print(json.dumps(batch(args.grids, args.tune_iters)), flush=True)
    if args.serve:
        print(json.dumps(serve(args.duration, args.rate, not args.no_70k,
                               not args.no_baseline, args.chunk, args.lanes)), flush=True)
    if args.track:
        print(json.dumps(track(["c2_2kbus", "c3_70kbus"], args.periods)), flush=True)
    if args.lanes_multigrid:
        print(json.dumps(lanes_multigrid()), flush=True)
    if args.grid_scaling:
        print(json.dumps(grid_scaling()), flush=True)
    if args.lanes_trace:
        print(json.dumps(lanes_trace()), flush=True)


if __name__ == "__main__":
    sys.exit(main())
