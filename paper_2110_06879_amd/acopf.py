"""Python binding of the HIP library ``libacopf.so`` (C ABI in include/acopf.h).

Argument marshalling only: every step of the ADMM iteration runs in the HIP
kernels behind the C ABI. There is no CPU fallback; if the library has not
been built, loading raises.
"""
from __future__ import annotations

import ctypes as C
import json
import os
from dataclasses import asdict, dataclass

import numpy as np

from .gridgen import Grid

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libacopf.so")

COLD, WARM, CONTINUE = 0, 1, 2
CONVERGED, MAX_ITER, NUMERICAL = 0, 1, 2
EINVAL, ENOMEM, EDEVICE, ESTATE, EBUDGET = -1, -2, -3, -4, -5
U, V, Z, Y, LAMBDA, BRANCH_X, BRANCH_LTIL, BRANCH_RTIL, SCALARS, PD, QD, HISTORY, STATS = range(13)
BRANCH_ALPHA = 13
SOLUTION = 14
STATE_CODES = {"u": U, "v": V, "z": Z, "y": Y, "lam": LAMBDA, "bx": BRANCH_X,
               "ltil": BRANCH_LTIL, "rtil": BRANCH_RTIL, "scalars": SCALARS,
               "pd": PD, "qd": QD, "calpha": BRANCH_ALPHA}
STATS_NAMES = ("branch_solves", "flops", "trig", "tron_calls", "tron_iters", "n_fgh",
               "n_f", "cauchy_trials", "cg_iters", "chol_attempts", "ps_trials",
               "al_iters", "tron_converged", "tron_maxit", "tron_stall", "reserved")
SCALAR_NAMES = ("beta", "znorm_prev", "r_pri", "r_dual", "r_z", "outer",
                "inner_total", "inner_in_outer", "status")
EXPORTS = ("acopf_default_params", "acopf_create", "acopf_solve", "acopf_update_loads",
           "acopf_get_state", "acopf_set_state", "acopf_get_sizes", "acopf_set_profiling",
           "acopf_get_timing", "acopf_destroy", "acopf_last_error", "acopf_start",
           "acopf_run", "acopf_poll", "acopf_copy_grid", "acopf_snapshot",
           "acopf_set_tuning", "acopf_get_tuning", "acopf_autotune", "acopf_quality",
           "acopf_update_gen_bounds", "acopf_set_counting", "acopf_peak_hbm",
           "acopf_peak_fp64", "acopf_quality_noalloc", "acopf_device_memory",
           "acopf_serving_plan", "acopf_server_create", "acopf_server_submit",
           "acopf_server_step", "acopf_server_poll", "acopf_server_info",
           "acopf_server_destroy")
QUALITY_NAMES = ("max_violation", "balance_p", "balance_q", "line_limit", "voltage_limit",
                 "angle_limit")


class AcopfError(RuntimeError):
    pass


class _Grid(C.Structure):
    _fields_ = [
        ("n_bus", C.c_int32), ("n_gen", C.c_int32), ("n_branch", C.c_int32),
        ("ref_bus", C.c_int32), ("base_mva", C.c_double),
    ] + [(n, C.c_void_p) for n in (
        "pd", "qd", "gs", "bs", "vmin", "vmax", "gen_bus", "pmin", "pmax", "qmin",
        "qmax", "c2", "c1", "c0", "br_from", "br_to", "r", "x", "b", "tap",
        "shift", "rate")]


class _Params(C.Structure):
    _fields_ = [
        ("rho_pq", C.c_double), ("rho_va", C.c_double), ("obj_scale", C.c_double),
        ("rate_scale", C.c_double), ("beta0", C.c_double), ("beta_gamma", C.c_double),
        ("beta_omega", C.c_double), ("beta_max", C.c_double), ("lambda_max", C.c_double),
        ("eps_pri", C.c_double), ("eps_dual", C.c_double), ("eps_z", C.c_double),
        ("max_outer", C.c_int32), ("max_inner", C.c_int32),
        ("tron_gtol", C.c_double), ("tron_ftol", C.c_double), ("tron_maxit", C.c_int32),
        ("al_rho0", C.c_double), ("al_rho_growth", C.c_double), ("al_rho_max", C.c_double),
        ("al_tol", C.c_double), ("al_shrink", C.c_double), ("al_maxit", C.c_int32),
    ]


class _Tuning(C.Structure):
    _fields_ = [("xstep_block", C.c_int32), ("bus_block", C.c_int32),
                ("chunk", C.c_int32), ("use_graph", C.c_int32), ("xstep_waves", C.c_int32),
                ("xstep_per_lane", C.c_int32), ("lanes", C.c_int32)]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


TUNING_FIELDS = tuple(n for n, _ in _Tuning._fields_)


class _Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("inner_iters", C.c_int32),
                ("outer_iters", C.c_int32), ("branch_failures", C.c_int32),
                ("objective", C.c_double), ("r_pri", C.c_double), ("r_dual", C.c_double),
                ("r_z", C.c_double), ("beta", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class _Served(C.Structure):
    _fields_ = [("request_id", C.c_int64), ("grid", C.c_int32), ("instance", C.c_int32),
                ("submitted", C.c_double), ("admitted", C.c_double), ("finished", C.c_double),
                ("result", _Result)]


@dataclass
class Params:
    """Method parameters; field names and order follow acopf_params."""
    rho_pq: float = 400.0
    rho_va: float = 4000.0
    obj_scale: float = 0.01
    rate_scale: float = 0.99
    beta0: float = 1e4
    beta_gamma: float = 6.0
    beta_omega: float = 0.8
    beta_max: float = 1e5
    lambda_max: float = 1e12
    eps_pri: float = 1e-4
    eps_dual: float = 1e-4
    eps_z: float = 1e-4
    max_outer: int = 20
    max_inner: int = 1000
    tron_gtol: float = 1e-6
    tron_ftol: float = 1e-12
    tron_maxit: int = 50
    al_rho0: float = 10.0
    al_rho_growth: float = 10.0
    al_rho_max: float = 1e8
    al_tol: float = 1e-6
    al_shrink: float = 0.25
    al_maxit: int = 20

    def c(self) -> _Params:
        return _Params(**asdict(self))


_lib = None


def load(path: str | None = None) -> C.CDLL:
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise AcopfError(f"{p} not built: run __graft_entry__.build() or "
                         "python -m paper_2110_06879_amd.build")
    lib = C.CDLL(p)
    vp, dp, i32, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64
    lib.acopf_default_params.argtypes = [C.POINTER(_Params)]
    lib.acopf_default_params.restype = None
    lib.acopf_create.argtypes = [C.POINTER(_Grid), i32, C.POINTER(_Params), i32, vp,
                                 C.POINTER(vp)]
    lib.acopf_solve.argtypes = [vp, i32, i32, C.POINTER(_Result)]
    lib.acopf_update_loads.argtypes = [vp, i32, dp, dp]
    lib.acopf_get_state.argtypes = [vp, i32, i32, dp, i64]
    lib.acopf_set_state.argtypes = [vp, i32, i32, dp, i64]
    lib.acopf_get_sizes.argtypes = [vp, i32, C.POINTER(C.c_int64)]
    lib.acopf_get_timing.argtypes = [vp, dp]
    lib.acopf_set_profiling.argtypes = [vp, i32]
    lib.acopf_start.argtypes = [vp, i32, i32, i32]
    lib.acopf_run.argtypes = [vp, i32, C.POINTER(i32)]
    lib.acopf_poll.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(_Result)]
    lib.acopf_copy_grid.argtypes = [vp, i32, i32]
    lib.acopf_snapshot.argtypes = [vp, i32]
    lib.acopf_set_tuning.argtypes = [vp, C.POINTER(_Tuning)]
    lib.acopf_get_tuning.argtypes = [vp, C.POINTER(_Tuning)]
    lib.acopf_autotune.argtypes = [vp, i32, C.POINTER(_Tuning)]
    lib.acopf_quality.argtypes = [vp, i32, dp]
    lib.acopf_quality_noalloc.argtypes = [vp, i32, dp]
    lib.acopf_update_gen_bounds.argtypes = [vp, i32, dp, dp]
    lib.acopf_set_counting.argtypes = [vp, i32]
    lib.acopf_destroy.argtypes = [vp]
    lib.acopf_destroy.restype = None
    lib.acopf_last_error.restype = C.c_char_p
    lib.acopf_peak_hbm.argtypes = [i64, i32, dp]
    lib.acopf_peak_fp64.argtypes = [i32, dp]
    lib.acopf_device_memory.argtypes = [i32, C.POINTER(C.c_int64)]
    lib.acopf_serving_plan.argtypes = [C.POINTER(_Grid), i32, C.c_double, i32,
                                       C.POINTER(i32), dp]
    lib.acopf_server_create.argtypes = [C.POINTER(_Grid), i32, C.POINTER(_Params), C.c_double,
                                        i32, i32, i32, C.POINTER(vp)]
    lib.acopf_server_submit.argtypes = [vp, i32, dp, dp, i64]
    lib.acopf_server_step.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
    lib.acopf_server_poll.argtypes = [vp, C.POINTER(_Served), i32, C.POINTER(i32)]
    lib.acopf_server_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(_Result),
                                      dp, C.POINTER(vp)]
    lib.acopf_server_destroy.argtypes = [vp]
    lib.acopf_server_destroy.restype = None
    for name in ("acopf_create", "acopf_solve", "acopf_update_loads", "acopf_get_state",
                 "acopf_set_state", "acopf_get_sizes", "acopf_get_timing",
                 "acopf_set_profiling", "acopf_start", "acopf_run", "acopf_poll",
                 "acopf_copy_grid", "acopf_snapshot", "acopf_set_tuning",
                 "acopf_get_tuning", "acopf_autotune", "acopf_quality",
                 "acopf_quality_noalloc",
                 "acopf_update_gen_bounds", "acopf_set_counting", "acopf_peak_hbm",
                 "acopf_peak_fp64", "acopf_device_memory", "acopf_serving_plan",
                 "acopf_server_create", "acopf_server_submit", "acopf_server_step",
                 "acopf_server_poll", "acopf_server_info"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def peak_hbm(nbytes: int = 1 << 30, iters: int = 20) -> float:
    """Achievable streaming-copy bandwidth of the current device, GB/s (read
    plus written bytes): a measurement helper, not part of the method."""
    lib = load()
    out = C.c_double(0.0)
    rc = lib.acopf_peak_hbm(int(nbytes), int(iters), C.byref(out))
    if rc != 0:
        raise AcopfError(f"acopf error {rc}: {lib.acopf_last_error().decode()}")
    return out.value


def device_memory(device: int = 0) -> tuple[int, int]:
    """(free, total) bytes of device memory (hipMemGetInfo)."""
    lib = load()
    out = (C.c_int64 * 2)()
    rc = lib.acopf_device_memory(device, out)
    if rc != 0:
        raise AcopfError(f"acopf_device_memory: {lib.acopf_last_error().decode()}")
    return int(out[0]), int(out[1])


def peak_fp64(iters: int = 200000) -> float:
    """Achievable FP64 fused multiply-add rate of the current device,
    TFLOP/s: a measurement helper, not part of the method."""
    lib = load()
    out = C.c_double(0.0)
    rc = lib.acopf_peak_fp64(int(iters), C.byref(out))
    if rc != 0:
        raise AcopfError(f"acopf error {rc}: {lib.acopf_last_error().decode()}")
    return out.value


def default_params() -> dict:
    p = _Params()
    load().acopf_default_params(C.byref(p))
    return {n: getattr(p, n) for n, _ in p._fields_}


def tuning_key(grids) -> str:
    """Workload shape that a launch tuning is chosen for: number of grids and
    their total buses, branches and rated branches."""
    gs = [grids] if isinstance(grids, Grid) else list(grids)
    nb = sum(int(g.n_bus) for g in gs)
    nl = sum(int(g.n_branch) for g in gs)
    n6 = sum(int(np.count_nonzero(np.asarray(g.rate) > 0)) for g in gs)
    return f"grids={len(gs)} buses={nb} branches={nl} rated={n6}"


def load_tuning(path: str, key: str) -> dict | None:
    """The tuning stored for `key` in the JSON file at `path`, or None (no
    file, no entry, or an entry without the tuning fields)."""
    try:
        with open(path) as fh:
            table = json.load(fh)
    except (OSError, ValueError):
        return None
    t = table.get(key) if isinstance(table, dict) else None
    if not isinstance(t, dict) or any(k not in t for k in TUNING_FIELDS):
        return None
    return {k: int(t[k]) for k in TUNING_FIELDS}


def save_tuning(path: str, key: str, tuning: dict) -> None:
    """Store `tuning` under `key` in the JSON file at `path`, keeping the other
    entries; written to a temporary file and renamed into place."""
    try:
        with open(path) as fh:
            table = json.load(fh)
        if not isinstance(table, dict):
            table = {}
    except (OSError, ValueError):
        table = {}
    table[key] = {k: int(tuning[k]) for k in TUNING_FIELDS}
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def grid_structs(grids: list[Grid]):
    """acopf_grid structs of the grids, and the arrays they point into (keep
    them alive for the call)."""
    keep = []
    cg = (_Grid * len(grids))()
    for k, g in enumerate(grids):
        arrs = {}
        for n in ("pd", "qd", "gs", "bs", "vmin", "vmax", "pmin", "pmax", "qmin",
                  "qmax", "c2", "c1", "c0", "r", "x", "b", "tap", "shift", "rate"):
            arrs[n] = np.ascontiguousarray(getattr(g, n), dtype=np.float64)
        for n in ("gen_bus", "br_from", "br_to"):
            arrs[n] = np.ascontiguousarray(getattr(g, n), dtype=np.int32)
        keep.append(arrs)
        cg[k] = _Grid(n_bus=g.n_bus, n_gen=g.n_gen, n_branch=g.n_branch,
                      ref_bus=g.ref_bus, base_mva=g.base_mva,
                      **{n: a.ctypes.data for n, a in arrs.items()})
    return cg, keep


class Solver:
    """A handle over one or more grids resident on one GPU."""

    def __init__(self, grids: Grid | list[Grid], params: Params | None = None,
                 device: int = 0, stream=None):
        self.lib = load()
        self.grids = [grids] if isinstance(grids, Grid) else list(grids)
        self.params = params or Params()
        cg, self._keep = grid_structs(self.grids)
        sp = None
        if stream is not None:
            sp = C.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        self._p = self.params.c()
        h = C.c_void_p()
        rc = self.lib.acopf_create(cg, len(self.grids), C.byref(self._p), device, sp,
                                   C.byref(h))
        self._check(rc)
        self.h = h
        self._keep = None
        self._owned = True

    @classmethod
    def view(cls, handle, grids: list[Grid], params: Params | None = None) -> "Solver":
        """A Solver over a handle owned elsewhere (a tracking server's): its
        calls act on that handle, and closing it leaves the handle alone."""
        self = cls.__new__(cls)
        self.lib = load()
        self.grids = list(grids)
        self.params = params or Params()
        self._keep = None
        self.h = handle
        self._owned = False
        return self

    def _check(self, rc: int):
        if rc != 0:
            raise AcopfError(f"acopf error {rc}: {self.lib.acopf_last_error().decode()}")

    def close(self):
        if getattr(self, "h", None):
            if getattr(self, "_owned", True):
                self.lib.acopf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def solve(self, mode: int = COLD, fixed_iters: int = 0) -> list[dict]:
        res = (_Result * len(self.grids))()
        self._check(self.lib.acopf_solve(self.h, mode, fixed_iters, res))
        return [r.as_dict() for r in res]

    def update_gen_bounds(self, grid: int, pmin, pmax):
        lo = np.ascontiguousarray(pmin, dtype=np.float64)
        hi = np.ascontiguousarray(pmax, dtype=np.float64)
        self._check(self.lib.acopf_update_gen_bounds(self.h, grid, _dp(lo), _dp(hi)))

    def update_loads(self, grid: int, pd, qd):
        pd = np.ascontiguousarray(pd, dtype=np.float64)
        qd = np.ascontiguousarray(qd, dtype=np.float64)
        self._check(self.lib.acopf_update_loads(self.h, grid, _dp(pd), _dp(qd)))

    def _size(self, grid: int, code: int) -> int:
        g = self.grids[grid]
        m = 2 * g.n_gen + 8 * g.n_branch
        return {U: m, V: m, Z: m, Y: m, LAMBDA: m, BRANCH_X: 6 * g.n_branch,
                BRANCH_LTIL: 2 * g.n_branch, BRANCH_RTIL: g.n_branch,
                BRANCH_ALPHA: g.n_branch, SCALARS: 9,
                PD: g.n_bus, QD: g.n_bus, STATS: 16,
                SOLUTION: 2 * g.n_gen + 2 * g.n_bus + 4 * g.n_branch}[code]

    def get(self, name: str, grid: int = 0) -> np.ndarray:
        code = STATE_CODES[name]
        out = np.empty(self._size(grid, code))
        self._check(self.lib.acopf_get_state(self.h, grid, code, _dp(out), out.size))
        return out

    def set(self, name: str, val, grid: int = 0):
        code = STATE_CODES[name]
        a = np.ascontiguousarray(val, dtype=np.float64)
        self._check(self.lib.acopf_set_state(self.h, grid, code, _dp(a), a.size))

    def solution(self, grid: int = 0) -> dict:
        """The recovered ADMM solution (Sec. IV-A) of one grid, input order:
        generator outputs pg, qg; bus voltage magnitudes vm and angles va;
        branch flows pij, qij, pji, qji recomputed from the bus voltages."""
        g = self.grids[grid]
        out = np.empty(self._size(grid, SOLUTION))
        self._check(self.lib.acopf_get_state(self.h, grid, SOLUTION, _dp(out), out.size))
        ng, nb, nl = g.n_gen, g.n_bus, g.n_branch
        cut = np.cumsum([ng, ng, nb, nb, nl, nl, nl, nl])[:-1]
        parts = np.split(out, cut)
        return dict(zip(("pg", "qg", "vm", "va", "pij", "qij", "pji", "qji"), parts))

    def scalars(self, grid: int = 0) -> dict:
        return dict(zip(SCALAR_NAMES, self.get("scalars", grid).tolist()))

    def history(self, grid: int = 0) -> np.ndarray:
        n = int(min(self.scalars(grid)["inner_total"], 1 << 15))
        out = np.empty(6 * n)
        self._check(self.lib.acopf_get_state(self.h, grid, HISTORY, _dp(out), out.size))
        return out.reshape(-1, 6)

    def stats(self) -> dict:
        out = np.empty(16)
        self._check(self.lib.acopf_get_state(self.h, 0, STATS, _dp(out), 16))
        return {n: int(v) for n, v in zip(STATS_NAMES, out)}

    # continuous batching -------------------------------------------------
    def start(self, grid: int, mode: int = WARM, fixed_iters: int = 0):
        self._check(self.lib.acopf_start(self.h, grid, mode, fixed_iters))

    def run(self, max_iters: int = 1 << 20) -> int:
        n = C.c_int32()
        self._check(self.lib.acopf_run(self.h, max_iters, C.byref(n)))
        return int(n.value)

    def poll(self, grid: int):
        """(is_running, result dict)."""
        r = _Result()
        n = C.c_int32()
        self._check(self.lib.acopf_poll(self.h, grid, C.byref(n), C.byref(r)))
        return bool(n.value), r.as_dict()

    def is_running(self, grid: int) -> bool:
        n = C.c_int32()
        self._check(self.lib.acopf_poll(self.h, grid, C.byref(n), None))
        return bool(n.value)

    def copy_grid(self, src: int, dst: int):
        self._check(self.lib.acopf_copy_grid(self.h, src, dst))

    def snapshot(self, restore: bool = False):
        self._check(self.lib.acopf_snapshot(self.h, 1 if restore else 0))

    def set_tuning(self, **kw):
        t = _Tuning(**{**self.tuning(), **kw})
        self._check(self.lib.acopf_set_tuning(self.h, C.byref(t)))

    def tuning(self) -> dict:
        t = _Tuning()
        self._check(self.lib.acopf_get_tuning(self.h, C.byref(t)))
        return t.as_dict()

    def quality(self, grid: int = 0) -> dict:
        """||c(x)||_inf over eq. acopf at the grid's current ADMM solution and
        its parts (power balance p and q, line, voltage and angle limits)."""
        out = np.zeros(6)
        self._check(self.lib.acopf_quality(self.h, grid, _dp(out)))
        return dict(zip(QUALITY_NAMES, out.tolist()))

    def autotune(self, iters: int = 32, cache: str | None = None) -> dict:
        """Measure the launch-shape candidates on this handle's grids and keep
        the fastest (state unchanged). With `cache`, a JSON file of earlier
        results keyed by the workload's shape (tuning_key): a hit applies
        the stored tuning without measuring, a miss measures and stores."""
        key = tuning_key(self.grids)
        if cache is not None:
            hit = load_tuning(cache, key)
            if hit is not None:
                self.set_tuning(**hit)
                return self.tuning()
        t = _Tuning()
        self._check(self.lib.acopf_autotune(self.h, iters, C.byref(t)))
        out = t.as_dict()
        if cache is not None:
            save_tuning(cache, key, out)
        return out

    def set_counting(self, on: bool = True):
        """Count algorithmic flops and TRON events into stats() (slower)."""
        self._check(self.lib.acopf_set_counting(self.h, 1 if on else 0))

    def set_profiling(self, on: bool = True):
        self._check(self.lib.acopf_set_profiling(self.h, int(on)))

    def timing(self) -> dict:
        out = np.zeros(5)
        self._check(self.lib.acopf_get_timing(self.h, _dp(out)))
        keys = ("xstep_ms", "bus_ms", "ctl_ms", "outer_ms")
        d = dict(zip(keys, out[:4].tolist()))
        d["iters"] = int(out[4])
        return d
