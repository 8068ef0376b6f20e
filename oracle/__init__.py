"""ctypes binding of the serial FP64 CPU oracle (``acopf_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the plain reference implementation that the HIP
path is checked against. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The product path
(``paper_2110_06879_amd``) never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, asdict, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "acopf_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")

__all__ = ["OracleParams", "Oracle", "build", "load", "branch_eval",
           "branch_solve", "tron_generic", "STATE"]


def build(verbose: bool = False) -> str:
    """Compile the oracle with g++ (-O2, no FP contraction). The explicit
    fused multiply-adds of the source (std::fma) use the FMA instructions of
    x86-64 (-mfma); they are correctly rounded either way, in hardware or in
    the C library."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    tmp = _LIB_PATH + ".tmp"
    cmd = ["g++", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c++17",
           "-mfma", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC]
    out = subprocess.run(cmd, capture_output=True, text=True)
    if out.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + out.stderr)
    os.replace(tmp, _LIB_PATH)
    if verbose:
        print("built", _LIB_PATH)
    return _LIB_PATH


QUALITY_NAMES = ("max_violation", "balance_p", "balance_q", "line_limit", "voltage_limit",
                 "angle_limit")


class _Params(C.Structure):
    _fields_ = [
        ("rho_pq", C.c_double), ("rho_va", C.c_double),
        ("obj_scale", C.c_double), ("rate_scale", C.c_double),
        ("beta0", C.c_double), ("beta_gamma", C.c_double),
        ("beta_omega", C.c_double), ("beta_max", C.c_double),
        ("lambda_max", C.c_double),
        ("eps_pri", C.c_double), ("eps_dual", C.c_double), ("eps_z", C.c_double),
        ("max_outer", C.c_int32), ("max_inner", C.c_int32),
        ("tron_gtol", C.c_double), ("tron_ftol", C.c_double),
        ("tron_maxit", C.c_int32),
        ("al_rho0", C.c_double), ("al_rho_growth", C.c_double),
        ("al_rho_max", C.c_double), ("al_tol", C.c_double),
        ("al_shrink", C.c_double), ("al_maxit", C.c_int32),
    ]


class _Stats(C.Structure):
    _fields_ = [(n, C.c_longlong) for n in (
        "branch_solves", "tron_calls", "tron_iters", "n_fgh", "n_f",
        "cauchy_trials", "cg_iters", "chol_attempts", "ps_trials", "al_iters",
        "tron_converged", "tron_maxit", "tron_stall", "flops", "trig")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class _Grid(C.Structure):
    _fields_ = [
        ("n_bus", C.c_int32), ("n_gen", C.c_int32), ("n_branch", C.c_int32),
        ("ref_bus", C.c_int32), ("base_mva", C.c_double),
    ] + [(n, C.c_void_p) for n in (
        "pd", "qd", "gs", "bs", "vmin", "vmax", "gen_bus", "pmin", "pmax",
        "qmin", "qmax", "c2", "c1", "c0", "br_from", "br_to", "r", "x", "b",
        "tap", "shift", "rate")]


@dataclass
class OracleParams:
    """Parameters of the method (readings of the paper where it is silent)."""
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


def load() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if (not os.path.exists(_LIB_PATH)
            or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        build()
    lib = C.CDLL(_LIB_PATH)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.c_int
    lib.ora_create.restype = vp
    lib.ora_create.argtypes = [C.POINTER(_Grid), C.POINTER(_Params)]
    for name in ("ora_destroy", "ora_cold_init", "ora_gen_step",
                 "ora_branch_step", "ora_bus_step", "ora_z_step", "ora_y_step",
                 "ora_residuals", "ora_outer_step", "ora_warm_reset",
                 "ora_reset_stats"):
        getattr(lib, name).argtypes = [vp]
        getattr(lib, name).restype = None
    lib.ora_objective.argtypes = [vp]
    lib.ora_objective.restype = C.c_double
    lib.ora_quality.argtypes = [vp, dp]
    lib.ora_quality.restype = None
    lib.ora_solution.argtypes = [vp, dp]
    lib.ora_solution.restype = None
    lib.ora_iterate.argtypes = [vp, ip]
    lib.ora_iterate.restype = ip
    lib.ora_solve.argtypes = [vp, ip]
    lib.ora_solve.restype = ip
    lib.ora_update_loads.argtypes = [vp, dp, dp]
    lib.ora_update_gen_bounds.argtypes = [vp, dp, dp]
    lib.ora_update_gen_bounds.restype = None
    lib.ora_get.argtypes = [vp, ip, dp, C.c_int64]
    lib.ora_get.restype = ip
    lib.ora_set.argtypes = [vp, ip, dp, C.c_int64]
    lib.ora_set.restype = ip
    lib.ora_get_scalars.argtypes = [vp, dp]
    lib.ora_set_scalars.argtypes = [vp, dp]
    lib.ora_hist_len.argtypes = [vp]
    lib.ora_hist_len.restype = C.c_int64
    lib.ora_get_hist.argtypes = [vp, dp]
    lib.ora_get_admittance.argtypes = [vp, dp]
    lib.ora_get_stats.argtypes = [vp, C.POINTER(_Stats)]
    lib.ora_set_count_flops.argtypes = [vp, ip]
    lib.ora_sincos.argtypes = [C.c_double, dp, dp]
    lib.ora_branch_eval.argtypes = [dp, ip, dp, C.c_double, dp, dp, dp, dp, dp]
    lib.ora_ldlt.argtypes = [ip, dp, dp, dp]
    lib.ora_ldlt.restype = ip
    lib.ora_ldlt_solve.argtypes = [ip, dp, dp, dp, dp]
    lib.ora_ldlt_solve.restype = ip
    lib.ora_model.argtypes = [ip, dp, dp, dp]
    lib.ora_model.restype = C.c_double
    lib.ora_branch_solve.argtypes = [dp, ip, dp, dp, dp, dp, dp, C.POINTER(_Params),
                                     C.POINTER(_Stats), ip]
    lib.ora_set_threads.argtypes = [vp, ip]
    lib.ora_set_threads.restype = None
    lib.ora_set_textbook.argtypes = [vp, ip]
    lib.ora_set_textbook.restype = None
    lib.ora_branch_eval_textbook.argtypes = [dp, ip, dp, C.c_double, dp, dp, dp, dp, dp]
    lib.ora_branch_eval_textbook.restype = None
    lib.ora_branch_solve_textbook.argtypes = [dp, ip, dp, dp, dp, dp, dp,
                                              C.POINTER(_Params), C.POINTER(_Stats)]
    lib.ora_branch_solve_textbook.restype = None
    lib.ora_chol_textbook.argtypes = [ip, dp, dp]
    lib.ora_chol_textbook.restype = ip
    lib.ora_precond_textbook.argtypes = [ip, dp, dp, dp, dp]
    lib.ora_precond_textbook.restype = ip
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


STATE = {"u": 0, "v": 1, "z": 2, "y": 3, "lam": 4, "rho": 5, "bx": 6,
         "ltil": 7, "rtil": 8, "vprev": 9, "pd": 10, "qd": 11, "calpha": 12}


class Oracle:
    """One grid's serial ADMM state (canonical coupling order)."""

    def __init__(self, grid, params: OracleParams | None = None, cold: bool = True):
        self.lib = load()
        self.grid = grid
        self.params = params or OracleParams()
        self._keep = {}
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)  # noqa: E731
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)  # noqa: E731
        arrs = {}
        for n in ("pd", "qd", "gs", "bs", "vmin", "vmax", "pmin", "pmax",
                  "qmin", "qmax", "c2", "c1", "c0", "r", "x", "b", "tap",
                  "shift", "rate"):
            arrs[n] = f64(getattr(grid, n))
        for n in ("gen_bus", "br_from", "br_to"):
            arrs[n] = i32(getattr(grid, n))
        self._keep = arrs
        g = _Grid(n_bus=grid.n_bus, n_gen=grid.n_gen, n_branch=grid.n_branch,
                  ref_bus=grid.ref_bus, base_mva=grid.base_mva,
                  **{k: v.ctypes.data for k, v in arrs.items()})
        self._cp = self.params.c()
        self.h = self.lib.ora_create(C.byref(g), C.byref(self._cp))
        if not self.h:
            raise ValueError("oracle rejected the grid")
        self.nb, self.ng, self.nl = grid.n_bus, grid.n_gen, grid.n_branch
        self.m = 2 * self.ng + 8 * self.nl
        if cold:
            self.cold_init()

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.ora_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _size(self, name):
        return {"bx": 6 * self.nl, "ltil": 2 * self.nl, "rtil": self.nl,
                "calpha": self.nl, "pd": self.nb, "qd": self.nb}.get(name, self.m)

    def get(self, name: str) -> np.ndarray:
        out = np.empty(self._size(name))
        if self.lib.ora_get(self.h, STATE[name], _dp(out), out.size) != 0:
            raise ValueError(name)
        return out

    def set(self, name: str, val) -> None:
        a = np.ascontiguousarray(val, dtype=np.float64)
        if self.lib.ora_set(self.h, STATE[name], _dp(a), a.size) != 0:
            raise ValueError(name)

    def scalars(self) -> dict:
        out = np.empty(9)
        self.lib.ora_get_scalars(self.h, _dp(out))
        keys = ("beta", "znorm_prev", "r_pri", "r_dual", "r_z", "outer",
                "inner_total", "inner_in_outer", "status")
        return dict(zip(keys, out.tolist()))

    def set_scalars(self, d: dict) -> None:
        keys = ("beta", "znorm_prev", "r_pri", "r_dual", "r_z", "outer",
                "inner_total", "inner_in_outer", "status")
        arr = np.array([float(d[k]) for k in keys])
        self.lib.ora_set_scalars(self.h, _dp(arr))

    def history(self) -> np.ndarray:
        n = self.lib.ora_hist_len(self.h)
        out = np.empty(n)
        if n:
            self.lib.ora_get_hist(self.h, _dp(out))
        return out.reshape(-1, 6)

    def admittance(self) -> np.ndarray:
        out = np.empty(9 * self.nl)
        self.lib.ora_get_admittance(self.h, _dp(out))
        return out.reshape(self.nl, 9)

    def stats(self) -> dict:
        s = _Stats()
        self.lib.ora_get_stats(self.h, C.byref(s))
        return s.as_dict()

    def reset_stats(self):
        self.lib.ora_reset_stats(self.h)

    def count_flops(self, on: bool = True):
        self.lib.ora_set_count_flops(self.h, int(on))

    def set_threads(self, n: int):
        """OpenMP threads for the loops over generators, branches, buses and
        couplings (1: serial, the default). Results are bitwise the same for
        any count."""
        self.lib.ora_set_threads(self.h, int(n))

    def set_textbook(self, on: bool = True):
        """Solve the branch subproblems by the textbook path (eq. branch
        summed term by term, libm sin/cos, plain arithmetic, Lin & More's
        scaled Cholesky preconditioner) instead of the fixed-sequence path."""
        self.lib.ora_set_textbook(self.h, int(on))

    # stages of one inner iteration (Algorithm 1)
    def cold_init(self):
        self.lib.ora_cold_init(self.h)

    def gen_step(self):
        self.lib.ora_gen_step(self.h)

    def branch_step(self):
        self.lib.ora_branch_step(self.h)

    def bus_step(self):
        self.lib.ora_bus_step(self.h)

    def z_step(self):
        self.lib.ora_z_step(self.h)

    def y_step(self):
        self.lib.ora_y_step(self.h)

    def residuals(self):
        self.lib.ora_residuals(self.h)

    def outer_step(self):
        self.lib.ora_outer_step(self.h)

    def objective(self) -> float:
        return float(self.lib.ora_objective(self.h))

    def quality(self) -> dict:
        """||c(x)||_inf over eq. acopf at the current ADMM solution and its
        parts (power balance p and q, line limits, voltage and angle limits)."""
        out = np.zeros(6)
        self.lib.ora_quality(self.h, _dp(out))
        return dict(zip(QUALITY_NAMES, out.tolist()))

    def solution(self) -> dict:
        """The ADMM solution of Sec. IV-A: generator outputs (pg, qg), bus
        voltage magnitudes and angles (vm = sqrt(w), va), and the branch flows
        recomputed from those voltages (pij, qij, pji, qji), input order."""
        nb, ng, nl = self.nb, self.ng, self.nl
        out = np.zeros(2 * ng + 2 * nb + 4 * nl)
        self.lib.ora_solution(self.h, _dp(out))
        parts = np.split(out, np.cumsum([ng, ng, nb, nb, nl, nl, nl, nl])[:-1])
        return dict(zip(("pg", "qg", "vm", "va", "pij", "qij", "pji", "qji"), parts))

    def iterate(self, fixed: bool = False) -> bool:
        return bool(self.lib.ora_iterate(self.h, int(fixed)))

    def solve(self, fixed_iters: int = 0) -> int:
        return int(self.lib.ora_solve(self.h, int(fixed_iters)))

    def update_gen_bounds(self, pmin, pmax):
        lo = np.ascontiguousarray(pmin, dtype=np.float64)
        hi = np.ascontiguousarray(pmax, dtype=np.float64)
        self.lib.ora_update_gen_bounds(self.h, _dp(lo), _dp(hi))

    def update_loads(self, pd, qd, warm_reset: bool = True):
        pd = np.ascontiguousarray(pd, dtype=np.float64)
        qd = np.ascontiguousarray(qd, dtype=np.float64)
        self.lib.ora_update_loads(self.h, _dp(pd), _dp(qd))
        if warm_reset:
            self.lib.ora_warm_reset(self.h)

    def snapshot(self) -> dict:
        snap = {k: self.get(k) for k in STATE}
        snap["_scalars"] = self.scalars()
        return snap

    def restore(self, snap: dict):
        for k in STATE:
            self.set(k, snap[k])
        self.set_scalars(snap["_scalars"])


# ---- single-branch entry points (tests) ------------------------------------

def pack_branch(adm8, lo6, hi6, vb8, z8, y8, rho8) -> np.ndarray:
    return np.ascontiguousarray(np.concatenate(
        [adm8, lo6, hi6, vb8, z8, y8, rho8]).astype(np.float64))


def branch_eval(data: np.ndarray, n: int, ltil, rtil: float, x, textbook: bool = False):
    """f, g, H and the coupling values a of eq. (branch) at x, on the
    fixed-sequence path or (textbook=True) on the textbook path."""
    lib = load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    lt = np.ascontiguousarray(ltil, dtype=np.float64)
    f = np.zeros(1)
    g = np.zeros(n)
    H = np.zeros(n * n)
    a = np.zeros(8)
    fn = lib.ora_branch_eval_textbook if textbook else lib.ora_branch_eval
    fn(_dp(data), n, _dp(lt), float(rtil), _dp(x), _dp(f), _dp(g), _dp(H), _dp(a))
    return f[0], g, H.reshape(n, n), a


def branch_solve(data: np.ndarray, n: int, x6, ltil, rtil: float,
                 params: OracleParams | None = None, count: bool = False,
                 alpha: float = 1.0, textbook: bool = False):
    """One branch solve from state (x6, ltil, rtil) with the trust-region
    Cauchy step length starting at `alpha`; returns the new x, ltil, rtil,
    the coupling values u and the counters (with the final step length under
    "alpha"). textbook=True takes the textbook path (no flop counting)."""
    lib = load()
    p = (params or OracleParams()).c()
    x = np.ascontiguousarray(x6, dtype=np.float64).copy()
    lt = np.ascontiguousarray(ltil, dtype=np.float64).copy()
    rt = np.array([rtil], dtype=np.float64)
    al = np.array([alpha], dtype=np.float64)
    u = np.zeros(8)
    st = _Stats()
    if textbook:
        lib.ora_branch_solve_textbook(_dp(data), n, _dp(x), _dp(lt), _dp(rt), _dp(al),
                                      _dp(u), C.byref(p), C.byref(st))
    else:
        lib.ora_branch_solve(_dp(data), n, _dp(x), _dp(lt), _dp(rt), _dp(al), _dp(u),
                             C.byref(p), C.byref(st), int(count))
    out = st.as_dict()
    out["alpha"] = float(al[0])
    return x, lt, rt[0], u, out


def ldlt(A):
    """The trust-region method's square-root-free Cholesky factorization of a
    symmetric matrix: (L unit lower, reciprocal pivots 1/e), or None at a
    non-positive pivot."""
    lib = load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    L = np.zeros((n, n))
    rd = np.zeros(n)
    ok = lib.ora_ldlt(n, _dp(A), _dp(L), _dp(rd))
    return (L, rd) if ok == 1 else None


def ldlt_solve(L, rd, r):
    """z = (L E L')^-1 r from the factors of ldlt."""
    lib = load()
    L = np.ascontiguousarray(L, dtype=np.float64)
    rd = np.ascontiguousarray(rd, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.zeros_like(r)
    lib.ora_ldlt_solve(len(r), _dp(L), _dp(rd), _dp(r), _dp(z))
    return z


def chol_textbook(A):
    """The textbook path's Cholesky factor L (A = L L'), or None at a
    non-positive pivot."""
    lib = load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    L = np.zeros((n, n))
    ok = lib.ora_chol_textbook(n, _dp(A), _dp(L))
    return L if ok == 1 else None


def precond_textbook(L, D, r):
    """z = D L'^-1 L^-1 D r, the textbook path's preconditioner solve."""
    lib = load()
    L = np.ascontiguousarray(L, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.zeros_like(r)
    lib.ora_precond_textbook(len(r), _dp(L), _dp(D), _dp(r), _dp(z))
    return z


def model(g, H, s):
    """The trust-region model q(s) = g's + s'Hs/2 as the oracle forms it."""
    lib = load()
    g = np.ascontiguousarray(g, dtype=np.float64)
    H = np.ascontiguousarray(H, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    return lib.ora_model(len(g), _dp(g), _dp(H), _dp(s))


def sincos(x: float):
    """The oracle's series sin/cos of a branch angle."""
    lib = load()
    s = C.c_double()
    c = C.c_double()
    lib.ora_sincos(float(x), C.byref(s), C.byref(c))
    return s.value, c.value


_F_CB = C.CFUNCTYPE(C.c_double, C.POINTER(C.c_double), C.c_void_p)
_G_CB = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.POINTER(C.c_double),
                    C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p)


def tron_generic(f, fgh, x0, lo, hi, params: OracleParams | None = None,
                 textbook: bool = False):
    """Run the oracle's TRON on Python callbacks f(x) and fgh(x)->(f,g,H),
    on the fixed-sequence path or (textbook=True) on the textbook path."""
    lib = load()
    n = len(x0)

    def _f(xp, _ctx):
        x = np.ctypeslib.as_array(xp, shape=(n,)).copy()
        return float(f(x))

    def _g(xp, fp, gp, hp, _ctx):
        x = np.ctypeslib.as_array(xp, shape=(n,)).copy()
        F, g, H = fgh(x)
        fp[0] = float(F)
        for i in range(n):
            gp[i] = float(g[i])
        Hf = np.asarray(H, dtype=np.float64).reshape(-1)
        for i in range(n * n):
            hp[i] = float(Hf[i])

    fcb, gcb = _F_CB(_f), _G_CB(_g)
    lib.ora_tron.argtypes = [C.c_int, C.POINTER(C.c_double),
                             C.POINTER(C.c_double), C.POINTER(C.c_double),
                             _F_CB, _G_CB, C.c_void_p, C.POINTER(_Params),
                             C.POINTER(_Stats)]
    lib.ora_tron.restype = C.c_int
    lib.ora_tron_textbook.argtypes = lib.ora_tron.argtypes
    lib.ora_tron_textbook.restype = C.c_int
    x = np.ascontiguousarray(x0, dtype=np.float64).copy()
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    p = (params or OracleParams()).c()
    st = _Stats()
    fn = lib.ora_tron_textbook if textbook else lib.ora_tron
    status = fn(n, _dp(x), _dp(lo), _dp(hi), fcb, gcb, None, C.byref(p), C.byref(st))
    return x, int(status), st.as_dict()
