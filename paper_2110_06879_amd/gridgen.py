"""Seeded synthetic power grids and load perturbations.

This module only draws inputs. It holds none of the solver's arithmetic: no
admittances, no flows, no scaling of ratings. Both the HIP path and the CPU
oracle receive the raw arrays it returns.

The grids stand in for the MATPOWER cases of the paper's Table 1 (pegase,
ACTIVSg25k/70k), which are not available here. The recipe (fixed draw order,
one ``numpy.random.default_rng(seed)`` per grid):

1. Topology: a random recursive spanning tree (a random permutation ``pi``;
   ``pi[k]`` attaches to ``pi[U{0..k-1}]``), then uniform random extra edges,
   rejecting self-loops and duplicates, until ``n_branch`` edges exist.
2. Branches: r ~ U(0.005, 0.05), x ~ U(0.02, 0.2), total charging
   b ~ U(0, 0.05) (p.u.). A seeded subset of round(rated_frac * n_branch)
   branches is rated with U(1, 3) p.u.; the rest have rate 0 (unlimited).
   tap = 1, shift = 0.
3. Generators on distinct buses, generator 0 at bus 0 (the reference bus):
   Pmin = 0, Pmax ~ U(0.5, 3), Q limits = +-Pmax, cost
   c2 ~ U(0.01, 0.1) $/MW^2h, c1 ~ U(10, 40) $/MWh, c0 = 0 (MATPOWER
   convention: cost on MW with baseMVA = 100).
4. Loads at every bus: Pd ~ load_factor * U(0, 0.5), Qd = 0.3 Pd. The five
   workloads use load_factor = 0.2: at the full U(0, 0.5) level these weak
   synthetic networks (x up to 0.2 p.u., a generator on one bus in five) are
   voltage-infeasible in remote radial pockets. Guard: if sum(Pd) > 0.75
   sum(Pmax), Pd and Qd are scaled so that the ratio is 0.75 (the factor is
   returned).
5. |V| in [0.94, 1.06], bus shunts 0, baseMVA 100.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["Grid", "gridgen", "perturb_loads", "config_grid", "batch_grids",
           "serving_grids", "CONFIGS"]


@dataclass
class Grid:
    """Raw grid data in per unit on ``base_mva``; SoA numpy arrays."""
    name: str
    base_mva: float
    ref_bus: int
    # buses
    pd: np.ndarray
    qd: np.ndarray
    gs: np.ndarray
    bs: np.ndarray
    vmin: np.ndarray
    vmax: np.ndarray
    # generators
    gen_bus: np.ndarray
    pmin: np.ndarray
    pmax: np.ndarray
    qmin: np.ndarray
    qmax: np.ndarray
    c2: np.ndarray
    c1: np.ndarray
    c0: np.ndarray
    # branches
    br_from: np.ndarray
    br_to: np.ndarray
    r: np.ndarray
    x: np.ndarray
    b: np.ndarray
    tap: np.ndarray
    shift: np.ndarray
    rate: np.ndarray
    load_scale: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def n_bus(self) -> int:
        return int(self.pd.shape[0])

    @property
    def n_gen(self) -> int:
        return int(self.gen_bus.shape[0])

    @property
    def n_branch(self) -> int:
        return int(self.br_from.shape[0])

    @property
    def n_rated(self) -> int:
        return int(np.count_nonzero(self.rate > 0))

    @property
    def n_coupling(self) -> int:
        return 2 * self.n_gen + 8 * self.n_branch

    def with_loads(self, pd: np.ndarray, qd: np.ndarray) -> "Grid":
        g = Grid(**{k: getattr(self, k) for k in self.__dataclass_fields__})
        g.pd = np.ascontiguousarray(pd, dtype=np.float64)
        g.qd = np.ascontiguousarray(qd, dtype=np.float64)
        return g


def _topology(rng: np.random.Generator, n_b: int, n_l: int):
    if n_l < n_b - 1:
        raise ValueError("need at least n_bus-1 branches for a spanning tree")
    max_edges = n_b * (n_b - 1) // 2
    if n_l > max_edges:
        raise ValueError("too many branches for a simple graph")
    perm = rng.permutation(n_b)
    # parent of perm[k] is perm[U{0..k-1}], k = 1..n_b-1
    ks = np.arange(1, n_b)
    parents = perm[(rng.random(n_b - 1) * ks).astype(np.int64)]
    frm = list(perm[1:].tolist())
    to = list(parents.tolist())
    seen = set()
    for a, b in zip(frm, to):
        seen.add((min(a, b), max(a, b)))
    while len(frm) < n_l:
        need = n_l - len(frm)
        cand = rng.integers(0, n_b, size=(2 * need + 8, 2))
        for a, b in cand.tolist():
            if a == b:
                continue
            key = (min(a, b), max(a, b))
            if key in seen:
                continue
            seen.add(key)
            frm.append(a)
            to.append(b)
            if len(frm) == n_l:
                break
    return np.asarray(frm, dtype=np.int32), np.asarray(to, dtype=np.int32)


def gridgen(n_bus: int, n_gen: int, n_branch: int, rated_frac: float,
            seed: int, name: str | None = None,
            load_guard: float = 0.75, load_factor: float = 1.0) -> Grid:
    """Draw one synthetic grid (recipe in the module docstring)."""
    if not (1 <= n_gen <= n_bus):
        raise ValueError("need 1 <= n_gen <= n_bus")
    rng = np.random.default_rng(seed)
    frm, to = _topology(rng, n_bus, n_branch)
    r = rng.uniform(0.005, 0.05, n_branch)
    x = rng.uniform(0.02, 0.2, n_branch)
    b = rng.uniform(0.0, 0.05, n_branch)
    n_rated = int(round(rated_frac * n_branch))
    rated = np.zeros(n_branch, dtype=bool)
    rated[rng.permutation(n_branch)[:n_rated]] = True
    rate_draw = rng.uniform(1.0, 3.0, n_branch)
    rate = np.where(rated, rate_draw, 0.0)
    others = rng.permutation(np.arange(1, n_bus))[: n_gen - 1]
    gen_bus = np.concatenate([[0], others]).astype(np.int32)
    pmax = rng.uniform(0.5, 3.0, n_gen)
    c2 = rng.uniform(0.01, 0.1, n_gen)
    c1 = rng.uniform(10.0, 40.0, n_gen)
    pd = load_factor * rng.uniform(0.0, 0.5, n_bus)
    qd = 0.3 * pd
    ratio = pd.sum() / pmax.sum()
    scale = 1.0
    if ratio > load_guard:
        scale = load_guard / ratio
        pd = pd * scale
        qd = qd * scale
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)  # noqa: E731
    return Grid(
        name=name or f"synth{n_bus}_s{seed}", base_mva=100.0, ref_bus=0,
        pd=f64(pd), qd=f64(qd), gs=np.zeros(n_bus), bs=np.zeros(n_bus),
        vmin=np.full(n_bus, 0.94), vmax=np.full(n_bus, 1.06),
        gen_bus=gen_bus, pmin=np.zeros(n_gen), pmax=f64(pmax),
        qmin=f64(-pmax), qmax=f64(pmax), c2=f64(c2), c1=f64(c1),
        c0=np.zeros(n_gen),
        br_from=frm, br_to=to, r=f64(r), x=f64(x), b=f64(b),
        tap=np.ones(n_branch), shift=np.zeros(n_branch), rate=f64(rate),
        load_scale=float(scale),
        meta=dict(n_bus=n_bus, n_gen=n_gen, n_branch=n_branch,
                  rated_frac=rated_frac, seed=seed,
                  load_ratio_before_guard=float(ratio)),
    )


def perturb_loads(grid: Grid, frac: float, seed: int):
    """Per-bus independent load change: Pd(1+d), Qd(1+d), d ~ U(-frac, frac)."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(-frac, frac, grid.n_bus)
    return grid.pd * (1.0 + d), grid.qd * (1.0 + d)


LOAD_FACTOR = 0.2

# The five workloads: 30-bus plain, 2k-bus, 70k-bus, 64-grid batch, serving.
CONFIGS = {
    "c1_30bus": dict(n_bus=30, n_gen=6, n_branch=41, rated_frac=1.0, seed=1,
                     load_factor=LOAD_FACTOR),
    "c2_2kbus": dict(n_bus=2000, n_gen=400, n_branch=2600, rated_frac=1.0, seed=2,
                     load_factor=LOAD_FACTOR),
    "c3_70kbus": dict(n_bus=70000, n_gen=10000, n_branch=88000, rated_frac=0.3, seed=3,
                      load_factor=LOAD_FACTOR),
    # the same grids at the stated load distribution Pd ~ U(0, 0.5) (load
    # factor 1, then the 0.75 total-load guard): remote radial pockets are
    # voltage-infeasible at this level, so these serve fixed-iteration runs
    "c2_2kbus_full": dict(n_bus=2000, n_gen=400, n_branch=2600, rated_frac=1.0, seed=2,
                          load_factor=1.0),
    "c3_70kbus_full": dict(n_bus=70000, n_gen=10000, n_branch=88000, rated_frac=0.3, seed=3,
                           load_factor=1.0),
}


def config_grid(name: str) -> Grid:
    return gridgen(name=name, **CONFIGS[name])


def batch_grids(n_grids: int = 64, seed: int = 4, lo: int = 500,
                hi: int = 20000, first_grid_seed: int = 400) -> list[Grid]:
    """Uneven multi-grid batch: n_bus log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    sizes = np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), n_grids)))
    out = []
    for k, nb in enumerate(sizes.astype(int).tolist()):
        ng = max(1, int(round(0.2 * nb)))
        nl = int(round(1.3 * nb))
        out.append(gridgen(nb, ng, nl, 1.0, first_grid_seed + k,
                           name=f"batch{k}_{nb}", load_factor=LOAD_FACTOR))
    return out


def serving_grids(n_grids: int = 16, seed: int = 5, lo: int = 2000,
                  hi: int = 70000, first_grid_seed: int = 500,
                  with_70k: bool = True) -> list[Grid]:
    """Resident grids for tracking requests; ends pinned at lo and hi."""
    rng = np.random.default_rng(seed)
    sizes = np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), n_grids)))
    sizes[0] = lo
    sizes[-1] = hi
    out = []
    for k, nb in enumerate(sizes.astype(int).tolist()):
        if nb == 70000 and with_70k:
            out.append(config_grid("c3_70kbus"))
            continue
        ng = max(1, int(round(0.2 * nb)))
        nl = int(round(1.3 * nb))
        rf = 0.3 if nb > 20000 else 1.0
        out.append(gridgen(nb, ng, nl, rf, first_grid_seed + k,
                           name=f"serve{k}_{nb}", load_factor=LOAD_FACTOR))
    return out
