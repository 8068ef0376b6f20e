"""Reader for MATPOWER case files (version 2 `.m` format) into the Grid of
gridgen, so that the grids of the paper's Table 1 run when a user supplies
the files (none ship here).

Only input handling: parsing and unit conversion, none of the solver's
arithmetic. Conventions (MATPOWER's): loads, shunts (at 1 p.u. voltage),
generator limits and ratings are in MW / MVAr / MVA and are divided by
baseMVA; branch `ratio` 0 means 1; `angle` is a phase shift in degrees
(converted to radians); `rateA` 0 means unlimited; elements with status 0
are dropped; polynomial costs (model 2) give c2, c1, c0 on P in MW. The
reference bus is the first bus of type 3. Bus numbers may be arbitrary and
are mapped to 0..n_bus-1 in file order.
"""
from __future__ import annotations

import math
import re

import numpy as np

from .gridgen import Grid

_BLOCK = re.compile(r"mpc\.(\w+)\s*=\s*\[(.*?)\]\s*;", re.S)
_SCALAR = re.compile(r"mpc\.baseMVA\s*=\s*([-+0-9.eE]+)\s*;")


def _rows(body: str) -> np.ndarray:
    rows = []
    for line in body.split("\n"):
        line = line.split("%", 1)[0]
        for part in line.split(";"):
            vals = part.replace(",", " ").split()
            if vals:
                rows.append([float(v) for v in vals])
    if not rows:
        return np.zeros((0, 0))
    width = max(len(r) for r in rows)
    if any(len(r) != width for r in rows):
        raise ValueError("ragged matrix in case file")
    return np.array(rows, dtype=np.float64)


def parse_case(text: str) -> dict:
    """The matrices and baseMVA of a MATPOWER case file's text."""
    text = re.sub(r"%[^\n]*", "", text)  # comments, also inside blocks
    m = _SCALAR.search(text)
    if not m:
        raise ValueError("case file has no mpc.baseMVA")
    out = {"baseMVA": float(m.group(1))}
    for name, body in _BLOCK.findall(text):
        out[name] = _rows(body)
    for need in ("bus", "gen", "branch", "gencost"):
        if need not in out:
            raise ValueError(f"case file has no mpc.{need}")
    return out


def grid_from_case(mpc: dict, name: str = "matpower") -> Grid:
    base = mpc["baseMVA"]
    bus, gen, br, cost = mpc["bus"], mpc["gen"], mpc["branch"], mpc["gencost"]
    if bus.shape[1] < 13 or gen.shape[1] < 10 or br.shape[1] < 11:
        raise ValueError("bus/gen/branch matrices have too few columns")
    if cost.shape[0] < gen.shape[0]:
        raise ValueError("gencost needs one row per generator")
    ids = {int(b): k for k, b in enumerate(bus[:, 0])}
    if len(ids) != bus.shape[0]:
        raise ValueError("duplicate bus numbers")
    refs = [k for k in range(bus.shape[0]) if int(bus[k, 1]) == 3]
    if not refs:
        raise ValueError("no reference bus (type 3)")
    g_on = [k for k in range(gen.shape[0]) if gen[k, 7] > 0]
    c2, c1, c0 = [], [], []
    for k in g_on:
        row = cost[k]
        if int(row[0]) != 2:
            raise ValueError(f"generator {k}: only polynomial costs (model 2) are supported")
        n = int(row[3])
        coef = list(row[4:4 + n])
        if len(coef) != n or n > 3:
            raise ValueError(f"generator {k}: polynomial cost of degree {n - 1} not supported")
        coef = [0.0] * (3 - n) + coef
        c2.append(coef[0]); c1.append(coef[1]); c0.append(coef[2])
    b_on = [k for k in range(br.shape[0]) if br[k, 10] > 0]
    tap = np.array([br[k, 8] if br[k, 8] != 0.0 else 1.0 for k in b_on])
    return Grid(
        name=name, base_mva=base, ref_bus=refs[0],
        pd=bus[:, 2] / base, qd=bus[:, 3] / base, gs=bus[:, 4] / base, bs=bus[:, 5] / base,
        vmin=bus[:, 12].copy(), vmax=bus[:, 11].copy(),
        gen_bus=np.array([ids[int(gen[k, 0])] for k in g_on], dtype=np.int32),
        pmin=np.array([gen[k, 9] for k in g_on]) / base,
        pmax=np.array([gen[k, 8] for k in g_on]) / base,
        qmin=np.array([gen[k, 4] for k in g_on]) / base,
        qmax=np.array([gen[k, 3] for k in g_on]) / base,
        c2=np.array(c2), c1=np.array(c1), c0=np.array(c0),
        br_from=np.array([ids[int(br[k, 0])] for k in b_on], dtype=np.int32),
        br_to=np.array([ids[int(br[k, 1])] for k in b_on], dtype=np.int32),
        r=np.array([br[k, 2] for k in b_on]), x=np.array([br[k, 3] for k in b_on]),
        b=np.array([br[k, 4] for k in b_on]), tap=tap,
        shift=np.array([math.radians(br[k, 9]) for k in b_on]),
        rate=np.array([br[k, 5] for k in b_on]) / base)


def load_case(path: str) -> Grid:
    """Read a MATPOWER version-2 case file into a Grid."""
    with open(path) as fh:
        text = fh.read()
    name = path.rsplit("/", 1)[-1].rsplit(".", 1)[0]
    return grid_from_case(parse_case(text), name)
