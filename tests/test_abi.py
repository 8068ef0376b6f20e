"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/acopf.h, fills default parameters, and rejects invalid
grids during validation (before any device call)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2110_06879_amd import acopf as A
from paper_2110_06879_amd.gridgen import config_grid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "acopf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(acopf_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = A.load()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(A.EXPORTS) == set(names)


def test_default_params_match_binding_defaults():
    d = A.default_params()
    p = A.Params()
    for k, v in d.items():
        assert getattr(p, k) == v, k


def _bad(mutator):
    g = config_grid("c1_30bus")
    mutator(g)
    with pytest.raises(A.AcopfError) as e:
        A.Solver(g)
    return str(e.value)


def test_validation_rejects_bad_grids():
    assert "-1" in _bad(lambda g: g.pd.__setitem__(3, np.nan))
    assert "-1" in _bad(lambda g: g.br_to.__setitem__(0, 999))
    assert "-1" in _bad(lambda g: (g.r.__setitem__(2, 0.0), g.x.__setitem__(2, 0.0)))
    assert "-1" in _bad(lambda g: g.vmin.__setitem__(1, 1.2))
    assert "-1" in _bad(lambda g: g.pmin.__setitem__(0, 5.0))
    assert "-1" in _bad(lambda g: g.gen_bus.__setitem__(0, -1))
    assert "-1" in _bad(lambda g: g.tap.__setitem__(0, 0.0))


def test_validation_rejects_isolated_bus():
    g = config_grid("c1_30bus")
    # move every branch end away from bus 7
    g.br_from[g.br_from == 7] = 8
    g.br_to[g.br_to == 7] = 9
    keep = g.br_from != g.br_to
    for n in ("br_from", "br_to", "r", "x", "b", "tap", "shift", "rate"):
        setattr(g, n, getattr(g, n)[keep])
    with pytest.raises(A.AcopfError, match="isolated|-1"):
        A.Solver(g)


def test_bad_params_rejected():
    g = config_grid("c1_30bus")
    with pytest.raises(A.AcopfError):
        A.Solver(g, A.Params(rho_pq=0.0))
    with pytest.raises(A.AcopfError):
        A.Solver(g, A.Params(max_inner=0))
