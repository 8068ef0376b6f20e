"""MATPOWER case reader (paper_2110_06879_amd.matpower) on a hand-made
5-bus case: unit conversions, element status, bus renumbering, costs; and a
solve of the read grid by the oracle."""
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2110_06879_amd import matpower as M

CASE = os.path.join(os.path.dirname(__file__), "golden", "case5_handmade.m")


def test_reader_conversions():
    g = M.load_case(CASE)
    assert g.name == "case5_handmade" and g.base_mva == 100.0
    assert g.n_bus == 5 and g.ref_bus == 1                  # bus 20 is type 3
    np.testing.assert_allclose(g.pd, [0.40, 0.0, 0.25, 0.30, 0.20])
    np.testing.assert_allclose(g.qd, [0.12, 0.0, 0.08, 0.09, 0.06])
    np.testing.assert_allclose(g.gs, [0, 0, 0, 0.01, 0]) and None
    np.testing.assert_allclose(g.bs, [0, 0, 0.05, 0, 0])
    # generator 4 is out of service; two generators on bus 30 (index 2)
    assert g.n_gen == 3
    np.testing.assert_array_equal(g.gen_bus, [1, 2, 2])
    np.testing.assert_allclose(g.pmax, [2.0, 0.8, 0.5])
    np.testing.assert_allclose(g.qmin, [-1.5, -0.6, -0.4])
    np.testing.assert_allclose(g.c2, [0.02, 0.05, 0.0])     # linear cost: c2 = 0
    np.testing.assert_allclose(g.c1, [20, 15, 30])
    # branch 6 (10-50) is out of service
    assert g.n_branch == 6
    np.testing.assert_array_equal(g.br_from, [1, 1, 0, 2, 3, 2])
    np.testing.assert_array_equal(g.br_to, [0, 2, 3, 3, 4, 4])
    np.testing.assert_allclose(g.tap, [1, 1, 1, 0.98, 1, 1])
    np.testing.assert_allclose(g.shift, [0, 0, 0, math.radians(2), 0, 0])
    np.testing.assert_allclose(g.rate, [2.5, 1.5, 0.0, 1.2, 1.0, 1.1])
    assert g.n_rated == 5


def test_reader_rejects_bad_cases():
    text = open(CASE).read()
    with pytest.raises(ValueError):
        M.parse_case(text.replace("mpc.baseMVA = 100;", ""))
    with pytest.raises(ValueError):
        M.grid_from_case(M.parse_case(text.replace("\t20\t3\t", "\t20\t1\t")))
    with pytest.raises(ValueError):   # piecewise-linear cost model
        M.grid_from_case(M.parse_case(text.replace("\t2\t0\t0\t3\t0.02", "\t1\t0\t0\t3\t0.02")))


def test_read_grid_solves_in_the_oracle():
    g = M.load_case(CASE)
    o = O.Oracle(g, O.OracleParams(rho_pq=400.0, rho_va=4000.0))
    q0 = o.quality()["max_violation"]
    status = o.solve(0)
    q = o.quality()
    assert np.isfinite(q["max_violation"]) and q["max_violation"] < q0
    assert o.scalars()["inner_total"] > 0
