"""Tracking horizon (Sec. IV-C) on the CPU: the load profile and the
ramp-limited bounds of paper_2110_06879_amd.tracking, and a short horizon
solved by the oracle, whose generator outputs must respect the ramp limits
|p_{t+1} - p_t| <= 2% of pmax between periods."""
import numpy as np

import oracle as O
from paper_2110_06879_amd import tracking as T
from paper_2110_06879_amd.gridgen import gridgen


def test_load_profile_shape():
    f = T.load_profile(30, 0.05)
    assert f.shape == (30,)
    assert f[0] == 1.0 and abs(f[-1] - 1.05) < 1e-15
    assert np.all(np.diff(f) >= 0)
    assert np.max(np.abs(f - 1.0)) <= 0.05 + 1e-15
    assert np.allclose(T.load_profile(1, 0.05), [1.0])


def test_ramp_bounds_properties():
    rng = np.random.default_rng(3)
    pmin = np.zeros(50)
    pmax = rng.uniform(0.5, 3.0, 50)
    p = rng.uniform(-0.1, 3.1, 50)   # also outside the bounds
    lo, hi = T.ramp_bounds(pmin, pmax, p, 0.02)
    assert np.all(lo <= hi)
    assert np.all(lo >= pmin) and np.all(hi <= pmax)
    pc = np.clip(p, pmin, pmax)
    assert np.all(hi - pc <= 0.02 * pmax + 1e-15) and np.all(pc - lo <= 0.02 * pmax + 1e-15)


def test_oracle_horizon_respects_ramp_limits():
    g = gridgen(60, 12, 80, 0.5, 71, load_factor=0.2)
    orc = O.Oracle(g, O.OracleParams())
    factor = T.load_profile(4, 0.05)
    p_prev = None
    for t in range(4):
        if t == 0:
            orc.update_gen_bounds(g.pmin, g.pmax)
        else:
            lo, hi = T.ramp_bounds(g.pmin, g.pmax, p_prev, 0.02)
            orc.update_gen_bounds(lo, hi)
        orc.update_loads(g.pd * factor[t], g.qd * factor[t], warm_reset=t > 0)
        orc.solve(0)
        p = T.generator_p(orc.get("u"), g.n_gen)
        if p_prev is not None:
            assert np.all(np.abs(p - p_prev) <= 0.02 * g.pmax * (1 + 1e-12)), t
        q = orc.quality()
        assert np.isfinite(q["max_violation"])
        p_prev = p
