"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.

Bar (norm-wise, per vector): ||X_gpu - X_oracle||_inf / ||X_oracle||_inf
<= 1e-9 after a fixed number of inner iterations, for u, v, z, y, lambda,
branch x and the line-limit multipliers; the objective at the same
iteration count within 1e-6 relative. Event counts of the branch solves
(TRON iterations, evaluations, ...) and the algorithmic flop count must match
the oracle's exactly when both sides take the same path.
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_2110_06879_amd import acopf as A
from paper_2110_06879_amd.gridgen import config_grid, gridgen, perturb_loads

pytestmark = pytest.mark.gpu

TOL = 1e-9
VECS = ("u", "v", "z", "y", "lam", "bx", "ltil", "calpha")


def oparams(p: A.Params) -> O.OracleParams:
    from dataclasses import asdict
    return O.OracleParams(**asdict(p))


def relerr(a, b):
    den = max(np.abs(b).max(), 1e-30)
    return float(np.abs(a - b).max() / den)


def compare(solver, orc, grid=0, tol=TOL, label=""):
    errs = {}
    for k in VECS:
        errs[k] = relerr(solver.get(k, grid), orc.get(k))
    print(label, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, e in errs.items():
        assert e <= tol, (label, k, e)
    return errs


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# x-step kernels: lane per branch (unlimited branches per lane automatic, or
# three per lane), and the persistent pool kernel
XSTEP = {"lane": dict(xstep_waves=0, xstep_per_lane=0), "lane3": dict(xstep_waves=0, xstep_per_lane=3),
         "pool": dict(xstep_waves=1, xstep_per_lane=0)}


@pytest.mark.parametrize("waves", list(XSTEP))
@pytest.mark.parametrize("name,iters", [("c1_30bus", 50), ("c2_2kbus", 50)])
def test_fixed_iterations_match_oracle(name, iters, waves):
    note(f"parity {name} cold {iters} fixed iterations, x-step {waves}")
    g = config_grid(name)
    p = A.Params(rho_pq=400.0, rho_va=400.0 if name == "c1_30bus" else 40000.0)
    orc = O.Oracle(g, oparams(p))
    orc.count_flops(True)
    orc.solve(iters)
    with A.Solver(g, p) as s:
        s.set_tuning(**XSTEP[waves])
        s.set_counting(True)
        res = s.solve(A.COLD, iters)[0]
        assert res["inner_iters"] == iters
        compare(s, orc, label=name)
        # residual history, iteration by iteration
        hg, ho = s.history(), orc.history()
        assert hg.shape == ho.shape
        np.testing.assert_allclose(hg[:, [0, 1, 2]], ho[:, [0, 1, 2]], rtol=1e-7, atol=1e-12)
        np.testing.assert_array_equal(hg[:, 5], ho[:, 5])
        # objective at the same iteration
        assert abs(res["objective"] - orc.objective()) <= 1e-6 * max(1.0, abs(orc.objective()))
        sg, so = s.stats(), orc.stats()
        note(f"gpu stats {sg}")
        note(f"oracle stats {so}")
        for k in ("branch_solves", "tron_calls", "tron_iters", "n_fgh", "n_f",
                  "cauchy_trials", "cg_iters", "chol_attempts", "ps_trials", "al_iters",
                  "trig"):
            assert sg[k] == so[k], (k, sg[k], so[k])
        assert sg["flops"] == so["flops"]


def test_outer_steps_match_oracle():
    """max_inner = 10 forces an outer step (lambda and beta update of
    Algorithm 1) every ten inner iterations: 55 iterations cross five."""
    note("parity c2 with an outer step every 10 inner iterations")
    g = config_grid("c2_2kbus")
    p = A.Params(max_inner=10)
    orc = O.Oracle(g, oparams(p))
    orc.solve(55)
    assert orc.history()[-1, 5] == 5
    with A.Solver(g, p) as s:
        s.solve(A.COLD, 55)
        compare(s, orc, label="c2 outer")
        assert np.abs(orc.get("lam")).max() > 0
        np.testing.assert_array_equal(s.history()[:, 5], orc.history()[:, 5])
        np.testing.assert_array_equal(s.history()[:, 4], orc.history()[:, 4])


def test_outer_steps_across_chunks_and_calls():
    """An outer step decided by an iteration's control is applied to lambda
    by the next bus step; one decided by the last iteration of a chunk waits
    for the next chunk, and one decided by the last iteration of a call is
    applied before the call returns. With max_inner = 8 and 16 iterations per
    chunk, outer steps fall on chunk ends (16, 32), and a run split after
    iteration 24 (an outer step) equals one run of 40 bit for bit and the
    oracle."""
    note("parity c2: outer steps on chunk ends and call ends")
    g = config_grid("c2_2kbus")
    p = A.Params(max_inner=8)
    orc = O.Oracle(g, oparams(p))
    orc.solve(24)
    with A.Solver(g, p) as s:
        assert s.tuning()["chunk"] == 16
        s.solve(A.COLD, 24)
        compare(s, orc, label="c2 outer x24")
        np.testing.assert_array_equal(s.history()[:, 5], orc.history()[:, 5])
        orc.solve(16)
        s.solve(A.CONTINUE, 16)
        compare(s, orc, label="c2 outer x24+16")
        np.testing.assert_array_equal(s.history()[:, 5], orc.history()[:, 5])
        split = {k: s.get(k) for k in VECS}
        s.solve(A.COLD, 40)
        for k in VECS:
            np.testing.assert_array_equal(s.get(k), split[k], err_msg=k)
    assert orc.history()[-1, 5] == 4  # outer steps at 8, 16, 24 and 32 before the 40th


def test_c1_200_iterations_objective():
    note("parity c1 200 iterations objective")
    g = config_grid("c1_30bus")
    p = A.Params(rho_pq=400.0, rho_va=400.0)
    orc = O.Oracle(g, oparams(p))
    orc.solve(200)
    with A.Solver(g, p) as s:
        res = s.solve(A.COLD, 200)[0]
        compare(s, orc, tol=1e-8, label="c1x200")
        assert abs(res["objective"] - orc.objective()) <= 1e-6 * max(1.0, abs(orc.objective()))


def test_continue_equals_one_run_and_determinism():
    note("continue/determinism c1")
    g = config_grid("c1_30bus")
    p = A.Params(rho_pq=400.0, rho_va=400.0)
    with A.Solver(g, p) as s1, A.Solver(g, p) as s2:
        s1.solve(A.COLD, 40)
        s2.solve(A.COLD, 25)
        s2.solve(A.CONTINUE, 15)
        for k in VECS + ("rtil",):
            np.testing.assert_array_equal(s1.get(k), s2.get(k))
        a = s1.get("u")
        s1.solve(A.COLD, 40)
        np.testing.assert_array_equal(a, s1.get("u"))


@pytest.mark.parametrize("waves", list(XSTEP))
def test_edge_grids_match_oracle(waves):
    note(f"edge grids, x-step {waves}")
    cases = []
    # two buses, one branch, one generator; ragged sizes; shunts and taps
    g = gridgen(2, 1, 1, 1.0, 31)
    cases.append(("2bus", g))
    g = gridgen(67, 9, 70, 0.5, 32)
    rng = np.random.default_rng(0)
    g.gs = rng.uniform(0, 0.02, g.n_bus)
    g.bs = rng.uniform(-0.02, 0.02, g.n_bus)
    g.tap = rng.uniform(0.95, 1.05, g.n_branch)
    g.shift = rng.uniform(-0.1, 0.1, g.n_branch)
    cases.append(("ragged_taps_shunts", g))
    g = gridgen(130, 20, 200, 0.0, 33)
    cases.append(("all_unrated", g))
    for name, g in cases:
        p = A.Params(rho_pq=400.0, rho_va=4000.0)
        orc = O.Oracle(g, oparams(p))
        orc.solve(30)
        with A.Solver(g, p) as s:
            s.set_tuning(**XSTEP[waves])
            s.solve(A.COLD, 30)
            compare(s, orc, tol=1e-9, label=name)


def structural_grid():
    """A 90-bus grid with the structures a MATPOWER case can hold and the
    synthetic recipe does not draw: eight parallel lines (half of them
    reversed, half rated), generators with a fixed real or reactive output
    (pmin = pmax, qmin = qmax), three generators on one bus, the reference at
    a generator bus other than bus 0, negative loads, and a bus with
    vmin = vmax (its w bound interval is a point)."""
    g = gridgen(90, 12, 120, 0.5, 36, load_factor=0.2)
    rng = np.random.default_rng(36)
    pick = rng.choice(g.n_branch, 8, replace=False)
    rev = np.arange(8) % 2 == 1
    f = np.where(rev, g.br_to[pick], g.br_from[pick])
    t = np.where(rev, g.br_from[pick], g.br_to[pick])
    g.br_from = np.concatenate([g.br_from, f]).astype(g.br_from.dtype)
    g.br_to = np.concatenate([g.br_to, t]).astype(g.br_to.dtype)
    g.r = np.concatenate([g.r, rng.uniform(0.005, 0.05, 8)])
    g.x = np.concatenate([g.x, rng.uniform(0.02, 0.2, 8)])
    g.b = np.concatenate([g.b, rng.uniform(0.0, 0.05, 8)])
    g.tap = np.concatenate([g.tap, np.ones(8)])
    g.shift = np.concatenate([g.shift, np.zeros(8)])
    g.rate = np.concatenate([g.rate, np.where(np.arange(8) < 4, rng.uniform(1, 3, 8), 0.0)])
    g.pmin[1:4] = g.pmax[1:4] = 0.5 * g.pmax[1:4]
    g.qmin[4] = g.qmax[4] = 0.1
    g.gen_bus[6:8] = g.gen_bus[0]
    g.ref_bus = int(g.gen_bus[5])
    g.pd[10:13] = -0.05
    g.qd[10:13] = -0.01
    g.vmin[20] = g.vmax[20] = 1.0
    return g


@pytest.mark.parametrize("waves", list(XSTEP))
def test_structural_edge_cases_match_oracle(waves):
    note(f"structural edge cases (parallel lines, fixed outputs, shared bus, reference, "
         f"point bounds), x-step {waves}")
    g = structural_grid()
    p = A.Params(rho_pq=400.0, rho_va=4000.0)
    orc = O.Oracle(g, oparams(p))
    orc.solve(30)
    with A.Solver(g, p) as s:
        s.set_tuning(**XSTEP[waves])
        s.solve(A.COLD, 30)
        compare(s, orc, tol=1e-9, label="structural")
        sg, so = s.solution(), orc.solution()
        for name, want in so.items():
            err = np.abs(sg[name] - want).max() / max(np.abs(want).max(), 1e-30)
            assert err <= 1e-13, (name, err)
        # the fixed outputs are the generator step's projections onto a point
        assert np.array_equal(sg["pg"][1:4], g.pmax[1:4]) and sg["qg"][4] == 0.1


def star_grid(n_leaf: int, n_gen: int, seed: int):
    """One hub bus joined to n_leaf leaves, with every generator on the hub:
    at a bus block of 64 lanes the hub's branch ends and generators exceed the
    bus kernel's LDS capacities, so its global-memory path runs."""
    g = gridgen(n_leaf + 1, n_gen, n_leaf, 0.3, seed, load_factor=0.2)
    g.br_from = np.zeros(n_leaf, dtype=g.br_from.dtype)
    g.br_to = np.arange(1, n_leaf + 1, dtype=g.br_to.dtype)
    g.gen_bus = np.zeros(n_gen, dtype=g.gen_bus.dtype)
    g.ref_bus = 0
    return g


def test_high_degree_bus_matches_oracle():
    note("star grid: hub of degree 300 with 40 generators, bus blocks 64 and 256")
    g = star_grid(300, 40, 35)
    p = A.Params(rho_pq=400.0, rho_va=4000.0)
    orc = O.Oracle(g, oparams(p))
    orc.solve(30)
    out = []
    for bb in (64, 256):
        with A.Solver(g, p) as s:
            s.set_tuning(bus_block=bb)
            s.solve(A.COLD, 30)
            compare(s, orc, tol=1e-9, label=f"star bus_block {bb}")
            out.append({k: s.get(k) for k in VECS + ("rtil",)})
    for k in out[0]:
        np.testing.assert_array_equal(out[0][k], out[1][k])


def test_batch_equals_alone():
    note("batch vs alone")
    gs = [gridgen(50 + 13 * k, 8 + k, 70 + 17 * k, 0.6, 40 + k) for k in range(3)]
    p = A.Params(rho_pq=400.0, rho_va=4000.0)
    with A.Solver(gs, p) as sb:
        sb.solve(A.COLD, 25)
        for k, g in enumerate(gs):
            with A.Solver(g, p) as sa:
                sa.solve(A.COLD, 25)
                for name in VECS + ("rtil",):
                    np.testing.assert_array_equal(sa.get(name), sb.get(name, k))


def test_warm_start_matches_oracle():
    note("warm start c2")
    g = config_grid("c2_2kbus")
    p = A.Params(rho_pq=400.0, rho_va=40000.0)
    orc = O.Oracle(g, oparams(p))
    orc.solve(40)
    pd, qd = perturb_loads(g, 0.05, 1001)
    orc.update_loads(pd, qd)
    orc.solve(30)
    with A.Solver(g, p) as s:
        s.solve(A.COLD, 40)
        s.update_loads(0, pd, qd)
        s.solve(A.WARM, 30)
        compare(s, orc, tol=1e-9, label="warm")
        np.testing.assert_array_equal(s.get("pd"), pd)


_ORACLE_70K = {}


def oracle_70k(p: A.Params, iters: int) -> "O.Oracle":
    """The oracle run from the cold start on the 70k-bus grid (once per
    module: about 0.25 s per iteration on one core)."""
    key = (iters, p.rho_va)
    if key not in _ORACLE_70K:
        orc = O.Oracle(config_grid("c3_70kbus"), oparams(p))
        orc.solve(iters)
        _ORACLE_70K[key] = orc
    return _ORACLE_70K[key]


@pytest.mark.parametrize("waves", list(XSTEP))
def test_70k_matches_oracle_from_cold(waves):
    """Full-size grid: the GPU and the oracle both run 6 iterations from the
    same cold start; every state vector must agree element by element."""
    note(f"parity c3 70k: 6 iterations from cold, x-step {waves}")
    g = config_grid("c3_70kbus")
    p = A.Params(rho_pq=400.0, rho_va=40000.0)
    orc = oracle_70k(p, 6)
    with A.Solver(g, p) as s:
        s.set_tuning(**XSTEP[waves])
        s.solve(A.COLD, 6)
        compare(s, orc, tol=1e-9, label="70k cold+6")
        for k in ("rtil",):
            np.testing.assert_allclose(s.get(k), orc.get(k), rtol=0, atol=0)


def assert_quality_equal(qg, qo, label):
    note(f"{label} gpu {qg}")
    note(f"{label} oracle {qo}")
    for k, vo in qo.items():
        assert abs(qg[k] - vo) <= 1e-13 * max(1.0, abs(vo)), (label, k, qg[k], vo)


def test_quality_matches_oracle():
    """||c(x)||_inf over eq. acopf (Sec. IV-A solution: generator outputs and
    bus voltages, flows recomputed) on the GPU against the oracle: the 2k grid
    after 50 iterations, and a three-grid batch including taps, phase shifters
    and shunts, each grid against its own oracle."""
    note("quality: c2 after 50 iterations")
    g = config_grid("c2_2kbus")
    p = A.Params()
    orc = O.Oracle(g, oparams(p))
    orc.solve(50)
    with A.Solver(g, p) as s:
        s.solve(A.COLD, 50)
        assert_quality_equal(s.quality(), orc.quality(), "c2")
    note("quality: three-grid batch with taps and shunts")
    gs = [gridgen(67, 9, 70, 0.5, 32, load_factor=0.2), gridgen(130, 20, 200, 0.0, 33),
          gridgen(90, 12, 120, 1.0, 34, load_factor=0.2)]
    rng = np.random.default_rng(0)
    gs[0].gs = rng.uniform(0, 0.02, gs[0].n_bus)
    gs[0].bs = rng.uniform(-0.02, 0.02, gs[0].n_bus)
    gs[0].tap = rng.uniform(0.95, 1.05, gs[0].n_branch)
    gs[0].shift = rng.uniform(-0.1, 0.1, gs[0].n_branch)
    with A.Solver(gs, p) as s:
        s.solve(A.COLD, 30)
        for k, gk in enumerate(gs):
            orc = O.Oracle(gk, oparams(p))
            orc.solve(30)
            assert_quality_equal(s.quality(k), orc.quality(), f"batch grid {k}")


@pytest.mark.parametrize("name", ["c3_70kbus", "c3_70kbus_full"])
def test_70k_default_launch_50_iterations_matches_oracle(name):
    """The 70k-bus grid in the launch configuration the benchmark times
    (default parameters and tuning: graph chunks of 16, automatic branches
    per lane), 50 iterations from the same cold start: every state vector,
    the residual history and the TRON event counts equal the oracle's. Also
    at the stated load distribution (load factor 1 and the 0.75 guard), where
    line limits bind and the branch AL loop takes extra rounds."""
    note(f"parity {name}: 50 iterations from cold, default launch, counting on")
    g = config_grid(name)
    p = A.Params()
    orc = O.Oracle(g, oparams(p))
    orc.count_flops(True)
    orc.solve(50)
    with A.Solver(g, p) as s:
        s.set_counting(True)
        s.solve(A.COLD, 50)
        compare(s, orc, tol=1e-9, label=f"{name} cold+50")
        np.testing.assert_array_equal(s.get("rtil"), orc.get("rtil"))
        hg, ho = s.history(), orc.history()
        np.testing.assert_array_equal(hg[:, [0, 1, 2]], ho[:, [0, 1, 2]])
        sg, so = s.stats(), orc.stats()
        for k in ("branch_solves", "tron_iters", "cauchy_trials", "cg_iters", "al_iters", "flops"):
            assert sg[k] == so[k], (k, sg[k], so[k])


def test_quality_70k_matches_oracle():
    note("quality: 70k grid after 6 iterations from cold, GPU and oracle")
    g = config_grid("c3_70kbus")
    p = A.Params(rho_pq=400.0, rho_va=40000.0)
    orc = oracle_70k(p, 6)
    with A.Solver(g, p) as s:
        s.solve(A.COLD, 6)
        assert_quality_equal(s.quality(), orc.quality(), "70k")


def test_70k_cold_solve_converges_with_default_parameters():
    """The benchmark's grid from a cold start to the termination test of
    Algorithm 1 with the library's default parameters (including the branch
    solver's tolerance readings): converged, residuals within the
    tolerances, the reported objective equal to the generator costs at the
    generator-side outputs, and a small constraint violation (Sec. IV-A)."""
    note("70k grid: cold solve to convergence with default parameters")
    g = config_grid("c3_70kbus")
    p = A.Params()
    with A.Solver(g, p) as s:
        res = s.solve(A.COLD)[0]
        assert res["status"] == A.CONVERGED, res
        assert res["r_pri"] <= p.eps_pri and res["r_dual"] <= p.eps_dual and res["r_z"] <= p.eps_z
        assert res["inner_iters"] < p.max_outer * p.max_inner
        u = s.get("u")
        pg = u[0:2 * g.n_gen:2] * g.base_mva
        cost = float(np.sum(g.c2 * pg * pg + g.c1 * pg + g.c0))
        assert abs(res["objective"] - cost) <= 1e-9 * abs(cost)
        q = s.quality()
        assert q["max_violation"] <= 1e-2, q
        assert q["line_limit"] <= 1e-6 and q["voltage_limit"] <= 1e-12, q


def test_tracking_horizon_matches_oracle():
    """Four periods of the tracking horizon (Sec. IV-C: loads drift, warm
    start, ramp-limited generator bounds) on the GPU and in the oracle: the
    same inner iterations and solution quality per period, the same final
    state, and ramp limits respected."""
    from paper_2110_06879_amd import tracking as T
    note("tracking: 60-bus grid, 4 periods")
    g = gridgen(60, 12, 80, 0.5, 71, load_factor=0.2)
    p = A.Params()
    with A.Solver(g, p) as s:
        recs = T.track(s, g, 0, periods=4)
        orc = O.Oracle(g, oparams(p))
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
            sc = orc.scalars()
            note(f"period {t}: gpu {recs[t]['inner_iters']} iters, oracle {int(sc['inner_total'])}")
            assert recs[t]["inner_iters"] == int(sc["inner_total"]), t
            qo = orc.quality()["max_violation"]
            assert abs(recs[t]["max_violation"] - qo) <= 1e-13 * max(1.0, qo), t
            assert recs[t]["ramp_ratio"] <= 1.0 + 1e-12
            p_prev = T.generator_p(orc.get("u"), g.n_gen)
        compare(s, orc, label="tracking final")


def test_matpower_case_matches_oracle():
    """A grid read from a MATPOWER case file (hand-made 5-bus case with a
    phase-shifting transformer, a shunt, two generators on one bus and
    out-of-service elements) on the GPU against the oracle."""
    import os
    from paper_2110_06879_amd import matpower as M
    note("MATPOWER case: 100 iterations")
    g = M.load_case(os.path.join(os.path.dirname(__file__), "golden", "case5_handmade.m"))
    p = A.Params(rho_pq=400.0, rho_va=4000.0)
    orc = O.Oracle(g, oparams(p))
    orc.solve(100)
    with A.Solver(g, p) as s:
        s.solve(A.COLD, 100)
        compare(s, orc, label="case5")
        assert_quality_equal(s.quality(), orc.quality(), "case5")


def test_beta_growth_and_lambda_clamp_match_oracle():
    """The outer level of Algorithm 1 (eq. two-level) with the beta rule
    active: beta0 = 1e3 below beta_max = 2e4, an outer step every ten inner
    iterations (max_inner = 10), and lambda_max = 20 so that the projection
    of lambda binds. After 60 iterations beta has grown twice (the second
    time to the cap), lambda sits at the clamp on some couplings, and every
    vector and the beta/outer history equal the oracle's."""
    note("parity c2: beta growth and lambda clamp, 60 iterations")
    g = config_grid("c2_2kbus")
    p = A.Params(beta0=1e3, beta_max=2e4, max_inner=10, lambda_max=20.0)
    orc = O.Oracle(g, oparams(p))
    orc.solve(60)
    ho = orc.history()
    betas = np.unique(ho[:, 4])
    assert list(betas) == [1e3, 6e3, 2e4], betas
    lam = orc.get("lam")
    assert (np.abs(lam) == 20.0).sum() > 100
    with A.Solver(g, p) as s:
        res = s.solve(A.COLD, 60)[0]
        compare(s, orc, label="c2 beta/lambda")
        hg = s.history()
        np.testing.assert_array_equal(hg[:, 4], ho[:, 4])
        np.testing.assert_array_equal(hg[:, 5], ho[:, 5])
        np.testing.assert_array_equal(s.get("lam"), lam)
        assert res["beta"] == orc.scalars()["beta"] == 2e4


def test_2k_cold_solve_to_convergence_matches_oracle():
    """A cold solve of the 2k-bus grid to the termination tests of Algorithm
    1: the same inner and outer iteration counts, the objective within 1e-6
    of the oracle's at that count, and the final state within 1e-9."""
    note("parity c2: cold solve to convergence")
    g = config_grid("c2_2kbus")
    p = A.Params()
    orc = O.Oracle(g, oparams(p))
    n = orc.solve(0)
    sc = orc.scalars()
    assert sc["status"] == 0
    with A.Solver(g, p) as s:
        res = s.solve(A.COLD)[0]
        note(f"gpu {res['inner_iters']} iterations, oracle {n}")
        assert res["status"] == A.CONVERGED
        assert res["inner_iters"] == n and res["outer_iters"] == int(sc["outer"])
        assert abs(res["objective"] - orc.objective()) <= 1e-6 * abs(orc.objective())
        compare(s, orc, label="c2 converged")


def test_70k_cold_solve_to_convergence_matches_oracle():
    """The benchmark's 70k-bus grid from a cold start to the termination tests
    of Algorithm 1, against the oracle run to its own termination (OpenMP
    over the host's threads, bitwise its serial results): the same inner and
    outer iteration counts, the objective within 1e-6 of the oracle's, and
    every state vector within the parity tolerance."""
    import os
    note("parity c3 70k: cold solve to convergence against the oracle")
    g = config_grid("c3_70kbus")
    p = A.Params()
    orc = O.Oracle(g, oparams(p))
    orc.set_threads(max(1, min(16, os.cpu_count() or 1)))
    n = orc.solve(0)
    sc = orc.scalars()
    assert sc["status"] == 0
    with A.Solver(g, p) as s:
        res = s.solve(A.COLD)[0]
        note(f"gpu {res['inner_iters']} iterations, oracle {n}")
        assert res["status"] == A.CONVERGED
        assert res["inner_iters"] == n and res["outer_iters"] == int(sc["outer"])
        assert abs(res["objective"] - orc.objective()) <= 1e-6 * abs(orc.objective())
        compare(s, orc, label="c3 converged")


def test_largest_grid_matches_oracle():
    """The largest single grid of the size scaling, 1.12 million buses
    (160,000 generators, 1,408,000 branches, 30% rated): the x-step puts one
    unlimited branch on each lane and its launch holds many rounds of
    wavefronts, and each decision block loops over thousands of tile slots.
    One graph chunk of 16 iterations from a cold start, in the default launch
    configuration, against the oracle (OpenMP over the host's threads)."""
    import os
    nb = 1120000
    note("parity 1.12M buses: 16 iterations in one graph chunk")
    g = gridgen(nb, nb // 7, int(round(nb * 88 / 70)), 0.3, 907, load_factor=0.2)
    p = A.Params()
    orc = O.Oracle(g, oparams(p))
    orc.set_threads(max(1, min(16, os.cpu_count() or 1)))
    orc.solve(16)
    with A.Solver(g, p) as s:
        assert s.tuning()["chunk"] == 16
        s.solve(A.COLD, 16)
        compare(s, orc, label="1.12M buses")


def tightened(name, factor):
    g = config_grid(name)
    g.rate = g.rate * factor
    return g


@pytest.mark.parametrize("name", ["c2_2kbus_tight", "c2_2kbus_full"])
def test_binding_line_limits_match_oracle(name):
    """Grids where line limits bind, so that the augmented-Lagrangian loop of
    eq. (branch) takes several rounds and its multipliers and penalties
    move: the 2k-bus grid with every rating scaled by 0.15, and the 2k-bus
    grid at the stated load distribution. 50 iterations from the cold start,
    element-wise against the oracle, with the AL event counts equal."""
    note(f"parity {name}: binding line limits, 50 iterations")
    g = tightened("c2_2kbus", 0.15) if name == "c2_2kbus_tight" else config_grid(name)
    p = A.Params()
    orc = O.Oracle(g, oparams(p))
    orc.solve(50)
    lt, rt = orc.get("ltil"), orc.get("rtil")
    n_bind = int((np.abs(lt) > 1e-3).sum())
    n_grow = int((rt > p.al_rho0).sum())
    note(f"{name}: {n_bind} binding multipliers, {n_grow} grown penalties")
    assert n_bind >= 10 and n_grow >= 20
    with A.Solver(g, p) as s:
        s.set_counting(True)
        s.solve(A.COLD, 50)
        compare(s, orc, label=name)
        np.testing.assert_array_equal(s.get("rtil"), rt)
        assert s.stats()["al_iters"] == orc.stats()["al_iters"] > 50 * g.n_branch


def uneven_batch():
    """Eight grids of uneven size (500 to 5,000 buses, log-spaced), with
    rated fractions 1, 0.3 and 0 mixed, at the default load factor."""
    sizes = np.round(np.exp(np.linspace(np.log(500), np.log(5000), 8))).astype(int)
    rf = [1.0, 0.3, 0.0, 1.0, 0.3, 1.0, 0.0, 0.3]
    out = []
    for k, nb in enumerate(sizes.tolist()):
        out.append(gridgen(nb, max(1, round(0.2 * nb)), round(1.3 * nb), rf[k], 600 + k,
                           load_factor=0.2))
    return out


def test_uneven_batch_with_staggered_starts_matches_oracles():
    """Batched launch (one handle, the same kernels for all grids) of eight
    uneven grids started at different iterations: each grid runs exactly 30
    iterations from its cold start, and every state vector of every grid
    equals its own oracle's."""
    note("batch of 8 uneven grids, staggered starts, each against its oracle")
    gs = uneven_batch()
    p = A.Params()
    with A.Solver(gs, p) as sb:
        for k in range(len(gs)):
            sb.start(k, A.COLD, 30)
            sb.run(5 + 3 * k)
        while sb.run(64) > 0:
            pass
        for k, g in enumerate(gs):
            running, res = sb.poll(k)
            assert not running and res["inner_iters"] == 30
            orc = O.Oracle(g, oparams(p))
            orc.solve(30)
            compare(sb, orc, grid=k, label=f"batch grid {k} ({g.n_bus} buses)")
            np.testing.assert_array_equal(sb.get("rtil", k), orc.get("rtil"))


def test_solution_view_matches_oracle():
    """acopf_get_state(ACOPF_SOLUTION): the ADMM solution of Sec. IV-A
    (generator outputs, |V| and theta from the bus problems, flows
    recomputed from the bus voltages) of each grid of a batch (taps, phase
    shifters and shunts on one of them) against the oracle's recovery."""
    note("solution view: 3-grid batch after 30 iterations")
    gs = [gridgen(67, 9, 70, 0.5, 32, load_factor=0.2), gridgen(130, 20, 200, 0.0, 33),
          gridgen(90, 12, 120, 1.0, 34, load_factor=0.2)]
    rng = np.random.default_rng(0)
    gs[0].gs = rng.uniform(0, 0.02, gs[0].n_bus)
    gs[0].bs = rng.uniform(-0.02, 0.02, gs[0].n_bus)
    gs[0].tap = rng.uniform(0.95, 1.05, gs[0].n_branch)
    gs[0].shift = rng.uniform(-0.1, 0.1, gs[0].n_branch)
    p = A.Params()
    with A.Solver(gs, p) as s:
        s.solve(A.COLD, 30)
        for k, gk in enumerate(gs):
            orc = O.Oracle(gk, oparams(p))
            orc.solve(30)
            sg, so = s.solution(k), orc.solution()
            for name, want in so.items():
                got = sg[name]
                assert got.shape == want.shape, name
                err = np.abs(got - want).max() / max(np.abs(want).max(), 1e-30)
                assert err <= 1e-13, (k, name, err)
