"""GPU tests of the driver: hipGraph chunks, continuous batching (per-grid
start/run/poll), device-side state copies and snapshots, the autotuner, and
the serving loop's alone-versus-mix equality. All comparisons are bitwise:
grids are independent problems, so their arithmetic cannot depend on the
launch shape or on the other grids in the batch."""
import sys

import numpy as np
import pytest

from paper_2110_06879_amd import acopf as A
from paper_2110_06879_amd import serve as S
from paper_2110_06879_amd.gridgen import config_grid, gridgen, perturb_loads

pytestmark = pytest.mark.gpu
VECS = ("u", "v", "z", "y", "lam", "bx", "ltil", "rtil", "calpha")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def states(s, grid=0):
    return {k: s.get(k, grid) for k in VECS}


def assert_same(a, b):
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_graph_replay_equals_plain_launches():
    note("graph vs plain, 2k grid, 48 iterations")
    g = config_grid("c2_2kbus")
    with A.Solver(g) as s1, A.Solver(g) as s2:
        s1.set_tuning(use_graph=1, chunk=16)
        s2.set_tuning(use_graph=0, chunk=16)
        s1.solve(A.COLD, 48)
        s2.solve(A.COLD, 48)
        assert_same(states(s1), states(s2))
        s1.set_tuning(use_graph=1, chunk=8, xstep_block=128, bus_block=512)
        s1.solve(A.CONTINUE, 40)
        s2.solve(A.CONTINUE, 40)
        assert_same(states(s1), states(s2))


def test_profiling_with_chunks_up_to_the_maximum():
    """Per-launch timing with the longest chunks set_tuning accepts (32 and
    64 iterations between readbacks): every iteration of a chunk has its own
    events, the timing comes back positive, and the iterates equal those of
    the default chunk."""
    note("profiling with chunks 32 and 64, 2k grid, 130 iterations")
    g = config_grid("c2_2kbus")
    with A.Solver(g) as ref:
        ref.solve(A.COLD, 130)
        want = states(ref)
    for chunk in (32, 64):
        with A.Solver(g) as s:
            s.set_tuning(chunk=chunk)
            s.set_profiling(True)
            s.solve(A.COLD, 130)
            t = s.timing()
            assert t["iters"] >= 130 and t["xstep_ms"] > 0.0 and t["bus_ms"] > 0.0, t
            assert_same(states(s), want)


@pytest.mark.parametrize("variant", [dict(xstep_waves=1), dict(xstep_waves=2),
                                     dict(xstep_per_lane=3), dict(xstep_per_lane=8, xstep_block=128)])
def test_xstep_variants_equal_lane_per_branch(variant):
    """The pool kernel and several branches per lane change which lane solves
    which branch, never the arithmetic of a solve: states, per-grid results
    and every event and flop count are bitwise those of one branch per lane,
    also while grids of the batch finish at different iterations."""
    note(f"x-step {variant} vs one branch per lane, 4-grid batch to convergence")
    gs = [gridgen(200 + 90 * k, 40 + 9 * k, 260 + 120 * k, 0.3 * k, 70 + k, load_factor=0.2)
          for k in range(4)]
    with A.Solver(gs) as s1, A.Solver(gs) as s2:
        s1.set_tuning(xstep_waves=0, xstep_per_lane=1)
        s2.set_tuning(**variant)
        s1.set_counting(True)
        s2.set_counting(True)
        r1 = s1.solve(A.COLD)
        r2 = s2.solve(A.COLD)
        for a, b in zip(r1, r2):
            for k in ("status", "inner_iters", "outer_iters", "branch_failures", "objective",
                      "r_pri", "r_dual", "r_z"):
                assert a[k] == b[k], (k, a[k], b[k])
        for k in range(len(gs)):
            assert_same(states(s1, k), states(s2, k))
        assert s1.stats() == s2.stats()


@pytest.mark.parametrize("waves", [0, 1])
def test_counting_leaves_results_unchanged(waves):
    """Counting flops and events (acopf_set_counting) only adds integer
    counters: every state is bitwise the same with and without it, and
    without it the counters stay zero."""
    note(f"counting on vs off, xstep_waves {waves}")
    g = config_grid("c2_2kbus")
    with A.Solver(g) as s1, A.Solver(g) as s2:
        s1.set_tuning(xstep_waves=waves)
        s2.set_tuning(xstep_waves=waves)
        s1.set_counting(True)
        s1.solve(A.COLD, 40)
        s2.solve(A.COLD, 40)
        assert_same(states(s1), states(s2))
        assert s1.stats()["branch_solves"] == 40 * g.n_branch
        assert all(v == 0 for v in s2.stats().values())


def test_staggered_starts_equal_alone():
    note("continuous batching: staggered starts")
    gs = [gridgen(300 + 50 * k, 60 + 10 * k, 390 + 60 * k, 1.0, 60 + k, load_factor=0.2)
          for k in range(3)]
    with A.Solver(gs) as sb:
        sb.start(0, A.COLD, 60)
        sb.run(16)
        sb.start(1, A.COLD, 60)
        sb.run(16)
        sb.start(2, A.COLD, 60)
        while sb.run(64) > 0:
            pass
        for k, g in enumerate(gs):
            running, res = sb.poll(k)
            assert not running and res["inner_iters"] == 60
            with A.Solver(g) as sa:
                sa.solve(A.COLD, 60)
                assert_same(states(sa), states(sb, k))


def test_copy_grid_and_snapshot_roundtrip():
    note("copy_grid and snapshot")
    g = gridgen(400, 80, 520, 1.0, 71, load_factor=0.2)
    with A.Solver([g, g]) as s:
        s.start(0, A.COLD, 30)
        while s.run(64) > 0:
            pass
        s.copy_grid(0, 1)
        assert_same(states(s, 0), states(s, 1))
        s.snapshot()
        base = states(s, 0)
        s.start(0, A.CONTINUE, 20)
        s.start(1, A.CONTINUE, 20)
        while s.run(64) > 0:
            pass
        assert_same(states(s, 0), states(s, 1))
        s.snapshot(restore=True)
        assert_same(states(s, 0), base)


def test_autotune_leaves_state_unchanged():
    note("autotune")
    g = config_grid("c2_2kbus")
    with A.Solver(g) as s:
        s.solve(A.COLD, 20)
        before = states(s)
        t = s.autotune(8)
        assert t["xstep_block"] in (64, 128, 256) and t["chunk"] in (8, 16, 32)
        assert_same(states(s), before)
        s.solve(A.CONTINUE, 10)
        with A.Solver(g) as r:
            r.solve(A.COLD, 30)
            assert_same(states(s), states(r))


def test_autotune_cache_round_trip(tmp_path):
    """autotune(cache=...) measures and stores on a miss; a second handle for
    the same workload applies the stored tuning without measuring."""
    note("autotune cache")
    g = config_grid("c2_2kbus")
    path = str(tmp_path / "tune.json")
    with A.Solver(g) as s:
        t1 = s.autotune(4, cache=path)
        assert A.load_tuning(path, A.tuning_key(g)) == t1
    with A.Solver(g) as r:
        r.set_tuning(xstep_block=256, chunk=8)
        t2 = r.autotune(4, cache=path)
        assert t2 == t1 and r.tuning() == t1


def test_serving_results_same_alone_and_in_mix():
    note("serving: alone vs mix")
    gs = [gridgen(250 + 40 * k, 50 + 8 * k, 325 + 52 * k, 1.0, 80 + k, load_factor=0.2)
          for k in range(3)]
    reqs = []
    for k in range(3):
        for t in range(2):
            pd, qd = perturb_loads(gs[k], 0.02, 900 + 10 * k + t)
            reqs.append(S.Request(len(reqs), k, 0.0, pd, qd))
    srv = S.TrackingServer(gs, max_slots_per_grid=2)
    out = srv.serve(reqs, realtime=False)
    assert out["requests"] == len(reqs)
    mix = {r.rid: r for r in out["done"]}
    # every request was admitted at once into its own slot, so each slot
    # still holds its request's final state
    assert len({r.slot for r in out["done"]}) == len(reqs)
    mixed_states = {r.rid: states(srv.solver, r.slot) for r in out["done"]}
    srv.close()
    for r in reqs:
        alone = S.TrackingServer(gs, max_slots_per_grid=2)
        one = S.Request(r.rid, r.grid, 0.0, r.pd, r.qd)
        o = alone.serve([one], realtime=False)["done"][0]
        got = states(alone.solver, o.slot)
        alone.close()
        for k in ("status", "inner_iters", "outer_iters", "objective", "r_pri", "r_dual", "r_z"):
            assert o.result[k] == mix[r.rid].result[k], (r.rid, k)
        assert_same(got, mixed_states[r.rid])


def test_served_request_matches_oracle_warm_start():
    """A served tracking request against the oracle: the server's resident
    state of a grid is its cold solve to convergence (bitwise the oracle's),
    a request warm-starts a copy of it with new loads (Sec. IV-C), and the
    result must equal the oracle's warm start from the same base state: the
    same iteration count and status, the objective within 1e-6, and every
    state vector within 1e-9."""
    import oracle as O
    from dataclasses import asdict
    note("serving: served warm start against the oracle")
    gs = [gridgen(300, 60, 390, 1.0, 85, load_factor=0.2),
          gridgen(420, 84, 546, 0.3, 86, load_factor=0.2)]
    p = A.Params()
    reqs = []
    for k in range(2):
        pd, qd = perturb_loads(gs[k], 0.03, 960 + k)
        reqs.append(S.Request(k, k, 0.0, pd, qd))
    srv = S.TrackingServer(gs, p, max_slots_per_grid=1)
    out = srv.serve(reqs, realtime=False)
    done = {r.rid: r for r in out["done"]}
    try:
        for k, g in enumerate(gs):
            orc = O.Oracle(g, O.OracleParams(**asdict(p)))
            n_cold = orc.solve(0)
            assert n_cold == srv.cold[k]["inner_iters"]
            orc.update_loads(reqs[k].pd, reqs[k].qd)
            n = orc.solve(0)
            r = done[k]
            note(f"grid {k}: served {r.result['inner_iters']} iterations, oracle {n}")
            assert r.result["status"] == A.CONVERGED and orc.scalars()["status"] == 0
            assert r.result["inner_iters"] == n
            assert abs(r.result["objective"] - orc.objective()) <= 1e-6 * abs(orc.objective())
            for name in VECS:
                a, b = srv.solver.get(name, r.slot), orc.get(name)
                err = np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)
                assert err <= 1e-9, (k, name, err)
    finally:
        srv.close()


def test_serving_budget_without_slots_runs_on_home():
    note("serving: budget allows no slots")
    gs = [gridgen(200, 40, 260, 1.0, 90, load_factor=0.2)]
    budget = S.instance_bytes(gs[0]) * 1.5
    srv = S.TrackingServer(gs, hbm_budget_bytes=budget)
    assert srv.slots_per_grid == [0]
    reqs = [S.Request(i, 0, 0.0, *perturb_loads(gs[0], 0.02, 950 + i)) for i in range(3)]
    out = srv.serve(reqs, realtime=False)
    srv.close()
    assert out["requests"] == 3 and out["converged"] == 3
    with pytest.raises(ValueError):
        S.TrackingServer(gs, hbm_budget_bytes=budget * 0.1)


def test_step_length_state_round_trip_and_validation():
    """The per-branch Cauchy step length is state like x and the AL terms:
    set_state/get_state round-trip positive values exactly, a new handle's
    cold state holds 1, and non-positive or non-finite values are refused."""
    note("calpha state: round trip and validation")
    g = config_grid("c1_30bus")
    with A.Solver(g) as s:
        s.solve(A.COLD, 5)
        a = s.get("calpha")
        assert a.shape == (g.n_branch,) and np.all(a > 0.0)
        want = np.linspace(0.25, 40.0, g.n_branch)
        s.set("calpha", want)
        np.testing.assert_array_equal(s.get("calpha"), want)
        for bad in (np.zeros(g.n_branch), -want, np.full(g.n_branch, np.nan)):
            with pytest.raises(A.AcopfError):
                s.set("calpha", bad)
        np.testing.assert_array_equal(s.get("calpha"), want)
    with A.Solver(g) as r:
        np.testing.assert_array_equal(r.get("calpha"), np.ones(g.n_branch))


def test_launches_over_running_subsets_equal_alone():
    """Launches sized to the running grids only: with every other grid of a
    16-grid batch running, the x-step takes its blocks from the work-item list
    (more than 12 segments), with three adjacent grids running from argument
    segments, and after each change of the running set the captured chunk's
    nodes are resized. Every grid's iterates equal those of the grid solved
    alone, and grids that did not run are untouched."""
    note("batch of 16: alternate grids, then three adjacent ones, against alone runs")
    gs = [gridgen(60 + 9 * k, 10 + k % 5, 80 + 12 * k, 0.5, 300 + k, load_factor=0.2)
          for k in range(16)]
    p = A.Params()
    want = {}
    for k, g in enumerate(gs):
        with A.Solver(g, p) as s:
            s.solve(A.COLD, 20)
            want[k] = states(s)
    with A.Solver(gs, p) as sb:
        sb.set_tuning(chunk=8)
        sb.solve(A.COLD, 1)  # every grid solved once, so WARM/CONTINUE starts are allowed
        before = {k: states(sb, k) for k in range(16)}
        for k in range(0, 16, 2):
            sb.start(k, A.COLD, 20)
        while sb.run(8) > 0:
            pass
        for k in range(16):
            if k % 2 == 0:
                assert_same(states(sb, k), want[k])
            else:
                assert_same(states(sb, k), before[k])
        for k in (5, 6, 7):
            sb.start(k, A.COLD, 20)
        while sb.run(8) > 0:
            pass
        for k in (5, 6, 7):
            assert_same(states(sb, k), want[k])


def test_server_commits_each_finished_slot_as_home():
    """The native tracking server: 30 requests over 3 grids with 2 slots
    each, all available at once. Every request converges on an instance of
    its own grid; the instance of each grid's last finished request is that
    grid's home afterwards; and a further request for a grid warm-starts from
    that home (its result equals a warm start of the same loads on a plain
    handle holding the home's state)."""
    note("native server: 30 requests, homes follow the finished slots")
    gs = [gridgen(120 + 30 * k, 20 + 4 * k, 156 + 39 * k, 0.5, 70 + k, load_factor=0.2)
          for k in range(3)]
    srv = S.TrackingServer(gs, max_slots_per_grid=2)
    try:
        assert srv.slots_per_grid == [2, 2, 2]
        inst = {j: [j] + [3 + 2 * j, 4 + 2 * j] for j in range(3)}
        reqs = []
        for r in range(30):
            j = r % 3
            pd, qd = perturb_loads(gs[j], 0.02, 700 + r)
            reqs.append(S.Request(r, j, 0.0, pd, qd))
        out = srv.serve(reqs, realtime=False)
        assert out["requests"] == 30 and out["converged"] == 30
        done = out["done"]
        for r in done:
            assert r.slot in inst[r.grid]
        home = srv.home()
        for j in range(3):
            assert home[j] == [r for r in done if r.grid == j][-1].slot
        # one more request for grid 1 starts from its home's state
        base = states(srv.solver, home[1])
        pd, qd = perturb_loads(gs[1], 0.02, 799)
        last = srv.serve([S.Request(99, 1, 0.0, pd, qd)], realtime=False)["done"][0]
        assert last.slot != home[1]
        with A.Solver(gs[1]) as ref:
            ref.solve(A.COLD, 1)
            for k, v in base.items():
                ref.set(k, v)
            ref.set("scalars", srv.solver.get("scalars", home[1]))
            ref.update_loads(0, pd, qd)
            want = ref.solve(A.WARM)[0]
            assert want["inner_iters"] == last.result["inner_iters"]
            assert want["objective"] == last.result["objective"]
            assert_same(states(ref), states(srv.solver, last.slot))
    finally:
        srv.close()


def test_two_handles_on_two_host_threads_equal_one_after_the_other():
    """Handles are independent: two handles on their own streams, driven from
    two host threads at once (cold solves, then warm starts after new loads),
    end with bitwise the iterates of the same solves run one after the
    other."""
    import threading
    gs = [gridgen(400 + 100 * k, 60 + 10 * k, 520 + 130 * k, 0.5, 140 + k, load_factor=0.2)
          for k in range(2)]
    loads = [perturb_loads(g, 0.02, 1400 + k) for k, g in enumerate(gs)]

    def run(g, ld, out, k):
        with A.Solver(g) as s:
            s.solve(A.COLD, 40)
            s.update_loads(0, *ld)
            out[k] = (s.solve(A.WARM, 30)[0], states(s))

    seq, par = {}, {}
    for k in range(2):
        run(gs[k], loads[k], seq, k)
    errs = []

    def guarded(k):
        try:
            run(gs[k], loads[k], par, k)
        except Exception as e:  # surfaced below
            errs.append(e)

    ts = [threading.Thread(target=guarded, args=(k,)) for k in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errs, errs
    for k in range(2):
        assert seq[k][0]["inner_iters"] == par[k][0]["inner_iters"]
        assert seq[k][0]["objective"] == par[k][0]["objective"]
        assert_same(seq[k][1], par[k][1])


@pytest.mark.parametrize("lanes", [2, 4])
def test_launch_lanes_equal_one_lane(lanes):
    """Launch lanes: the grids of a handle split into groups launched on
    streams of their own, whose chunks run concurrently. Grids of different
    lanes share no data, so every grid's results, iterates and branch state
    are bitwise those of one lane, through convergence at different
    iterations, staggered starts and a running set that changes."""
    note(f"5 uneven grids: {lanes} lanes against one")
    gs = [gridgen(150 + 70 * k, 30 + 6 * k, 200 + 95 * k, 0.4, 700 + k, load_factor=0.2)
          for k in range(5)]
    with A.Solver(gs) as s1, A.Solver(gs) as s2:
        s1.set_tuning(lanes=1)
        s2.set_tuning(lanes=lanes)
        assert s1.tuning()["lanes"] == 1 and s2.tuning()["lanes"] == lanes
        r1 = s1.solve(A.COLD)
        r2 = s2.solve(A.COLD)
        for a, b in zip(r1, r2):
            for k in ("status", "inner_iters", "outer_iters", "branch_failures", "objective",
                      "r_pri", "r_dual", "r_z"):
                assert a[k] == b[k], (k, a[k], b[k])
        for s in (s1, s2):
            s.start(3, A.WARM, 40)
            s.run(16)
            s.start(0, A.WARM, 25)
            while s.run(64) > 0:
                pass
        for k in range(len(gs)):
            assert_same(states(s1, k), states(s2, k))


def test_launch_lanes_clamped_and_persistent_kernel_one_lane():
    """More lanes than grids are reduced to the number of grids, and the
    persistent branch kernel, which pools every branch of the handle, runs as
    one lane."""
    note("lanes clamped to the grids; persistent kernel as one lane")
    gs = [gridgen(120 + 40 * k, 20, 160 + 50 * k, 0.3, 750 + k, load_factor=0.2)
          for k in range(3)]
    with A.Solver(gs) as s:
        assert s.tuning()["lanes"] == 2
        s.set_tuning(lanes=4)
        assert s.tuning()["lanes"] == 3
        s.set_tuning(xstep_waves=1)
        assert s.tuning()["lanes"] == 1
        with pytest.raises(A.AcopfError):
            s.set_tuning(lanes=5)
    with A.Solver(gs[0]) as s:
        assert s.tuning()["lanes"] == 1
