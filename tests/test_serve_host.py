"""CPU tests of the serving scheduler (paper_2110_06879_amd.serve): slot
allocation under the HBM budget, admission, commits (the finished slot becomes
the home) and the home-only
path, with a stand-in for the device solver that only counts iterations.
The arithmetic of a solve is covered by the GPU tests; here only the host
logic runs."""
import numpy as np
import pytest

from paper_2110_06879_amd import acopf as A
from paper_2110_06879_amd import serve as S
from paper_2110_06879_amd.gridgen import gridgen


class FakeSolver:
    """Instances (homes then slots) that each need a fixed number of
    iterations per start; records every call the server makes."""

    def __init__(self, inst, params=None, device=0):
        self.inst = inst
        self.remaining = [0] * len(inst)
        self.state = list(range(len(inst)))   # which commit each instance holds
        self.loads = [None] * len(inst)
        self.log = []
        self.iters_per_start = {A.COLD: 7, A.WARM: 3}

    def tuning(self):
        return {"xstep_block": 64, "bus_block": 256, "chunk": 2, "use_graph": 1,
                "xstep_waves": 0}

    def start(self, grid, mode=A.WARM, fixed_iters=0):
        assert self.remaining[grid] == 0, "start on a running instance"
        self.remaining[grid] = self.iters_per_start[mode]
        self.log.append(("start", grid, mode))

    def run(self, max_iters=1 << 20):
        n = 0
        for k in range(len(self.remaining)):
            if self.remaining[k] > 0:
                self.remaining[k] = max(0, self.remaining[k] - max_iters)
                n += self.remaining[k] > 0
        return n

    def is_running(self, grid):
        return self.remaining[grid] > 0

    def poll(self, grid):
        return self.is_running(grid), {"status": A.CONVERGED, "inner_iters": 3,
                                       "r_pri": 0.0, "r_dual": 0.0, "r_z": 0.0,
                                       "state": self.state[grid], "loads": self.loads[grid]}

    def copy_grid(self, src, dst):
        assert self.remaining[dst] == 0, "copy into a running instance"
        self.state[dst] = self.state[src]
        self.loads[dst] = self.loads[src]
        self.log.append(("copy", src, dst))

    def update_loads(self, grid, pd, qd):
        assert self.remaining[grid] == 0
        self.loads[grid] = float(np.asarray(pd)[0])
        self.log.append(("loads", grid))

    def close(self):
        pass


@pytest.fixture
def fake(monkeypatch):
    monkeypatch.setattr(A, "Solver", FakeSolver)


def grids3():
    return [gridgen(40 + 20 * k, 6, 50 + 25 * k, 0.3, 90 + k, load_factor=0.2) for k in range(3)]


def test_slots_follow_budget(fake):
    gs = grids3()
    sizes = [S.instance_bytes(g) for g in gs]
    # room for the homes and exactly one slot of the smallest grid
    srv = S.TrackingServer(gs, hbm_budget_bytes=sum(sizes) + min(sizes), max_slots_per_grid=4)
    assert srv.slots_per_grid == [1, 0, 0]
    assert srv.bytes_used <= sum(sizes) + min(sizes)
    # a large budget stops at the per-grid cap
    srv = S.TrackingServer(gs, hbm_budget_bytes=1e12, max_slots_per_grid=2)
    assert srv.slots_per_grid == [2, 2, 2]
    # the handle holds homes first, then each grid's slots
    assert len(srv.solver.inst) == 3 + 6
    assert srv.slot_ids == [[3, 4], [5, 6], [7, 8]]


def test_budget_below_homes_rejected(fake):
    gs = grids3()
    with pytest.raises(ValueError):
        S.TrackingServer(gs, hbm_budget_bytes=S.instance_bytes(gs[0]))


def test_every_request_served_and_committed_in_order(fake):
    gs = grids3()
    srv = S.TrackingServer(gs, hbm_budget_bytes=1e12, max_slots_per_grid=2)
    assert [e[2] for e in srv.solver.log[:3]] == [A.COLD] * 3
    rng = np.random.default_rng(0)
    reqs = []
    for r in range(30):
        j = int(rng.integers(3))
        pd = np.full(gs[j].n_bus, 100.0 + r)
        reqs.append(S.Request(r, j, 0.001 * r, pd, pd * 0.3))
    out = srv.serve(reqs, realtime=False)
    assert out["requests"] == 30 and out["converged"] == 30
    done = out["done"]
    assert sorted(r.rid for r in done) == list(range(30))
    for r in done:
        assert r.finished >= r.admitted >= 0.0
        assert r.result["loads"] == 100.0 + r.rid   # solved with its own loads
        assert r.slot in [r.grid] + srv.slot_ids[r.grid]
    log = srv.solver.log
    # every admission copies the grid's home into another instance of the
    # grid before starting it; a completion makes its instance the new home
    # and copies nothing, so there is exactly one copy per request
    grid_of = {i: j for j in range(3) for i in [j] + srv.slot_ids[j]}
    for k, e in enumerate(log):
        if e[0] == "start" and e[2] == A.WARM:
            slot = e[1]
            copies = [c for c in log[:k] if c[0] == "copy" and c[2] == slot]
            assert copies and copies[-1][1] != slot and grid_of[copies[-1][1]] == grid_of[slot]
    assert len([e for e in log if e[0] == "copy"]) == 30
    # the home of each grid is the instance of its last finished request, and
    # every other instance is free again
    for j in range(3):
        last = [r for r in done if r.grid == j][-1]   # `done` is in completion order
        assert srv.home[j] == last.slot
        assert sorted(list(srv.free[j]) + [srv.home[j]]) == sorted([j] + srv.slot_ids[j])


def test_grid_without_slots_runs_on_home_one_at_a_time(fake):
    gs = grids3()
    sizes = [S.instance_bytes(g) for g in gs]
    srv = S.TrackingServer(gs, hbm_budget_bytes=sum(sizes) * 1.0001)
    assert srv.slots_per_grid == [0, 0, 0]
    reqs = [S.Request(r, 1, 0.0, np.full(gs[1].n_bus, float(r)), np.zeros(gs[1].n_bus))
            for r in range(4)]
    out = srv.serve(reqs, realtime=False)
    assert out["requests"] == 4
    starts = [e for e in srv.solver.log if e[0] == "start" and e[2] == A.WARM]
    assert [e[1] for e in starts] == [1, 1, 1, 1]   # the home instance, serially
    assert [r.result["loads"] for r in sorted(out["done"], key=lambda r: r.rid)] == [0, 1, 2, 3]
