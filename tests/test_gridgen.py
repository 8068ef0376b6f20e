"""CPU tests of the seeded input recipe: the workloads have the sizes they are
named for, every grid is connected and simple, the draws stay in their stated
ranges, the load guard holds, and a seed always gives the same arrays."""
import numpy as np
import pytest

from paper_2110_06879_amd.gridgen import (CONFIGS, LOAD_FACTOR, batch_grids, config_grid,
                                          gridgen, perturb_loads, serving_grids)


def connected(g) -> bool:
    parent = np.arange(g.n_bus)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a, b in zip(g.br_from.tolist(), g.br_to.tolist()):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    return len({find(i) for i in range(g.n_bus)}) == 1


def check_recipe(g, rated_frac, load_factor):
    n_b, n_g, n_l = g.n_bus, g.n_gen, g.n_branch
    assert connected(g)
    assert np.all(g.br_from != g.br_to)
    keys = set(zip(np.minimum(g.br_from, g.br_to).tolist(), np.maximum(g.br_from, g.br_to).tolist()))
    assert len(keys) == n_l  # no parallel lines
    assert np.all((g.r >= 0.005) & (g.r <= 0.05)) and np.all((g.x >= 0.02) & (g.x <= 0.2))
    assert np.all((g.b >= 0.0) & (g.b <= 0.05))
    rated = g.rate > 0
    assert rated.sum() == int(round(rated_frac * n_l))
    assert np.all((g.rate[rated] >= 1.0) & (g.rate[rated] <= 3.0))
    assert np.all(g.tap == 1.0) and np.all(g.shift == 0.0)
    assert g.gen_bus[0] == 0 and g.ref_bus == 0 and len(set(g.gen_bus.tolist())) == n_g
    assert np.all(g.pmin == 0.0) and np.all((g.pmax >= 0.5) & (g.pmax <= 3.0))
    assert np.array_equal(g.qmax, g.pmax) and np.array_equal(g.qmin, -g.pmax)
    assert np.all((g.c2 >= 0.01) & (g.c2 <= 0.1)) and np.all((g.c1 >= 10) & (g.c1 <= 40))
    assert np.all(g.c0 == 0.0)
    assert np.all(g.pd >= 0.0) and np.all(g.pd <= load_factor * 0.5 * g.load_scale + 1e-15)
    np.testing.assert_allclose(g.qd, 0.3 * g.pd, rtol=1e-15)
    assert g.pd.sum() <= 0.75 * g.pmax.sum() * (1 + 1e-12)
    assert np.all(g.vmin == 0.94) and np.all(g.vmax == 1.06)
    assert np.all(g.gs == 0.0) and np.all(g.bs == 0.0) and g.base_mva == 100.0


@pytest.mark.parametrize("name", ["c1_30bus", "c2_2kbus", "c2_2kbus_full"])
def test_config_grids_follow_the_recipe(name):
    c = CONFIGS[name]
    g = config_grid(name)
    assert (g.n_bus, g.n_gen, g.n_branch) == (c["n_bus"], c["n_gen"], c["n_branch"])
    check_recipe(g, c["rated_frac"], c["load_factor"])


def test_benchmark_grid_sizes_and_guard():
    """The 70k-bus benchmark grid: 70,000 buses, 10,000 generators, 88,000
    branches of which 26,400 rated; at the stated load distribution the
    0.75 guard scales the loads (factor below 1), at factor 0.2 it does not."""
    g = config_grid("c3_70kbus")
    assert (g.n_bus, g.n_gen, g.n_branch, int((g.rate > 0).sum())) == (70000, 10000, 88000, 26400)
    check_recipe(g, 0.3, LOAD_FACTOR)
    assert g.load_scale == 1.0
    f = config_grid("c3_70kbus_full")
    assert f.load_scale < 1.0
    np.testing.assert_allclose(f.pd.sum() / f.pmax.sum(), 0.75, rtol=1e-12)
    # the same topology and branch data at both load levels
    assert np.array_equal(f.br_from, g.br_from) and np.array_equal(f.r, g.r)


def test_seeds_are_deterministic_and_distinct():
    a, b = gridgen(300, 40, 400, 0.5, 11), gridgen(300, 40, 400, 0.5, 11)
    c = gridgen(300, 40, 400, 0.5, 12)
    for k in ("br_from", "br_to", "r", "x", "b", "rate", "gen_bus", "pmax", "c2", "c1", "pd"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    assert not np.array_equal(a.r, c.r)


def test_batch_and_serving_grids():
    gs = batch_grids(64)
    sizes = [g.n_bus for g in gs]
    assert len(gs) == 64 and min(sizes) >= 500 and max(sizes) <= 20000
    assert len({g.name for g in gs}) == 64
    ss = serving_grids()
    assert len(ss) == 16 and min(g.n_bus for g in ss) == 2000 and max(g.n_bus for g in ss) == 70000
    for g in gs[:4] + ss[:2]:
        assert connected(g)


def test_perturbation_is_bounded_and_seeded():
    g = config_grid("c2_2kbus")
    pd1, qd1 = perturb_loads(g, 0.05, 1001)
    pd2, _ = perturb_loads(g, 0.05, 1001)
    assert np.array_equal(pd1, pd2)
    nz = g.pd > 0
    d = pd1[nz] / g.pd[nz] - 1.0
    assert np.all(np.abs(d) <= 0.05 + 1e-12) and np.abs(d).max() > 0.04
    np.testing.assert_allclose(qd1[nz] / g.qd[nz], pd1[nz] / g.pd[nz], rtol=1e-12)


def test_topology_rejects_impossible_sizes():
    with pytest.raises(ValueError):
        gridgen(10, 2, 8, 0.5, 1)  # fewer branches than a spanning tree needs
    with pytest.raises(ValueError):
        gridgen(4, 2, 7, 0.5, 1)  # more branches than a simple graph holds
    with pytest.raises(ValueError):
        gridgen(4, 5, 4, 0.5, 1)  # more generators than buses
