"""CPU tests of the tracking server's planning (acopf_serving_plan in the
library, no device needed): slots per grid under the HBM budget, the
per-grid cap, and the EBUDGET error when the homes alone do not fit. The
admission, commit and batching behaviour needs a device and is covered by
the GPU tests in test_gpu_batching.py."""
import pytest

from paper_2110_06879_amd import serve as S
from paper_2110_06879_amd.gridgen import gridgen


def grids3():
    return [gridgen(40 + 20 * k, 6, 50 + 25 * k, 0.3, 90 + k, load_factor=0.2) for k in range(3)]


def test_instance_footprint_grows_with_the_grid():
    gs = grids3()
    sizes = [S.instance_bytes(g) for g in gs]
    assert 0 < sizes[0] < sizes[1] < sizes[2]
    # the history of 2^15 iterations x 6 doubles is part of every instance
    assert sizes[0] > 6 * 8 * (1 << 15)


def test_slots_follow_budget():
    gs = grids3()
    sizes = [S.instance_bytes(g) for g in gs]
    # room for the homes and exactly one slot of the smallest grid
    slots, used = S.serving_plan(gs, sum(sizes) + min(sizes), 4)
    assert slots == [1, 0, 0]
    assert used == pytest.approx(sum(sizes) + min(sizes))
    # room for a slot of each of the two smaller grids: smallest first, round robin
    slots, used = S.serving_plan(gs, sum(sizes) + sizes[0] + sizes[1] + 1.0, 4)
    assert slots == [1, 1, 0]
    # a large budget stops at the per-grid cap
    slots, used = S.serving_plan(gs, 1e12, 2)
    assert slots == [2, 2, 2]
    assert used == pytest.approx(3 * sum(sizes))
    # a budget that holds only the homes leaves every grid without slots
    slots, _ = S.serving_plan(gs, sum(sizes) * 1.0001, 4)
    assert slots == [0, 0, 0]


def test_budget_below_homes_rejected():
    gs = grids3()
    with pytest.raises(ValueError, match="budget"):
        S.serving_plan(gs, S.instance_bytes(gs[0]), 4)
