"""The oracle's optional OpenMP loops (the all-core CPU baseline) give the
serial oracle's results bit for bit: generators, branches and buses are
independent elements, the residuals are maxima and the event counters
integer sums, so no result depends on the thread count (CPU only)."""
import numpy as np
import pytest

import oracle as O
from paper_2110_06879_amd.gridgen import config_grid


@pytest.mark.parametrize("textbook", [False, True])
def test_threads_give_bitwise_serial_results(textbook):
    g = config_grid("c2_2kbus")
    g.rate = g.rate * 0.15  # binding limits: AL rounds differ per branch
    p = O.OracleParams(max_inner=10)  # outer steps inside the run
    a = O.Oracle(g, p)
    b = O.Oracle(g, p)
    a.set_textbook(textbook)
    b.set_textbook(textbook)
    b.set_threads(4)
    a.solve(25)
    b.solve(25)
    for k in ("u", "v", "z", "y", "lam", "bx", "ltil", "rtil", "calpha"):
        np.testing.assert_array_equal(a.get(k), b.get(k), err_msg=k)
    np.testing.assert_array_equal(a.history(), b.history())
    assert a.stats() == b.stats()
    assert a.scalars() == b.scalars()
