"""acopf_quality_noalloc, the allocation-free variant of acopf_quality for
callers that cannot allocate device memory: its kernels use the library's
fixed device scratch instead of the buffer acopf_quality allocates. Called
through the C ABI and checked against acopf_quality on two calls in a row,
the second on a smaller handle, then on a handle beyond the scratch."""
import ctypes as C

import numpy as np
import pytest

from paper_2110_06879_amd import acopf as A
from paper_2110_06879_amd.gridgen import config_grid, gridgen

pytestmark = pytest.mark.gpu


def quality_pair(s, grid):
    lib = s.lib
    want = np.zeros(6)
    got = np.full(6, np.nan)
    assert lib.acopf_quality(s.h, grid, want.ctypes.data_as(C.POINTER(C.c_double))) == 0
    rc = lib.acopf_quality_noalloc(s.h, grid, got.ctypes.data_as(C.POINTER(C.c_double)))
    assert rc == 0, lib.acopf_last_error().decode()
    return got, want


def test_noalloc_quality_equals_quality_on_two_calls():
    print("noalloc quality: 2k grid after 40 iterations, then a smaller batch", flush=True)
    with A.Solver(config_grid("c2_2kbus")) as s:
        s.solve(A.COLD, 40)
        got, want = quality_pair(s, 0)
        np.testing.assert_array_equal(got, want)
        assert want[0] > 0.0
    gs = [gridgen(60, 10, 80, 1.0, 91, load_factor=0.2),
          gridgen(45, 8, 60, 0.0, 92, load_factor=0.2)]
    with A.Solver(gs) as s:
        s.solve(A.COLD, 25)
        for k in range(2):
            got, want = quality_pair(s, k)
            np.testing.assert_array_equal(got, want)


def test_noalloc_quality_rejects_handles_beyond_the_scratch():
    print("noalloc quality: a handle too large for the fixed scratch", flush=True)
    g = gridgen(180000, 100, 200000, 0.0, 93, load_factor=0.2)
    with A.Solver(g) as s:
        lib = s.lib
        out = np.zeros(6)
        rc = lib.acopf_quality_noalloc(s.h, 0, out.ctypes.data_as(C.POINTER(C.c_double)))
        assert rc == A_EINVAL
        assert "scratch" in lib.acopf_last_error().decode()


A_EINVAL = -1
