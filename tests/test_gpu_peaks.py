"""GPU tests of the measurement helpers that report the device's achievable
streaming bandwidth and FP64 rate beside the published peaks (8 TB/s HBM3E,
78.6 TFLOP/s FP64 vector): plausible values, invalid arguments refused."""
import sys

import pytest

from paper_2110_06879_amd import acopf as A

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_peak_rates_are_plausible_and_arguments_checked():
    note("measurement helpers: 1 GiB copy, FP64 FMA loop")
    bw = A.peak_hbm(1 << 30, 5)
    assert 1000.0 < bw < 10000.0, bw
    tf = A.peak_fp64(50000)
    assert 10.0 < tf < 80.0, tf
    for bad in (lambda: A.peak_hbm(1000, 5), lambda: A.peak_hbm(1 << 30, 0),
                lambda: A.peak_fp64(0)):
        with pytest.raises(A.AcopfError):
            bad()
