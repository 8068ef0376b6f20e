"""CPU tests of bench.py's host logic: the kernel-source hash that ties the
committed profile summaries to the sources, the HBM traffic figure read from
the counter summary (null once the sources differ from the ones profiled),
and the refusal of more than one GPU."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_profile_summaries_name_their_sources_and_command():
    """Every summary names the kernel sources it was measured on (a 16-digit
    hash, which bench.py compares with the current sources) and the command
    that produced it."""
    assert re.fullmatch(r"[0-9a-f]{16}", bench.sources_hash())
    pdir = os.path.join(ROOT, "profiles")
    for name in os.listdir(pdir):
        txt = open(os.path.join(pdir, name)).read()
        assert re.search(r"sha256\[:16\] = `[0-9a-f]{16}`", txt), name
        assert "```" in txt and ("python3" in txt or "rocprofv3" in txt), name


def test_traffic_comes_from_the_counter_summary_and_goes_null_on_other_sources(tmp_path,
                                                                             monkeypatch):
    txt = open(bench.COUNTERS_MD).read()
    want = int(re.search(r"xstep_kernel HBM bytes per launch: (\d+)", txt).group(1))
    fresh = tmp_path / "fresh.md"
    fresh.write_text(re.sub(r"sha256\[:16\] = `[0-9a-f]{16}`",
                            f"sha256[:16] = `{bench.sources_hash()}`", txt))
    monkeypatch.setattr(bench, "COUNTERS_MD", str(fresh))
    assert bench.measured_traffic() == want and 30e6 < want < 50e6
    stale = tmp_path / "counters.md"
    stale.write_text(txt.replace(bench.sources_hash(), "0" * 16))
    monkeypatch.setattr(bench, "COUNTERS_MD", str(stale))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "COUNTERS_MD", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert "one GPU" in (r.stdout + r.stderr)
