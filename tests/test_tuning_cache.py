"""Host logic of the autotuner's JSON cache (no GPU): the workload key, a
store and load round trip, other entries kept, and damaged or incomplete
files treated as a miss."""
import json

from paper_2110_06879_amd import acopf as A
from paper_2110_06879_amd.gridgen import gridgen

TUNE = {"xstep_block": 128, "bus_block": 512, "chunk": 32, "use_graph": 1,
        "xstep_waves": 0, "xstep_per_lane": 2, "lanes": 2}


def test_key_counts_the_workload_shape():
    g1 = gridgen(40, 6, 50, 0.5, 1)
    g2 = gridgen(70, 9, 90, 1.0, 2)
    k = A.tuning_key([g1, g2])
    n6 = int((g1.rate > 0).sum() + (g2.rate > 0).sum())
    assert k == f"grids=2 buses=110 branches=140 rated={n6}"
    assert A.tuning_key(g1) == A.tuning_key([g1])
    assert A.tuning_key([g1, g2]) != A.tuning_key([g2])


def test_store_and_load_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    assert A.load_tuning(path, "k1") is None          # no file yet
    A.save_tuning(path, "k1", TUNE)
    A.save_tuning(path, "k2", {**TUNE, "chunk": 8})
    assert A.load_tuning(path, "k1") == TUNE
    assert A.load_tuning(path, "k2")["chunk"] == 8
    assert A.load_tuning(path, "k3") is None          # other workload
    with open(path) as fh:
        assert set(json.load(fh)) == {"k1", "k2"}


def test_damaged_or_incomplete_files_are_a_miss(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert A.load_tuning(str(path), "k1") is None
    path.write_text(json.dumps({"k1": {"chunk": 16}}))
    assert A.load_tuning(str(path), "k1") is None
    old = {k: v for k, v in TUNE.items() if k != "lanes"}  # stored before lanes existed
    path.write_text(json.dumps({"k1": old}))
    assert A.load_tuning(str(path), "k1") is None
    path.write_text(json.dumps([1, 2, 3]))
    assert A.load_tuning(str(path), "k1") is None
    A.save_tuning(str(path), "k1", TUNE)              # replaces the damaged file
    assert A.load_tuning(str(path), "k1") == TUNE
