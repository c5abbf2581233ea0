"""Host logic of the column-schedule tuner: shape classes, the choice of the
faster schedule, reuse of a recorded choice, and the JSON cache (fake runners
and a fake timer stand in for the kernels)."""
import json

from paper_2307_11648_amd import autotune


def test_shape_key_follows_kernel_instantiation():
    k1 = autotune.shape_key(3, 3, 1_000_000, 512, 32, "mixed")
    assert k1 == "d3/nu3/pool512/k32/mixed/T2^20"
    # strides of one rows-per-lane class and picks of one capacity class share a key
    assert autotune.shape_key(3, 3, 1_000_000, 300, 20, "mixed") == autotune.shape_key(3, 3, 1_000_000, 512, 32,
                                                                                        "mixed")
    assert autotune.shape_key(3, 3, 1_000_000, 128, 32, "mixed") != k1
    assert autotune.shape_key(3, 3, 1_000_000, 512, 16, "mixed") != k1
    assert autotune.shape_key(3, 3, 1_000_000, 512, 32, "fp64") != k1
    assert autotune.shape_key(2, 3, 1_000_000, 512, 32, "mixed") != k1
    assert autotune.shape_key(3, 5, 1_000_000, 512, 32, "mixed") != k1
    assert autotune.shape_key(3, 3, 600_000, 512, 32, "mixed") == k1
    assert autotune.shape_key(3, 3, 400_000, 512, 32, "mixed") != k1
    assert autotune.shape_key(3, 3, 0, 64, 1, "mixed").endswith("T2^0")


class _Fake:
    """Runners that count their calls; a timer that reads fixed times."""

    def __init__(self, ms):
        self.ms = ms
        self.calls = {name: 0 for name in ms}

    def runners(self):
        def make(name):
            def run():
                self.calls[name] += 1
            run.ms = self.ms[name]
            return run
        return {name: make(name) for name in self.ms}

    @staticmethod
    def timer(run, stream):
        run()
        return run.ms


def test_choose_times_each_once_and_reuses(tmp_path):
    f = _Fake({"natural": 73.0, "spatial": 68.0})
    t = autotune.SelectTuner(timer=f.timer)
    assert t.choose("a", f.runners()) == "spatial"
    assert f.calls == {"natural": 2, "spatial": 2}  # one warm-up and one timed run each
    assert t.tuning_runs == 1
    assert t.choose("a", f.runners()) == "spatial"
    assert f.calls == {"natural": 2, "spatial": 2}
    assert t.choices["a"]["ms"] == {"natural": 73.0, "spatial": 68.0}
    # another class is timed on its own; a tie goes to the natural order
    g = _Fake({"natural": 12.0, "spatial": 12.0})
    assert t.choose("b", g.runners()) == "natural"
    assert t.tuning_runs == 2


def test_json_cache_round_trip_and_bad_files(tmp_path):
    path = str(tmp_path / "tune.json")
    f = _Fake({"natural": 10.0, "spatial": 12.5})
    t = autotune.SelectTuner(path=path, timer=f.timer)
    assert t.choose("x", f.runners()) == "natural"
    doc = json.load(open(path))
    assert doc["version"] == 2 and doc["choices"]["x"]["schedule"] == "natural"
    # a new process reads the choice back and times nothing
    g = _Fake({"natural": 99.0, "spatial": 1.0})
    t2 = autotune.SelectTuner(path=path, timer=g.timer)
    assert t2.choose("x", g.runners()) == "natural"
    assert g.calls == {"natural": 0, "spatial": 0} and t2.tuning_runs == 0
    # unreadable, other-version or malformed files are ignored
    for text in ("not json", json.dumps({"version": 7, "choices": {"x": {"schedule": "spatial"}}}),
                 json.dumps({"version": 2, "choices": {"x": {"schedule": "sideways"}}})):
        open(path, "w").write(text)
        assert autotune.SelectTuner(path=path, timer=g.timer).choices == {}


def test_order_must_be_a_permutation():
    import pytest
    import torch

    autotune.check_permutation(torch.tensor([2, 0, 1], dtype=torch.int32), 3)
    autotune.check_permutation(torch.zeros(0, dtype=torch.int32), 0)
    for bad in ([0, 1], [0, 1, 1], [0, 1, 3], [0, -1, 2]):
        with pytest.raises(ValueError):
            autotune.check_permutation(torch.tensor(bad, dtype=torch.int32), 3)


def test_four_schedules_fastest_wins_and_ties_go_to_the_earlier():
    f = _Fake({"natural": 30.0, "spatial": 28.0, "natural/mw": 21.0, "spatial/mw": 20.5})
    t = autotune.SelectTuner(timer=f.timer)
    assert t.choose("m", f.runners()) == "spatial/mw"
    g = _Fake({"natural": 10.0, "spatial": 12.0, "natural/mw": 10.0, "spatial/mw": 11.0})
    assert t.choose("n", g.runners()) == "natural"
    assert set(autotune.SCHEDULES) == {"natural", "spatial", "natural/mw", "spatial/mw"}


def test_aggregated_shape_key_and_schedules(tmp_path):
    """Multi-target shape classes round the group count and the rows per group
    (pool + members) up to powers of two; the aggregated schedule names
    survive the JSON cache, and the fastest of them wins."""
    k1 = autotune.agg_shape_key(2, 5, 64, 2048, 64, 128, "fp64", True)
    assert k1 == "agg/d2/nu5/G2^6/rows2^12/m64/k128/fp64/pv1"
    assert autotune.agg_shape_key(2, 5, 60, 2000, 64, 128, "fp64", True) == k1
    assert autotune.agg_shape_key(2, 5, 65, 2048, 64, 128, "fp64", True) != k1
    assert autotune.agg_shape_key(2, 5, 64, 2048, 64, 128, "mixed", False) != k1
    path = str(tmp_path / "tune.json")
    f = _Fake({"one_group": 30.0, "split256": 8.0, "split512": 7.0, "split1024": 7.0})
    t = autotune.SelectTuner(path=path, timer=f.timer)
    assert t.choose(k1, f.runners()) == "split512"  # a tie goes to the earlier schedule
    t2 = autotune.SelectTuner(path=path, timer=f.timer)
    assert t2.choices[k1]["schedule"] == "split512"
