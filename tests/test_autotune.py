"""The launch-shape tuner's selection and JSON cache (CPU: a stand-in timer)."""
import json

from paper_1401_1112_amd import autotune as A


def _fake_timer(costs):
    def timer(candidates, apply, run, repeats, stream):
        out = {}
        for c in candidates:
            apply(c)
            out[json.dumps(c, sort_keys=True)] = costs[c["max_blocks"]]
        return out
    return timer


def test_tune_picks_fastest_and_caches(tmp_path, monkeypatch):
    monkeypatch.setenv("AMRFLD_TUNE_CACHE", str(tmp_path / "tune.json"))
    applied = []
    cands = [{"max_blocks": b} for b in (256, 1024, 4096)]
    costs = {256: 3.0, 1024: 1.5, 4096: 2.0}
    best, ms, cached = A.tune("k", cands, applied.append, lambda: None, timer=_fake_timer(costs), device="dev0")
    assert best == {"max_blocks": 1024} and not cached
    assert applied[-1] == best
    assert json.load(open(tmp_path / "tune.json"))["dev0|k"]["best"] == best
    # a second call returns the cached choice without timing
    def no_timer(*a):
        raise AssertionError("timed again")
    best2, _, cached2 = A.tune("k", cands, applied.append, lambda: None, timer=no_timer, device="dev0")
    assert best2 == best and cached2 and applied[-1] == best
    # another device or workload is timed anew
    best3, _, cached3 = A.tune("k", cands, applied.append, lambda: None,
                               timer=_fake_timer({256: 1.0, 1024: 2.0, 4096: 3.0}), device="dev1")
    assert best3 == {"max_blocks": 256} and not cached3


def test_workload_key_separates_sizes_and_precision():
    a = A.workload_key("batch", [8, 16, 32], 0)
    assert a == A.workload_key("batch", [8, 16, 32], 0)
    assert a != A.workload_key("batch", [8, 16, 34], 0)
    assert a != A.workload_key("batch", [8, 16, 32], 1)
    assert a != A.workload_key("levels", [8, 16, 32], 0)
