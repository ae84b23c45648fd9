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
    best, ms, src = A.tune("k", cands, applied.append, lambda: None, timer=_fake_timer(costs), device="dev0",
                           arch="none")
    assert best == {"max_blocks": 1024} and src == "timed"
    assert applied[-1] == best
    assert json.load(open(tmp_path / "tune.json"))["dev0|k"]["best"] == best
    # a second call returns the cached choice without timing
    def no_timer(*a):
        raise AssertionError("timed again")
    best2, _, src2 = A.tune("k", cands, applied.append, lambda: None, timer=no_timer, device="dev0", arch="none")
    assert best2 == best and src2 == "cache" and applied[-1] == best
    # another device or workload is timed anew
    best3, _, src3 = A.tune("k", cands, applied.append, lambda: None,
                            timer=_fake_timer({256: 1.0, 1024: 2.0, 4096: 3.0}), device="dev1", arch="none")
    assert best3 == {"max_blocks": 256} and src3 == "timed"


def test_workload_key_separates_sizes_and_precision():
    a = A.workload_key("batch", [8, 16, 32], 0)
    assert a == A.workload_key("batch", [8, 16, 32], 0)
    assert a != A.workload_key("batch", [8, 16, 34], 0)
    assert a != A.workload_key("batch", [8, 16, 32], 1)
    assert a != A.workload_key("levels", [8, 16, 32], 0)


def test_shipped_table_applies_on_its_architecture(tmp_path, monkeypatch):
    monkeypatch.setenv("AMRFLD_TUNE_CACHE", str(tmp_path / "tune.json"))
    table = tmp_path / "shipped.json"
    table.write_text(json.dumps({"arch": "gfx950", "entries": {"w": {"best": {"max_blocks": 512}, "ms": {}}}}))
    monkeypatch.setattr(A, "SHIPPED", str(table))
    applied = []

    def no_timer(*a):
        raise AssertionError("timed")
    best, _, src = A.tune("w", [{"max_blocks": 512}], applied.append, lambda: None, timer=no_timer,
                          device="d", arch="gfx950:sramecc+:xnack-")
    assert best == {"max_blocks": 512} and src == "shipped" and applied == [best]
    # another architecture, or another workload, is timed
    best, _, src = A.tune("w", [{"max_blocks": 1024}], applied.append, lambda: None,
                          timer=_fake_timer({1024: 1.0}), device="d", arch="gfx942")
    assert src == "timed"


def test_shipped_table_keys_match_the_benchmark_workloads():
    # the shipped entries are keyed by the benchmark workloads' sizes
    from synth.configs import patch_sizes
    d = json.load(open(A.SHIPPED))
    assert d["arch"] == "gfx950"
    keys = set(d["entries"])
    assert A.workload_key("levels", [262144, 1250000, 1250000, 1250000], 0) in keys
    assert A.workload_key("batch", [int(max(2, n)) for n in patch_sizes(4000, 512)], 0) in keys


def test_shipped_entries_are_candidates():
    # every shipped choice is one of the shapes its tuner times
    table = json.load(open(A.SHIPPED))
    inner = tuple({"inner_tol": t} for t in A.INNER_TOLS)
    cands = {"levels": A.LEVEL_CANDIDATES, "batch": A.BATCH_SHAPES, "level-shapes": A.LEVEL_SHAPES,
             "refinement-levels": inner, "refinement-batch": inner, "refinement-collapse": inner}
    for key, e in table["entries"].items():
        assert e["best"] in [dict(c) for c in cands[key.split("|")[0]]], key
        assert json.dumps(e["best"], sort_keys=True) in e["ms"], key


def test_shipped_table_can_be_skipped(monkeypatch):
    monkeypatch.setenv("AMRFLD_TUNE_SHIPPED", "0")
    key = next(iter(json.load(open(A.SHIPPED))["entries"]))
    assert A._shipped(key, arch="gfx950") is None
