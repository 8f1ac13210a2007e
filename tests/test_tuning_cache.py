"""The JSON plan cache of the autotuner (host logic only)."""
import json

from paper_1707_05062_amd import tuning


def test_workload_class():
    assert tuning.workload_class([(3456, 5184)]) == "single:24"
    assert tuning.workload_class([(256, 256)]) == "single:16"
    assert tuning.workload_class([(256, 256)] * 96).startswith("batch:7:")


def test_plan_key_separates_families_and_workloads():
    a = tuning.plan_key("gfx950", 256, 1, 256, 4, [(3456, 5184)])
    assert a != tuning.plan_key("gfx950", 256, 1, 256, 8, [(3456, 5184)])
    assert a != tuning.plan_key("gfx950", 256, 1, 256, 4, [(1080, 1920)])
    assert a != tuning.plan_key("gfx942", 304, 1, 256, 4, [(3456, 5184)])


def test_store_and_load_roundtrip(tmp_path):
    path = str(tmp_path / "plans.json")
    assert tuning.load(path) == {}
    plan = {"form": 1, "band": 32, "block": 512, "grid": 512, "px_per_lane": 4, "replicas": 16}
    tuning.store("k1", plan, 34.5, path)
    tuning.store("k2", dict(plan, band=16), 40.0, path)
    data = tuning.load(path)
    assert data["k1"] == {"plan": plan, "us": 34.5}
    assert data["k2"]["plan"]["band"] == 16
    with open(path) as f:
        assert json.load(f) == data


def test_corrupt_cache_is_ignored(tmp_path):
    path = tmp_path / "plans.json"
    path.write_text("{not json")
    assert tuning.load(str(path)) == {}
