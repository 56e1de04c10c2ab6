"""The autotuner cache (no GPU): keys, lookup, and the shape of stored entries."""
import json

from paper_2102_03494_amd import tune


def test_ring_key_and_lookup(tmp_path):
    path = tmp_path / "cache.json"
    assert tune.lookup(8192, (30, 30), 40, str(path)) is None
    key = tune.ring_key(8192, (30, 30), 40)
    assert key == "n8192_q30-30_p40"
    path.write_text(json.dumps({key: {"p_groups": {"2": 1}, "ms_per_step": {"2": {"1": 0.5}}, "batch": 8,
                                      "device": "x"}}))
    assert tune.lookup(8192, (30, 30), 40, str(path)) == {2: 1}
    assert tune.lookup(8192, (30, 30, 30), 40, str(path)) is None


def test_committed_cache_entries_are_legal():
    for key, entry in tune.load_cache().items():
        assert key.startswith("n") and "_q" in key and "_p" in key
        for level, pg in entry["p_groups"].items():
            assert 1 <= pg <= min(int(level), 4)
            assert str(pg) in entry["ms_per_step"][level]
            times = entry["ms_per_step"][level]
            assert times[str(pg)] == min(times.values())
