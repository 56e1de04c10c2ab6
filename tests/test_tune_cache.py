"""The autotuner cache (no GPU): keys, lookup, staleness, and the shape of
stored entries."""
import json

from paper_2102_03494_amd import tune


def _entry(sha, pg=None, halves=None):
    return {"p_groups": pg or {"2": 1}, "modup_halves": halves or {"2": 0}, "split_streams": 1,
            "ms_per_step": {"2": {"h0_pg1": 0.5, "h1_pg1": 0.6}}, "batch": 8, "device": "x", "kernel_sha256": sha}


def test_ring_key_and_lookup(tmp_path):
    path = tmp_path / "cache.json"
    assert tune.lookup(8192, (30, 30), 40, str(path)) == (None, "no entry")
    key = tune.ring_key(8192, (30, 30), 40)
    assert key == "n8192_q30-30_p40"
    path.write_text(json.dumps({key: _entry(tune.kernel_sha256())}))
    entry, status = tune.lookup(8192, (30, 30), 40, str(path))
    assert status == "cache" and entry["p_groups"] == {"2": 1}
    assert tune.lookup(8192, (30, 30, 30), 40, str(path)) == (None, "no entry")


def test_stale_entry_is_rejected(tmp_path):
    """An entry measured on other kernel sources is ignored."""
    path = tmp_path / "cache.json"
    key = tune.ring_key(8192, (30, 30), 40)
    path.write_text(json.dumps({key: _entry("0" * 64)}))
    assert tune.lookup(8192, (30, 30), 40, str(path)) == (None, "stale cache")
    assert tune.lookup(8192, (30, 30), 40, str(path), sha="0" * 64)[1] == "cache"


def test_kernel_hash_is_stable_and_covers_sources():
    a = tune.kernel_sha256()
    assert a == tune.kernel_sha256() and len(a) == 64


def test_committed_cache_entries_are_legal():
    for key, entry in tune.load_cache().items():
        assert key.startswith("n") and "_q" in key and "_p" in key
        assert len(entry["kernel_sha256"]) == 64
        assert entry["split_streams"] in (0, 1)
        assert entry.get("split_parts", 2) in (2, 3, 4)
        for level, pg in entry["p_groups"].items():
            hv = entry["modup_halves"][level]
            assert 1 <= pg <= min(int(level), 4) and hv in (0, 1)
            times = entry["ms_per_step"][level]
            assert times[f"h{hv}_pg{pg}"] == min(times.values())
