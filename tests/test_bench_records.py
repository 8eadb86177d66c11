"""Host checks of bench.py's stored-record logic: counter traffic recorded in
profiles/hbm_traffic.json is used only while the kernel sources it was
measured on are unchanged (no GPU needed)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write(tmp_path, rec):
    d = tmp_path / "profiles"
    d.mkdir()
    (d / "hbm_traffic.json").write_text(json.dumps(rec))
    return str(d)


def test_stored_traffic_follows_the_source_hashes(tmp_path, monkeypatch):
    plain = bench.source_hash()
    batch = bench.source_hash(bench.BATCH_PATH_SOURCES)
    assert plain != batch
    rec = {"source_hash": plain, "large": {"fwd_kernel": 1, "inv_kernel": 2},
           "batch_default_tiles": {"source_hash": batch, "fwd_batch_kernel": 3}}
    monkeypatch.setattr(bench, "PROFILES", _write(tmp_path, rec))
    assert bench.stored_traffic("large")["fwd_kernel"] == 1
    assert bench.stored_traffic("batch_default_tiles", bench.BATCH_PATH_SOURCES)["fwd_batch_kernel"] == 3
    # an entry measured on other sources is not used
    assert bench.stored_traffic("batch_default_tiles") is None
    assert bench.stored_traffic("missing") is None


def test_stale_records_are_ignored(tmp_path, monkeypatch):
    rec = {"source_hash": "0" * 16, "large": {"fwd_kernel": 1},
           "batch_default_tiles": {"source_hash": "1" * 16, "fwd_batch_kernel": 3}}
    monkeypatch.setattr(bench, "PROFILES", _write(tmp_path, rec))
    assert bench.stored_traffic("large") is None
    assert bench.stored_traffic("batch_default_tiles", bench.BATCH_PATH_SOURCES) is None


def test_committed_records_match_the_committed_sources():
    """The committed traffic figures belong to the committed kernels."""
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as f:
        rec = json.load(f)
    assert rec["source_hash"] == bench.source_hash()
    assert rec["batch_default_tiles"]["source_hash"] == bench.source_hash(bench.BATCH_PATH_SOURCES)
