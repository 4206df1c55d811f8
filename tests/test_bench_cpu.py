"""Host-side checks of bench.py's measurement bookkeeping (no GPU): the
recorded HBM traffic is reported only while every source it was measured
with is unchanged, and its calibration arithmetic."""
import hashlib
import json
import os
import shutil
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _copy_tree(tmp_path, names):
    for n in names:
        src = os.path.join(ROOT, n)
        dst = tmp_path / n
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copyfile(src, dst)


def test_committed_records_match_their_sources():
    with open(os.path.join(ROOT, "profiles", "scan_traffic.json")) as f:
        recs = json.load(f)
    for name, rec in recs.items():
        sources = rec.get("sources") or {rec["source"]: rec["source_sha256"]}
        for src, digest in sources.items():
            with open(os.path.join(ROOT, src), "rb") as f:
                assert hashlib.sha256(f.read()).hexdigest() == digest, (name, src)
        got = bench.recorded_traffic(name)
        # reads scaled by the copy's 1 GiB over its FETCH reading, writes likewise
        want = (rec["fetch_kib"] * rec["copy_bytes_each"] / rec["copy_fetch_kib"] +
                rec["write_kib"] * rec["copy_bytes_each"] / rec["copy_write_kib"])
        assert got == round(want), name


def test_traffic_is_dropped_when_a_source_changes(tmp_path):
    with open(os.path.join(ROOT, "profiles", "scan_traffic.json")) as f:
        recs = json.load(f)
    files = {"bench.py", "profiles/scan_traffic.json"}
    for rec in recs.values():
        files.update(rec.get("sources") or {rec["source"]: None})
    _copy_tree(tmp_path, sorted(files))
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_copy", tmp_path / "bench.py")
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    for name, rec in recs.items():
        assert b.recorded_traffic(name) is not None
        for src in rec.get("sources") or {rec["source"]: None}:
            with open(tmp_path / src, "rb") as f:
                keep = f.read()
            with open(tmp_path / src, "ab") as f:
                f.write(b"\n")
            assert b.recorded_traffic(name) is None, (name, src)
            with open(tmp_path / src, "wb") as f:
                f.write(keep)
        assert b.recorded_traffic(name) is not None
    assert b.recorded_traffic("no such kernel") is None
