"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a message before any device work."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_summary_matches_sources_and_guards_changes(tmp_path, monkeypatch):
    """A counter summary carries the hash of the pass kernel's sources:
    bench.py reports its HBM bytes only while the hash agrees with them."""
    sys.path.insert(0, ROOT)
    import bench
    text = open(bench.TRAFFIC_SUMMARY).read()
    fresh = tmp_path / "fresh.md"
    stale = tmp_path / "stale.md"
    lines = [ln for ln in text.splitlines() if not ln.startswith("- kernel_sources_sha256:")]
    fresh.write_text("\n".join(lines + [f"- kernel_sources_sha256: `{bench.kernel_source_hash()}`"]))
    stale.write_text("\n".join(lines + ["- kernel_sources_sha256: `" + "0" * 64 + "`"]))
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(fresh))
    got = bench.counted_traffic()
    assert got is not None and abs(got / (1 << 30) - 1.0) < 0.01   # ~1 GiB per pass
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(stale))
    assert bench.counted_traffic() is None
