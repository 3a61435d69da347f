"""bench.py's host logic (no GPU): the HBM traffic of the roofline comes from a committed
counter summary only while the kernel sources are those the counters were taken with, and a
run on more than one GPU is refused."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _sha():
    h = hashlib.sha256()
    for f in ("kernels.hip", "setup.cpp"):
        h.update(open(os.path.join(ROOT, "paper_1111_0983_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def test_traffic_is_reported_only_for_the_current_sources(tmp_path, monkeypatch):
    b = _bench()
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"kernel": "k", "traffic_bytes": 123456789, "source_sha": _sha()}
    (prof / "now.txt").write_text("# command\nsummary line\n" + json.dumps(rec) + "\n")
    rec_old = dict(rec, source_sha="0000000000000000")
    (prof / "old.txt").write_text("summary\n" + json.dumps(rec_old) + "\n")
    # the summaries are looked up under ROOT/profiles; the sources under ROOT/paper_.../csrc
    (tmp_path / "paper_1111_0983_amd").symlink_to(os.path.join(ROOT, "paper_1111_0983_amd"))
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.measured_traffic("now.txt") == 123456789
    assert b.measured_traffic("old.txt") is None
    assert b.measured_traffic("missing.txt") is None


def test_committed_relaxation_counters_name_their_sources():
    path = os.path.join(ROOT, "profiles", "k_relax_tank384_level0_counters.txt")
    rec = json.loads(open(path).read().strip().splitlines()[-1])
    assert rec["traffic_bytes"] > 0 and len(rec["source_sha"]) == 16
    assert rec["fetch_scale"] > 0 and rec["write_scale"] > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
