"""bench.py host logic (CPU): the one-GPU command-line contract and the rule
that counter-measured HBM traffic is reported only for the kernel source it
was measured on."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def _fake_root(tmp_path, source_text, recorded_text):
    csrc = tmp_path / "paper_2007_14228_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k_spmm.hip").write_text(source_text)
    (tmp_path / "profiles").mkdir()
    sha = hashlib.sha256(recorded_text.encode()).hexdigest()[:16]
    rec = {"k_spmm_shift@c3": {"kernel": "k_spmm_halo<double, 1>", "bytes_per_launch": 5781812918,
                               "source": "k_spmm.hip", "source_sha": sha}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))


def test_traffic_is_reported_for_the_measured_source(tmp_path, monkeypatch):
    _fake_root(tmp_path, "kernel v1\n", "kernel v1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profiles("k_spmm_shift", "c3")["bytes"] == 5781812918


def test_traffic_is_null_once_the_source_changes(tmp_path, monkeypatch):
    _fake_root(tmp_path, "kernel v2\n", "kernel v1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profiles("k_spmm_shift", "c3") is None


def test_traffic_is_null_without_a_record(tmp_path, monkeypatch):
    _fake_root(tmp_path, "kernel v1\n", "kernel v1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profiles("k_spmm_shift", "c2") is None
    os.remove(tmp_path / "profiles" / "traffic.json")
    assert bench.traffic_from_profiles("k_spmm_shift", "c3") is None
