"""Host logic of bench.py that runs without a GPU: the one-GPU guard and the
lookup of a kernel's HBM traffic from the committed counter summary, which
must give a figure only while the kernel's sources still hash to the value
recorded with the counters."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "single GPU" in r.stderr


def _summary(tmp_path, files, entries, top_files):
    (tmp_path / "profiles").mkdir()
    for name, text in files.items():
        (tmp_path / name).write_text(text)

    def digest(names):
        h = hashlib.sha256()
        for n in names:
            h.update((tmp_path / n).read_bytes())
        return h.hexdigest()

    for e in entries:
        if "kernel_sources" in e:
            e["kernel_source_sha256"] = digest(e["kernel_sources"])
    d = {"kernel_sources": top_files, "kernel_source_sha256": digest(top_files), "entries": entries}
    (tmp_path / "profiles" / "pair_kernel_f32_angular_n65536_hbm.json").write_text(json.dumps(d))


def test_traffic_lookup_follows_the_recorded_source_hashes(tmp_path, monkeypatch):
    files = {"a.hip": "kernel a", "b.hip": "kernel b"}
    entries = [{"kernel": "ka", "n": 64, "tile": [2, 8], "traffic_bytes_per_dispatch": 123.0},
               {"kernel": "kb", "n": 64, "tile": [0, 1], "traffic_bytes_per_dispatch": 456.0,
                "kernel_sources": ["b.hip"]}]
    _summary(tmp_path, files, entries, ["a.hip"])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.hbm_traffic("ka", 64, [2, 8]) == 123.0
    assert bench.hbm_traffic("kb", 64, (0, 1)) == 456.0
    assert bench.hbm_traffic("ka", 64, [1, 8]) is None          # no entry for that tile
    assert bench.hbm_traffic("ka", 128, [2, 8]) is None         # nor for that N
    (tmp_path / "b.hip").write_text("kernel b, changed")
    assert bench.hbm_traffic("kb", 64, [0, 1]) is None          # its own sources changed
    assert bench.hbm_traffic("ka", 64, [2, 8]) == 123.0         # the other entry is unaffected
    (tmp_path / "a.hip").write_text("kernel a, changed")
    assert bench.hbm_traffic("ka", 64, [2, 8]) is None


def test_traffic_lookup_without_a_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.hbm_traffic("ka", 64, [2, 8]) is None
