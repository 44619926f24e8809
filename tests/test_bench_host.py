"""Host-side logic of bench.py (no GPU): the kernel-source hash that guards
the committed HBM byte counters, the lookup of those counters, and the
one-GPU guard."""
import json
import os
import shutil
import subprocess
import sys

import bench
from paper_2206_15454_amd import inputs


def _tree(tmp_path):
    """A copy of the hashed sources and an empty profiles/ under tmp_path."""
    for p in bench.KERNEL_SOURCES:
        (tmp_path / os.path.dirname(p)).mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, p), tmp_path / p)
    (tmp_path / "profiles").mkdir()


def test_kernel_hash_tracks_every_source(monkeypatch, tmp_path):
    """A code edit in any hashed source changes the hash; comments, blank
    lines and trailing blanks do not (they leave the compiled kernels as
    they were)."""
    _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_hash()
    assert len(h0) == 16 and h0 == bench.kernel_hash()
    seen = {h0}
    for i, p in enumerate(bench.KERNEL_SOURCES):
        seen_last = bench.kernel_hash()
        with open(tmp_path / p, "a") as f:
            f.write("\n// a comment\n/* another\n   one */   \n\n")
        assert bench.kernel_hash() == seen_last, p
        with open(tmp_path / p, "a") as f:
            f.write(f"static int edit_{i};\n")
        h = bench.kernel_hash()
        assert h not in seen, p
        seen.add(h)


def test_measured_traffic_only_for_the_current_kernel_and_workload(monkeypatch, tmp_path):
    _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    path = tmp_path / "profiles" / "traffic_counters.json"
    w = inputs.C2
    assert bench.measured_traffic("f32", w) is None  # no counters committed
    rec = {"entries": {f"{w.name}/f32": {"kernel_hash": bench.kernel_hash(), "cells": w.n,
                                         "bytes_per_launch": 2_516_582_400}}}
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("f32", w) == 2_516_582_400
    assert bench.measured_traffic("bf16s", w) is None           # another storage type
    assert bench.measured_traffic("f32", inputs.FOREST) is None  # another workload
    rec["entries"][f"{w.name}/f32"]["cells"] = w.n + 1
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("f32", w) is None             # another grid
    rec["entries"][f"{w.name}/f32"].update(cells=w.n, kernel_hash="0" * 16)
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("f32", w) is None             # taken on other kernels
    path.write_text("not json")
    assert bench.measured_traffic("f32", w) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bytes_per_population():
    # algorithmic bytes per lattice update are 2 * 19 * these
    assert bench.BYTES_PER_ELT == {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2, "bf16sr": 2}
