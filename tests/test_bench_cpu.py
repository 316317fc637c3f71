"""Host logic of bench.py that needs no GPU: the one-GPU contract and the
use of the committed counter traffic."""
import json
import os
import subprocess
import sys

import bench
from paper_1812_10499_amd.build import kernel_source_hash

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_refused():
    """A run on more than one GPU exits with a message, before any GPU work."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_the_built_kernel(tmp_path, monkeypatch):
    """The counter traffic of the committed summary is used only while its
    source hash is the round kernel's; a stale summary gives None."""
    src = os.path.join(ROOT, "profiles", "rounds_kernel_rmat22_traffic.json")
    with open(src) as fh:
        d = json.load(fh)
    want = float(d["hbm_bytes_per_launch"]) if d["source_sha"] == kernel_source_hash() else None
    assert bench.measured_traffic("rmat22") == want
    (tmp_path / "profiles").mkdir()
    for sha, expect in ((kernel_source_hash(), 123.0), ("0" * 16, None)):
        with open(tmp_path / "profiles" / "rounds_kernel_x_traffic.json", "w") as fh:
            json.dump({"source_sha": sha, "hbm_bytes_per_launch": 123.0}, fh)
        monkeypatch.setattr(bench, "ROOT", str(tmp_path))
        assert bench.measured_traffic("x") == expect
    assert bench.measured_traffic("absent") is None
