"""Host-side checks of bench.py (no GPU needed): it refuses more than one GPU
before touching the device, and an HBM-traffic record is used only while its
hash (kernel sources and compile flags) matches."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_traffic_records_are_used_only_for_their_hash():
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for kernel in ("vix_kernel", "viewshed_kernel"):
        h = d[kernel]["source_hash"]
        assert bench.traffic_from_profiles(kernel, h) == d[kernel]["bytes_per_launch"]
        assert bench.traffic_from_profiles(kernel, "0" * 16) is None
    assert bench.traffic_from_profiles("no_such_kernel", "0" * 16) is None


def test_source_hash_follows_compile_flags(monkeypatch):
    from paper_2006_16783_amd import build as B
    before = bench.source_hash(["vix.hip", "common.hpp"])
    monkeypatch.setitem(B.FILE_FLAGS, "vix.hip", [])
    assert bench.source_hash(["vix.hip", "common.hpp"]) != before
