"""The measurement side of bench.py, on the CPU: the single-GPU contract, the
arithmetic of the roofline figures, and the tie between the committed
profiles and the kernel sources they were taken on."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


# two passes: [rays traced, inner nodes, triangles, rays continued, LDS node reads, spills]
COUNTS = np.array([[100, 1000, 300, 60, 400, 0],
                   [60, 500, 200, 0, 150, 2]], dtype=np.uint64)


def test_algorithmic_ops_counts_each_unit_once():
    # 160 rays, 1500 node visits, 500 triangle tests
    assert bench.algorithmic_ops(COUNTS) == 150 * 160 + 53 * 1500 + 54 * 500


def test_algorithmic_bytes_by_engine():
    # pass 0: 112*1000 + 48*300 + 32*100, and 40 converged pixels fill image 1: 16*40
    # pass 1: 112*500 + 48*200 + 32*60 (the last pass fills nothing)
    chain = 112 * 1000 + 48 * 300 + 32 * 100 + 16 * 40 + 112 * 500 + 48 * 200 + 32 * 60
    assert bench.algorithmic_bytes(COUNTS, "chain") == chain
    # the per-pass engine also moves its 16-byte state entries: 60 written at
    # pass 0, 60 read at pass 1
    assert bench.algorithmic_bytes(COUNTS, "passes") == chain + 16 * 60 + 16 * 60


def test_logical_bytes_split_lds_from_caches():
    tiers = bench.logical_bytes_by_tier(COUNTS)
    assert tiers["lds"] == 112 * 550
    assert tiers["l1_l2"] == 112 * (1500 - 550) + 48 * 500 + 16 * 160


def test_source_hash_ignores_comments_and_spacing(tmp_path, monkeypatch):
    a, b = tmp_path / "a.hip", tmp_path / "b.hip"
    a.write_text("int f(int x) {  // one\n  return x + 1; /* two */\n}\n")
    b.write_text("int f(int x) { return x + 1; }   // other words\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(a)])
    ha = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(b)])
    assert bench.kernel_source_hash() == ha
    b.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_source_hash() != ha


def test_load_profile_checks_hash_and_workload(tmp_path):
    p = tmp_path / "prof.json"
    p.write_text(json.dumps({"kernel_source_sha256": bench.kernel_source_hash(), "workload": "terrain1m", "x": 1}))
    assert bench.load_profile(str(p), "terrain1m")["x"] == 1
    assert bench.load_profile(str(p), "terrain4m") is None
    p.write_text(json.dumps({"kernel_source_sha256": "0" * 64, "workload": "terrain1m"}))
    assert bench.load_profile(str(p), "terrain1m") is None
    assert bench.load_profile(str(tmp_path / "missing.json"), "terrain1m") is None


@pytest.mark.parametrize("name", ["k_chain_terrain1m_traffic.json", "k_chain_terrain1m_counters.json"])
def test_committed_profiles_match_the_kernel_sources(name):
    """The bench line reports HBM traffic and VALU issue only from profiles
    taken on the current kernels; the committed ones must be current."""
    pr = bench.load_profile(os.path.join(ROOT, "profiles", name), "terrain1m")
    assert pr is not None, f"profiles/{name} was taken on other kernel sources"
