"""Host-side pieces of bench.py (no GPU): argument handling, the operator
bond of a chunk, the roofline record and the traffic guard."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_mpo_bond_max():
    assert bench.mpo_bond_max({"layers_per_round": 1}) == 4
    assert bench.mpo_bond_max({"layers_per_round": 2}) == 4
    assert bench.mpo_bond_max({"layers_per_round": 3}) == 16


def test_roofline_record():
    n = len(bench.CLASSES)
    launches = np.ones(n)
    ms = np.ones(n)
    flops = np.full(n, 1e9)
    byts = np.full(n, 1e6)
    ms[bench.CLASSES.index("qr")] = 10.0
    rl = bench.roofline((launches, ms, flops, byts), "c64")
    assert rl["bound"] == "alu" and rl["unit"] == "TFLOP/s"
    assert abs(rl["achieved"] - 1e9 / 10e-3 / 1e12) < 1e-3
    assert abs(rl["frac"] - rl["achieved"] / rl["peak"]) < 1e-3
    assert rl["traffic"] is None            # counters only on the default workload
    ms[bench.CLASSES.index("gemm_nt")] = 20.0
    rl = bench.roofline((launches, ms, flops, byts), "bf16x3")
    assert rl["bound"] == "mfma" and abs(rl["peak"] - 2500.0 / 3) < 1e-9


def test_traffic_guard_matches_sources():
    t = bench.measured_traffic("qr")
    assert t is None or 1e9 < t < 1e11
    assert bench.measured_traffic("no such class") is None


def test_tree_overlap_is_the_state_vector_overlap():
    from oracle import ttn as OT
    from paper_2609_26516_amd.engine import TreeTopology
    for lv in ([1, 3, 9], [1, 2, 4, 8]):
        tr, tp = OT.Tree(lv), TreeTopology(lv)
        a, b = OT.generic_bra(tr, 4, 1), OT.generic_bra(tr, 4, 2)
        b = [x * (1 + 0.3j) if i == 0 else x for i, x in enumerate(b)]
        assert abs(bench.tree_overlap(tp, a, b) - OT.overlap(tr, a, b)) < 1e-14
