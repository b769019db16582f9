"""The paper's worked examples and closed forms as oracle pins: teleportation
(Sec. V-A) and dynamic GHZ preparation (Sec. V-B), plus branch-ensemble
invariants and single-path sampling statistics."""
import json
import os

import numpy as np
import pytest

from inputs import circuits as C
from inputs.randomness import shot_uniforms
from oracle import dynamic as D
from oracle import mps as M
from oracle import statevector as SV

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _bob_state(mps):
    """Reduced state of qubit 2 when qubits 0 and 1 are in a basis state."""
    v = M.to_statevector(mps).reshape(4, 2)
    row = v[np.argmax(np.linalg.norm(v, axis=1))]
    return row / np.linalg.norm(row)


def test_teleport_four_paths():
    g = _gold("teleport.json")
    res = D.run_multi_path(C.teleportation(False), D.Simulator(3, 2, k=20, n_sweeps=2))
    br = res["branches"]
    assert [b["path"] for b in br] == [(0, 0), (0, 1), (1, 0), (1, 1)]
    for b in br:
        assert abs(b["p"] - g["printed"]["p_path4"]) < 1e-12
        assert abs(b["F"] - 1) < 1e-12
    (a, bb) = [complex(*x) for x in g["input_amplitudes"]]
    nrm = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
    want = np.array([a, bb]) / nrm
    for b in br:                                  # Bob holds the input state
        assert abs(abs(np.vdot(want, _bob_state(b["mps"]))) - 1) < 1e-12


def test_teleport_eight_paths():
    g = _gold("teleport.json")
    res = D.run_multi_path(C.teleportation(True), D.Simulator(3, 2, k=20, n_sweeps=2))
    br = res["branches"]
    assert len(br) == 8
    (a, bb) = [complex(*x) for x in g["input_amplitudes"]]
    p0 = abs(a) ** 2 / (abs(a) ** 2 + abs(bb) ** 2)
    for b in br:
        exact = 0.25 * (p0 if b["path"][2] == 0 else 1 - p0)
        printed = g["printed"]["p_path8_bob0" if b["path"][2] == 0 else "p_path8_bob1"]
        assert abs(b["p"] - exact) < 1e-12
        assert abs(b["p"] - printed) < g["printed_rounding"]["p_path8"]
    assert abs(p0 - g["printed"]["bob_p0"]) < g["printed_rounding"]["bob"]
    assert abs(sum(b["p"] for b in br) - 1) < 1e-12


@pytest.mark.parametrize("n", _gold("ghz.json")["sizes"])
def test_ghz_paths_equiprobable(n):
    prm = _gold("ghz.json")["params"]
    circ = C.ghz_dynamic(n)
    r = (n - 1) // 2
    res = D.run_multi_path(circ, D.Simulator(n, prm["chi"], k=prm["k"], n_sweeps=prm["s"]))
    br = res["branches"]
    assert len(br) == 2 ** r
    for b in br:
        assert abs(b["p"] - 2.0 ** -r) < 1e-12
        # reset outcomes equal the mid-circuit outcomes (deterministic)
        assert b["c"][r:] == b["c"][:r]
        assert abs(b["F"] - 1) < 1e-10
    assert abs(sum(b["p"] for b in br) - 1) < 1e-12


@pytest.mark.parametrize("n", [5, 7, 9])
def test_ghz_final_parity(n):
    circ = C.ghz_dynamic(n, final_measure=True)
    r = (n - 1) // 2
    res = D.run_multi_path(circ, D.Simulator(n, 4, k=25, n_sweeps=2))
    br = res["branches"]
    assert len(br) == 2 ** (r + 1)
    tot = {0: 0.0, 1: 0.0}
    for b in br:
        fin = b["c"][2 * r:]
        assert len(set(fin)) == 1                 # all odd qubits agree
        tot[fin[0]] += b["p"]
    assert abs(tot[0] - 0.5) < 1e-12 and abs(tot[1] - 0.5) < 1e-12


@pytest.mark.parametrize("n,cap", _gold("ghz.json")["cap_cases"])
def test_ghz_branch_cap_tvd_closed_form(n, cap):
    circ = C.ghz_dynamic(n)
    r = (n - 1) // 2
    res = D.run_multi_path(circ, D.Simulator(n, 4, k=25, n_sweeps=2), max_branches=cap)
    br = res["branches"]
    kept = min(cap, 2 ** r)
    assert len(br) == kept
    ideal = {b["path"]: 2.0 ** -r for b in SV.branches(circ)} if n <= 11 else None
    sim = {b["path"]: b["p"] for b in br}
    raw = 0.5 * (1 - kept * 2.0 ** -r)
    assert abs(sum(sim.values()) + res["dropped"] - 1) < 1e-12
    if ideal is not None:
        assert abs(D.tvd(ideal, sim) - raw) < 1e-12
        ptot = sum(sim.values())
        renorm = {k: v / ptot for k, v in sim.items()}
        assert abs(D.tvd(ideal, renorm) - 2 * raw) < 1e-12
    else:
        assert abs(res["dropped"] - (1 - kept * 2.0 ** -r)) < 1e-12
    if kept == 2 ** r:
        assert raw == 0.0


def test_multi_path_matches_statevector_branches():
    circ, p = C.workload("cfg1_n10_chi16", n=6, depth=4, chi=8)
    res = D.run_multi_path(circ, D.Simulator(6, 8, k=1000))
    ref = {b["path"]: b for b in SV.branches(circ)}
    assert {b["path"] for b in res["branches"]} == set(ref)
    for b in res["branches"]:
        assert abs(b["p"] - ref[b["path"]]["p"]) < 1e-12
        v = M.to_statevector(b["mps"])
        assert abs(abs(np.vdot(ref[b["path"]]["psi"], v)) ** 2 - 1) < 1e-11


def test_single_path_sampling_statistics():
    """Empirical path frequencies of single-path runs against the exact
    teleportation distribution (chi-square at fixed seeds)."""
    circ = C.teleportation(True)
    sim = D.Simulator(3, 2, k=20, n_sweeps=2)
    exact = {b["path"]: b["p"] for b in SV.branches(circ)}
    n_shots = 1500
    counts = {}
    for s in range(n_shots):
        r = D.run_single_path(circ, sim, uniforms=shot_uniforms(77, s, 3))
        counts[tuple(r["outcomes"])] = counts.get(tuple(r["outcomes"]), 0) + 1
        assert abs(r["p"] - exact[tuple(r["outcomes"])]) < 1e-12
    chi2 = sum((counts.get(k, 0) - n_shots * v) ** 2 / (n_shots * v) for k, v in exact.items())
    assert chi2 < 24.3                      # 7 degrees of freedom, p = 0.001
    emp = {k: v / n_shots for k, v in counts.items()}
    assert D.tvd(exact, emp) < 0.06


def test_single_path_tvd_shrinks_with_runs():
    circ = C.ghz_dynamic(5)
    sim = D.Simulator(5, 4, k=25, n_sweeps=2)
    exact = {b["path"]: b["p"] for b in SV.branches(circ)}
    res = []
    for n_runs in (4, 64, 512):
        counts = {}
        for s in range(n_runs):
            r = D.run_single_path(circ, sim, uniforms=shot_uniforms(5, s, 8))
            counts[tuple(r["outcomes"])] = counts.get(tuple(r["outcomes"]), 0) + 1
        res.append(D.tvd(exact, {k: v / n_runs for k, v in counts.items()}))
    assert res[2] < res[0] and res[2] < 0.1
