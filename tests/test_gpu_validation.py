"""The paper's validation studies (Sec. V) driven through the GPU path.

Pins: the multi-path probabilities of teleportation (four paths of 1/4;
eight with Bob's qubit measured, 0.25 x the normalised input's |alpha|^2 and
|beta|^2) and of the dynamic GHZ preparation (2^r paths of 2^-r); the GHZ
branch-cap distances in closed form (raw 1/2 (1 - M 2^-r), renormalised
1 - M 2^-r, zero once M >= 2^r); the single-path outcome sequences and hence
the whole distance curve equal to the oracle's on the same seeded uniforms
(complex128, exact regime); and the statistical shape of the curve (the
expected distance of N samples shrinks like N^-1/2).
"""
import numpy as np
import pytest

from inputs import circuits as C
from inputs.randomness import shot_uniforms
from oracle import dynamic as OD

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_26516_amd import engine as E
    e = E.Engine(0)
    yield e
    e.close()


def _V():
    from paper_2609_26516_amd import validation as V
    return V


def test_teleport_distributions(eng):
    V = _V()
    d = V.path_distribution(eng, C.teleportation(False), 2, 20)["p"]
    assert sorted(d) == [(0, 0), (0, 1), (1, 0), (1, 1)]
    assert max(abs(v - 0.25) for v in d.values()) < 1e-12
    a, b = C.teleportation(True).meta["amplitudes"]
    d8 = V.path_distribution(eng, C.teleportation(True), 2, 20)["p"]
    assert len(d8) == 8
    for path, v in d8.items():
        want = 0.25 * (abs(a) ** 2 if path[2] == 0 else abs(b) ** 2)
        assert abs(v - want) < 1e-12
    assert abs(0.25 * abs(a) ** 2 - 0.0929228) < 5e-8      # R13 values


@pytest.mark.parametrize("circ_name,chi,k", [("teleport", 2, 20), ("teleport_bob", 2, 20),
                                             ("ghz7", 4, 25)])
def test_tvd_curve_matches_oracle(eng, circ_name, chi, k):
    """Same seeded uniforms on both sides: identical outcome sequences, so the
    GPU curve equals the curve formed from the oracle's runs."""
    V = _V()
    circ = {"teleport": C.teleportation(False), "teleport_bob": C.teleportation(True),
            "ghz7": C.ghz_dynamic(7)}[circ_name]
    ns, reps, seed = [1, 2, 4, 8, 16, 32], 4, 3
    r = V.tvd_vs_shots(eng, circ, ns, reps, chi, k, seed=seed)
    sim = OD.Simulator(circ.n_qubits, chi, k=k, n_sweeps=2)
    nm = circ.n_measurements()
    paths = []
    for s in range(max(ns) * reps):
        o = OD.run_single_path(circ, sim, uniforms=shot_uniforms(seed, s, nm))
        paths.append(tuple(int(m) for m in o["outcomes"]))
    exact = {tuple(int(c) for c in key): v for key, v in r["exact"].items()}
    ref = V.tvd_curve(paths, exact, ns, reps)
    for got, want in zip(r["curve"], ref):
        assert got["N"] == want["N"]
        np.testing.assert_allclose(got["tvd"], want["tvd"], atol=1e-12)


def test_tvd_shrinks_with_runs(eng):
    """Teleportation, 64 repetitions: the mean distance falls from N = 1
    (1 - 1/4 for any single path) to about sqrt(3 / (2 pi N)) at N = 256."""
    V = _V()
    r = V.tvd_vs_shots(eng, C.teleportation(False), [1, 16, 256], 64, 2, 20, seed=11)
    c = {row["N"]: row["tvd_mean"] for row in r["curve"]}
    assert abs(c[1] - 0.75) < 1e-12
    expect256 = 2 * np.sqrt(2 * 0.25 * 0.75 / (np.pi * 256)) # E|f - p| summed / 2 over 4 paths
    assert 0.5 * expect256 < c[256] < 2.0 * expect256
    assert c[256] < c[16] < c[1]


@pytest.mark.parametrize("n,caps", [(9, [1, 4, 8, 16, 64]), (11, [8, 32, 64]), (13, [16, 64])])
def test_ghz_cap_closed_form(eng, n, caps):
    V = _V()
    r = (n - 1) // 2
    res = V.ghz_tvd_vs_cap(eng, n, caps)
    assert res["paths"] == 2 ** r
    for row in res["rows"]:
        m = min(row["M"], 2 ** r)
        assert row["kept"] == m
        assert abs(row["tvd_raw"] - 0.5 * (1 - m * 2.0 ** -r)) < 1e-12
        assert abs(row["tvd_renormalised"] - (1 - m * 2.0 ** -r)) < 1e-12
        assert abs(row["dropped"] - (1 - m * 2.0 ** -r)) < 1e-12


def test_ghz_scaling_rows(eng):
    V = _V()
    rows = V.ghz_scaling(eng, [5, 9, 13], repeats=1)
    assert [row["paths"] for row in rows] == [4, 16, 64]
    assert all(row["seconds"] > 0 for row in rows)
    mem = [row["state_bytes"] for row in rows]
    assert mem[0] < mem[1] < mem[2]


def test_random_circuit_study_rows_match_oracle(eng):
    """Random dynamic circuits: the study's single-path mean fidelity and
    multi-path fidelity equal the oracle's for the same circuits, uniforms
    and starting guesses (complex128); the exact bond cap gives F = 1."""
    from inputs.randomness import shot_uniforms
    V = _V()
    n, runs = 8, 3
    rows = V.random_circuit_study(eng, n, [2, 3], [4, 16], circuits=2, runs=runs,
                                  max_branches=8)
    assert [(r["depth"], r["chi"]) for r in rows] == [(2, 4), (2, 16), (3, 4), (3, 16)]
    for r in rows:
        if r["chi"] == 16:
            assert abs(r["F_sp"] - 1) < 1e-10 and abs(r["F_mp"] - 1) < 1e-10
        assert r["seconds_sp"] > 0 and r["bytes_mp"] > r["bytes_per_run_sp"]
    r = rows[2]
    for c in range(2):
        circ = C.random_dynamic(n, 3, c)
        sim = OD.Simulator(n, 4, 20, 2, 7 + c, w_cap=16)
        nm = circ.n_measurements()
        f = [OD.run_single_path(circ, sim, uniforms=shot_uniforms(1, s, nm))["F"]
             for s in range(runs)]
        assert abs(r["F_sp_each"][c] - np.mean(f)) < 1e-9
        mp = OD.run_multi_path(circ, sim, max_branches=8)
        assert abs(r["F_mp_each"][c] - mp["F_mp"]) < 1e-9
