"""Pins of the oracle's gates on distant or reversed qubit pairs, the
operator-bond chunk rule and the adaptive pruning rule.

Each check takes an independent route: the entry-wise definition of an
embedded gate (<i|U|j> from the gate's matrix where i and j agree elsewhere),
the SWAP identity, brute-force statevector replay in the exact regime, and
hand-worked weight lists for the pruning rule."""
import numpy as np
import pytest

from inputs import circuits as C
from oracle import dynamic as D
from oracle import mps as M
from oracle import statevector as SV


def _mpo_full_operator(mpo):
    t = mpo[0][0].reshape(2, 2, -1)
    d = 2
    for w in mpo[1:]:
        t = np.einsum("ijw,wstv->isjtv", t, w).reshape(d * 2, d * 2, -1)
        d *= 2
    return t[:, :, 0]


@pytest.mark.parametrize("pair", [(0, 3), (3, 0), (1, 4), (4, 2), (2, 1)])
def test_apply_gate_matches_entrywise_embedding(pair):
    rng = np.random.default_rng(sum(pair))
    n = 5
    u = C.haar_unitary(rng, 4)
    psi = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
    full = SV.full_operator(n, pair, u)
    np.testing.assert_allclose(SV.apply_gate(psi, n, pair, u), full @ psi, atol=1e-12)
    assert np.allclose(full.conj().T @ full, np.eye(2 ** n))


def test_cnot_far_apart_truth_table():
    """CNOT with control qubit 0 and target qubit 3 of 4 flips bit 3 exactly
    when bit 0 is set; with the pair reversed the roles swap."""
    n = 4
    for i in range(2 ** n):
        e = np.zeros(2 ** n)
        e[i] = 1
        out = SV.apply_gate(e, n, (0, 3), C.CNOT_01)
        j = i ^ 1 if (i >> 3) & 1 else i
        assert out[j] == 1
        out = SV.apply_gate(e, n, (3, 0), C.CNOT_01)
        j = i ^ 8 if i & 1 else i
        assert out[j] == 1


@pytest.mark.parametrize("pair", [(0, 4), (4, 0), (1, 3), (3, 1), (2, 3), (3, 2)])
def test_swap_routing_is_the_same_operator(pair):
    rng = np.random.default_rng(7 + pair[0] * 5 + pair[1])
    n = 5
    u = C.haar_unitary(rng, 4)
    routed = M.route_swaps([(pair, u)])
    assert all(len(q) == 1 or q[1] == q[0] + 1 for q, _ in routed)
    full = np.eye(2 ** n, dtype=complex)
    for q, m in routed:
        full = SV.full_operator(n, q, m) @ full
    np.testing.assert_allclose(full, SV.full_operator(n, pair, u), atol=1e-12)
    np.testing.assert_allclose(_mpo_full_operator(M.chunk_mpo(n, [(pair, u)])), full,
                               atol=1e-12)


def test_gate_ranks_and_span_bonds():
    rng = np.random.default_rng(3)
    assert M.gate_rank(C.CNOT_01) == 2
    assert M.gate_rank(M.SWAP) == 4
    assert M.gate_rank(np.kron(C.H, C.Z)) == 1
    assert M.gate_rank(C.haar_unitary(rng, 4)) == 4
    n = 6
    ops = [((0, 3), C.CNOT_01), ((5, 2), C.haar_unitary(rng, 4)), ((1,), C.H),
           ((4, 5), np.kron(C.X, C.X))]
    # bonds w_0..w_6: CNOT spans bonds 1..3 (x2), the Haar gate bonds 3..5 (x4)
    assert list(M.span_bonds(n, ops)) == [1, 2, 2, 8, 4, 4, 1]


def test_chunk_rule_closes_before_the_cap():
    rng = np.random.default_rng(4)
    sim = D.Simulator(6, 4, 20, w_cap=16)
    g1 = ((0, 4), C.haar_unitary(rng, 4))
    g2 = ((1, 5), C.haar_unitary(rng, 4))
    g3 = ((2, 3), C.CNOT_01)
    assert not sim.closes_chunk([], g1)
    assert not sim.closes_chunk([g1], g2)          # bonds 2..4 reach 16
    assert sim.closes_chunk([g1, g2], g3)          # bond 3 would be 32
    assert not sim.closes_chunk([g1, g2], ((0,), C.X))
    with pytest.raises(ValueError):
        D.Simulator(6, 4, 20, w_cap=2).closes_chunk([], g1)
    assert not D.Simulator(6, 4, 20).closes_chunk([g1, g2], g3)


@pytest.mark.parametrize("seed", [0, 1])
def test_random_dynamic_exact_regime_replays_statevector(seed):
    """Distant and reversed pairs, measured subsets and parity conditions: in
    the exact regime (chi = 2^(n/2)) the single-path run equals the
    statevector replay of its outcomes, whatever the chunk boundaries."""
    n = 7
    circ = C.random_dynamic(n, 4, seed)
    assert any(len(o.qubits) == 2 and abs(o.qubits[1] - o.qubits[0]) > 1
               for o in circ.ops if isinstance(o, C.Gate))
    u = np.random.default_rng(seed).random(circ.n_measurements())
    r = D.run_single_path(circ, D.Simulator(n, 8, 20, w_cap=16), uniforms=u)
    ref = SV.replay(circ, r["outcomes"])
    assert abs(r["p"] - ref["p"]) < 1e-11
    assert abs(r["F"] - 1) < 1e-10
    v = M.to_statevector(r["mps"])
    assert abs(abs(np.vdot(ref["psi"], v)) ** 2 - 1) < 1e-10
    r4 = D.run_single_path(circ, D.Simulator(n, 8, 20, w_cap=4), uniforms=u)
    assert r4["outcomes"] == r["outcomes"]
    assert len(r4["fids"]) > len(r["fids"])
    assert abs(abs(M.overlap(r4["mps"], r["mps"])) ** 2 - 1) < 1e-10


def test_prune_adaptive_rules():
    w = [0.05, 0.4, 0.1, 0.4, 0.05]
    keep, d = D.prune_adaptive(w, 5)                 # no rule: all, stable order
    assert keep == [1, 3, 2, 0, 4] and d == 0.0
    keep, d = D.prune_adaptive(w, 3)                 # = top-3
    assert (keep, d) == D.topk_by_weight(w, 3)
    keep, d = D.prune_adaptive(w, 5, mass_tol=0.15)  # stop once 0.85 of the mass is kept
    assert keep == [1, 3, 2] and abs(d - 0.1) < 1e-15
    keep, d = D.prune_adaptive(w, 5, mass_tol=0.2)   # 0.8 reached after two
    assert keep == [1, 3] and abs(d - 0.2) < 1e-15
    keep, d = D.prune_adaptive(w, 5, rel_min=0.2)    # drop below 0.08
    assert keep == [1, 3, 2] and abs(d - 0.1) < 1e-15
    keep, d = D.prune_adaptive([0.0, 0.0], 2, mass_tol=0.5, rel_min=1.0)
    assert keep == [0]                               # the heaviest is always kept
    assert D.prune_adaptive([], 3) == ([], 0.0)


def test_multi_path_prune_keeps_the_mass():
    n = 6
    circ = C.random_dynamic(n, 3, 5)
    sim = D.Simulator(n, 8, 20, w_cap=16)
    full = D.run_multi_path(circ, sim)
    pr = D.run_multi_path(circ, sim, prune=(0.2, 0.0))
    tot = sum(b["p"] for b in pr["branches"])
    assert abs(tot + pr["dropped"] - 1) < 1e-10
    assert len(pr["branches"]) <= len(full["branches"])
    exact = {b["path"]: b["p"] for b in full["branches"]}
    for b in pr["branches"]:
        assert abs(b["p"] - exact[b["path"]]) < 1e-10
