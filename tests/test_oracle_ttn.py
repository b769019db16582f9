"""Pins of the tree-tensor-network oracle: statevector in the exact regime,
the direct overlap and the Schmidt bound of every edge in the truncated one,
non-decreasing sweeps, canonical starting guess, measurement and collapse
against the statevector, and agreement with the MPS oracle where both are
exact."""
import numpy as np
import pytest

from inputs import circuits as C
from oracle import dynamic as D
from oracle import mps as M
from oracle import statevector as SV
from oracle import ttn as T


def _rand_ops(rng, n, count, far=True):
    ops = []
    for _ in range(count):
        if far:
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        else:
            a = int(rng.integers(n - 1)); b = a + 1
        ops.append(((a, b), C.haar_unitary(rng, 4)))
        ops.append(((int(rng.integers(n)),), C.haar_unitary(rng, 2)))
    return ops


def _apply(n, psi, ops):
    for q, m in ops:
        psi = SV.apply_gate(psi, n, q, m)
    return psi


def test_tree_structure():
    tr = T.Tree([1, 3, 9, 27])
    assert tr.n_nodes == 13 and tr.n == 27
    assert tr.children[0] == [1, 2, 3] and tr.children[2] == [7, 8, 9]
    assert tr.qubits[2] == list(range(9, 18)) and tr.qubits[12] == [24, 25, 26]
    assert tr.leaf_of(13) == (8, 2)
    assert tr.shape(0, 32) == (1, 32, 32, 32) and tr.shape(5, 32) == (8, 2, 2, 2)
    assert tr.edge_dim(1, 1024) == 2 ** 9
    w = tr.walk()
    assert w[0] == 0 and w[-1] == 0 and len(w) == 2 * (tr.n_nodes - 1) + 1
    assert all(b == tr.parent[a] or a == tr.parent[b] for a, b in zip(w, w[1:]))
    with pytest.raises(ValueError):
        T.Tree([1, 3, 8])


def test_zero_state_and_generic_bra():
    tr = T.Tree([1, 2, 4, 8])
    sv = T.to_statevector(tr, T.zero_state(tr, 4))
    assert sv[0] == 1 and np.sum(np.abs(sv)) == 1
    g = T.generic_bra(tr, 4, 5)
    assert abs(T.norm_sq(tr, g) - 1) < 1e-12
    for v in range(1, tr.n_nodes):                # isometries from lower legs to the upper edge
        m = g[v].reshape(g[v].shape[0], -1)
        np.testing.assert_allclose(m @ m.conj().T, np.eye(m.shape[0]), atol=1e-12)


@pytest.mark.parametrize("levels,chi", [([1, 2, 4], 4), ([1, 3, 9], 8), ([1, 2, 4, 8], 16),
                                        ([1, 5], 1)])
def test_compress_exact_regime(levels, chi):
    """Bond caps at the full Schmidt rank: the compression reproduces U psi."""
    tr = T.Tree(levels)
    rng = np.random.default_rng(sum(levels) + chi)
    ket = T.zero_state(tr, chi)
    ops = _rand_ops(rng, tr.n, 3)
    new, f, centre = T.compress(tr, ket, ops, T.generic_bra(tr, chi, 3), 2)
    want = _apply(tr.n, T.to_statevector(tr, ket), ops)
    got = T.to_statevector(tr, new)
    assert centre == 0 and abs(f - 1) < 1e-10
    assert abs(abs(np.vdot(want, got)) ** 2 - 1) < 1e-10
    assert abs(np.linalg.norm(got) - 1) < 1e-10


def _schmidt_bound(n, psi, qubits, cap):
    rest = [q for q in range(n) if q not in qubits]
    t = psi.reshape((2,) * n).transpose(qubits + rest).reshape(2 ** len(qubits), -1)
    s = np.linalg.svd(t, compute_uv=False)
    return float(np.sum(s[:cap] ** 2))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_truncated_fidelity_is_overlap_and_within_every_edge_bound(seed):
    tr = T.Tree([1, 2, 4, 8])
    chi = 2
    rng = np.random.default_rng(seed)
    ket, _, _ = T.compress(tr, T.zero_state(tr, chi), _rand_ops(rng, 8, 2, far=False),
                           T.generic_bra(tr, chi, 1), 2)
    ops = _rand_ops(rng, 8, 3)
    new, f, _ = T.compress(tr, ket, ops, T.generic_bra(tr, chi, 1), 2)
    target = _apply(8, T.to_statevector(tr, ket), ops)
    got = T.to_statevector(tr, new)
    assert abs(np.linalg.norm(got) - 1) < 1e-10
    assert abs(f - abs(np.vdot(got, target)) ** 2) < 1e-10      # f is the squared overlap
    assert f < 1 - 1e-4                                          # truncation is real here
    for v in range(1, tr.n_nodes):
        assert f <= _schmidt_bound(8, target, tr.qubits[v], tr.edge_dim(v, chi)) + 1e-10


def test_sweeps_do_not_lower_the_fidelity():
    tr = T.Tree([1, 3, 9])
    chi = 3
    rng = np.random.default_rng(7)
    ket, _, _ = T.compress(tr, T.zero_state(tr, chi), _rand_ops(rng, 9, 2),
                           T.generic_bra(tr, chi, 2), 2)
    ops = _rand_ops(rng, 9, 3)
    fs = [T.compress(tr, ket, ops, T.generic_bra(tr, chi, 2), s)[1] for s in (1, 2, 3, 4)]
    assert all(b >= a - 1e-12 for a, b in zip(fs, fs[1:]))


def test_measure_and_collapse_match_statevector():
    tr = T.Tree([1, 2, 4, 8])
    rng = np.random.default_rng(4)
    psi, _, _ = T.compress(tr, T.zero_state(tr, 16), _rand_ops(rng, 8, 4),
                           T.generic_bra(tr, 16, 2), 2)
    sv = T.to_statevector(tr, psi)
    for q in (0, 3, 7):
        n0, n1 = T.outcome_norms(tr, psi, q)
        s0, s1 = SV.outcome_norms(sv, 8, q)
        assert abs(n0 - s0) < 1e-13 and abs(n1 - s1) < 1e-13
        for m, nm in ((0, n0), (1, n1)):
            post = T.to_statevector(tr, T.collapse(tr, psi, q, m, nm))
            np.testing.assert_allclose(post, SV.project(sv, 8, q, m, nm), atol=1e-12)


def test_single_path_on_a_tree_matches_mps_and_statevector():
    """Both networks exact: the same outcomes, probabilities and final state."""
    circ = C.random_dynamic(8, 3, 6)
    u = np.random.default_rng(3).random(circ.n_measurements())
    rt = D.run_single_path(circ, D.Simulator(8, 16, 20, 2, 7, tree=[1, 2, 4, 8]), uniforms=u)
    rm = D.run_single_path(circ, D.Simulator(8, 16, 20, 2, 7), uniforms=u)
    ref = SV.replay(circ, rt["outcomes"])
    assert rt["outcomes"] == rm["outcomes"]
    assert abs(rt["p"] - ref["p"]) < 1e-11 and abs(rt["F"] - 1) < 1e-10
    tree = T.Tree([1, 2, 4, 8])
    v = T.to_statevector(tree, rt["mps"])
    assert abs(abs(np.vdot(ref["psi"], v)) ** 2 - 1) < 1e-10
    assert abs(abs(np.vdot(M.to_statevector(rm["mps"]), v)) ** 2 - 1) < 1e-10
