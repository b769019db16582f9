"""Pins of the statevector reference against textbook facts and against the
explicit Kronecker-product embedding of Def. III.2."""
import numpy as np
import pytest

from inputs import circuits as C
from oracle import statevector as SV


def test_gate_embedding_matches_kronecker():
    rng = np.random.default_rng(3)
    n = 5
    psi = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
    psi /= np.linalg.norm(psi)
    for q in range(n):
        u = C.haar_unitary(rng, 2)
        ref = SV.full_operator(n, (q,), u) @ psi
        np.testing.assert_allclose(SV.apply_gate(psi, n, (q,), u), ref, atol=1e-14)
    for q in range(n - 1):
        u = C.haar_unitary(rng, 4)
        ref = SV.full_operator(n, (q, q + 1), u) @ psi
        np.testing.assert_allclose(SV.apply_gate(psi, n, (q, q + 1), u), ref, atol=1e-14)


def test_textbook_states():
    # H|0> = |+>; CNOT (control q0) on |+>|0> = Bell state (|00> + |11>)/sqrt 2
    psi = SV.zero_state(2)
    psi = SV.apply_gate(psi, 2, (0,), C.H)
    np.testing.assert_allclose(psi, [1 / np.sqrt(2), 0, 1 / np.sqrt(2), 0], atol=1e-15)
    psi = SV.apply_gate(psi, 2, (0, 1), C.CNOT_01)
    np.testing.assert_allclose(psi, [1 / np.sqrt(2), 0, 0, 1 / np.sqrt(2)], atol=1e-15)
    n0, n1 = SV.outcome_norms(psi, 2, 1)
    assert abs(n0 - 0.5) < 1e-15 and abs(n1 - 0.5) < 1e-15
    post = SV.project(psi, 2, 1, 1, n1)
    np.testing.assert_allclose(post, [0, 0, 0, 1], atol=1e-15)


@pytest.mark.parametrize("mat,table", [
    (C.CNOT_01, {0: 0, 1: 1, 2: 3, 3: 2}),
    (C.CNOT_10, {0: 0, 1: 3, 2: 2, 3: 1}),
])
def test_cnot_truth_tables(mat, table):
    for src, dst in table.items():
        e = np.zeros(4, dtype=complex)
        e[src] = 1
        out = SV.apply_gate(e, 2, (0, 1), mat)
        assert abs(out[dst] - 1) < 1e-15


def test_measurement_definition():
    rng = np.random.default_rng(5)
    n = 4
    psi = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
    psi /= np.linalg.norm(psi)
    for q in range(n):
        n0, n1 = SV.outcome_norms(psi, n, q)
        # P_m built explicitly as diag over basis states with bit q = m
        bits = (np.arange(2 ** n) >> (n - 1 - q)) & 1
        for m, nm in ((0, n0), (1, n1)):
            pm = np.diag((bits == m).astype(float))
            assert abs(np.vdot(psi, pm @ psi).real - nm) < 1e-14
            np.testing.assert_allclose(SV.project(psi, n, q, m, nm), pm @ psi / np.sqrt(nm),
                                       atol=1e-14)
        assert abs(n0 + n1 - 1) < 1e-14
