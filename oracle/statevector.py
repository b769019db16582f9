"""Brute-force statevector reference (oracle; test infrastructure only).

The state of n qubits is a normalised vector in C^(2^n) (Def. III.1); qubit 0
(the paper's Q_1) is the most significant bit of the basis index.  Gates are
applied by embedding them with identities (Def. III.2); a measurement has
outcome probability p_m = <psi|P_m|psi> and post-measurement state
P_m psi / sqrt(p_m) (Def. III.3).  Classically controlled gates are applied
when their condition holds (Def. III.4); branches carry (p, c, psi)
(Def. III.6).
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from inputs.circuits import CGate, Circuit, Gate, Measure


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def apply_gate(psi: np.ndarray, n: int, qubits, mat: np.ndarray) -> np.ndarray:
    """psi <- U psi with U acting on the listed qubits (one, or two distinct
    qubits in the order of the matrix's basis) and the identity elsewhere."""
    k = len(qubits)
    t = np.moveaxis(psi.reshape((2,) * n), list(qubits), list(range(k)))
    shape = t.shape
    t = (mat @ t.reshape(2 ** k, -1)).reshape(shape)
    return np.moveaxis(t, list(range(k)), list(qubits)).reshape(-1)


def full_operator(n: int, qubits, mat: np.ndarray) -> np.ndarray:
    """The gate embedded in the full 2^n space.  For one qubit or an
    adjacent pair (q, q+1) by Kronecker products with identities; otherwise
    entry by entry: <i|U|j> = mat[(i_q0 i_q1), (j_q0 j_q1)] when i and j
    agree on every other qubit, else 0 (small n only)."""
    q = qubits[0]
    k = len(qubits)
    if k == 1 or qubits[1] == q + 1:
        return np.kron(np.kron(np.eye(2 ** q), mat), np.eye(2 ** (n - q - k)))
    a, b = qubits
    bit = lambda x, j: (x >> (n - 1 - j)) & 1                         # noqa: E731
    full = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    for i in range(2 ** n):
        for j in range(2 ** n):
            if all(bit(i, o) == bit(j, o) for o in range(n) if o not in (a, b)):
                full[i, j] = mat[2 * bit(i, a) + bit(i, b), 2 * bit(j, a) + bit(j, b)]
    return full


def outcome_norms(psi: np.ndarray, n: int, q: int) -> Tuple[float, float]:
    """<psi|P_m|psi> for m = 0, 1 on qubit q."""
    t = psi.reshape(2 ** q, 2, 2 ** (n - q - 1))
    return float(np.sum(np.abs(t[:, 0, :]) ** 2)), float(np.sum(np.abs(t[:, 1, :]) ** 2))


def project(psi: np.ndarray, n: int, q: int, m: int, norm_m: float) -> np.ndarray:
    """P_m psi / sqrt(norm_m)."""
    t = psi.reshape(2 ** q, 2, 2 ** (n - q - 1)).copy()
    t[:, 1 - m, :] = 0.0
    t /= np.sqrt(norm_m)
    return t.reshape(-1)


def holds(cond, c) -> bool:
    return (sum(int(c[b]) for b in cond.bits) % 2) == int(cond.value)


def replay(circ: Circuit, outcomes: List[int]) -> Dict:
    """Run the circuit exactly along a fixed sequence of outcomes.

    Returns the path probability, the per-measurement p_m, the classical
    register and the final normalised state."""
    n = circ.n_qubits
    psi = zero_state(n)
    c = [0] * circ.n_bits
    p = 1.0
    pms = []
    it = iter(outcomes)
    for op in circ.ops:
        if isinstance(op, CGate):
            if holds(op.cond, c):
                psi = apply_gate(psi, n, op.gate.qubits, op.gate.mat)
        elif isinstance(op, Gate):
            psi = apply_gate(psi, n, op.qubits, op.mat)
        elif isinstance(op, Measure):
            m = next(it)
            n0, n1 = outcome_norms(psi, n, op.qubit)
            nm = (n0, n1)[m]
            pm = nm / (n0 + n1)
            pms.append(pm)
            psi = project(psi, n, op.qubit, m, nm)
            p *= pm
            c[op.bit] = m
    return {"p": p, "pms": pms, "c": c, "psi": psi}


def branches(circ: Circuit, eps: float = 1e-10) -> List[Dict]:
    """Exact branch ensemble {(path, p, c, psi)} of the dynamic circuit: every
    measurement splits each branch into its outcomes with p_m > eps."""
    n = circ.n_qubits
    live = [{"path": (), "p": 1.0, "c": [0] * circ.n_bits, "psi": zero_state(n)}]
    for op in circ.ops:
        nxt = []
        for b in live:
            if isinstance(op, CGate):
                if holds(op.cond, b["c"]):
                    b["psi"] = apply_gate(b["psi"], n, op.gate.qubits, op.gate.mat)
                nxt.append(b)
            elif isinstance(op, Gate):
                b["psi"] = apply_gate(b["psi"], n, op.qubits, op.mat)
                nxt.append(b)
            else:
                n0, n1 = outcome_norms(b["psi"], n, op.qubit)
                for m, nm in ((0, n0), (1, n1)):
                    pm = nm / (n0 + n1)
                    if pm > eps:
                        c = list(b["c"])
                        c[op.bit] = m
                        nxt.append({"path": b["path"] + (m,), "p": b["p"] * pm, "c": c,
                                    "psi": project(b["psi"], n, op.qubit, m, nm)})
        live = nxt
    return live
