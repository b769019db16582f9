"""Dynamic-circuit description and seeded circuit generators.

A dynamic circuit D = (Q, C, O) (Def. III.5) is an ordered list of operations
over n qubits and m classical bits.  Operation kinds (Sec. III-A, Sec. IV-B):

* ``Gate``     unitary on one qubit or on two distinct qubits (q0, q1), in
               any order and at any distance.  The matrix is row-major in the
               basis |q0 q1>, q0 the most significant bit (Def. III.2).
* ``Measure``  computational-basis measurement of one qubit whose outcome is
               written to one classical bit (Def. III.3).
* ``CGate``    a ``Gate`` applied only when its condition holds (Def. III.4).
               A condition is the XOR-parity of a set of bits compared with a
               value; a single bit equal to 1 is the common case.

Reset (Sec. IV-B3) is emitted as a measurement into a scratch bit followed by
an X gate conditioned on that bit.

Qubit Q_i of the paper is site i-1 of the chain (MPS tensors T^[0..n-1]).
Generators build the paper's two fixed circuits (teleportation, Sec. V-A;
dynamic GHZ preparation, Sec. V-B) and the seeded Haar-brickwork stand-ins for
the random dynamic circuits of Sec. V-C.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
# CNOT with control on the first (more significant) qubit of the pair
CNOT_01 = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]],
                   dtype=np.complex128)
# CNOT with control on the second qubit of the pair
CNOT_10 = np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0]],
                   dtype=np.complex128)


@dataclass(frozen=True)
class Gate:
    qubits: Tuple[int, ...]          # (q,) or (q0, q1), q0 != q1
    mat: np.ndarray = field(compare=False)

    def __post_init__(self):
        k = len(self.qubits)
        if k not in (1, 2):
            raise ValueError("gates act on one or two qubits")
        if k == 2 and self.qubits[1] == self.qubits[0]:
            raise ValueError("a two-qubit gate acts on two distinct qubits")
        if self.mat.shape != (2 ** k, 2 ** k):
            raise ValueError("gate matrix shape does not match its qubits")


@dataclass(frozen=True)
class Measure:
    qubit: int
    bit: int


@dataclass(frozen=True)
class Cond:
    bits: Tuple[int, ...]
    value: int = 1


@dataclass(frozen=True)
class CGate:
    cond: Cond
    gate: Gate


@dataclass
class Circuit:
    n_qubits: int
    n_bits: int
    ops: List[object]
    name: str = ""
    meta: dict = field(default_factory=dict)

    def n_measurements(self) -> int:
        return sum(isinstance(o, Measure) for o in self.ops)


def haar_unitary(rng: np.random.Generator, d: int) -> np.ndarray:
    """Haar-random d x d unitary: QR of a complex Ginibre matrix with the
    phases of diag(R) moved into Q (Mezzadri, Notices AMS 54, 2007)."""
    g = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2.0)
    q, r = np.linalg.qr(g)
    dg = np.diag(r)
    return q * (dg / np.abs(dg))[None, :]


def _state_prep(alpha: complex, beta: complex) -> np.ndarray:
    """Single-qubit unitary with first column (alpha, beta)."""
    return np.array([[alpha, -np.conj(beta)], [beta, np.conj(alpha)]], dtype=np.complex128)


TELEPORT_INPUT = (0.61 + 0j, 0.59 + 0.53j)   # Sec. V-A, un-normalised as printed


def teleportation(final_measure: bool = False,
                  amplitudes: Tuple[complex, complex] = TELEPORT_INPUT) -> Circuit:
    """Teleportation protocol of Sec. V-A on three qubits.

    Q1 holds the input state, (Q2, Q3) the Bell pair; Alice measures Q1 and Q2,
    Bob corrects Q3 with X if C2 and Z if C1.  The printed input amplitudes are
    normalised before use (their squared norm is 1.0011).  With
    ``final_measure`` Bob's qubit is measured into C3 afterwards.
    """
    a, b = amplitudes
    nrm = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    a, b = a / nrm, b / nrm
    ops = [
        Gate((0,), _state_prep(a, b)),
        Gate((1,), H),
        Gate((1, 2), CNOT_01),
        Gate((0, 1), CNOT_01),
        Gate((0,), H),
        Measure(0, 0),
        Measure(1, 1),
        CGate(Cond((1,), 1), Gate((2,), X)),
        CGate(Cond((0,), 1), Gate((2,), Z)),
    ]
    n_bits = 2
    if final_measure:
        ops.append(Measure(2, 2))
        n_bits = 3
    return Circuit(3, n_bits, ops, name="teleport" + ("_bob" if final_measure else ""),
                   meta={"amplitudes": (a, b)})


def ghz_dynamic(n: int, with_reset: bool = True, final_measure: bool = False) -> Circuit:
    """Constant-depth dynamic GHZ preparation of Sec. V-B for odd n.

    H on the odd qubits Q1, Q3, ..., Qn; CNOT Q_{2i-1} -> Q_{2i} and
    CNOT Q_{2i+1} -> Q_{2i} so that each even qubit carries the parity of its
    neighbours; measure Q_{2i} into C_i (r = (n-1)/2 measurements); X on
    Q_{2j+1} when C_1 xor ... xor C_j; then reset every even qubit.
    With ``final_measure`` every odd qubit is measured at the end.
    """
    if n < 3 or n % 2 == 0:
        raise ValueError("dynamic GHZ needs an odd n >= 3")
    r = (n - 1) // 2
    ops: List[object] = []
    for q in range(0, n, 2):                      # odd Q -> even sites
        ops.append(Gate((q,), H))
    for i in range(1, r + 1):                     # CNOT Q_{2i-1} -> Q_{2i}
        ops.append(Gate((2 * i - 2, 2 * i - 1), CNOT_01))
    for i in range(1, r + 1):                     # CNOT Q_{2i+1} -> Q_{2i}
        ops.append(Gate((2 * i - 1, 2 * i), CNOT_10))
    for i in range(1, r + 1):                     # measure Q_{2i} -> C_i
        ops.append(Measure(2 * i - 1, i - 1))
    for j in range(1, r + 1):                     # X on Q_{2j+1} if parity(C_1..C_j)
        ops.append(CGate(Cond(tuple(range(j)), 1), Gate((2 * j,), X)))
    n_bits = r
    if with_reset:
        for i in range(1, r + 1):                 # reset Q_{2i}
            ops.append(Measure(2 * i - 1, n_bits))
            ops.append(CGate(Cond((n_bits,), 1), Gate((2 * i - 1,), X)))
            n_bits += 1
    if final_measure:
        for q in range(0, n, 2):
            ops.append(Measure(q, n_bits))
            n_bits += 1
    return Circuit(n, n_bits, ops, name=f"ghz{n}", meta={"r": r})


def brickwork(n: int, depth: int, layers_per_round: int, meas_per_round: int,
              feedforward: str, seed: int, meas_range: Optional[Tuple[int, int]] = None,
              name: str = "") -> Circuit:
    """Seeded Haar brickwork with rounds of mid-circuit measurements.

    Layer l (0-based) applies independent Haar 4x4 unitaries on pairs (2i, 2i+1)
    when l is even and on (2i+1, 2i+2) when l is odd, drawn layer-major then
    pair-ascending.  After every ``layers_per_round`` layers a round measures
    ``meas_per_round`` distinct qubits drawn without replacement from
    ``meas_range`` (inclusive bounds), in ascending qubit order, each into a
    fresh bit; then, per measured qubit q in the same order, the feed-forward
    gates conditioned on that bit:
      'x_right'          X on q+1
      'x_right_z_left'   X on q+1 and Z on q-1
    """
    rng = np.random.default_rng([int(seed), 0xC1C])
    if meas_range is None:
        meas_range = (0, n - 2)
    lo, hi = meas_range
    ops: List[object] = []
    n_bits = 0
    for layer in range(depth):
        start = layer % 2
        for q in range(start, n - 1, 2):
            ops.append(Gate((q, q + 1), haar_unitary(rng, 4)))
        if (layer + 1) % layers_per_round == 0:
            qs = np.sort(rng.choice(np.arange(lo, hi + 1), size=meas_per_round, replace=False))
            bits = []
            for q in qs:
                ops.append(Measure(int(q), n_bits))
                bits.append(n_bits)
                n_bits += 1
            for q, b in zip(qs, bits):
                q = int(q)
                if feedforward in ("x_right", "x_right_z_left"):
                    ops.append(CGate(Cond((b,), 1), Gate((q + 1,), X)))
                if feedforward == "x_right_z_left":
                    ops.append(CGate(Cond((b,), 1), Gate((q - 1,), Z)))
    return Circuit(n, n_bits, ops, name=name or f"brick{n}x{depth}",
                   meta={"seed": seed, "layers_per_round": layers_per_round})


def random_dynamic(n: int, depth: int, seed: int, p_two: float = 0.5, p_round: float = 0.75,
                   meas_max: Optional[int] = None, cond_max: int = 4,
                   name: str = "") -> Circuit:
    """Seeded random dynamic circuit in the style of the random-circuit study
    (Sec. V-C): gates on arbitrary qubit pairs, measured subsets of varying
    size and one or more classically controlled gates.

    Each of the `depth` layers walks a random permutation of the qubits; with
    probability p_two the next two qubits of the walk (in walk order, so at
    any distance and in either order) get a Haar 4x4 gate, else the next
    qubit gets a Haar 2x2 gate.  After a layer, with probability p_round a
    measurement round follows: a random subset of 1..meas_max qubits (default
    max(1, n // 3)), ascending, each into a fresh bit; then 1..cond_max
    gates, each X, Z or a Haar 2x2 on a random qubit, conditioned on the
    parity of a random non-empty subset of the round's bits equalling a
    random value."""
    rng = np.random.default_rng([int(seed), 0xD1A])
    meas_max = max(1, n // 3) if meas_max is None else meas_max
    ops: List[object] = []
    n_bits = 0
    for _ in range(depth):
        walk = [int(q) for q in rng.permutation(n)]
        i = 0
        while i < n:
            if i + 1 < n and rng.random() < p_two:
                ops.append(Gate((walk[i], walk[i + 1]), haar_unitary(rng, 4)))
                i += 2
            else:
                ops.append(Gate((walk[i],), haar_unitary(rng, 2)))
                i += 1
        if rng.random() < p_round:
            size = int(rng.integers(1, meas_max + 1))
            qs = np.sort(rng.choice(n, size=size, replace=False))
            bits = []
            for q in qs:
                ops.append(Measure(int(q), n_bits))
                bits.append(n_bits)
                n_bits += 1
            for _ in range(int(rng.integers(1, cond_max + 1))):
                nb = int(rng.integers(1, len(bits) + 1))
                cb = tuple(sorted(int(b) for b in rng.choice(bits, size=nb, replace=False)))
                kind = int(rng.integers(3))
                mat = (X, Z)[kind] if kind < 2 else haar_unitary(rng, 2)
                ops.append(CGate(Cond(cb, int(rng.integers(2))), Gate((int(rng.integers(n)),), mat)))
    return Circuit(n, n_bits, ops, name=name or f"random{n}x{depth}",
                   meta={"seed": seed, "depth": depth})


# Synthetic workloads with the shapes of the five benchmark configurations.
# Each entry: circuit recipe + simulator parameters.  k=None means "chunks
# break only at measurements" (k at least the longest unitary segment).
WORKLOADS = {
    "cfg1_n10_chi16": dict(n=10, depth=10, layers_per_round=2, meas_per_round=2,
                           feedforward="x_right", meas_range=None, chi=16, seed=1001,
                           mode="single", shots=1, precision="c128", init_seed=7),
    "cfg2_n40_chi256": dict(n=40, depth=20, layers_per_round=2, meas_per_round=4,
                            feedforward="x_right_z_left", meas_range=(1, 38), chi=256,
                            seed=2001, mode="single", shots=1, precision="c64", init_seed=14),
    "cfg3_n32_mp64": dict(n=32, depth=16, layers_per_round=2, meas_per_round=2,
                          feedforward="x_right", meas_range=None, chi=256, seed=3001,
                          mode="multi", max_branches=64, chi_choices=tuple(range(32, 257, 16)),
                          precision="c64", init_seed=21),
    "cfg4_n24_chi64_x1024": dict(n=24, depth=12, layers_per_round=1, meas_per_round=1,
                                 feedforward="x_right", meas_range=None, chi=64, seed=4001,
                                 mode="single", shots=1024, precision="c64", init_seed=28),
    "cfg5_n60_chi1024": dict(n=60, depth=24, layers_per_round=3, meas_per_round=1,
                             feedforward="x_right", meas_range=None, chi=1024, seed=5001,
                             mode="single", shots=1, precision="bf16x3", init_seed=35),
    # tree tensor network [1, 3, 9, 27] at bond cap 32 (the tree and cap of the
    # paper's tree runs on 27 qubits), seeded brickwork standing in for its
    # random dynamic circuits
    "ttn27_chi32": dict(n=27, depth=8, layers_per_round=2, meas_per_round=2,
                        feedforward="x_right", meas_range=None, chi=32, seed=6001,
                        mode="single", shots=64, precision="c64", init_seed=42,
                        tree=(1, 3, 9, 27)),
}


def workload(name: str, **override) -> Tuple[Circuit, dict]:
    """Circuit and simulator parameters of a named workload; keyword overrides
    (e.g. n, depth, chi) give reduced slices of the same recipe."""
    p = dict(WORKLOADS[name])
    p.update(override)
    mr = p.get("meas_range")
    if mr is not None:
        mr = (mr[0], min(mr[1], p["n"] - 2))
    circ = brickwork(p["n"], p["depth"], p["layers_per_round"], p["meas_per_round"],
                     p["feedforward"], p["seed"], mr, name=name)
    return circ, p


def segment_max(circ: Circuit) -> int:
    """Longest run of unitary operations (gates and controlled gates) between
    measurements; a chunk size at least this large breaks chunks only at
    measurements."""
    best = cur = 0
    for o in circ.ops:
        if isinstance(o, Measure):
            cur = 0
        else:
            cur += 1
            best = max(best, cur)
    return best


def ops_summary(circ: Circuit) -> Sequence[int]:
    n_g = sum(isinstance(o, Gate) for o in circ.ops)
    n_c = sum(isinstance(o, CGate) for o in circ.ops)
    return n_g, n_c, circ.n_measurements()
