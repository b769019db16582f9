"""FP64 tree-tensor-network reference (oracle; test infrastructure only).

The paper names the tree ansatz and its structure but leaves its
compression step to the work it builds on; the step below is a reading: the
single-node form of the MPS step (Sec. III-C) on a tree.  Its pins: the
statevector in the exact regime, the direct overlap, the Schmidt bound of
every edge, non-decreasing sweeps.

Tree (Sec. II-B, TTN paragraph): structure (n_0, ..., n_L) with n_0 = 1 and
n_L = n qubits, regular: a node of layer l has d_l = n_{l+1} / n_l children;
tensors sit in layers 0 .. L-1 and those of layer L-1 carry the physical
legs.  Readings: the qubits are the leaves in order (node i of layer L-1
holds qubits i d .. i d + d - 1, d = d_{L-1}; node i of layer l < L-1 has
children d_l i .. d_l i + d_l - 1); a node tensor's legs are [edge to the
parent (dimension 1 at the root), children or physical legs in order]; the
edge above a node whose subtree holds s qubits has the fixed, zero-padded
dimension min(chi, 2^s, 2^(n-s)).

Compression step (readings): the starting guess is canonical toward the
root (every other node an isometry from its lower legs to its upper edge),
built from seeded Gaussians by QR from the bottom up; a sweep is the walk
that starts at the root and returns to it passing every edge twice
(depth-first, children in order); every node on the walk is set to
T = F / sqrt(<F|F>), F the derivative of <phi|U|psi> by conj(phi_v) (here
formed by brute force on the 2^n statevector: F[x] = <B_x|U psi>, B_x the
network with node v replaced by the unit tensor e_x), and the centre moves
to the next node of the walk by a QR of T with the edge towards that node as
its column index; the last update (at the root) keeps T and gives
f = <F|F>.  Measurement and collapse as for the MPS: n_m from the
statevector, the leg of the measured qubit projected in its node and the node
scaled by 1 / sqrt(n_m).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from . import statevector as SV


class Tree:
    """Node ids in layer order (root 0); parent, children, qubit range."""

    def __init__(self, levels: Sequence[int]):
        levels = [int(x) for x in levels]
        if not levels or levels[0] != 1 or len(levels) < 2:
            raise ValueError("levels start at 1 and end at the number of qubits")
        for a, b in zip(levels, levels[1:]):
            if b % a or b < a:
                raise ValueError("each layer must divide the next")
        self.levels, self.n, self.L = levels, levels[-1], len(levels) - 1
        self.offset = [sum(levels[:l]) for l in range(self.L)]
        self.n_nodes = sum(levels[:self.L])
        self.layer, self.parent, self.children, self.qubits = [], [], [], []
        for l in range(self.L):
            d = levels[l + 1] // levels[l]
            for i in range(levels[l]):
                self.layer.append(l)
                self.parent.append(-1 if l == 0 else self.offset[l - 1] + i // (levels[l] // levels[l - 1]))
                if l + 1 < self.L:
                    self.children.append([self.offset[l + 1] + d * i + c for c in range(d)])
                    self.qubits.append(None)
                else:
                    self.children.append([])
                    self.qubits.append(list(range(d * i, d * i + d)))
        for v in reversed(range(self.n_nodes)):     # inner nodes: union of their children
            if self.children[v]:
                self.qubits[v] = [q for c in self.children[v] for q in self.qubits[c]]

    def edge_dim(self, v: int, chi: int) -> int:
        if v == 0:
            return 1
        s = len(self.qubits[v])
        return min(chi, 2 ** s, 2 ** (self.n - s))

    def shape(self, v: int, chi: int) -> Tuple[int, ...]:
        lower = ([self.edge_dim(c, chi) for c in self.children[v]] if self.children[v]
                 else [2] * len(self.qubits[v]))
        return (self.edge_dim(v, chi), *lower)

    def leaf_of(self, q: int) -> Tuple[int, int]:
        """(node, leg) of qubit q: the physical leg is leg 1 + position."""
        d = self.levels[-1] // self.levels[-2]
        return self.offset[self.L - 1] + q // d, 1 + q % d

    def walk(self) -> List[int]:
        """Root, then every subtree in order, returning through each node."""
        out = [0]

        def rec(v):
            for c in self.children[v]:
                out.append(c)
                rec(c)
                out.append(v)
        rec(0)
        return out


def zero_state(tree: Tree, chi: int) -> List[np.ndarray]:
    out = []
    for v in range(tree.n_nodes):
        t = np.zeros(tree.shape(v, chi), dtype=np.complex128)
        t[(0,) * t.ndim] = 1.0
        out.append(t)
    return out


def _subtree_vec(tree: Tree, state, v: int) -> np.ndarray:
    """(edge dim, 2^s) matrix of node v's subtree: row a is the subtree's
    state over its qubits (first qubit most significant) for edge index a."""
    t = state[v]
    if not tree.children[v]:
        return t.reshape(t.shape[0], -1)
    acc = t
    for c in tree.children[v]:
        sub = _subtree_vec(tree, state, c)                 # (dim_c, 2^{s_c})
        acc = np.tensordot(acc, sub, axes=([1], [0]))      # leg c consumed, its qubits appended
    return acc.reshape(t.shape[0], -1)


def to_statevector(tree: Tree, state) -> np.ndarray:
    return _subtree_vec(tree, state, 0).reshape(-1)


def overlap(tree: Tree, a, b) -> complex:
    return complex(np.vdot(to_statevector(tree, a), to_statevector(tree, b)))


def norm_sq(tree: Tree, state) -> float:
    return float(np.real(overlap(tree, state, state)))


def _isometry_towards(t: np.ndarray, leg: int) -> np.ndarray:
    """Q of the QR of t with `leg` as the column index, in t's leg order."""
    moved = np.moveaxis(t, leg, -1)
    rows = int(np.prod(moved.shape[:-1]))
    cols = moved.shape[-1]
    if rows < cols:
        raise ValueError("edge wider than the rest of the node")
    q, _ = np.linalg.qr(moved.reshape(rows, cols))
    return np.moveaxis(q.reshape(moved.shape), -1, leg)


def generic_bra(tree: Tree, chi: int, seed: int) -> List[np.ndarray]:
    """Seeded Gaussian nodes made canonical toward the root: from the deepest
    layer up, each node is replaced by the Q of its QR with the upper edge
    as the column index and R is absorbed into the parent's leg; the root is
    normalised."""
    from inputs.randomness import gaussians_for_shapes
    shapes = [tree.shape(v, chi) for v in range(tree.n_nodes)]
    g = gaussians_for_shapes(shapes, seed, 0x7EE)
    for v in reversed(range(1, tree.n_nodes)):
        moved = g[v].reshape(g[v].shape[0], -1).T            # (lower legs, upper edge)
        q, r = np.linalg.qr(moved)
        g[v] = q.T.reshape(g[v].shape)
        p = tree.parent[v]
        leg = 1 + tree.children[p].index(v)
        g[p] = np.moveaxis(np.tensordot(r, g[p], axes=([1], [leg])), 0, leg)
    g[0] = g[0] / np.sqrt(np.sum(np.abs(g[0]) ** 2))
    return g


def environment(tree: Tree, bra, v: int, target: np.ndarray) -> np.ndarray:
    """F[x] = <B_x | target>, B_x the statevector of the bra with node v
    replaced by the unit tensor e_x (brute force)."""
    shp = bra[v].shape
    f = np.zeros(shp, dtype=np.complex128).reshape(-1)
    trial = list(bra)
    for x in range(f.size):
        e = np.zeros(f.size, dtype=np.complex128)
        e[x] = 1.0
        trial[v] = e.reshape(shp)
        f[x] = np.vdot(to_statevector(tree, trial), target)
    return f.reshape(shp)


def compress(tree: Tree, ket, ops, bra, n_sweeps: int):
    """Compression step of the chunk `ops` ((qubits, matrix) in time order)
    applied to `ket`, from the starting guess `bra`.  Returns the new state,
    f and the centre (the root)."""
    target = to_statevector(tree, ket)
    for qubits, mat in ops:
        target = SV.apply_gate(target, tree.n, qubits, np.asarray(mat, dtype=np.complex128))
    visits = []
    for _ in range(n_sweeps):
        visits.extend(tree.walk() if not visits else tree.walk()[1:])
    cur = [np.array(t, dtype=np.complex128) for t in bra]
    f = 0.0
    for i, v in enumerate(visits):
        F = environment(tree, cur, v, target)
        nrm2 = float(np.sum(np.abs(F) ** 2))
        t = F / np.sqrt(nrm2) if nrm2 > 0 else F
        if i + 1 == len(visits):
            cur[v] = t
            f = nrm2
            break
        u = visits[i + 1]
        leg = 0 if u == tree.parent[v] else 1 + tree.children[v].index(u)
        cur[v] = _isometry_towards(t, leg)
    return cur, f, visits[-1]


def outcome_norms(tree: Tree, state, q: int) -> Tuple[float, float]:
    return SV.outcome_norms(to_statevector(tree, state), tree.n, q)


def collapse(tree: Tree, state, q: int, m: int, norm_m: float) -> List[np.ndarray]:
    v, leg = tree.leaf_of(q)
    out = [np.array(t) for t in state]
    t = np.moveaxis(out[v], leg, 0).copy()
    t[1 - m] = 0.0
    t /= np.sqrt(norm_m)
    out[v] = np.moveaxis(t, 0, leg)
    return out
