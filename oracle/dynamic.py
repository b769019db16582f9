"""Single-path (Alg. 1) and multi-path (Alg. 2) drivers of the oracle.

Oracle -- test infrastructure only (see the package docstring).

Chunk construction (Sec. IV-C): operations are scanned in order; unitary gates
are appended to the branch's chunk; a classically controlled gate is appended
when its condition holds on the branch's register and skipped otherwise
(Sec. IV-B2); a chunk is compressed when it holds k operations, or, when it is
non-empty, before a measurement; a residual chunk is compressed at the end.
With an operator-bond cap w_cap (a reading, for gates on distant qubits whose
operator bonds multiply): a gate that would make some bond of the chunk's
operator exceed w_cap (M.span_bonds) first closes the current chunk, which is
compressed, and then starts the next one.

Single path (Alg. 1): a measurement samples outcome m with probability p_m
(here: m = 0 when the supplied uniform u < p_0), p <- p p_m, the outcome is
written to its bit, and the fidelity estimate is the product of the partial
fidelities (Sec. III-C).

Multi path (Alg. 2): a measurement replaces each branch by one child per
outcome with p_m > eps (m = 0 first), each with p p_m, the updated register,
the parent's fidelity and an empty chunk; after the measurement, if more than
M branches are live only the M with the largest p are kept (stable order on
ties; no renormalisation, the dropped mass is reported).  Multi-path fidelity
is the probability-weighted mean of the branch fidelities (Sec. V-C).
"""
from __future__ import annotations

from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from inputs.circuits import CGate, Circuit, Gate, Measure
from inputs.randomness import bra_init_gaussians

from . import mps as M
from . import ttn as T

EPS_BRANCH = 1e-10


def holds(cond, c) -> bool:
    """Condition phi(c): XOR of the selected bits equals the stated value."""
    return (sum(int(c[b]) for b in cond.bits) % 2) == int(cond.value)


class Simulator:
    """Parameters shared by both strategies: bond cap chi, chunk size k,
    sweeps s, the seed of the starting guess."""

    def __init__(self, n: int, chi: int, k: int, n_sweeps: int = 2, init_seed: int = 7,
                 warm_eta: Optional[float] = None, w_cap: Optional[int] = None,
                 tree: Optional[Sequence[int]] = None):
        self.n, self.chi, self.k, self.s, self.init_seed = n, chi, k, n_sweeps, init_seed
        self.warm_eta = warm_eta   # None: generic guess; else warm start (M.warm_bra)
        self.w_cap = w_cap         # None: no operator-bond cap on a chunk
        # None: MPS; else the levels (n_0 = 1, ..., n_L = n) of a tree network (oracle.ttn)
        self.tree = T.Tree(tree) if tree is not None else None
        if self.tree is not None and (self.tree.n != n or warm_eta is not None):
            raise ValueError("the tree must hold n qubits; warm start is an MPS option")
        self._bra = {}

    def zero(self, chi: int):
        return T.zero_state(self.tree, chi) if self.tree else M.zero_state(self.n, chi)

    def norms(self, state, q: int):
        return T.outcome_norms(self.tree, state, q) if self.tree else M.outcome_norms(state, q)

    def collapse(self, state, q: int, m: int, nm: float):
        return T.collapse(self.tree, state, q, m, nm) if self.tree else M.collapse(state, q, m, nm)

    def closes_chunk(self, chunk, gate) -> bool:
        """True when appending `gate` to the non-empty `chunk` would push an
        operator bond past w_cap.  A gate over the cap on its own is an
        error."""
        if self.w_cap is None or len(gate[0]) == 1:
            return False
        if M.span_bonds(self.n, [gate]).max() > self.w_cap:
            raise ValueError("a single gate exceeds the operator-bond cap")
        return bool(chunk) and M.span_bonds(self.n, list(chunk) + [gate]).max() > self.w_cap

    def bra_init(self, chi: int) -> List[np.ndarray]:
        if chi not in self._bra:
            self._bra[chi] = (T.generic_bra(self.tree, chi, self.init_seed) if self.tree else
                              M.generic_bra(bra_init_gaussians(self.n, chi, self.init_seed)))
        return self._bra[chi]

    def compress(self, state, chunk, chi: int):
        if self.tree is not None:
            new, f, _ = T.compress(self.tree, state, chunk, self.bra_init(chi), self.s)
            return new, f
        mpo = M.chunk_mpo(self.n, chunk)
        bra = self.bra_init(chi)
        if self.warm_eta is not None and all(
                k.shape[0] <= b.shape[0] and k.shape[2] <= b.shape[2] for k, b in zip(state, bra)):
            bra = M.warm_bra(state, bra, self.warm_eta)
        new, f, centre = M.compress(state, mpo, bra, self.s)
        return new, f


def _unitary(op):
    g = op.gate if isinstance(op, CGate) else op
    return (tuple(g.qubits), g.mat)


def run_single_path(circ: Circuit, sim: Simulator, uniforms: Optional[Sequence[float]] = None,
                    outcomes: Optional[Sequence[int]] = None,
                    chi_ladder: Optional[Sequence[int]] = None, f_target: float = 0.0,
                    chis: Optional[Sequence[int]] = None) -> Dict:
    """Alg. 1.  Outcomes come from ``outcomes`` when given (replay), else from
    ``uniforms`` (m = 0 iff u < p_0).  Returns the fidelity estimate, path
    probability, register, final MPS and the per-measurement records.
    Adaptive bond cap (a reading; the paper fixes chi per run): with
    ``chi_ladder`` (ascending from sim.chi), a compression whose partial
    fidelity is below ``f_target`` moves the run one rung up for the next
    compressions; "chis" records the cap of every compression.
    Bond-cap schedule: ``chis`` (exclusive with ``chi_ladder``) gives the cap
    of each compression in order, e.g. the caps a multi-path branch used along
    its path (each child compresses into its own cap, the ket keeping its
    parent's bonds); a run needing more compressions than listed is an
    error."""
    if chis is not None and chi_ladder is not None:
        raise ValueError("chis and chi_ladder are exclusive")
    state = sim.zero(sim.chi)
    c = [0] * circ.n_bits
    p, fid = 1.0, 1.0
    chunk: List = []
    rec = {"outcomes": [], "pms": [], "p0s": [], "fids": [], "chis": []}
    i_meas = 0
    rung = 0
    ladder = list(chi_ladder) if chi_ladder is not None else [sim.chi]

    def flush():
        nonlocal state, fid, chunk, rung
        if chis is not None:
            if len(rec["chis"]) >= len(chis):
                raise ValueError("the bond-cap schedule is shorter than the run")
            cap = int(chis[len(rec["chis"])])
        else:
            cap = ladder[rung]
        state, f = sim.compress(state, chunk, cap)
        fid *= f
        rec["fids"].append(f)
        rec["chis"].append(cap)
        chunk = []
        if f < f_target and rung + 1 < len(ladder):
            rung += 1

    for op in circ.ops:
        if isinstance(op, CGate) and not holds(op.cond, c):
            continue
        if isinstance(op, Measure):
            if chunk:
                flush()
            n0, n1 = sim.norms(state, op.qubit)
            p0 = n0 / (n0 + n1)
            if outcomes is not None:
                m = int(outcomes[i_meas])
            else:
                m = 0 if uniforms[i_meas] < p0 else 1
            nm = (n0, n1)[m]
            pm = nm / (n0 + n1)
            if pm <= EPS_BRANCH:
                raise ValueError("sampled an outcome of vanishing probability")
            state = sim.collapse(state, op.qubit, m, nm)
            p *= pm
            c[op.bit] = m
            rec["outcomes"].append(m)
            rec["pms"].append(pm)
            rec["p0s"].append(p0)
            i_meas += 1
        else:
            g = _unitary(op)
            if sim.closes_chunk(chunk, g):
                flush()
            chunk.append(g)
            if len(chunk) == sim.k:
                flush()
    if chunk:
        flush()
    return {"F": fid, "p": p, "c": c, "mps": state, **rec}


def topk_by_weight(weights: Sequence[float], k: int):
    """Indices of the k largest weights in descending order, ties kept in
    list order (stable), and the total weight of the rest."""
    order = sorted(range(len(weights)), key=lambda i: -weights[i])   # stable
    keep = order[:k]
    dropped = float(sum(weights[i] for i in order[k:]))
    return keep, dropped


def prune_adaptive(weights: Sequence[float], k_max: int, mass_tol: float = 0.0,
                   rel_min: float = 0.0):
    """Adaptive pruning beyond top-M (a reading of the open direction in the
    conclusion): walk the weights from the largest down (ties in list order)
    and keep each while fewer than k_max are kept, it is at least rel_min
    times the largest weight, and, for mass_tol > 0, the mass kept before it
    is below (1 - mass_tol) times the total (summed in list order).  The
    largest is always kept.  Returns the kept indices and the dropped mass."""
    order = sorted(range(len(weights)), key=lambda i: -weights[i])   # stable
    total = 0.0
    for w in weights:
        total += float(w)
    keep, kept = [], 0.0
    for i in order:
        w = float(weights[i])
        if len(keep) == k_max:
            break
        if keep and (w < rel_min * float(weights[order[0]])
                     or (mass_tol > 0 and kept >= (1.0 - mass_tol) * total)):
            break
        keep.append(i)
        kept += w
    dropped = 0.0
    for i in order[len(keep):]:
        dropped += float(weights[i])
    return keep, dropped


def run_multi_path(circ: Circuit, sim: Simulator, max_branches: Optional[int] = None,
                   chi_of: Optional[Callable[[tuple], int]] = None,
                   eps: float = EPS_BRANCH, chi_ladder: Optional[Sequence[int]] = None,
                   f_target: float = 0.0, prune: Optional[Sequence[float]] = None) -> Dict:
    """Alg. 2.  ``chi_of(path)`` gives a child's bond cap (default: sim.chi).
    ``prune = (mass_tol, rel_min)`` replaces the top-M step by
    prune_adaptive(p, max_branches or all, mass_tol, rel_min), applied after
    every measurement.
    With ``chi_ladder`` (ascending from sim.chi; a reading, the paper fixes
    chi per run) a branch whose compression fidelity falls below ``f_target``
    takes the next rung for its later compressions and passes its rung to
    its children; "chis" records each branch's caps along its path.
    Returns the live branches (path, p, c, F, mps, chi, and p0s: the p_0 of
    every measurement along the branch's path, taken on its ancestor), the
    dropped mass and the probability-weighted fidelity."""
    ladder = list(chi_ladder) if chi_ladder is not None else [sim.chi]
    live = [{"path": (), "p": 1.0, "c": [0] * circ.n_bits, "F": 1.0, "chunk": [],
             "mps": sim.zero(sim.chi), "chi": sim.chi, "rung": 0,
             "chis": [], "p0s": []}]
    dropped = 0.0
    n_compress = 0

    def flush(b):
        nonlocal n_compress
        b["mps"], f = sim.compress(b["mps"], b["chunk"], b["chi"])
        b["F"] *= f
        b["chunk"] = []
        b["chis"].append(b["chi"])
        n_compress += 1
        if chi_ladder is not None and f < f_target and b["rung"] + 1 < len(ladder):
            b["rung"] += 1
            b["chi"] = ladder[b["rung"]]

    for op in circ.ops:
        nxt = []
        for b in live:
            if isinstance(op, CGate) and not holds(op.cond, b["c"]):
                nxt.append(b)
                continue
            if isinstance(op, Measure):
                if b["chunk"]:
                    flush(b)
                n0, n1 = sim.norms(b["mps"], op.qubit)
                for m, nm in ((0, n0), (1, n1)):
                    pm = nm / (n0 + n1)
                    if pm > eps:
                        c = list(b["c"])
                        c[op.bit] = m
                        path = b["path"] + (m,)
                        nxt.append({"path": path, "p": b["p"] * pm, "c": c, "F": b["F"],
                                    "chunk": [], "mps": sim.collapse(b["mps"], op.qubit, m, nm),
                                    "chi": chi_of(path) if chi_of else b["chi"],
                                    "rung": b["rung"], "chis": list(b["chis"]),
                                    "p0s": b["p0s"] + [n0 / (n0 + n1)]})
            else:
                g = _unitary(op)
                if sim.closes_chunk(b["chunk"], g):
                    flush(b)
                b["chunk"].append(g)
                if len(b["chunk"]) == sim.k:
                    flush(b)
                nxt.append(b)
        live = nxt
        if isinstance(op, Measure) and prune is not None:
            keep, d = prune_adaptive([b["p"] for b in live], max_branches or len(live),
                                     prune[0], prune[1])
            dropped += d
            live = [live[i] for i in keep]
        elif isinstance(op, Measure) and max_branches is not None and len(live) > max_branches:
            keep, d = topk_by_weight([b["p"] for b in live], max_branches)
            dropped += d
            live = [live[i] for i in keep]
    for b in live:
        if b["chunk"]:
            flush(b)
    ptot = sum(b["p"] for b in live)
    fmp = sum(b["p"] * b["F"] for b in live) / ptot if ptot > 0 else float("nan")
    return {"branches": live, "dropped": dropped, "F_mp": fmp, "n_compress": n_compress}


def tvd(p: Dict, q: Dict) -> float:
    """Total variation distance 1/2 sum |p_g - q_g| over the union of paths."""
    keys = set(p) | set(q)
    return 0.5 * sum(abs(p.get(k, 0.0) - q.get(k, 0.0)) for k in keys)
