"""Drivers of the dynamic-circuit strategies over the C ABI.

The classical side of the method stays here, on the host: scanning the
operation list, evaluating the Boolean conditions of classically controlled
gates on each branch's register (Sec. IV-B2), building chunks (Sec. IV-C),
sampling outcomes (Alg. 1) or branching on them (Alg. 2) and keeping the
top-M branches.  Every tensor operation (compression step, measurement
probability, collapse) runs in libdcs.so on the GPU; PyTorch only provides
the device buffer and the stream.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from inputs.circuits import CGate, Circuit, Gate, Measure

from . import capi

EPS_BRANCH = 1e-10
PRECISIONS = {"c128": capi.DCS_C128, "c64": capi.DCS_C64, "bf16x3": capi.DCS_BF16X3}


def _cond_true(cond, regs: np.ndarray) -> np.ndarray:
    """phi evaluated on every row of a (branches x bits) register array."""
    par = np.zeros(regs.shape[0], dtype=np.int64)
    for b in cond.bits:
        par ^= regs[:, b].astype(np.int64)
    return par == int(cond.value)


def _gate_of(op) -> Gate:
    return op.gate if isinstance(op, CGate) else op


class Engine:
    """One HIP device: the library context plus a cache of compiled chunks."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("a ROCm GPU is required")
        self.device = device
        torch.cuda.set_device(device)
        self.ctx = capi.dcs_ctx_create(device)
        self._chunks: Dict[tuple, tuple] = {}

    def stream(self) -> int:
        return torch.cuda.current_stream(self.device).cuda_stream

    def chunk(self, circ: Circuit, op_ids: Sequence[int]) -> int:
        """Compiled chunk of the listed operations (cached by circuit and op
        indices; the cache holds the circuit, so its id is not reused)."""
        key = (id(circ), tuple(op_ids))
        hit = self._chunks.get(key)
        if hit is not None and hit[0] is circ:
            return hit[1]
        if hit is not None:
            capi.dcs_chunk_destroy(hit[1])
        q0, q1, mats = [], [], []
        for i in op_ids:
            g = _gate_of(circ.ops[i])
            q0.append(g.qubits[0])
            q1.append(g.qubits[1] if len(g.qubits) == 2 else -1)
            mats.append(np.asarray(g.mat, dtype=np.complex128).reshape(-1))
        h = capi.dcs_chunk_compile(self.ctx, circ.n_qubits, q0, q1, np.concatenate(mats))
        self._chunks[key] = (circ, h)
        return h

    def span(self, circ: Circuit, li: int):
        """(lo, hi, r) of operation li: the qubit range a two-qubit gate's
        operator bond spans and its operator-Schmidt rank (dcs_gate_rank);
        None for a one-qubit gate."""
        key = (id(circ), "span")
        hit = self._chunks.get(key)
        if hit is None or hit[0] is not circ:
            hit = (circ, {})
            self._chunks[key] = hit
        cache = hit[1]
        if li not in cache:
            g = _gate_of(circ.ops[li])
            if len(g.qubits) == 1:
                cache[li] = None
            else:
                cache[li] = (min(g.qubits), max(g.qubits), capi.dcs_gate_rank(g.mat))
        return cache[li]

    def clear_chunks(self) -> None:
        for _, h in self._chunks.values():
            if not isinstance(h, dict):
                capi.dcs_chunk_destroy(h)
        self._chunks.clear()

    def tuning(self, enabled: bool, reps: int = 3) -> None:
        """Online autotuning of the contraction tile shapes (on by default)."""
        capi.dcs_ctx_set_tuning(self.ctx, enabled, reps)

    def save_tuning(self, path: str) -> None:
        capi.dcs_ctx_tuning_save(self.ctx, path)

    def load_tuning(self, path: str) -> None:
        capi.dcs_ctx_tuning_load(self.ctx, path)

    def graphs(self, enabled: bool) -> None:
        """Replay recurring compression steps from captured HIP graphs."""
        capi.dcs_ctx_set_graphs(self.ctx, enabled)

    def timing(self, enabled: bool) -> None:
        capi.dcs_ctx_set_timing(self.ctx, enabled)

    def timing_stats(self, reset: bool = False):
        return capi.dcs_ctx_timing(self.ctx, reset)

    def close(self) -> None:
        self.clear_chunks()
        if self.ctx:
            capi.dcs_ctx_destroy(self.ctx)
            self.ctx = 0


class State:
    """Branch slots of one circuit size in a caller-owned device buffer."""

    def __init__(self, eng: Engine, precision: str, n_qubits: int, capacity: int, chi_max: int,
                 mpo_bond_max: int = 4, init_chis: Sequence[int] = (), init_seed: int = 7,
                 gaussians=None):
        self.eng, self.n, self.capacity, self.chi_max = eng, n_qubits, capacity, chi_max
        self.wmax = mpo_bond_max
        self.precision = PRECISIONS[precision]
        chis = sorted(set(init_chis)) or [chi_max]
        nbytes = capi.dcs_state_bytes(self.precision, n_qubits, capacity, chi_max, mpo_bond_max,
                                      len(chis))
        self.nbytes = nbytes
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=f"cuda:{eng.device}")
        ptr = self.buf.data_ptr()
        self.ptr = (ptr + 255) // 256 * 256
        self.h = capi.dcs_state_create(eng.ctx, self.precision, n_qubits, capacity, chi_max,
                                       mpo_bond_max, len(chis), self.ptr, nbytes, eng.stream())
        if gaussians is None:
            from inputs.randomness import bra_init_gaussians
            gaussians = lambda chi: bra_init_gaussians(n_qubits, chi, init_seed)  # noqa: E731
        for chi in chis:
            g = gaussians(chi)
            flat = np.concatenate([np.ascontiguousarray(a).reshape(-1) for a in g])
            capi.dcs_state_set_init(self.h, chi, flat, eng.stream())
        self.free = list(range(capacity - 1, -1, -1))

    def warm_start(self, eta: Optional[float]) -> None:
        """Starting guess of later compression steps: None the generic guess,
        else the ket plus eta times the generic guess (dcs_state_set_warm_start)."""
        capi.dcs_state_set_warm_start(self.h, eta is not None, 0.0 if eta is None else eta)

    def alloc(self, k: int = 1) -> List[int]:
        if len(self.free) < k:
            raise capi.DcsError(capi.DCS_ECAPACITY, "no free branch slot")
        return [self.free.pop() for _ in range(k)]

    def release(self, ids: Sequence[int]) -> None:
        if len(ids):
            capi.dcs_branch_release(self.h, ids)
            self.free.extend(int(i) for i in ids)

    def reset(self) -> None:
        capi.dcs_branch_release(self.h, list(range(self.capacity)))
        self.free = list(range(self.capacity - 1, -1, -1))

    def export(self, bid: int):
        return capi.dcs_export_mps(self.h, bid, self.n, self.chi_max, self.eng.stream())

    # operations the drivers use (TreeState provides the same ones)
    bond_rule = True            # chunks close before the MPS operator bond passes wmax

    def chunk(self, circ: Circuit, op_ids: Sequence[int]) -> int:
        return self.eng.chunk(circ, op_ids)

    def init_zero(self, ids, chis) -> None:
        capi.dcs_branch_init_zero(self.h, ids, chis, self.eng.stream())

    def set_chi(self, ids, chis) -> None:
        capi.dcs_branch_set_chi(self.h, ids, chis)

    def compress(self, ids, chunks, n_sweeps: int) -> np.ndarray:
        return capi.dcs_compress_step(self.h, ids, chunks, n_sweeps, self.eng.stream())

    def measure(self, ids, qubits) -> np.ndarray:
        return capi.dcs_measure_prob(self.h, ids, qubits, self.eng.stream())

    def collapse(self, src, qubits, outcomes, dst, eps: float) -> np.ndarray:
        return capi.dcs_collapse(self.h, src, qubits, outcomes, dst, eps, self.eng.stream())

    def close(self) -> None:
        if self.h:
            capi.dcs_state_destroy(self.h)
            self.h = 0
            self.buf = None


class TreeTopology:
    """Node numbering and shapes of a regular tree (levels n_0 = 1, ..., n_L =
    n), as the library lays them out (dcs_tree_* in include/dcs.h): nodes in
    layer order, leaves holding consecutive qubits, node legs [edge above,
    children's edges or physical legs]."""

    def __init__(self, levels: Sequence[int]):
        self.levels = [int(x) for x in levels]
        self.n, self.L = self.levels[-1], len(self.levels) - 1
        self.kids: List[List[int]] = []
        self.qn: List[int] = []
        off = [sum(self.levels[:l]) for l in range(self.L)]
        for l in range(self.L):
            for i in range(self.levels[l]):
                self.qn.append(self.n // self.levels[l])
                if l + 1 < self.L:
                    dk = self.levels[l + 1] // self.levels[l]
                    self.kids.append([off[l + 1] + dk * i + c for c in range(dk)])
                else:
                    self.kids.append([])
        self.N = len(self.kids)
        self.d = self.levels[-1] // self.levels[-2]

    def edges(self, chi: int) -> List[int]:
        return [1 if v == 0 else min(chi, 2 ** self.qn[v], 2 ** (self.n - self.qn[v]))
                for v in range(self.N)]

    def shapes(self, e: Sequence[int]) -> List[tuple]:
        return [(e[v], *([e[c] for c in self.kids[v]] if self.kids[v] else [2] * self.d))
                for v in range(self.N)]


class TreeState:
    """Branch slots of a tree tensor network in a caller-owned device buffer
    (dcs_tree_* calls); the drivers below run on it as on an MPS State.
    Scratch for the contraction intermediates is sized from the circuit: the
    largest need of any run of unitaries between measurements (every
    controlled gate included) compressed into any of the bond caps."""

    bond_rule = False

    def __init__(self, eng: Engine, precision: str, levels: Sequence[int], capacity: int,
                 chi_max: int, mpo_bond_max: int = 16, init_chis: Sequence[int] = (),
                 init_seed: int = 7, circ: Optional[Circuit] = None, scratch_elems: int = 0):
        if precision not in ("c128", "c64"):
            raise ValueError("trees run in complex128 or complex64")
        self.eng, self.capacity, self.chi_max = eng, capacity, chi_max
        self.topo = TreeTopology(levels)
        self.levels, self.n, self.wmax = self.topo.levels, self.topo.n, mpo_bond_max
        self.precision = PRECISIONS[precision]
        self._chunks: Dict[tuple, tuple] = {}
        chis = sorted(set(init_chis)) or [chi_max]
        if circ is not None:
            for seg in _segments(circ):
                h = self.chunk(circ, seg)
                for c in chis:
                    scratch_elems = max(scratch_elems,
                                        capi.dcs_tree_chunk_scratch(h, c, chi_max))
        scratch_elems = max(int(scratch_elems), 1)
        self.scratch_elems = scratch_elems
        nbytes = capi.dcs_tree_state_bytes(self.precision, self.levels, capacity, chi_max,
                                           mpo_bond_max, scratch_elems, len(chis))
        self.nbytes = nbytes
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=f"cuda:{eng.device}")
        self.ptr = (self.buf.data_ptr() + 255) // 256 * 256
        self.h = capi.dcs_tree_create(eng.ctx, self.precision, self.levels, capacity, chi_max,
                                      mpo_bond_max, scratch_elems, len(chis), self.ptr, nbytes,
                                      eng.stream())
        from inputs.randomness import gaussians_for_shapes
        for chi in chis:
            g = gaussians_for_shapes(self.topo.shapes(self.topo.edges(chi)), init_seed, 0x7EE)
            flat = np.concatenate([np.ascontiguousarray(a).reshape(-1) for a in g])
            capi.dcs_tree_set_init(self.h, chi, flat, eng.stream())
        self.free = list(range(capacity - 1, -1, -1))

    def alloc(self, k: int = 1) -> List[int]:
        if len(self.free) < k:
            raise capi.DcsError(capi.DCS_ECAPACITY, "no free branch slot")
        return [self.free.pop() for _ in range(k)]

    def release(self, ids: Sequence[int]) -> None:
        if len(ids):
            capi.dcs_tree_branch_release(self.h, ids)
            self.free.extend(int(i) for i in ids)

    def reset(self) -> None:
        capi.dcs_tree_branch_release(self.h, list(range(self.capacity)))
        self.free = list(range(self.capacity - 1, -1, -1))

    def export(self, bid: int):
        cap = sum(int(np.prod(s)) for s in self.topo.shapes(self.topo.edges(self.chi_max)))
        return capi.dcs_tree_export(self.h, bid, self.topo.shapes, self.topo.N, cap,
                                    self.eng.stream())

    def chunk(self, circ: Circuit, op_ids: Sequence[int]) -> int:
        key = (id(circ), tuple(op_ids))
        hit = self._chunks.get(key)
        if hit is not None and hit[0] is circ:
            return hit[1]
        q0, q1, mats = [], [], []
        for i in op_ids:
            g = _gate_of(circ.ops[i])
            q0.append(g.qubits[0])
            q1.append(g.qubits[1] if len(g.qubits) == 2 else -1)
            mats.append(np.asarray(g.mat, dtype=np.complex128).reshape(-1))
        h = capi.dcs_tree_chunk_compile(self.eng.ctx, self.levels, q0, q1,
                                        np.concatenate(mats) if mats else np.zeros(0, complex))
        if hit is not None:
            capi.dcs_tchunk_destroy(hit[1])
        self._chunks[key] = (circ, h)
        return h

    def init_zero(self, ids, chis) -> None:
        capi.dcs_tree_branch_init_zero(self.h, ids, chis, self.eng.stream())

    def set_chi(self, ids, chis) -> None:
        capi.dcs_tree_branch_set_chi(self.h, ids, chis)

    def compress(self, ids, chunks, n_sweeps: int) -> np.ndarray:
        return capi.dcs_tree_compress_step(self.h, ids, chunks, n_sweeps, self.eng.stream())

    def measure(self, ids, qubits) -> np.ndarray:
        return capi.dcs_tree_measure_prob(self.h, ids, qubits, self.eng.stream())

    def collapse(self, src, qubits, outcomes, dst, eps: float) -> np.ndarray:
        return capi.dcs_tree_collapse(self.h, src, qubits, outcomes, dst, eps, self.eng.stream())

    def close(self) -> None:
        for _, h in self._chunks.values():
            capi.dcs_tchunk_destroy(h)
        self._chunks.clear()
        if self.h:
            capi.dcs_tree_destroy(self.h)
            self.h = 0
            self.buf = None


def _segments(circ: Circuit) -> List[List[int]]:
    """Operation indices of every maximal run of unitaries (gates and
    controlled gates) between measurements."""
    out, cur = [], []
    for li, op in enumerate(circ.ops):
        if isinstance(op, Measure):
            if cur:
                out.append(cur)
            cur = []
        else:
            cur.append(li)
    if cur:
        out.append(cur)
    return out


def _bond_rule_active(eng: Engine, circ: Circuit, wmax: int) -> bool:
    """False when no chunk of the circuit can have an operator bond above
    wmax: every run of unitaries between measurements, all its controlled
    gates included, stays within it.  Then the per-gate bond bookkeeping
    below is skipped.  A gate whose own rank exceeds wmax raises."""
    w = np.ones(circ.n_qubits + 1, dtype=np.int64)
    active = False
    for li, op in enumerate(circ.ops):
        if isinstance(op, Measure):
            w[:] = 1
            continue
        sp = eng.span(circ, li)
        if sp is None:
            continue
        lo, hi, r = sp
        if r > wmax:
            raise ValueError(f"gate {li} has operator rank {r} > mpo_bond_max {wmax}")
        w[lo + 1:hi + 1] *= r
        active = active or int(w.max()) > wmax
    return active


class _Bonds:
    """Operator bonds of the open chunks of a set of runs, entry j + 1 the
    bond between qubits j and j + 1: the product of the ranks of the gates
    spanning it (as dcs_chunk_compile builds it).  A gate that would push a
    bond of a non-empty chunk past the state's mpo_bond_max closes that chunk
    first."""

    def __init__(self, eng: Engine, circ: Circuit, wmax: int, runs: int):
        self.eng, self.circ, self.wmax = eng, circ, wmax
        self.w = np.ones((runs, circ.n_qubits + 1), dtype=np.int64)

    def closes(self, li: int, rows: np.ndarray, nonempty: np.ndarray) -> np.ndarray:
        """Rows (of `rows`) whose open chunk must be compressed before li."""
        sp = self.eng.span(self.circ, li)
        if sp is None or len(rows) == 0:
            return rows[:0]
        lo, hi, r = sp
        over = self.w[rows, lo + 1:hi + 1].max(axis=1) * r > self.wmax
        return rows[over & nonempty]

    def add(self, li: int, rows: np.ndarray) -> None:
        sp = self.eng.span(self.circ, li)
        if sp is not None:
            self.w[rows, sp[0] + 1:sp[1] + 1] *= sp[2]

    def reset(self, rows) -> None:
        self.w[rows] = 1


def run_single_path(eng: Engine, st: State, circ: Circuit, shots: int, chi: int, k: int,
                    n_sweeps: int = 2, uniforms: Optional[np.ndarray] = None,
                    outcomes: Optional[np.ndarray] = None, device_sampling: bool = False,
                    chi_ladder: Optional[Sequence[int]] = None, f_target: float = 0.0) -> Dict:
    """Alg. 1 for `shots` independent trajectories advanced in lockstep.

    Outcome of measurement i of shot s: outcomes[s, i] when given (replay),
    else 0 if uniforms[s, i] < p_0 and 1 otherwise.  Chunks of all shots that
    are due at the same operation are compressed in one batched call.  With
    device_sampling the draw and the collapse happen on the GPU
    (dcs_measure_sample_collapse); only the outcomes come back, for the
    classical register (p_0 is then not reported: NaN).

    Adaptive bond cap: with `chi_ladder` (ascending, chi its first rung, every
    rung registered in the state), a run whose compression returns a partial
    fidelity below `f_target` compresses with the next rung from then on;
    "chis" lists each run's caps, one per compression."""
    stream = eng.stream()
    if chi_ladder is not None:
        chi_ladder = [int(c) for c in chi_ladder]
        if chi_ladder[0] != chi or any(a >= b for a, b in zip(chi_ladder, chi_ladder[1:])):
            raise ValueError("chi_ladder must ascend from chi")
    rung = np.zeros(shots, dtype=np.int64)
    chis: List[List[int]] = [[] for _ in range(shots)]
    if device_sampling:
        if uniforms is None:
            raise ValueError("device sampling draws from given uniforms")
        dev = torch.device("cuda", eng.device)
        u_dev = torch.tensor(np.ascontiguousarray(np.asarray(uniforms, dtype=np.float64).T),
                             device=dev)
        m_dev = torch.empty(u_dev.shape, dtype=torch.int32, device=dev)
        pm_dev = torch.empty(u_dev.shape, dtype=torch.float64, device=dev)
    if device_sampling and not st.bond_rule:
        raise ValueError("device sampling is an MPS option")
    rule = st.bond_rule and _bond_rule_active(eng, circ, st.wmax)   # raises before any slot is taken
    ids = np.array(st.alloc(shots), dtype=np.int32)
    st.init_zero(ids, np.full(shots, chi))
    regs = np.zeros((shots, max(circ.n_bits, 1)), dtype=np.int8)
    p = np.ones(shots)
    fid = np.ones(shots)
    chunk: List[List[int]] = [[] for _ in range(shots)]
    bonds = _Bonds(eng, circ, st.wmax, shots) if rule else None
    rec_out, rec_p0, rec_f = [], [], []
    i_meas = 0

    def compress(sel: np.ndarray) -> None:
        if len(sel) == 0:
            return
        hs = [st.chunk(circ, chunk[s]) for s in sel]
        f = st.compress(ids[sel], hs, n_sweeps)
        fid[sel] *= f
        f_all = np.full(shots, np.nan)
        f_all[sel] = f
        rec_f.append(f_all)
        if bonds is not None:
            bonds.reset(sel)
        for s in sel:
            chunk[s] = []
            chis[s].append(chi_ladder[rung[s]] if chi_ladder else chi)
        if chi_ladder is not None:
            up = [s for s, fv in zip(sel, f) if fv < f_target and rung[s] + 1 < len(chi_ladder)]
            if up:
                rung[up] += 1
                st.set_chi(ids[up], [chi_ladder[rung[s]] for s in up])

    try:
        for li, op in enumerate(circ.ops):
            if isinstance(op, Measure):
                compress(np.array([s for s in range(shots) if chunk[s]], dtype=np.int64))
                q = np.full(shots, op.qubit)
                if device_sampling:
                    capi.dcs_measure_sample_collapse(st.h, ids, q, u_dev[i_meas].data_ptr(),
                                                     EPS_BRANCH, m_dev[i_meas].data_ptr(),
                                                     pm_dev[i_meas].data_ptr(), stream)
                    m = m_dev[i_meas].cpu().numpy()
                    pm = pm_dev[i_meas].cpu().numpy()
                    if np.any(m < 0):
                        raise capi.DcsError(capi.DCS_ENUMERIC, "state norm vanished")
                    p0 = np.full(shots, np.nan)
                else:
                    p0 = st.measure(ids, q)
                    if outcomes is not None:
                        m = np.asarray(outcomes[:, i_meas], dtype=np.int32)
                    else:
                        m = (uniforms[:, i_meas] >= p0).astype(np.int32)
                    pm = st.collapse(ids, q, m, ids, EPS_BRANCH)
                p *= pm
                regs[:, op.bit] = m
                rec_out.append(m.copy())
                rec_p0.append(p0.copy())
                i_meas += 1
                continue
            if isinstance(op, CGate):
                active = np.nonzero(_cond_true(op.cond, regs))[0]
            else:
                active = np.arange(shots)
            if bonds is not None:
                nonempty = np.array([len(chunk[s]) > 0 for s in active], dtype=bool)
                compress(bonds.closes(li, active, nonempty))
                bonds.add(li, active)
            due = []
            for s in active:
                chunk[s].append(li)
                if len(chunk[s]) == k:
                    due.append(s)
            compress(np.array(due, dtype=np.int64))
        compress(np.array([s for s in range(shots) if chunk[s]], dtype=np.int64))
    except Exception:
        st.release(ids)
        raise
    return {"ids": ids, "F": fid, "p": p, "regs": regs,
            "outcomes": np.array(rec_out).T if rec_out else np.zeros((shots, 0), np.int32),
            "p0s": np.array(rec_p0).T if rec_p0 else np.zeros((shots, 0)),
            "fids": rec_f, "chis": chis}


def run_multi_path(eng: Engine, st: State, circ: Circuit, chi: int, k: int, n_sweeps: int = 2,
                   max_branches: Optional[int] = None, chi_of=None,
                   eps: float = EPS_BRANCH, chi_ladder: Optional[Sequence[int]] = None,
                   f_target: float = 0.0, prune: Optional[Sequence[float]] = None) -> Dict:
    """Alg. 2: every measurement splits each live branch into its outcomes with
    p_m > eps (m = 0 kept in place, m = 1 copied to a new slot); after the
    measurement at most `max_branches` branches with the largest p are kept,
    or, with `prune = (mass_tol, rel_min)`, the branches dcs_prune_adaptive
    keeps (at most `max_branches`, if given).
    `chi_of(path)` gives a new child's bond cap.  Chunks of all branches due
    at the same operation are compressed in one batched call.

    Adaptive bond cap: with `chi_ladder` (ascending from chi), a branch whose
    compression returns a partial fidelity below `f_target` moves one rung up
    for its later compressions, and its children start on its rung.  Each
    branch's "chi" is its current cap, "chis" the caps of the compressions
    on its path and "p0s" the p_0 of every measurement on its path (taken on
    its ancestor at that measurement).  If anything raises, every slot the run
    holds is released before the exception propagates."""
    if chi_ladder is not None:
        chi_ladder = [int(c) for c in chi_ladder]
        if chi_of is not None:
            raise ValueError("chi_ladder and chi_of are exclusive")
        if chi_ladder[0] != chi or any(a >= b for a, b in zip(chi_ladder, chi_ladder[1:])):
            raise ValueError("chi_ladder must ascend from chi")
    rule = st.bond_rule and _bond_rule_active(eng, circ, st.wmax)   # raises before any slot is taken
    first = st.alloc(1)[0]
    st.init_zero([first], [chi])
    new_bonds = (lambda: _Bonds(eng, circ, st.wmax, 1)) if rule else (lambda: None)  # noqa: E731
    one = np.zeros(1, dtype=np.int64)
    br = [{"id": first, "path": (), "p": 1.0, "c": np.zeros(max(circ.n_bits, 1), np.int8),
           "F": 1.0, "chunk": [], "rung": 0, "chi": chi, "chis": [], "p0s": [],
           "w": new_bonds()}]
    dropped = 0.0

    def compress(sel: List[dict]) -> None:
        if not sel:
            return
        hs = [st.chunk(circ, b["chunk"]) for b in sel]
        f = st.compress([b["id"] for b in sel], hs, n_sweeps)
        up = []
        for b, fv in zip(sel, f):
            b["F"] *= float(fv)
            b["chunk"] = []
            if b["w"] is not None:
                b["w"].reset(one)
            b["chis"].append(b["chi"])
            if chi_ladder and fv < f_target and b["rung"] + 1 < len(chi_ladder):
                b["rung"] += 1
                b["chi"] = chi_ladder[b["rung"]]
                up.append(b)
        if up:
            st.set_chi([b["id"] for b in up], [b["chi"] for b in up])

    # slots this run holds: the live branches plus children allocated before
    # they join them; all are released if anything below raises
    held = {first}

    def take() -> int:
        sid = st.alloc(1)[0]
        held.add(sid)
        return sid

    def let_go(sids) -> None:
        sids = [int(x) for x in sids]
        st.release(sids)
        held.difference_update(sids)

    try:
        for li, op in enumerate(circ.ops):
            if isinstance(op, Measure):
                compress([b for b in br if b["chunk"]])
                ids = [b["id"] for b in br]
                q = [op.qubit] * len(br)
                p0 = st.measure(ids, q)
                src, dst, outc, qq, kids = [], [], [], [], []
                for b, pz in zip(br, p0):
                    opts = [m for m, pm in ((0, pz), (1, 1.0 - pz)) if pm > eps]
                    for j, m in enumerate(opts):
                        did = b["id"] if j == 0 else take()
                        src.append(b["id"])
                        dst.append(did)
                        outc.append(m)
                        qq.append(op.qubit)
                        kids.append((b, m, did, float(pz)))
                pm = st.collapse(src, qq, outc, dst, eps)
                nxt = []
                for (b, m, did, pz), pmv in zip(kids, pm):
                    c = b["c"].copy()
                    c[op.bit] = m
                    nxt.append({"id": did, "path": b["path"] + (m,), "p": b["p"] * float(pmv),
                                "c": c, "F": b["F"], "chunk": [], "rung": b["rung"],
                                "chi": chi_of(b["path"] + (m,)) if chi_of else b["chi"],
                                "chis": list(b["chis"]), "p0s": b["p0s"] + [pz],
                                "w": new_bonds()})
                br = nxt
                if chi_of is not None:
                    st.set_chi([b["id"] for b in br], [b["chi"] for b in br])
                if prune is not None or (max_branches is not None and len(br) > max_branches):
                    if prune is not None:
                        keep, disc = capi.dcs_prune_adaptive([b["p"] for b in br],
                                                             max_branches or len(br),
                                                             prune[0], prune[1])
                    else:
                        keep, disc = capi.dcs_topk_by_weight([b["p"] for b in br],
                                                             max_branches)
                    dropped += disc
                    kept = set(int(i) for i in keep)
                    let_go([b["id"] for i, b in enumerate(br) if i not in kept])
                    br = [br[int(i)] for i in keep]
                continue
            act = [b for b in br
                   if not (isinstance(op, CGate) and not _cond_true(op.cond, b["c"][None, :])[0])]
            if rule:
                compress([b for b in act
                          if len(b["w"].closes(li, one, np.array([bool(b["chunk"])])))])
            due = []
            for b in act:
                b["chunk"].append(li)
                if rule:
                    b["w"].add(li, one)
                if len(b["chunk"]) == k:
                    due.append(b)
            compress(due)
        compress([b for b in br if b["chunk"]])
    except BaseException:
        let_go(sorted(held))
        raise
    ptot = sum(b["p"] for b in br)
    fmp = sum(b["p"] * b["F"] for b in br) / ptot if ptot > 0 else float("nan")
    return {"branches": br, "dropped": dropped, "F_mp": fmp}
