"""FP64 MPS reference of the compression step and the dynamic operations.

Oracle -- test infrastructure only (see the package docstring).

State (Sec. III-B, MPS paragraph): site tensors A_j of shape
(chi_j, 2, chi_{j+1}), index order [left bond, physical, right bond], with
fixed padded bond dimensions chi_b = min(chi, 2^b, 2^(n-b)).

Compression step (Sec. III-C, Defs. "Unitary chunk" / "Compression step"):
the chunk is written as one layered operator per site (gates as local tensor
operators); the target U_chunk |psi~> is never formed; the new state is
optimised one site tensor at a time with all others fixed: the environment
F (everything but the optimised tensor contracted) gives the optimum
T = F / sqrt(<F|F>); a fixed number s of sweeps; the partial fidelity of the
chunk is |<psi~'| U |psi~>|^2.

Readings taken where the paper is silent:
  * single-site updates with the bond dimensions held at chi_b (zero padded);
  * the starting guess is a generic right-canonical MPS built from seeded
    Gaussians, the same for every chunk;
  * sweeps alternate left-to-right / right-to-left starting left-to-right;
    the orthogonality centre moves by QR (LQ) of the normalised site tensor;
    the turning site is not optimised twice; the last update of the last
    sweep keeps T as the centre and gives f = <F|F>, the squared overlap,
    since every other site tensor is then an isometry;
  * gate splitting: each two-qubit gate is split by an SVD across its two
    qubits (singular values above 1e-14 of the largest kept); one-qubit gates
    become single-site operators; gates are placed in ASAP layers and the
    layers multiplied site by site.

Measurement (Sec. IV-B1): n_m = <psi|P_m|psi> by contracting the network with
the projector on the measured leg, p_m = n_m / (n_0 + n_1); collapse projects
the local tensor and rescales it by 1/sqrt(n_m).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

SPLIT_CUTOFF = 1e-14


def bond_dims(n: int, chi: int) -> List[int]:
    return [min(chi, 2 ** b, 2 ** (n - b)) for b in range(n + 1)]


def zero_state(n: int, chi: int) -> List[np.ndarray]:
    """|0...0> as an MPS with padded bonds: A_j[0, 0, 0] = 1, zeros elsewhere."""
    d = bond_dims(n, chi)
    out = []
    for j in range(n):
        a = np.zeros((d[j], 2, d[j + 1]), dtype=np.complex128)
        a[0, 0, 0] = 1.0
        out.append(a)
    return out


def dims_of(mps: Sequence[np.ndarray]) -> List[int]:
    return [mps[0].shape[0]] + [a.shape[2] for a in mps]


# ---------------------------------------------------------------------------
# QR / LQ (Householder, LAPACK convention, through numpy)

def qr_q(t: np.ndarray) -> np.ndarray:
    """Thin Q of the QR factorisation of a tall or square matrix."""
    q, _ = np.linalg.qr(t, mode="reduced")
    return q


def lq_q(t: np.ndarray) -> np.ndarray:
    """Q with orthonormal rows of the LQ factorisation T = L Q (wide or
    square T), computed as the conjugate transpose of QR(T^H)."""
    q, _ = np.linalg.qr(t.conj().T, mode="reduced")
    return q.conj().T


# ---------------------------------------------------------------------------
# Starting guess of the compression step

def generic_bra(gauss: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Right-canonical generic MPS from Gaussian tensors G_j: for j >= 1 the
    site tensor is the orthonormal-row factor of LQ(G_j as chi_j x 2chi_{j+1});
    site 0 is G_0 normalised (it is optimised before it is ever read)."""
    out = []
    for j, g in enumerate(gauss):
        dl, _, dr = g.shape
        if j == 0:
            out.append(g / np.linalg.norm(g))
        else:
            out.append(lq_q(g.reshape(dl, 2 * dr)).reshape(dl, 2, dr))
    return out


def warm_bra(ket: Sequence[np.ndarray], generic: Sequence[np.ndarray],
             eta: float) -> List[np.ndarray]:
    """Warm-start guess (a reading: the paper does not fix the starting state
    of the variational compression): M_j = the ket's site embedded in the
    bond dims of ``generic`` (zero outside the ket's block) plus eta times
    the generic site, then, from the right, M_j = L_j Q_j by LQ, B_j = Q_j and
    L_j absorbed into M_{j-1}; site 0 keeps what is left.  The result
    represents the same state as the MPS M, with every site but 0
    right-canonical."""
    n = len(generic)
    m = []
    for j in range(n):
        dl, _, dr = generic[j].shape
        kl, _, kr = ket[j].shape
        if kl > dl or kr > dr:
            raise ValueError("ket bond wider than the starting guess")
        t = eta * np.asarray(generic[j], dtype=np.complex128)
        t[:kl, :, :kr] += ket[j]
        m.append(t)
    for j in range(n - 1, 0, -1):
        dl, _, dr = m[j].shape
        mj = m[j].reshape(dl, 2 * dr)
        q = lq_q(mj)
        lf = mj @ q.conj().T
        m[j] = q.reshape(dl, 2, dr)
        m[j - 1] = np.einsum("asb,bc->asc", m[j - 1], lf)
    return m


# ---------------------------------------------------------------------------
# Chunk -> one layered operator per site

def split_two_qubit(mat: np.ndarray, cutoff: float = SPLIT_CUTOFF) -> Tuple[np.ndarray, np.ndarray]:
    """Operator-Schmidt split of a 4x4 gate on (q, q+1).

    G[(s s'), (t t')] with s, t of qubit q is regrouped as M[(s t), (s' t')]
    and factored by SVD, M = U S V^H.  Returns W_q of shape (1, 2, 2, r) with
    W_q[0, s, t, w] = (U S)[(s t), w] and W_{q+1} of shape (r, 2, 2, 1) with
    W_{q+1}[w, s', t', 0] = V^H[w, (s' t')]."""
    g = mat.reshape(2, 2, 2, 2)                      # [s, s', t, t']
    m = g.transpose(0, 2, 1, 3).reshape(4, 4)        # [(s t), (s' t')]
    u, sv, vh = np.linalg.svd(m)
    r = int(np.sum(sv > cutoff * sv[0]))
    left = (u[:, :r] * sv[:r]).reshape(1, 2, 2, r)
    right = vh[:r, :].reshape(r, 2, 2, 1)
    return left, right


SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)


def route_swaps(ops: Sequence[Tuple[Tuple[int, ...], np.ndarray]]) -> List:
    """Nearest-neighbour form of a gate list by SWAP routing: a gate on
    (q0, q1) that is not (q, q+1) becomes the SWAPs (j, j+1) that carry the
    content of qubit q1 (if q1 > q0) or of qubit q0 (if q0 > q1) next to the
    other qubit, the gate on the adjacent pair in the order of its own
    qubits, and the same SWAPs undone in reverse order."""
    out = []
    for qubits, mat in ops:
        if len(qubits) == 1 or qubits[1] == qubits[0] + 1:
            out.append((tuple(qubits), mat))
            continue
        a, b = qubits
        if a < b:          # move q1 from b down to a + 1
            swaps = [(j, j + 1) for j in range(b - 1, a, -1)]
            pair = (a, a + 1)
        else:              # move q0 from a down to b; q1 then sits at b + 1
            swaps = [(j, j + 1) for j in range(a - 1, b - 1, -1)]
            pair = (b, b + 1)
        out.extend((sw, SWAP) for sw in swaps)
        out.append((pair, mat))
        out.extend((sw, SWAP) for sw in reversed(swaps))
    return out


def gate_rank(mat: np.ndarray, cutoff: float = SPLIT_CUTOFF) -> int:
    """Operator-Schmidt rank of a 4x4 gate: the number of singular values of
    its regrouped matrix (as in split_two_qubit) above cutoff times the
    largest."""
    return split_two_qubit(np.asarray(mat, dtype=np.complex128), cutoff)[0].shape[3]


def span_bonds(n: int, ops: Sequence[Tuple[Tuple[int, ...], np.ndarray]]) -> np.ndarray:
    """Operator bond of a chunk with non-adjacent gates carried exactly across
    the sites they span: entry j + 1, the bond between qubits j and j+1, is
    the product of the operator-Schmidt ranks of the two-qubit gates whose
    qubits lie on both sides of it.  Entries 0 and n are 1."""
    w = np.ones(n + 1, dtype=np.int64)
    for qubits, mat in ops:
        if len(qubits) == 2:
            lo, hi = min(qubits), max(qubits)
            w[lo + 1:hi + 1] *= gate_rank(mat)
    return w


def asap_layers(ops: Sequence[Tuple[Tuple[int, ...], np.ndarray]]) -> List[List]:
    """Place each gate in the first layer after the last layer that touches
    any of its qubits (time order preserved per qubit)."""
    last = {}
    layers: List[List] = []
    for qubits, mat in ops:
        lay = 1 + max((last.get(q, -1) for q in qubits), default=-1)
        while len(layers) <= lay:
            layers.append([])
        layers[lay].append((qubits, mat))
        for q in qubits:
            last[q] = lay
    return layers


def chunk_mpo(n: int, ops: Sequence[Tuple[Tuple[int, ...], np.ndarray]]) -> List[np.ndarray]:
    """Layered operator of a chunk: W_j[w_l, s(out), t(in), w_r] per site.

    Gates on non-adjacent or reversed pairs are first SWAP-routed to
    nearest-neighbour gates (route_swaps).  Each layer gives one operator per
    site (identity where no gate acts); the
    per-site operators of successive layers are multiplied in time order, the
    combined bond index being (earlier layer, later layer) with the earlier
    layer most significant."""
    ident = np.eye(2, dtype=np.complex128).reshape(1, 2, 2, 1)
    total = [ident.copy() for _ in range(n)]
    for layer in asap_layers(route_swaps(ops)):
        site_ops = [ident for _ in range(n)]
        for qubits, mat in layer:
            if len(qubits) == 1:
                site_ops[qubits[0]] = np.asarray(mat, dtype=np.complex128).reshape(1, 2, 2, 1)
            else:
                lft, rgt = split_two_qubit(np.asarray(mat, dtype=np.complex128))
                site_ops[qubits[0]] = lft
                site_ops[qubits[0] + 1] = rgt
        for j in range(n):
            a, b = total[j], site_ops[j]                 # a acts first, then b
            c = np.einsum("wsuv,xuty->wxstvy", b, a)     # b[w,s,u,v] a[x,u,t,y]
            # combined index order: earlier (a) most significant -> (x, w)
            c = c.transpose(1, 0, 2, 3, 5, 4)            # [x, w, s, t, y, v]
            wl = a.shape[0] * b.shape[0]
            wr = a.shape[3] * b.shape[3]
            total[j] = np.ascontiguousarray(c.reshape(wl, 2, 2, wr))
    return total


# ---------------------------------------------------------------------------
# Environments and the local optimisation

def site_tensor(lenv, ket, w, renv) -> np.ndarray:
    """F[a, s, c] = sum L[a,w,x] K[x,t,y] W[w,s,t,v] R[c,v,y]."""
    x = np.einsum("awx,xty->awty", lenv, ket, optimize=True)
    x = np.einsum("awty,wstv->asvy", x, w, optimize=True)
    return np.einsum("asvy,cvy->asc", x, renv, optimize=True)


def left_env_step(lenv, bra, ket, w) -> np.ndarray:
    """L'[c, v, y] = sum conj(B[a,s,c]) L[a,w,x] K[x,t,y] W[w,s,t,v]."""
    x = np.einsum("awx,xty->awty", lenv, ket, optimize=True)
    x = np.einsum("awty,wstv->asvy", x, w, optimize=True)
    return np.einsum("asc,asvy->cvy", bra.conj(), x, optimize=True)


def right_env_step(renv, bra, ket, w) -> np.ndarray:
    """R'[a, w, x] = sum conj(B[a,s,c]) K[x,t,y] W[w,s,t,v] R[c,v,y]."""
    x = np.einsum("xty,cvy->xtcv", ket, renv, optimize=True)
    x = np.einsum("xtcv,wstv->xwsc", x, w, optimize=True)
    return np.einsum("asc,xwsc->awx", bra.conj(), x, optimize=True)


def sweep_visits(n: int, n_sweeps: int) -> List[int]:
    """Site order of s sweeps: odd sweeps run left to right (sites 0..n-1 for
    the first, 1..n-1 afterwards), even sweeps right to left (n-2..0)."""
    visits: List[int] = []
    for t in range(1, n_sweeps + 1):
        if t % 2 == 1:
            visits.extend(range(0 if t == 1 else 1, n))
        else:
            visits.extend(range(n - 2, -1, -1))
    return visits


def compress(ket: Sequence[np.ndarray], mpo: Sequence[np.ndarray],
             bra_init: Sequence[np.ndarray], n_sweeps: int):
    """One compression step: returns (new MPS, partial fidelity f, centre).

    The new state has the bond dimensions of ``bra_init``; ``ket`` may have
    other bond dimensions.  Environments: L_0 = R_n = [[1]]; the right
    environments of the starting guess are built first; at each visited site
    F is formed, T = F/|F|; if another visit follows on the right, T is
    QR-factored and its Q becomes the site tensor and extends the left
    environment; if the next visit is on the left, LQ and the right
    environment; at the final visit T itself is kept and f = |F|^2."""
    n = len(ket)
    if n_sweeps < 1:
        raise ValueError("at least one sweep")
    bra = [b.copy() for b in bra_init]
    env: List[np.ndarray] = [None] * (n + 1)
    env[0] = np.ones((1, 1, 1), dtype=np.complex128)
    env[n] = np.ones((1, 1, 1), dtype=np.complex128)
    for j in range(n - 1, 0, -1):
        env[j] = right_env_step(env[j + 1], bra[j], ket[j], mpo[j])
    visits = sweep_visits(n, n_sweeps)
    f = None
    centre = None
    for i, j in enumerate(visits):
        f_site = site_tensor(env[j], ket[j], mpo[j], env[j + 1])
        nu = np.linalg.norm(f_site)
        if nu == 0.0:
            raise FloatingPointError("environment tensor vanished")
        t = f_site / nu
        dl, _, dr = t.shape
        if i == len(visits) - 1:
            bra[j] = t
            f = float(nu * nu)
            centre = j
            break
        nxt = visits[i + 1]
        if nxt == j + 1:
            bra[j] = qr_q(t.reshape(dl * 2, dr)).reshape(dl, 2, dr)
            env[j + 1] = left_env_step(env[j], bra[j], ket[j], mpo[j])
        elif nxt == j - 1:
            bra[j] = lq_q(t.reshape(dl, 2 * dr)).reshape(dl, 2, dr)
            env[j] = right_env_step(env[j + 1], bra[j], ket[j], mpo[j])
        else:
            raise AssertionError("visits must move by one site")
    return bra, f, centre


# ---------------------------------------------------------------------------
# Measurement and collapse

def outcome_norms(mps: Sequence[np.ndarray], q: int) -> Tuple[float, float]:
    """n_m = <psi|P_m^(q)|psi>, m = 0, 1, by contracting bra, projector and
    ket from left to right."""
    out = []
    for m in (0, 1):
        e = np.ones((1, 1), dtype=np.complex128)
        for j, a in enumerate(mps):
            if j == q:
                am = a[:, m, :]
                e = np.einsum("ab,ac,bd->cd", e, am.conj(), am, optimize=True)
            else:
                e = np.einsum("ab,asc,bsd->cd", e, a.conj(), a, optimize=True)
        out.append(float(e[0, 0].real))
    return out[0], out[1]


def collapse(mps: Sequence[np.ndarray], q: int, m: int, norm_m: float) -> List[np.ndarray]:
    """P_m applied to the physical leg of site q, rescaled by 1/sqrt(n_m)."""
    out = [a.copy() for a in mps]
    a = out[q]
    a[:, 1 - m, :] = 0.0
    a[:, m, :] /= np.sqrt(norm_m)
    return out


# ---------------------------------------------------------------------------
# Checks on small states

def overlap(a: Sequence[np.ndarray], b: Sequence[np.ndarray]) -> complex:
    """<a|b> by left-to-right transfer."""
    e = np.ones((1, 1), dtype=np.complex128)
    for x, y in zip(a, b):
        e = np.einsum("ab,asc,bsd->cd", e, x.conj(), y, optimize=True)
    return complex(e[0, 0])


def to_statevector(mps: Sequence[np.ndarray]) -> np.ndarray:
    """Contract the chain into the 2^n amplitude vector (qubit 0 most
    significant)."""
    v = mps[0][0]                                   # (2, chi_1), chi_0 = 1
    for a in mps[1:]:
        v = np.einsum("pa,asb->psb", v, a, optimize=True).reshape(-1, a.shape[2])
    return v[:, 0].copy()


def norm_sq(mps: Sequence[np.ndarray]) -> float:
    return float(overlap(mps, mps).real)
