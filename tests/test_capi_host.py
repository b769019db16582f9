"""Host-side checks of the C ABI (no GPU): the library loads and exports every
function the header declares; host-only entry points and their error paths."""
import os
import re

import numpy as np
import pytest

from inputs import circuits as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dcs.h")
HEADER_TESTING = os.path.join(ROOT, "include", "dcs_testing.h")


def _declared(path=HEADER):
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dcs_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_and_library_exports():
    capi = pytest.importorskip("paper_2609_26516_amd.capi")
    import ctypes
    lib = ctypes.CDLL(capi.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(capi.EXPORTED) == names
    tnames = _declared(HEADER_TESTING)
    for name in tnames:
        assert hasattr(lib, name), name
    assert sorted(capi.EXPORTED_TESTING) == tnames


def test_version():
    from paper_2609_26516_amd import capi
    assert capi.dcs_version() >= 100


def test_topk_by_weight():
    from paper_2609_26516_amd import capi
    keep, disc = capi.dcs_topk_by_weight([0.1, 0.3, 0.3, 0.05, 0.25], 3)
    assert list(keep) == [1, 2, 4] and abs(disc - 0.15) < 1e-15
    keep, disc = capi.dcs_topk_by_weight([0.2] * 5, 2)
    assert list(keep) == [0, 1] and abs(disc - 0.6) < 1e-15
    keep, disc = capi.dcs_topk_by_weight([0.5, 0.5], 8)
    assert list(keep) == [0, 1] and disc == 0.0
    keep, disc = capi.dcs_topk_by_weight([], 3)
    assert len(keep) == 0 and disc == 0.0


def test_topk_matches_stable_sort_random():
    from paper_2609_26516_amd import capi
    rng = np.random.default_rng(0)
    for _ in range(50):
        w = rng.integers(0, 6, size=rng.integers(1, 40)).astype(float) / 8
        k = int(rng.integers(0, 45))
        keep, disc = capi.dcs_topk_by_weight(w, k)
        order = sorted(range(len(w)), key=lambda i: -w[i])
        assert list(keep) == order[:k]
        assert abs(disc - sum(w[i] for i in order[k:])) < 1e-12


def test_chunk_compile_bonds_and_errors():
    from paper_2609_26516_amd import capi
    rng = np.random.default_rng(1)
    n = 6
    # two brickwork layers of Haar gates: every inner bond straddled once, rank 4
    ops = [(q, q + 1) for q in range(0, n - 1, 2)] + [(q, q + 1) for q in range(1, n - 1, 2)]
    mats = np.concatenate([C.haar_unitary(rng, 4).reshape(-1) for _ in ops])
    h = capi.dcs_chunk_compile(0, n, [a for a, _ in ops], [b for _, b in ops], mats)
    assert list(capi.dcs_chunk_bonds(h, n)) == [1, 4, 4, 4, 4, 4, 1]
    capi.dcs_chunk_destroy(h)
    # CNOT has operator-Schmidt rank 2; a product gate rank 1; 1q gates add nothing
    mats = np.concatenate([C.CNOT_01.reshape(-1), np.kron(C.H, C.X).reshape(-1),
                           C.X.reshape(-1)])
    h = capi.dcs_chunk_compile(0, 4, [0, 2, 1], [1, 3, -1], mats)
    assert list(capi.dcs_chunk_bonds(h, 4)) == [1, 2, 1, 1, 1]
    capi.dcs_chunk_destroy(h)
    # stacked gates on one bond multiply ranks
    mats = np.concatenate([C.CNOT_01.reshape(-1), C.CNOT_10.reshape(-1)])
    h = capi.dcs_chunk_compile(0, 3, [1, 1], [2, 2], mats)
    assert list(capi.dcs_chunk_bonds(h, 3)) == [1, 1, 4, 1]
    capi.dcs_chunk_destroy(h)
    with pytest.raises(capi.DcsError) as e:
        capi.dcs_chunk_compile(0, 4, [2], [2], C.CNOT_01.reshape(-1))
    assert e.value.code == capi.DCS_EQUBITS == capi.DCS_ENONLOCAL
    # a distant pair spans its bonds: CNOT (0, 2) and reversed CNOT (3, 1)
    mats = np.concatenate([C.CNOT_01.reshape(-1), C.CNOT_01.reshape(-1)])
    h = capi.dcs_chunk_compile(0, 4, [0, 3], [2, 1], mats)
    assert list(capi.dcs_chunk_bonds(h, 4)) == [1, 2, 4, 2, 1]
    capi.dcs_chunk_destroy(h)
    with pytest.raises(capi.DcsError) as e:
        capi.dcs_chunk_compile(0, 4, [4], [-1], C.X.reshape(-1))
    assert e.value.code == capi.DCS_EINVAL


def test_state_bytes_validation():
    from paper_2609_26516_amd import capi
    b64 = capi.dcs_state_bytes(capi.DCS_C64, 40, 8, 256, 4, 1)
    b128 = capi.dcs_state_bytes(capi.DCS_C128, 40, 8, 256, 4, 1)
    assert 1.5 < b128 / b64 < 2.1
    for bad in [(7, 4, 1, 8, 4, 1), (0, 0, 1, 8, 4, 1), (0, 4, 0, 8, 4, 1), (0, 4, 1, 2048, 4, 1),
                (0, 4, 1, 8, 32, 1), (0, 4, 1, 8, 4, 0)]:
        with pytest.raises(capi.DcsError) as e:
            capi.dcs_state_bytes(*bad)
        assert e.value.code == capi.DCS_EINVAL


def _op_matrix(mpo):
    t = mpo[0][0].reshape(2, 2, -1)
    d = 2
    for w in mpo[1:]:
        t = np.einsum("ijw,wstv->isjtv", t, w).reshape(d * 2, d * 2, -1)
        d *= 2
    return t[:, :, 0]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_long_range_chunk_operator(seed):
    """The compiled operator of a chunk with distant and reversed pairs is the
    product of the gates embedded entry by entry (statevector definition)."""
    from oracle import statevector as SV
    from paper_2609_26516_amd import capi
    rng = np.random.default_rng(seed)
    n = 5
    pairs = [(0, 4), (3, 1), (2, 3), (4, 2), (1, 0)]
    ops = [(p, C.haar_unitary(rng, 4)) for p in pairs[seed:seed + 3]]
    ops.insert(1, ((2,), C.haar_unitary(rng, 2)))
    full = np.eye(2 ** n, dtype=complex)
    for q, m in ops:
        full = SV.full_operator(n, q, m) @ full
    q0 = [q[0] for q, _ in ops]
    q1 = [q[1] if len(q) == 2 else -1 for q, _ in ops]
    h = capi.dcs_chunk_compile(0, n, q0, q1, np.concatenate([m.reshape(-1) for _, m in ops]))
    np.testing.assert_allclose(_op_matrix(capi.dcs_chunk_export(h, n)), full, atol=1e-12)
    capi.dcs_chunk_destroy(h)


def test_gate_rank():
    from paper_2609_26516_amd import capi
    rng = np.random.default_rng(5)
    assert capi.dcs_gate_rank(C.CNOT_01) == 2
    assert capi.dcs_gate_rank(C.CNOT_10) == 2
    assert capi.dcs_gate_rank(np.kron(C.H, C.X)) == 1
    assert capi.dcs_gate_rank(C.haar_unitary(rng, 4)) == 4
    swap = np.eye(4)[[0, 2, 1, 3]]
    assert capi.dcs_gate_rank(swap) == 4
    bad = C.CNOT_01.copy()
    bad[1, 1] = np.nan
    with pytest.raises(capi.DcsError):
        capi.dcs_gate_rank(bad)
    with pytest.raises(capi.DcsError) as e:
        capi.dcs_chunk_compile(0, 3, [0], [2], bad.reshape(-1))
    assert e.value.code == capi.DCS_EINVAL


def test_prune_adaptive_matches_oracle():
    """Kept indices and dropped mass bit-exact against the oracle's rule on
    random weights with ties."""
    from oracle import dynamic as D
    from paper_2609_26516_amd import capi
    rng = np.random.default_rng(9)
    for trial in range(300):
        n = int(rng.integers(0, 40))
        w = rng.choice([0.0, 0.25, 0.5], size=n) if trial % 3 == 0 else rng.random(n) ** 4
        k = int(rng.integers(1, 50))
        tol = float(rng.choice([0.0, 0.01, 0.1, 0.5]))
        rel = float(rng.choice([0.0, 0.001, 0.1, 1.0]))
        keep, d = capi.dcs_prune_adaptive(w, k, tol, rel)
        ref_keep, ref_d = D.prune_adaptive(list(w), k, tol, rel)
        assert list(keep) == ref_keep, (trial, n, k, tol, rel)
        assert d == ref_d
    for bad in [(1.0, 0.0), (-0.1, 0.0), (0.0, 1.5)]:
        with pytest.raises(capi.DcsError):
            capi.dcs_prune_adaptive([0.5, 0.5], 2, *bad)
    with pytest.raises(capi.DcsError):
        capi.dcs_prune_adaptive([0.5, -0.1], 2)
    with pytest.raises(capi.DcsError):
        capi.dcs_prune_adaptive([0.5], 0)


def test_library_makes_no_device_allocation():
    """Every device buffer the product library uses lies in the caller's state
    buffer: no hipMalloc / hipFree outside the kernel-test entry points."""
    import glob
    csrc = os.path.join(ROOT, "paper_2609_26516_amd", "csrc")
    for path in glob.glob(os.path.join(csrc, "*")):
        if os.path.basename(path) == "testing.cpp":
            continue
        txt = re.sub(r"//[^\n]*|/\*.*?\*/", "", open(path).read(), flags=re.S)
        for call in ("hipMalloc(", "hipFree(", "hipMallocAsync(", "hipExtMallocWithFlags("):
            assert call not in txt, (path, call)


def test_tree_topology_matches_the_oracle_numbering():
    """The driver's tree layout (node order, shapes for a bond cap) is the one
    the FP64 tree oracle uses, and the library counts the same nodes."""
    from oracle import ttn as OT
    from paper_2609_26516_amd import capi
    from paper_2609_26516_amd.engine import TreeTopology
    for levels in ([1, 2, 4], [1, 3, 9], [1, 2, 4, 8], [1, 3, 9, 27], [1, 2, 8]):
        tr, tp = OT.Tree(levels), TreeTopology(levels)
        assert tp.N == tr.n_nodes == capi.dcs_tree_n_nodes(levels)
        for chi in (1, 2, 4, 32, 1024):
            assert tp.shapes(tp.edges(chi)) == [tr.shape(v, chi) for v in range(tr.n_nodes)]


def test_tree_chunk_bonds_and_scratch():
    """Operator bond of every tree edge: the product of the operator-Schmidt
    ranks of the gates whose leaves lie on both sides of it; a gate inside one
    leaf adds none.  The contraction scratch grows with the bond caps."""
    from oracle import mps as OM
    from paper_2609_26516_amd import capi
    rng = np.random.default_rng(3)
    levels = [1, 3, 9]            # root 0, leaves 1, 2, 3 with qubits 0-2, 3-5, 6-8
    gates = [((2, 3), C.haar_unitary(rng, 4)),    # leaf 1 - leaf 2
             ((4, 5), C.haar_unitary(rng, 4)),    # inside leaf 2
             ((8, 0), C.CNOT_01),                 # leaf 3 - leaf 1, reversed order
             ((7,), C.H)]
    mats = np.concatenate([np.asarray(m, complex).reshape(-1) for _, m in gates])
    q0 = [g[0][0] for g in gates]
    q1 = [g[0][1] if len(g[0]) == 2 else -1 for g in gates]
    ch = capi.dcs_tree_chunk_compile(None, levels, q0, q1, mats)
    w = capi.dcs_tchunk_bonds(ch, 4)
    r0, r2 = OM.gate_rank(gates[0][1]), OM.gate_rank(gates[2][1])
    assert (r0, r2) == (4, 2)
    np.testing.assert_array_equal(w, [1, r0 * r2, r0, r2])
    s4 = capi.dcs_tree_chunk_scratch(ch, 4, 4)
    s8 = capi.dcs_tree_chunk_scratch(ch, 8, 8)
    assert 0 < s4 < s8
    capi.dcs_tchunk_destroy(ch)
    with pytest.raises(capi.DcsError) as e:
        capi.dcs_tree_chunk_compile(None, levels, [1], [1], np.eye(4, dtype=complex).reshape(-1))
    assert e.value.code == capi.DCS_EQUBITS
    with pytest.raises(capi.DcsError):
        capi.dcs_tree_n_nodes([1, 3, 8])
