"""Pins of the oracle's MPS compression step and dynamic operations against
brute force, closed forms and the Eckart-Young bound (no oracle formula is
re-typed here: each check uses an independent route to the same number)."""
import numpy as np
import pytest

from inputs import circuits as C
from inputs.randomness import bra_init_gaussians
from oracle import dynamic as D
from oracle import mps as M
from oracle import statevector as SV


def _random_chunk(rng, n, layers, one_qubit=True):
    ops = []
    for layer in range(layers):
        for q in range(layer % 2, n - 1, 2):
            ops.append(((q, q + 1), C.haar_unitary(rng, 4)))
        if one_qubit:
            q = int(rng.integers(n))
            ops.append(((q,), C.haar_unitary(rng, 2)))
    return ops


def _mpo_full_operator(mpo):
    """Contract the layered operator into a 2^n x 2^n matrix."""
    t = mpo[0][0]                                   # [s, t, w]
    out_dim = 2
    t = t.reshape(2, 2, -1)
    for w in mpo[1:]:
        t = np.einsum("ijw,wstv->isjtv", t, w).reshape(out_dim * 2, out_dim * 2, -1)
        out_dim *= 2
    return t[:, :, 0]


def test_split_ranks():
    rng = np.random.default_rng(1)
    assert M.split_two_qubit(C.haar_unitary(rng, 4))[0].shape[3] == 4
    assert M.split_two_qubit(C.CNOT_01)[0].shape[3] == 2
    assert M.split_two_qubit(np.kron(C.H, C.X))[0].shape[3] == 1


@pytest.mark.parametrize("layers", [1, 2, 3])
def test_chunk_operator_equals_gate_product(layers):
    rng = np.random.default_rng(10 + layers)
    n = 5
    ops = _random_chunk(rng, n, layers)
    full = np.eye(2 ** n, dtype=complex)
    for qubits, mat in ops:
        full = SV.full_operator(n, qubits, mat) @ full
    np.testing.assert_allclose(_mpo_full_operator(M.chunk_mpo(n, ops)), full, atol=1e-12)


def test_asap_layering_order():
    # a 1q gate between two 2q gates on the same qubit must stay between them
    g = np.eye(4)
    ops = [((0, 1), g), ((1,), np.eye(2)), ((1, 2), g), ((0,), np.eye(2))]
    lay = M.asap_layers(ops)
    assert [len(x) for x in lay] == [1, 2, 1]
    assert lay[1][0][0] == (1,) and lay[1][1][0] == (0,)


def test_generic_bra_is_right_canonical():
    b = M.generic_bra(bra_init_gaussians(9, 8, 3))
    for j in range(1, 9):
        a = b[j].reshape(b[j].shape[0], -1)
        np.testing.assert_allclose(a @ a.conj().T, np.eye(a.shape[0]), atol=1e-13)


def _exact_case(n, n_sweeps, seed):
    rng = np.random.default_rng(seed)
    chi = 2 ** (n // 2)
    circ_ops = _random_chunk(rng, n, 3)
    # a random normalised input MPS (exactly representable at this chi)
    psi0 = [rng.standard_normal(a.shape) + 1j * rng.standard_normal(a.shape)
            for a in M.zero_state(n, chi)]
    nrm = np.sqrt(M.norm_sq(psi0))
    psi0[0] = psi0[0] / nrm
    new, f, centre = M.compress(psi0, M.chunk_mpo(n, circ_ops), M.generic_bra(
        bra_init_gaussians(n, chi, seed)), n_sweeps)
    sv = M.to_statevector(psi0)
    for qubits, mat in circ_ops:
        sv = SV.apply_gate(sv, n, qubits, mat)
    return new, f, centre, sv


@pytest.mark.parametrize("n,n_sweeps", [(4, 1), (6, 1), (6, 2), (8, 2), (10, 2), (7, 3)])
def test_compress_exact_regime(n, n_sweeps):
    new, f, centre, sv = _exact_case(n, n_sweeps, seed=100 + n)
    v = M.to_statevector(new)
    assert abs(np.linalg.norm(v) - 1) < 1e-12
    assert abs(abs(np.vdot(sv, v)) ** 2 - 1) < 1e-12
    assert abs(f - 1) < 1e-12
    assert centre == (n - 1 if n_sweeps % 2 == 1 else 0)


def test_compress_gauge_after_sweeps():
    n = 8
    for s, expect in ((1, "left"), (2, "right")):
        new, f, centre, _ = _exact_case(n, s, seed=7)
        for j in range(n):
            if j == centre:
                continue
            a = new[j]
            if expect == "left":
                m = a.reshape(-1, a.shape[2])
                np.testing.assert_allclose(m.conj().T @ m, np.eye(m.shape[1]), atol=1e-12)
            else:
                m = a.reshape(a.shape[0], -1)
                np.testing.assert_allclose(m @ m.conj().T, np.eye(m.shape[0]), atol=1e-12)


@pytest.mark.parametrize("chi,s", [(2, 1), (4, 2), (3, 2), (4, 4)])
def test_truncated_fidelity_is_overlap(chi, s):
    """f equals |<psi~'|U|psi~>|^2 computed from contracted vectors."""
    n = 8
    rng = np.random.default_rng(chi * 10 + s)
    psi = M.zero_state(n, chi)
    ops0 = _random_chunk(rng, n, 2, one_qubit=False)
    sim_init = M.generic_bra(bra_init_gaussians(n, chi, 1))
    psi, _, _ = M.compress(psi, M.chunk_mpo(n, ops0), sim_init, 2)
    ops = _random_chunk(rng, n, 2)
    new, f, _ = M.compress(psi, M.chunk_mpo(n, ops), sim_init, s)
    target = M.to_statevector(psi)
    for qubits, mat in ops:
        target = SV.apply_gate(target, n, qubits, mat)
    v = M.to_statevector(new)
    assert abs(np.linalg.norm(v) - 1) < 1e-12
    assert abs(abs(np.vdot(v, target)) ** 2 - f) < 1e-12
    assert 0.0 < f <= 1.0 + 1e-12


def test_eckart_young_single_bond():
    """Truncation at one bond only: f never exceeds the sum of the kept squared
    Schmidt coefficients and reaches it when the sweeps converge."""
    n, chi = 4, 2
    rng = np.random.default_rng(42)
    start = [((0,), C.H), ((0, 1), C.CNOT_01), ((2,), C.H), ((2, 3), C.CNOT_01)]
    init = M.generic_bra(bra_init_gaussians(n, chi, 5))
    psi, f0, _ = M.compress(M.zero_state(n, chi), M.chunk_mpo(n, start), init, 2)
    assert abs(f0 - 1) < 1e-12
    gate = [((1, 2), C.haar_unitary(rng, 4))]
    target = M.to_statevector(psi)
    target = SV.apply_gate(target, n, (1, 2), gate[0][1])
    sv = np.linalg.svd(target.reshape(4, 4), compute_uv=False)
    bound = float(np.sum(sv[:chi] ** 2))
    assert bound < 1 - 1e-3                        # the gate really is truncated
    for s in (1, 2, 3):
        _, f, _ = M.compress(psi, M.chunk_mpo(n, gate), init, s)
        assert f <= bound + 1e-12
    prev = 0.0
    for s in (4, 8, 16):                           # monotone approach
        _, f, _ = M.compress(psi, M.chunk_mpo(n, gate), init, s)
        assert prev - 1e-14 <= f <= bound + 1e-12
        prev = f
    _, f40, _ = M.compress(psi, M.chunk_mpo(n, gate), init, 40)
    assert abs(f40 - bound) < 1e-12


def test_measure_and_collapse_match_statevector():
    n, chi = 7, 8
    rng = np.random.default_rng(9)
    psi = M.zero_state(n, chi)
    init = M.generic_bra(bra_init_gaussians(n, chi, 2))
    psi, _, _ = M.compress(psi, M.chunk_mpo(n, _random_chunk(rng, n, 3)), init, 2)
    sv = M.to_statevector(psi)
    for q in range(n):
        n0, n1 = M.outcome_norms(psi, q)
        s0, s1 = SV.outcome_norms(sv, n, q)
        assert abs(n0 - s0) < 1e-13 and abs(n1 - s1) < 1e-13
        for m, nm in ((0, n0), (1, n1)):
            post = M.to_statevector(M.collapse(psi, q, m, nm))
            np.testing.assert_allclose(post, SV.project(sv, n, q, m, nm), atol=1e-12)


def test_single_path_exact_regime_replays_statevector():
    circ, p = C.workload("cfg1_n10_chi16", n=8, depth=8, chi=16)
    sim = D.Simulator(8, 16, k=1000, n_sweeps=2, init_seed=7)
    u = np.random.default_rng(11).random(64)
    r = D.run_single_path(circ, sim, uniforms=u)
    ref = SV.replay(circ, r["outcomes"])
    assert abs(r["p"] - ref["p"]) < 1e-12
    np.testing.assert_allclose(r["pms"], ref["pms"], atol=1e-12)
    assert abs(r["F"] - 1) < 1e-11
    v = M.to_statevector(r["mps"])
    assert abs(abs(np.vdot(ref["psi"], v)) ** 2 - 1) < 1e-11


def test_single_path_chunking_with_small_k():
    """Chunk size 3 forces compressions in the middle of unitary segments; in
    the exact regime the result must not change."""
    circ, p = C.workload("cfg1_n10_chi16", n=6, depth=6, chi=8)
    u = np.random.default_rng(2).random(64)
    r1 = D.run_single_path(circ, D.Simulator(6, 8, k=1000), uniforms=u)
    r2 = D.run_single_path(circ, D.Simulator(6, 8, k=3), uniforms=u)
    assert r1["outcomes"] == r2["outcomes"]
    assert len(r2["fids"]) > len(r1["fids"])
    assert abs(abs(M.overlap(r1["mps"], r2["mps"])) ** 2 - 1) < 1e-11


def test_topk_stable_and_mass():
    keep, dropped = D.topk_by_weight([0.1, 0.3, 0.3, 0.05, 0.25], 3)
    assert keep == [1, 2, 4]
    assert abs(dropped - 0.15) < 1e-15
    keep, dropped = D.topk_by_weight([0.2] * 5, 2)
    assert keep == [0, 1] and abs(dropped - 0.6) < 1e-15


def _random_mps(rng, n, chi):
    """A normalised MPS with every bond at min(chi, 2^b, 2^(n-b)) and generic
    (full-rank) bonds."""
    dims = M.bond_dims(n, chi)
    t = [rng.normal(size=(dims[j], 2, dims[j + 1])) + 1j * rng.normal(size=(dims[j], 2, dims[j + 1]))
         for j in range(n)]
    v = M.to_statevector(t)
    t[0] = t[0] / np.linalg.norm(v)
    return t


def test_warm_bra_keeps_the_state_and_is_right_canonical():
    """eta = 0: the LQ chain with absorbed L factors represents the ket
    exactly; eta > 0: it represents the site-wise sum M_j = ket_j + eta G_j;
    sites 1..n-1 have orthonormal rows in both cases."""
    rng = np.random.default_rng(8)
    n, chi = 7, 6
    ket = _random_mps(rng, n, chi)
    gen = M.generic_bra(bra_init_gaussians(n, chi, 3))
    for eta in (0.0, 0.3):
        b = M.warm_bra(ket, gen, eta)
        msum = [k + eta * g for k, g in zip(ket, gen)]
        np.testing.assert_allclose(M.to_statevector(b), M.to_statevector(msum), atol=1e-12)
        for j in range(1, n):
            dl, _, dr = b[j].shape
            q = b[j].reshape(dl, 2 * dr)
            np.testing.assert_allclose(q @ q.conj().T, np.eye(dl), atol=1e-12)


def test_warm_bra_pads_a_narrower_ket():
    """A ket of smaller bonds sits in the top-left block of each site; the
    rest is eta G (seeded completion); the chain keeps that state."""
    rng = np.random.default_rng(9)
    n = 6
    ket = _random_mps(rng, n, 2)
    gen = M.generic_bra(bra_init_gaussians(n, 4, 3))
    eta = 0.05
    b = M.warm_bra(ket, gen, eta)
    assert [t.shape for t in b] == [t.shape for t in gen]
    msum = []
    for k, g in zip(ket, gen):
        t = eta * g.copy()
        t[:k.shape[0], :, :k.shape[2]] += k
        msum.append(t)
    np.testing.assert_allclose(M.to_statevector(b), M.to_statevector(msum), atol=1e-12)
    with pytest.raises(ValueError):
        M.warm_bra(_random_mps(rng, n, 8), gen, eta)


def test_warm_start_one_sweep_reproduces_the_ket():
    """Identity chunk, warm start with eta = 0 from a ket of full-rank bonds:
    the bra spans the ket's right subspaces, so one left-to-right sweep
    returns the ket with f = 1."""
    rng = np.random.default_rng(10)
    n, chi = 6, 4
    ket = _random_mps(rng, n, chi)
    gen = M.generic_bra(bra_init_gaussians(n, chi, 3))
    ident = M.chunk_mpo(n, [((0,), np.eye(2, dtype=complex))])
    new, f, _ = M.compress(ket, ident, M.warm_bra(ket, gen, 0.0), 1)
    assert abs(f - 1) < 1e-12
    ov = np.vdot(M.to_statevector(new), M.to_statevector(ket))
    assert abs(abs(ov) ** 2 - 1) < 1e-12


def test_chi_ladder_reduces_to_fixed_cap():
    """A ladder that never climbs (target 0) or has one rung is the fixed-cap
    run: same outcomes, fidelities and state."""
    circ, p = C.workload("cfg1_n10_chi16", n=6, depth=6, chi=2)
    u = np.random.default_rng(5).random(64)
    ref = D.run_single_path(circ, D.Simulator(6, 2, k=3), uniforms=u)
    for ladder, target in (([2, 4, 8], 0.0), ([2], 2.0)):
        r = D.run_single_path(circ, D.Simulator(6, 2, k=3), uniforms=u, chi_ladder=ladder,
                              f_target=target)
        assert r["outcomes"] == ref["outcomes"]
        np.testing.assert_allclose(r["fids"], ref["fids"], atol=1e-13)
        assert r["chis"] == [2] * len(ref["fids"])
        assert abs(abs(M.overlap(r["mps"], ref["mps"])) ** 2 - 1) < 1e-11


def test_chi_ladder_climbs_to_exact_cap():
    """A target above 1 climbs one rung per compression; on 6 qubits the top
    rung 8 is the exact bond dimension, so every later step has fidelity 1
    and the estimate is the product of the truncated steps alone."""
    circ, p = C.workload("cfg1_n10_chi16", n=6, depth=6, chi=2)
    u = np.random.default_rng(5).random(64)
    r = D.run_single_path(circ, D.Simulator(6, 2, k=6), uniforms=u, chi_ladder=[2, 4, 8],
                          f_target=2.0)
    fixed = D.run_single_path(circ, D.Simulator(6, 2, k=6), uniforms=u)
    nc = len(r["fids"])
    assert nc >= 3
    assert r["chis"] == [2, 4] + [8] * (nc - 2)
    assert r["fids"][0] < 1 - 1e-3
    assert abs(r["fids"][0] - fixed["fids"][0]) < 1e-13
    np.testing.assert_allclose(r["fids"][2:], 1.0, atol=1e-11)
    assert abs(r["F"] - np.prod(r["fids"])) < 1e-14
    mp = D.run_multi_path(circ, D.Simulator(6, 2, k=3), chi_ladder=[2, 8], f_target=2.0)
    assert abs(sum(b["p"] for b in mp["branches"]) - 1) < 1e-11
    for b in mp["branches"]:
        assert b["chis"][0] == 2 and all(c == 8 for c in b["chis"][1:])
        assert b["chi"] == 8


def test_chi_ladder_multi_path_matches_single_path_replay():
    """Each multi-path branch, replayed as a single path with the same ladder
    and its outcomes, climbs the same rungs and reaches the same fidelity."""
    circ, p = C.workload("cfg1_n10_chi16", n=6, depth=4, chi=2)
    sim = D.Simulator(6, 2, k=3)
    mp = D.run_multi_path(circ, sim, chi_ladder=[2, 4, 8], f_target=0.999)
    for b in mp["branches"][:4]:
        r = D.run_single_path(circ, sim, outcomes=list(b["path"]), chi_ladder=[2, 4, 8],
                              f_target=0.999)
        assert r["chis"] == b["chis"]
        assert abs(r["F"] - b["F"]) < 1e-12


@pytest.mark.parametrize("chi_bra", [4, 8])
def test_compress_into_narrower_bra(chi_bra):
    """A ket of bond cap 16 compressed into a bra of cap 4 or 8 (what every
    multi-path child with a smaller cap than its parent does): the result has
    the bra's bond dims and unit norm, and f equals |<psi~'|U|psi~>|^2 from
    contracted state vectors."""
    n = 10
    rng = np.random.default_rng(300 + chi_bra)
    ket = _random_mps(rng, n, 16)
    assert M.dims_of(ket) == M.bond_dims(n, 16)
    ops = _random_chunk(rng, n, 2)
    bra = M.generic_bra(bra_init_gaussians(n, chi_bra, 4))
    for s in (1, 2, 3):
        new, f, _ = M.compress(ket, M.chunk_mpo(n, ops), bra, s)
        assert M.dims_of(new) == M.bond_dims(n, chi_bra)
        target = M.to_statevector(ket)
        for qubits, mat in ops:
            target = SV.apply_gate(target, n, qubits, mat)
        v = M.to_statevector(new)
        assert abs(np.linalg.norm(v) - 1) < 1e-12
        assert abs(abs(np.vdot(v, target)) ** 2 - f) < 1e-12
        assert 0.0 < f < 1.0 - 1e-3             # the bra really truncates


def _mps_from_statevector(psi, n, chi):
    """Exact MPS of a state vector by successive SVDs, each bond zero-padded
    to min(chi, 2^b, 2^(n-b)) (chi at least every Schmidt rank)."""
    dims = M.bond_dims(n, chi)
    out, rest, left = [], psi.reshape(1, -1), 1
    for j in range(n - 1):
        m = rest.reshape(left * 2, -1)
        u, s, vh = np.linalg.svd(m, full_matrices=False)
        r = int(np.sum(s > 1e-14 * s[0]))
        assert r <= dims[j + 1]
        a = np.zeros((dims[j], 2, dims[j + 1]), dtype=complex)
        a[:left, :, :r] = u[:, :r].reshape(left, 2, r)
        out.append(a)
        rest = (s[:r, None] * vh[:r]).reshape(r, -1)
        left = r
    last = np.zeros((dims[n - 1], 2, 1), dtype=complex)
    last[:left, :, 0] = rest.reshape(left, 2)
    out.append(last)
    return out


def test_narrower_bra_reaches_eckart_young_bound():
    """Ket stored at cap 16 whose Schmidt ranks are at most 4 on every bond but
    the middle one (rank 8: three partially entangled pairs across it), a
    chunk of one-qubit gates (ranks unchanged), bra of cap 4: only the middle
    bond truncates, so f never exceeds the sum of the 4 largest squared
    Schmidt coefficients there and reaches it as the sweeps converge."""
    n = 8
    rng = np.random.default_rng(77)
    psi = np.zeros(2 ** n, dtype=complex)
    psi[0] = 1.0
    for (a, b), th in zip(((3, 4), (2, 5), (1, 6)), (0.35, 0.6, 0.9)):
        # cos th |00> + sin th |11> on (a, b), placed by two exact gates
        psi = SV.apply_gate(psi, n, (a,), np.array([[np.cos(th), -np.sin(th)],
                                                     [np.sin(th), np.cos(th)]]))
        cnot_far = SV.full_operator(n, (a,), np.diag([1.0, 0.0])) + \
            SV.full_operator(n, (a,), np.diag([0.0, 1.0])) @ SV.full_operator(n, (b,), C.X)
        psi = cnot_far @ psi
    for q in range(n):
        psi = SV.apply_gate(psi, n, (q,), C.haar_unitary(rng, 2))
    ket = _mps_from_statevector(psi, n, 16)
    assert M.dims_of(ket) == M.bond_dims(n, 16)
    ranks = [np.linalg.matrix_rank(psi.reshape(2 ** b, -1), tol=1e-12) for b in range(1, n)]
    assert ranks == [1, 2, 4, 8, 4, 2, 1]
    ops = [((q,), C.haar_unitary(rng, 2)) for q in range(n)]
    target = psi.copy()
    for qubits, mat in ops:
        target = SV.apply_gate(target, n, qubits, mat)
    sv = np.linalg.svd(target.reshape(16, 16), compute_uv=False)
    bound = float(np.sum(sv[:4] ** 2))
    assert bound < 1 - 1e-3
    bra = M.generic_bra(bra_init_gaussians(n, 4, 6))
    mpo = M.chunk_mpo(n, ops)
    prev = 0.0
    for s in (1, 2, 4, 8, 16):
        _, f, _ = M.compress(ket, mpo, bra, s)
        assert f <= bound + 1e-12
        if s >= 4:
            assert prev - 1e-14 <= f
        prev = f
    _, f_conv, _ = M.compress(ket, mpo, bra, 60)
    assert abs(f_conv - bound) < 1e-10


def test_chi_schedule_exact_caps_replay_statevector():
    """A bond-cap schedule that never cuts below the state's Schmidt ranks
    (cap 4 after the first two brickwork layers, 16 after four, then 32)
    leaves the run exact: every p_m and the final state match the state
    vector, each compression has f = 1 and the final bonds are those of the
    last cap."""
    n = 10
    circ, _ = C.workload("cfg1_n10_chi16", n=n, depth=10, chi=32)
    sim = D.Simulator(n, 32, k=1000, n_sweeps=2, init_seed=7)
    u = np.random.default_rng(12).random(64)
    first = D.run_single_path(circ, sim, uniforms=u)
    nc = len(first["fids"])
    sched = [4, 16] + [32] * (nc - 2)
    r = D.run_single_path(circ, sim, outcomes=first["outcomes"], chis=sched)
    assert r["chis"] == sched
    np.testing.assert_allclose(r["fids"], 1.0, atol=1e-11)
    ref = SV.replay(circ, r["outcomes"])
    np.testing.assert_allclose(r["pms"], ref["pms"], atol=1e-12)
    assert M.dims_of(r["mps"]) == M.bond_dims(n, 32)
    v = M.to_statevector(r["mps"])
    assert abs(abs(np.vdot(ref["psi"], v)) ** 2 - 1) < 1e-11


def test_chi_schedule_truncates_where_the_cap_is_too_small():
    """The schedule's caps apply in order: a cap of 2 at the second
    compression (Schmidt ranks up to 16 by then) is the only truncated step;
    a schedule shorter than the run is an error."""
    n = 10
    circ, _ = C.workload("cfg1_n10_chi16", n=n, depth=10, chi=32)
    sim = D.Simulator(n, 32, k=1000, n_sweeps=2, init_seed=7)
    u = np.random.default_rng(12).random(64)
    first = D.run_single_path(circ, sim, uniforms=u)
    nc = len(first["fids"])
    sched = [4, 2] + [32] * (nc - 2)
    r = D.run_single_path(circ, sim, outcomes=first["outcomes"], chis=sched)
    assert r["chis"] == sched
    assert abs(r["fids"][0] - 1) < 1e-11
    assert r["fids"][1] < 1 - 1e-3
    assert M.bond_dims(n, 2) != M.bond_dims(n, 32)
    with pytest.raises(ValueError):
        D.run_single_path(circ, sim, outcomes=first["outcomes"], chis=sched[:-1])


def test_multi_path_branches_record_p0_and_replay_with_their_schedule():
    """Each multi-path branch with per-child caps records p_0 of every
    measurement on its path; the single-path run replaying its outcomes with
    its cap schedule reproduces those p_0, its weight, fidelity and state
    (the replay the full-size GPU checks rely on)."""
    from inputs.randomness import branch_chi_draw
    circ, prm = C.workload("cfg3_n32_mp64", n=8, depth=6, chi=16)
    choices = (4, 8, 12, 16)
    chi_of = lambda path: branch_chi_draw(prm["seed"], path, choices)  # noqa: E731
    k = C.segment_max(circ)
    sim = D.Simulator(8, 16, k, 2, prm["init_seed"])
    mp = D.run_multi_path(circ, sim, max_branches=5, chi_of=chi_of)
    nm = circ.n_measurements()
    for b in mp["branches"]:
        assert len(b["p0s"]) == nm == len(b["path"])
        pm = [p0 if m == 0 else 1 - p0 for p0, m in zip(b["p0s"], b["path"])]
        assert abs(np.prod(pm) - b["p"]) < 1e-12
        r = D.run_single_path(circ, sim, outcomes=list(b["path"]), chis=b["chis"])
        np.testing.assert_allclose(r["p0s"], b["p0s"], atol=1e-12)
        assert abs(r["p"] - b["p"]) < 1e-12 and abs(r["F"] - b["F"]) < 1e-12
        assert abs(abs(M.overlap(r["mps"], b["mps"])) ** 2 - 1) < 1e-11
