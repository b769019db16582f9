"""Degenerate inputs through the C ABI: empty chunks and empty branch lists,
one- and two-qubit states, circuits without measurements or without gates,
against the oracle and the statevector definition."""
import numpy as np
import pytest

from inputs import circuits as C
from inputs.randomness import bra_init_gaussians, shot_uniforms
from oracle import dynamic as OD
from oracle import mps as OM
from oracle import statevector as SV

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_26516_amd import engine as E
    e = E.Engine(0)
    yield e
    e.close()


def _E():
    from paper_2609_26516_amd import engine as E
    return E


def _capi():
    from paper_2609_26516_amd import capi
    return capi


def _fid_err(a, b):
    return abs(1 - abs(OM.overlap(a, b)) ** 2 / (OM.norm_sq(a) * OM.norm_sq(b)))


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_empty_chunk_keeps_the_state(eng, prec):
    """A chunk of no operations is the identity: compressing a state of the
    bra's own bond dims returns it with f = 1."""
    capi = _capi()
    n, chi = 8, 8
    rng = np.random.default_rng(2)
    init = OM.generic_bra(bra_init_gaussians(n, chi, 5))
    ops = [((q, q + 1), C.haar_unitary(rng, 4)) for q in range(0, n - 1, 2)]
    psi, _, _ = OM.compress(OM.zero_state(n, chi), OM.chunk_mpo(n, ops), init, 2)
    h = capi.dcs_chunk_compile(eng.ctx, n, [], [], np.zeros(0, np.complex128))
    assert list(capi.dcs_chunk_bonds(h, n)) == [1] * (n + 1)
    st = _E().State(eng, prec, n, 1, chi, 4, [chi], 5)
    capi.dcs_import_mps(st.h, 0, chi, psi, eng.stream())
    f = capi.dcs_compress_step(st.h, [0], [h], 2, eng.stream())
    assert abs(f[0] - 1) < (1e-12 if prec == "c128" else 1e-5)
    assert _fid_err(st.export(0), psi) < (1e-12 if prec == "c128" else 1e-6)
    capi.dcs_chunk_destroy(h)
    st.close()


def test_empty_branch_lists(eng):
    capi = _capi()
    st = _E().State(eng, "c64", 6, 2, 4, 4, [4], 5)
    assert len(capi.dcs_compress_step(st.h, [], [], 2, eng.stream())) == 0
    assert len(capi.dcs_measure_prob(st.h, [], [], eng.stream())) == 0
    assert len(capi.dcs_collapse(st.h, [], [], [], [], 1e-10, eng.stream())) == 0
    capi.dcs_branch_init_zero(st.h, [], [], eng.stream())
    capi.dcs_branch_release(st.h, [])
    st.close()


@pytest.mark.parametrize("n", [1, 2])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_one_and_two_qubit_runs(eng, n, prec):
    """Single-path runs on the smallest chains equal the statevector replay
    (every bond is exact at chi = 2)."""
    rng = np.random.default_rng(n)
    ops = [C.Gate((0,), C.haar_unitary(rng, 2)), C.Measure(0, 0)]
    if n == 2:
        ops = [C.Gate((0, 1), C.haar_unitary(rng, 4)), C.Measure(1, 0),
               C.CGate(C.Cond((0,), 1), C.Gate((0,), C.X)), C.Gate((1, 0), C.haar_unitary(rng, 4)),
               C.Measure(0, 1)]
    circ = C.Circuit(n, 2 if n == 2 else 1, ops, name=f"tiny{n}")
    u = np.stack([shot_uniforms(3, s, circ.n_measurements()) for s in range(4)])
    st = _E().State(eng, prec, n, 4, 2, 4, [2], 5)
    res = _E().run_single_path(eng, st, circ, 4, 2, 20, 2, uniforms=u)
    for s in range(4):
        ref = SV.replay(circ, list(res["outcomes"][s]))
        assert abs(res["p"][s] - ref["p"]) < (1e-12 if prec == "c128" else 1e-6)
        v = OM.to_statevector(st.export(int(res["ids"][s])))
        assert abs(abs(np.vdot(ref["psi"], v)) ** 2 - 1) < (1e-12 if prec == "c128" else 1e-6)
    st.close()


def test_no_measurements_and_no_gates(eng):
    """A circuit without measurements is one compression per chunk; one
    without gates only measures |0...0> (outcome 0, p = 1, no compression)."""
    n = 6
    circ, _ = C.workload("cfg1_n10_chi16", n=n, depth=4, chi=8)
    gates = C.Circuit(n, 0, [o for o in circ.ops if isinstance(o, C.Gate)], name="gates")
    st = _E().State(eng, "c128", n, 2, 8, 4, [8], 7)
    res = _E().run_single_path(eng, st, gates, 1, 8, 5, 2)
    ref = OD.run_single_path(gates, OD.Simulator(n, 8, 5, 2, 7))
    assert len(res["chis"][0]) == len(ref["fids"])
    assert abs(res["F"][0] - ref["F"]) < 1e-10
    assert _fid_err(st.export(int(res["ids"][0])), ref["mps"]) < 1e-10
    st.release(res["ids"])
    meas = C.Circuit(n, 2, [C.Measure(0, 0), C.Measure(5, 1)], name="meas")
    res = _E().run_single_path(eng, st, meas, 1, 8, 5, 2, uniforms=np.array([[0.99, 0.99]]))
    assert list(res["outcomes"][0]) == [0, 0] and res["p"][0] == 1.0
    assert res["chis"][0] == []
    st.close()
