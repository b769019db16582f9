"""Full-size check of the benchmark workload (40 qubits, depth-20 brickwork, 4
measurements every 2 layers, bond cap 256): GPU shots in complex64 and
complex128 against the FP64 oracle replaying the same outcomes.

Sampled outputs: every measurement probability p_0 of the shot, the final
state (fidelity error 1 - |<gpu|oracle>|^2) and the fidelity estimate.
Complex64 targets of the precision form: probability error and state-fidelity
error at most 1e-6; complex128 agrees to rounding (1e-9)."""
import time

import numpy as np
import pytest

from inputs import circuits as C
from inputs.randomness import shot_uniforms
from oracle import dynamic as OD
from oracle import mps as OM

pytestmark = pytest.mark.gpu

WORKLOAD = "cfg2_n40_chi256"


@pytest.fixture(scope="module")
def runs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_26516_amd import engine as E
    circ, prm = C.workload(WORKLOAD)
    n, chi = prm["n"], prm["chi"]
    k = C.segment_max(circ) + 1
    shots = 2
    u = np.stack([shot_uniforms(prm["seed"], s, circ.n_measurements()) for s in range(shots)])
    eng = E.Engine(0)
    out = {}
    st = E.State(eng, "c64", n, shots, chi, 4, [chi], prm["init_seed"])
    t = time.time()
    r64 = E.run_single_path(eng, st, circ, shots, chi, k, 2, uniforms=u)
    print(f"c64 {shots} shots: {time.time() - t:.1f} s", flush=True)
    out["c64"] = (r64, [st.export(int(i)) for i in r64["ids"]])
    st.close()
    st = E.State(eng, "c128", n, shots, chi, 4, [chi], prm["init_seed"])
    t = time.time()
    r128 = E.run_single_path(eng, st, circ, shots, chi, k, 2, outcomes=r64["outcomes"])
    print(f"c128 replay: {time.time() - t:.1f} s", flush=True)
    out["c128"] = (r128, [st.export(int(i)) for i in r128["ids"]])
    st.close()
    eng.close()
    t = time.time()
    ref = OD.run_single_path(circ, OD.Simulator(n, chi, k, 2, prm["init_seed"]),
                             outcomes=r64["outcomes"][0])
    print(f"oracle shot 0: {time.time() - t:.1f} s", flush=True)
    out["oracle"] = ref
    return out


def _fid_err(a, b):
    return abs(1 - abs(OM.overlap(a, b)) ** 2 / (OM.norm_sq(a) * OM.norm_sq(b)))


def test_truncated_regime_reached(runs):
    ref = runs["oracle"]
    assert len(ref["p0s"]) == 40
    assert min(ref["fids"]) < 0.999          # bond cap 256 really truncates
    assert 0.0 < ref["F"] < 1.0


def test_complex128_matches_oracle(runs):
    r, mps = runs["c128"]
    ref = runs["oracle"]
    np.testing.assert_allclose(r["p0s"][0], ref["p0s"], atol=1e-9, rtol=0)
    assert abs(r["F"][0] - ref["F"]) < 1e-8
    assert _fid_err(mps[0], ref["mps"]) < 1e-9


def test_complex64_meets_precision_targets(runs):
    r, mps = runs["c64"]
    ref = runs["oracle"]
    dp = np.max(np.abs(r["p0s"][0] - np.array(ref["p0s"])))
    fe = _fid_err(mps[0], ref["mps"])
    print(f"complex64 vs FP64 oracle: max |dp| = {dp:.3e}, state fidelity error = {fe:.3e}, "
          f"F = {r['F'][0]:.6f} vs {ref['F']:.6f}")
    assert dp <= 1e-6
    assert fe <= 1e-6
    assert abs(r["F"][0] - ref["F"]) < 1e-4


def test_complex64_vs_complex128_second_shot(runs):
    r64, m64 = runs["c64"]
    r128, m128 = runs["c128"]
    dp = np.max(np.abs(r64["p0s"][1] - r128["p0s"][1]))
    fe = _fid_err(m64[1], m128[1])
    assert dp <= 1e-6
    assert fe <= 1e-6
