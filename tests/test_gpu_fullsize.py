"""Full-size check of the benchmark workload (40 qubits, depth-20 brickwork, 4
measurements every 2 layers, bond cap 256) in the launch configuration of the
benchmark step: 256 complex64 shots in one batch with the tile autotuner on.
Sampled shots (the first and the last of the batch) are replayed by the
FP64 oracle on the same outcomes, and by the complex128 GPU path.

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
SHOTS = 256
SAMPLED = (0, SHOTS - 1)


@pytest.fixture(scope="module")
def runs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_26516_amd import engine as E
    circ, prm = C.workload(WORKLOAD)
    n, chi = prm["n"], prm["chi"]
    k = C.segment_max(circ) + 1
    nm = circ.n_measurements()
    u = np.stack([shot_uniforms(prm["seed"], s, nm) for s in range(SHOTS)])
    eng = E.Engine(0)
    eng.tuning(True)
    out = {}
    st = E.State(eng, "c64", n, SHOTS, chi, 4, [chi], prm["init_seed"])
    t = time.time()
    r64 = E.run_single_path(eng, st, circ, SHOTS, chi, k, 2, uniforms=u)
    print(f"c64 {SHOTS} shots: {time.time() - t:.1f} s", flush=True)
    out["c64"] = (r64, {s: st.export(int(r64["ids"][s])) for s in SAMPLED})
    st.close()
    st = E.State(eng, "c128", n, len(SAMPLED), chi, 4, [chi], prm["init_seed"])
    t = time.time()
    r128 = E.run_single_path(eng, st, circ, len(SAMPLED), chi, k, 2,
                             outcomes=r64["outcomes"][list(SAMPLED)])
    print(f"c128 replay of shots {SAMPLED}: {time.time() - t:.1f} s", flush=True)
    out["c128"] = (r128, [st.export(int(i)) for i in r128["ids"]])
    st.close()
    eng.close()
    out["oracle"] = {}
    for s in SAMPLED:
        t = time.time()
        out["oracle"][s] = OD.run_single_path(circ, OD.Simulator(n, chi, k, 2, prm["init_seed"]),
                                              outcomes=r64["outcomes"][s])
        print(f"oracle shot {s}: {time.time() - t:.1f} s", flush=True)
    out["u"] = u
    return out


def _fid_err(a, b):
    return abs(1 - abs(OM.overlap(a, b)) ** 2 / (OM.norm_sq(a) * OM.norm_sq(b)))


def test_truncated_regime_reached(runs):
    for ref in runs["oracle"].values():
        assert len(ref["p0s"]) == 40
        assert min(ref["fids"]) < 0.999          # bond cap 256 really truncates
        assert 0.0 < ref["F"] < 1.0


def test_outcomes_follow_the_uniforms(runs):
    """Each sampled shot's outcome is 1 exactly when its uniform is at least
    the oracle's p_0 (no uniform falls within the tolerance of p_0 here)."""
    r, _ = runs["c64"]
    for s, ref in runs["oracle"].items():
        p0 = np.array(ref["p0s"])
        assert np.min(np.abs(runs["u"][s] - p0)) > 1e-6
        np.testing.assert_array_equal(r["outcomes"][s], (runs["u"][s] >= p0).astype(np.int8))


def test_complex128_matches_oracle(runs):
    r, mps = runs["c128"]
    for i, s in enumerate(SAMPLED):
        ref = runs["oracle"][s]
        np.testing.assert_allclose(r["p0s"][i], ref["p0s"], atol=1e-9, rtol=0)
        assert abs(r["F"][i] - ref["F"]) < 1e-8
        assert _fid_err(mps[i], ref["mps"]) < 1e-9


def test_complex64_meets_precision_targets(runs):
    r, mps = runs["c64"]
    for s in SAMPLED:
        ref = runs["oracle"][s]
        dp = np.max(np.abs(r["p0s"][s] - np.array(ref["p0s"])))
        fe = _fid_err(mps[s], ref["mps"])
        print(f"shot {s}: complex64 vs FP64 oracle: max |dp| = {dp:.3e}, state fidelity error "
              f"= {fe:.3e}, F = {r['F'][s]:.6f} vs {ref['F']:.6f}")
        assert dp <= 1e-6
        assert fe <= 1e-6
        assert abs(r["F"][s] - ref["F"]) < 1e-4


def test_complex64_batch_properties(runs):
    """Every shot of the batch: probabilities in [0, 1] and fidelity estimates
    (products of partial fidelities, each at most 1) in (0, 1]."""
    r, _ = runs["c64"]
    p = np.asarray(r["p0s"])
    assert p.shape == (SHOTS, 40)
    assert np.all(p >= -1e-12) and np.all(p <= 1 + 1e-12)
    F = np.asarray(r["F"])
    assert np.all(F > 0.0) and np.all(F <= 1.0 + 1e-12)
