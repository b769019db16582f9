"""Full-size checks of the other three workloads, each in the launch
configuration its benchmark run uses:

* 24 qubits, bond cap 64, one-layer chunks, 1024 complex64 shots in one batch
  (autotuner on): the first, a middle and the last shot replayed by the FP64
  oracle on the same outcomes;
* the 32-qubit multi-path run (Alg. 2, top-M with M = 64, per-branch bond caps
  drawn from {32, 48, ..., 256}): complex64 against the complex128 path, plus
  the mass balance of the branch weights; the heaviest kept branch and the
  branch at the cut (the lightest kept) of the complex64 run replayed by the
  FP64 oracle's single-path driver with that branch's outcomes and bond-cap
  schedule, held to the precision form's targets (every measurement's p_0
  within 1e-6, state-fidelity error at most 1e-6);
* 60 qubits, bond cap 1024, three-layer chunks, one split-BF16 shot: against
  the complex128 GPU path replaying its outcomes (the oracle cannot hold this
  size; the complex128 path is held to it at 1e-9 on every smaller case).

Tolerances: complex64 1e-6 on probabilities and state-fidelity error, 1e-4 on
a whole run's fidelity estimate; branch weights (products of up to 16
probabilities) 1e-5.  Split-BF16: 1e-4 on probabilities (first order in the
3 * 2^-18 error of a split product), 1e-6 on the state-fidelity error (second
order), 1e-3 on the product of a whole run's 24 partial fidelities."""
import time

import numpy as np
import pytest

from inputs import circuits as C
from inputs.randomness import branch_chi_draw, shot_uniforms
from oracle import dynamic as OD
from oracle import mps as OM

pytestmark = pytest.mark.gpu


def _fid_err(a, b):
    return abs(1 - abs(OM.overlap(a, b)) ** 2 / (OM.norm_sq(a) * OM.norm_sq(b)))


def _engine():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_26516_amd import engine as E
    return E, E.Engine(0)


def test_24_qubits_1024_shots_sampled_against_oracle():
    E, eng = _engine()
    circ, prm = C.workload("cfg4_n24_chi64_x1024")
    n, chi, shots = prm["n"], prm["chi"], 1024
    assert (n, chi, prm["layers_per_round"]) == (24, 64, 1)
    k = C.segment_max(circ) + 1
    nm = circ.n_measurements()
    u = np.stack([shot_uniforms(prm["seed"], s, nm) for s in range(shots)])
    eng.tuning(True)
    st = E.State(eng, "c64", n, shots, chi, 4, [chi], prm["init_seed"])
    t = time.time()
    r = E.run_single_path(eng, st, circ, shots, chi, k, 2, uniforms=u)
    print(f"c64 {shots} shots: {time.time() - t:.2f} s", flush=True)
    sampled = (0, shots // 2 - 1, shots - 1)
    mps = {s: st.export(int(r["ids"][s])) for s in sampled}
    st.close()
    eng.close()
    p = np.asarray(r["p0s"])
    assert p.shape == (shots, nm)
    assert np.all(p >= 0.0) and np.all(p <= 1.0)
    assert np.all(np.asarray(r["F"]) > 0.0) and np.all(np.asarray(r["F"]) <= 1.0 + 1e-12)
    for s in sampled:
        ref = OD.run_single_path(circ, OD.Simulator(n, chi, k, 2, prm["init_seed"]),
                                 outcomes=r["outcomes"][s])
        dp = np.max(np.abs(p[s] - np.array(ref["p0s"])))
        fe = _fid_err(mps[s], ref["mps"])
        print(f"shot {s}: max |dp| = {dp:.3e}, state fidelity error = {fe:.3e}, "
              f"F = {r['F'][s]:.6f} vs {ref['F']:.6f}", flush=True)
        assert dp <= 1e-6
        assert fe <= 1e-6
        assert abs(r["F"][s] - ref["F"]) < 1e-4
        # the outcomes are the ones the uniforms select under the oracle's p_0
        p0 = np.array(ref["p0s"])
        assert np.min(np.abs(u[s] - p0)) > 1e-6
        np.testing.assert_array_equal(r["outcomes"][s], (u[s] >= p0).astype(np.int8))


def _multi_path(E, eng, prec, tuning):
    """One full-size run; the heaviest kept branch and the lightest kept one
    (the cut) are exported before the state is freed."""
    circ, prm = C.workload("cfg3_n32_mp64")
    n, chi, M = prm["n"], prm["chi"], prm["max_branches"]
    choices = prm["chi_choices"]
    k = C.segment_max(circ) + 1
    chi_of = lambda path: branch_chi_draw(prm["seed"], path, choices)  # noqa: E731
    eng.tuning(tuning)
    st = E.State(eng, prec, n, 2 * M, chi, 4, list(choices) + [chi], prm["init_seed"])
    t = time.time()
    res = E.run_multi_path(eng, st, circ, chi, k, 2, max_branches=M, chi_of=chi_of)
    print(f"{prec} multi-path run: {time.time() - t:.2f} s, {len(res['branches'])} branches, "
          f"dropped {res['dropped']:.6f}", flush=True)
    w = [b["p"] for b in res["branches"]]
    picked = {"heaviest": res["branches"][int(np.argmax(w))],
              "cut": res["branches"][int(np.argmin(w))]}
    res["picked"] = {name: (b, st.export(b["id"])) for name, b in picked.items()}
    st.close()
    return res, M


@pytest.fixture(scope="module")
def multi_path_runs():
    E, eng = _engine()
    r64, M = _multi_path(E, eng, "c64", True)
    r128, _ = _multi_path(E, eng, "c128", False)
    eng.close()
    return r64, r128, M


@pytest.mark.parametrize("which", ["heaviest", "cut"])
def test_32_qubit_multi_path_kept_branch_against_oracle(multi_path_runs, which):
    """A kept branch of the full-size complex64 run against the FP64 oracle
    replaying its outcomes with its bond-cap schedule (the root's cap for the
    first compression, then the cap each child drew)."""
    r64, _, _ = multi_path_runs
    b, mps = r64["picked"][which]
    circ, prm = C.workload("cfg3_n32_mp64")
    n, chi = prm["n"], prm["chi"]
    k = C.segment_max(circ) + 1
    nm = circ.n_measurements()
    assert b["chis"][0] == chi and len(set(b["chis"])) > 1    # uneven caps on the path
    t = time.time()
    ref = OD.run_single_path(circ, OD.Simulator(n, chi, k, 2, prm["init_seed"]),
                             outcomes=list(b["path"]), chis=b["chis"])
    assert ref["chis"] == b["chis"]
    dp = np.max(np.abs(np.array(b["p0s"]) - np.array(ref["p0s"])))
    fe = _fid_err(mps, ref["mps"])
    print(f"{which} branch (p = {b['p']:.3e}, caps {b['chis']}): oracle {time.time() - t:.1f} s, "
          f"max |dp| = {dp:.3e}, state fidelity error = {fe:.3e}, "
          f"F = {b['F']:.6f} vs {ref['F']:.6f}", flush=True)
    assert len(b["p0s"]) == nm
    assert dp <= 1e-6
    assert fe <= 1e-6
    assert abs(b["p"] - ref["p"]) <= nm * 1e-6 * max(ref["p"], 1e-300) / min(ref["pms"])
    assert abs(b["F"] - ref["F"]) < 1e-4


def test_32_qubit_multi_path_complex64_against_complex128(multi_path_runs):
    r64, r128, M = multi_path_runs
    for res in (r64, r128):
        w = np.array([b["p"] for b in res["branches"]])
        assert len(w) == M                      # the cap binds at this size
        assert np.all(w > 0.0)
        # every split conserves the weight; top-M moves the rest to "dropped"
        assert abs(w.sum() + res["dropped"] - 1.0) < 1e-9
        assert 0.0 < res["F_mp"] <= 1.0 + 1e-12
    got = {b["path"]: b for b in r64["branches"]}
    want = {b["path"]: b for b in r128["branches"]}
    # kept sets agree except for paths tied with the cut within the tolerance
    for paths, res in ((set(got) - set(want), r64), (set(want) - set(got), r128)):
        cut = min(b["p"] for b in res["branches"])
        for pth in paths:
            b = (got if res is r64 else want)[pth]
            assert b["p"] - cut < 2e-5, (pth, b["p"], cut)
    common = set(got) & set(want)
    assert len(common) >= M - 2
    for pth in common:
        assert abs(got[pth]["p"] - want[pth]["p"]) < 1e-5
        assert abs(got[pth]["F"] - want[pth]["F"]) < 1e-4
        assert got[pth]["chi"] == want[pth]["chi"]
    assert abs(r64["dropped"] - r128["dropped"]) < 1e-5 * M
    assert abs(r64["F_mp"] - r128["F_mp"]) < 1e-4


def test_60_qubits_chi_1024_split_bf16_against_complex128():
    E, eng = _engine()
    from paper_2609_26516_amd import capi
    circ, prm = C.workload("cfg5_n60_chi1024")
    n, chi = prm["n"], prm["chi"]
    assert (n, chi, prm["layers_per_round"]) == (60, 1024, 3)
    w = 16                                  # two rank-4 gates across a bond per chunk
    k = C.segment_max(circ) + 1
    u = shot_uniforms(prm["seed"], 0, circ.n_measurements())[None, :]
    st = E.State(eng, "bf16x3", n, 1, chi, w, [chi], prm["init_seed"])
    t = time.time()
    rb = E.run_single_path(eng, st, circ, 1, chi, k, 2, uniforms=u)
    print(f"split-BF16 shot: {time.time() - t:.1f} s", flush=True)
    mps_b = st.export(int(rb["ids"][0]))
    st.close()
    st = E.State(eng, "c128", n, 2, chi, w, [chi], prm["init_seed"])
    t = time.time()
    rd = E.run_single_path(eng, st, circ, 1, chi, k, 2, outcomes=rb["outcomes"])
    print(f"complex128 replay: {time.time() - t:.1f} s", flush=True)
    i64 = int(rd["ids"][0])
    other = st.alloc(1)[0]
    capi.dcs_import_mps(st.h, other, chi, mps_b, eng.stream())
    ov = capi.dcs_overlap(st.h, i64, other, eng.stream())
    na = capi.dcs_overlap(st.h, i64, i64, eng.stream()).real
    nb = capi.dcs_overlap(st.h, other, other, eng.stream()).real
    st.close()
    eng.close()
    fe = abs(1 - abs(ov) ** 2 / (na * nb))
    dp = np.max(np.abs(rb["p0s"][0] - rd["p0s"][0]))
    print(f"split-BF16 vs complex128: max |dp| = {dp:.3e}, state fidelity error = {fe:.3e}, "
          f"F = {rb['F'][0]:.6f} vs {rd['F'][0]:.6f}", flush=True)
    assert abs(na - 1.0) < 1e-9 and abs(nb - 1.0) < 1e-6
    assert rd["F"][0] < 0.999                # the bond cap really truncates
    assert dp <= 1e-4
    assert fe <= 1e-6
    assert abs(rb["F"][0] - rd["F"][0]) < 1e-3
