#!/usr/bin/env python3
"""Throughput of the dynamic-circuit simulation hot path on one MI355X.

Workload (the precision form): 40-qubit chain, depth-20 Haar brickwork, a
round of 4 mid-circuit Z measurements (qubits 1..38) every 2 layers with X on
the right and Z on the left neighbour when the outcome is 1; bond cap 256;
single-path sampling (Alg. 1), two sweeps per compression step, chunks broken
only at measurements.  One step = one batch of `--shots` independent shots
simulated in lockstep from |0...0> to the end of the circuit (every
compression step, measurement probability and collapse of every shot).

The timed form stores and contracts in complex64 (FP32 MFMA, FP32
accumulation) with FP64 QR, norms and renormalisation; the plain FP64 path
(complex128 on FP64 MFMA) is timed beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "cfg2_n40_chi256"
# other workload shapes reachable with --workload (parity-test configurations,
# not the headline line)
SINGLE_PATH = {"sp40": "cfg2_n40_chi256", "sp24": "cfg4_n24_chi64_x1024",
               "sp10": "cfg1_n10_chi16"}
MULTI_PATH = {"mp32": "cfg3_n32_mp64"}
LARGE_CHI = {"sp60": "cfg5_n60_chi1024"}
TREE = {"tt27": "ttn27_chi32"}
PEAK = {"c64": (157.3, "fp32 dense MFMA"), "c128": (78.6, "fp64 dense MFMA"),
        "bf16x3": (2500.0 / 3.0, "bf16 dense MFMA / 3 products per real product")}
HBM_PEAK_GBS = 8000.0
CLASSES = ["gemm_nn", "gemm_nt", "gemm_cn", "gemm_jt", "gate_operator", "qr", "measure",
           "other"]
# rocprofv3 kernel names of the timed classes (complex64 path)
KERNEL_NAMES = {
    "gemm_nn": "gemm_kernel<0, 0, 0, float, 0, 0>", "gemm_nt": "gemm_kernel<0, 0, 0, float, 0, 1>",
    "gemm_cn": "gemm_kernel<0, 0, 0, float, 2, 0>", "gemm_jt": "gemm_kernel<0, 0, 0, float, 3, 1>",
    "gate_operator": "mpo_right_kernel / mpo_left_kernel", "qr": "qr_left_kernel<0, 0, 512 | 256>",
}


TUNE = {"enabled": True, "save": None}


# HBM bytes of the dominant kernel from two rocprofv3 --pmc passes (FETCH_SIZE,
# then WRITE_SIZE, KiB per dispatch, averaged over the kernel's dispatches in
# one default step), each scaled by what the counter reads for a plain copy
# of known size.  Valid only for the kernel source they were taken on.
TRAFFIC = {
    "qr": {"src": ["paper_2609_26516_amd/csrc/kernels.hip", "paper_2609_26516_amd/csrc/qr_panel.h",
                   "paper_2609_26516_amd/csrc/qr_cholpanel.h", "paper_2609_26516_amd/csrc/kernel_util.h"],
           "sha256": "c83839423b301ba0c9187665c893ee8c5b6bb761681f887b94c1238a938f87da",
           "fetch_kib": 2501359.8, "write_kib": 979570.9,
           "fetch_factor": 1048576 / 524300.5, "write_factor": 1048576 / 1048576.3},
}


def measured_traffic(cls):
    import hashlib
    t = TRAFFIC.get(cls)
    if t is None:
        return None
    h = hashlib.sha256()
    for src in t["src"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != t["sha256"]:
        return None       # kernel changed since the counters were taken
    return (t["fetch_kib"] * t["fetch_factor"] + t["write_kib"] * t["write_factor"]) * 1024.0


def mpo_bond_max(prm) -> int:
    """Operator bond of a chunk of L Haar brickwork layers: a bond is
    straddled by ceil(L / 2) two-qubit gates of operator-Schmidt rank 4."""
    return 4 ** ((prm["layers_per_round"] + 1) // 2)


def run_gpu(prec: str, shots: int, steps: int, warmup: int, timing: bool, workload=WORKLOAD,
            graphs: bool = False, sampled=()):
    """W warm-up steps, then K timed steps with no per-launch instrumentation.
    With `timing`, one more step after the timed ones records per-class launch
    durations with HIP events (the roofline figures); the shots listed in
    `sampled` are exported from that step (or from the last timed one)."""
    import torch
    from inputs import circuits as C
    from inputs.randomness import shot_uniforms
    from paper_2609_26516_amd import engine as E

    circ, prm = C.workload(workload)
    n, chi = prm["n"], prm["chi"]
    k = C.segment_max(circ) + 1      # chunks break only at measurements
    eng = E.Engine(0)
    eng.graphs(graphs)
    eng.tuning(TUNE["enabled"])
    st = E.State(eng, prec, n, shots, chi, mpo_bond_max(prm), [chi], prm["init_seed"])
    nm = circ.n_measurements()
    samples = {}

    def one_step(step, export=False):
        u = np.stack([shot_uniforms(prm["seed"], step * shots + s, nm) for s in range(shots)])
        res = E.run_single_path(eng, st, circ, shots, chi, k, 2, uniforms=u)
        if export:
            for s in sampled:
                samples[s] = {"outcomes": res["outcomes"][s].copy(), "p0s": res["p0s"][s].copy(),
                              "F": float(res["F"][s]), "mps": st.export(int(res["ids"][s]))}
        st.release(res["ids"])
        return res

    for w in range(warmup):
        one_step(10_000 + w)
    torch.cuda.synchronize()
    eng.timing(False)
    t0 = time.perf_counter()
    fids = []
    for s in range(steps):
        r = one_step(s, export=(s == steps - 1 and not timing))
        fids.append(float(np.mean(r["F"])))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = None
    if timing:
        eng.timing(True)
        eng.timing_stats(reset=True)
        one_step(steps, export=True)
        torch.cuda.synchronize()
        stats = eng.timing_stats(reset=True)
        eng.timing(False)
    if TUNE["save"] and prec == "c64":
        eng.save_tuning(TUNE["save"])
    st.close()
    eng.close()
    return dt, stats, fids, samples


def precision_vs_fp64(workload: str, samples: dict):
    """Sampled shots of a reduced-precision run against the complex128 GPU path
    replaying their outcomes (the complex128 path is itself held to the FP64
    oracle): every measurement probability, and the state-fidelity error
    1 - |<a|b>|^2 / (<a|a><b|b>) from the FP64 overlap of the two final states
    (the reduced-precision state imported into a complex128 state)."""
    from inputs import circuits as C
    from paper_2609_26516_amd import capi
    from paper_2609_26516_amd import engine as E

    circ, prm = C.workload(workload)
    n, chi = prm["n"], prm["chi"]
    k = C.segment_max(circ) + 1
    shots = sorted(samples)
    eng = E.Engine(0)
    st = E.State(eng, "c128", n, 2 * len(shots), chi, mpo_bond_max(prm), [chi],
                 prm["init_seed"])
    outs = np.stack([samples[s]["outcomes"] for s in shots])
    r = E.run_single_path(eng, st, circ, len(shots), chi, k, 2, outcomes=outs)
    dp, fe, df = [], [], []
    for i, s in enumerate(shots):
        ref_id = int(r["ids"][i])
        other = st.alloc(1)[0]
        capi.dcs_import_mps(st.h, other, chi, samples[s]["mps"], eng.stream())
        ov = capi.dcs_overlap(st.h, ref_id, other, eng.stream())
        na = capi.dcs_overlap(st.h, ref_id, ref_id, eng.stream()).real
        nb = capi.dcs_overlap(st.h, other, other, eng.stream()).real
        fe.append(float(abs(1 - abs(ov) ** 2 / (na * nb))))
        dp.append(float(np.max(np.abs(samples[s]["p0s"] - r["p0s"][i]))))
        df.append(float(abs(samples[s]["F"] - r["F"][i])))
    st.close()
    eng.close()
    return {"reference": "GPU FP64 path (complex128, FP64 MFMA) replaying the outcomes",
            "shots": shots, "max_abs_probability_error": max(dp),
            "state_fidelity_error": max(fe), "fidelity_estimate_abs_error": max(df),
            "targets": {"max_abs_probability_error": 1e-6, "state_fidelity_error": 1e-6}}


def run_gpu_multipath(prec: str, steps: int, warmup: int, timing: bool, workload: str):
    """Alg. 2 runs of the uneven-bond-cap multi-path workload; one step = one
    run from |0...0> to the end with top-M retention after every measurement."""
    import torch
    from inputs import circuits as C
    from inputs.randomness import branch_chi_draw
    from paper_2609_26516_amd import engine as E

    circ, prm = C.workload(workload)
    n, chi, M = prm["n"], prm["chi"], prm["max_branches"]
    choices = prm["chi_choices"]
    k = C.segment_max(circ) + 1
    chi_of = lambda path: branch_chi_draw(prm["seed"], path, choices)  # noqa: E731
    eng = E.Engine(0)
    eng.tuning(TUNE["enabled"])
    st = E.State(eng, prec, n, 2 * M, chi, 4, list(choices) + [chi], prm["init_seed"])
    info = {}

    def one_run():
        st.reset()
        res = E.run_multi_path(eng, st, circ, chi, k, 2, max_branches=M, chi_of=chi_of)
        info["branches"] = len(res["branches"])
        info["dropped"] = res["dropped"]
        info["F_mp"] = res["F_mp"]
        return res

    for _ in range(warmup):
        one_run()
    torch.cuda.synchronize()
    eng.timing(False)
    t0 = time.perf_counter()
    for _ in range(steps):
        one_run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = None
    if timing:   # one instrumented run after the timed ones
        eng.timing(True)
        eng.timing_stats(reset=True)
        one_run()
        torch.cuda.synchronize()
        stats = eng.timing_stats(reset=True)
        eng.timing(False)
    st.close()
    eng.close()
    return dt, stats, info


def roofline(stats, prec, counters=False, names=None):
    """counters: the HBM counters in TRAFFIC were taken on this workload;
    names: kernel names of the classes where they differ from KERNEL_NAMES."""
    launches, ms, flops, byts = stats
    dom = int(np.argmax(ms))
    avg_ms = ms[dom] / max(1, launches[dom])
    per_launch_flops = flops[dom] / max(1, launches[dom])
    per_launch_bytes = byts[dom] / max(1, launches[dom])
    if CLASSES[dom].startswith("gemm") or CLASSES[dom] == "measure":
        peak, _ = PEAK[prec]
        ach = per_launch_flops / (avg_ms * 1e-3) / 1e12
        rl = {"bound": "mfma", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
              "frac": round(ach / peak, 4), "traffic": None}
    elif CLASSES[dom] == "qr":
        ach = per_launch_flops / (avg_ms * 1e-3) / 1e12
        rl = {"bound": "alu", "achieved": round(ach, 3), "peak": 78.6, "unit": "TFLOP/s",
              "frac": round(ach / 78.6, 4), "traffic": None}
    else:
        ach = per_launch_bytes / (avg_ms * 1e-3) / 1e9
        rl = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None}
    tr = measured_traffic(CLASSES[dom]) if counters else None
    if tr is not None:
        rl["traffic"] = round(tr)
        rl["traffic_over_algorithmic"] = round(tr / max(1.0, per_launch_bytes), 2)
    rl["kernel"] = {**KERNEL_NAMES, **(names or {})}.get(CLASSES[dom], CLASSES[dom])
    rl["avg_launch_ms"] = round(avg_ms, 5)
    rl["launches"] = int(launches[dom])
    rl["time_share"] = round(ms[dom] / max(1e-12, sum(ms)), 4)
    rl["classes_ms"] = {c: round(v, 2) for c, v in zip(CLASSES, ms)}
    tot_f = sum(flops[:4])
    tot_ms = sum(ms[:4])
    rl["all_contraction_gemms"] = {"achieved_tflops": round(tot_f / (tot_ms * 1e-3) / 1e12, 3),
                                   "frac": round(tot_f / (tot_ms * 1e-3) / 1e12 / PEAK[prec][0], 4)}
    return rl


def run_large_chi(workload: str, steps: int, warmup: int, timing: bool, graphs: bool = False):
    """Single-path shots of the large-chi workload in the split-BF16 form,
    then the FP64 path replaying the first shot's outcomes; the two final
    states are compared by the FP64 overlap in one complex128 state."""
    import torch
    from inputs import circuits as C
    from inputs.randomness import shot_uniforms
    from paper_2609_26516_amd import capi
    from paper_2609_26516_amd import engine as E

    circ, prm = C.workload(workload)
    n, chi = prm["n"], prm["chi"]
    k = C.segment_max(circ) + 1
    w = mpo_bond_max(prm)
    nm = circ.n_measurements()
    u = lambda shot: shot_uniforms(prm["seed"], shot, nm)[None, :]  # noqa: E731
    eng = E.Engine(0)
    eng.graphs(graphs)
    st = E.State(eng, "bf16x3", n, 1, chi, w, [chi], prm["init_seed"])
    for i in range(warmup):
        st.release(E.run_single_path(eng, st, circ, 1, chi, k, 2, uniforms=u(10_000 + i))["ids"])
    torch.cuda.synchronize()
    eng.timing(False)
    t0 = time.perf_counter()
    first = None
    for i in range(steps):
        r = E.run_single_path(eng, st, circ, 1, chi, k, 2, uniforms=u(i))
        if first is None:
            first = (r, st.export(int(r["ids"][0])))
        st.release(r["ids"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = None
    if timing:   # one instrumented shot after the timed ones
        eng.timing(True)
        eng.timing_stats(reset=True)
        st.release(E.run_single_path(eng, st, circ, 1, chi, k, 2, uniforms=u(steps))["ids"])
        torch.cuda.synchronize()
        stats = eng.timing_stats(reset=True)
        eng.timing(False)
    st.close()
    r_bf, mps_bf = first
    st64 = E.State(eng, "c128", n, 2, chi, w, [chi], prm["init_seed"])
    t1 = time.perf_counter()
    r64 = E.run_single_path(eng, st64, circ, 1, chi, k, 2, outcomes=r_bf["outcomes"])
    torch.cuda.synchronize()
    dt64 = time.perf_counter() - t1
    i64 = int(r64["ids"][0])
    other = st64.alloc(1)[0]
    capi.dcs_import_mps(st64.h, other, chi, mps_bf, eng.stream())
    ov = capi.dcs_overlap(st64.h, i64, other, eng.stream())
    na = capi.dcs_overlap(st64.h, i64, i64, eng.stream()).real
    nb = capi.dcs_overlap(st64.h, other, other, eng.stream()).real
    st64.close()
    eng.close()
    cmp = {"reference": "GPU FP64 path (complex128, FP64 MFMA) replaying the outcomes",
           "state_fidelity_error": float(abs(1 - abs(ov) ** 2 / (na * nb))),
           "max_abs_probability_error": float(np.max(np.abs(r_bf["p0s"][0] - r64["p0s"][0]))),
           "fidelity_estimate": float(r_bf["F"][0]), "fidelity_estimate_fp64": float(r64["F"][0])}
    return dt, dt64, stats, cmp


def _oracle_shot_sample(rounds: int):
    """Wall time of the FP64 oracle (numpy, complex128) on a bounded sample of
    one shot of the headline workload: its first `rounds` measurement rounds
    (each one compression step and 4 measurements), then the compression of
    the last round's feed-forward gates, the one compression step a shot has
    beyond its rounds.  Returns (seconds of the rounds, seconds of the final
    compression)."""
    from inputs import circuits as C
    from inputs.randomness import shot_uniforms
    from oracle import dynamic as OD

    circ, prm = C.workload(WORKLOAD)
    n, chi = prm["n"], prm["chi"]
    ops, seen = [], 0
    for op in circ.ops:
        ops.append(op)
        if isinstance(op, C.Measure):
            seen += 1
            if seen == rounds * prm["meas_per_round"]:
                break
    sub = C.Circuit(circ.n_qubits, circ.n_bits, ops, name="prefix")
    sim = OD.Simulator(n, chi, C.segment_max(circ), 2, prm["init_seed"])
    sim.bra_init(chi)   # starting guess built before the clock starts
    u = shot_uniforms(prm["seed"], 0, circ.n_measurements())
    t0 = time.perf_counter()
    r = OD.run_single_path(sub, sim, uniforms=u)
    t_rounds = time.perf_counter() - t0
    # the last round's feed-forward gates, all of them (an upper bound of what fires)
    last = max(i for i, op in enumerate(circ.ops) if isinstance(op, C.Measure))
    tail = [(tuple(op.gate.qubits), op.gate.mat) for op in circ.ops[last + 1:]
            if isinstance(op, C.CGate)]
    t0 = time.perf_counter()
    sim.compress(r["mps"], tail, chi)
    t_final = time.perf_counter() - t0
    return t_rounds, t_final


def tree_overlap(topo, a, b) -> complex:
    """<a|b> of two tree states (node tensors in node order) by contraction
    from the leaves up: E_v = conj(A_v) B_v over v's lower legs, the children's
    E's inserted."""
    E = [None] * topo.N
    for v in reversed(range(topo.N)):
        x = b[v]
        for i, c in enumerate(topo.kids[v]):
            # replace lower leg i + 1 (ket index) by the bra index through E_c
            x = np.moveaxis(np.tensordot(E[c], x, axes=([1], [i + 1])), 0, i + 1)
        lower = tuple(range(1, a[v].ndim))
        E[v] = np.tensordot(a[v].conj(), x, axes=(lower, lower))
    return complex(E[0].reshape(-1)[0])


def run_gpu_tree(prec: str, shots: int, steps: int, warmup: int, timing: bool, workload: str,
                 sampled=(), outcomes=None):
    """Single-path shots on the tree tensor network state: W warm-up steps, K
    timed steps without instrumentation, one instrumented step with timing;
    `outcomes` replays given outcome rows instead of sampling (one step)."""
    import torch
    from inputs import circuits as C
    from inputs.randomness import shot_uniforms
    from paper_2609_26516_amd import engine as E

    circ, prm = C.workload(workload)
    chi, levels = prm["chi"], prm["tree"]
    k = C.segment_max(circ) + 1
    eng = E.Engine(0)
    eng.tuning(TUNE["enabled"])
    st = E.TreeState(eng, prec, levels, shots, chi, 16, [chi], prm["init_seed"], circ=circ)
    nm = circ.n_measurements()
    samples = {}

    def one_step(step, export=False):
        if outcomes is not None:
            res = E.run_single_path(eng, st, circ, shots, chi, k, 2, outcomes=outcomes)
        else:
            u = np.stack([shot_uniforms(prm["seed"], step * shots + s, nm) for s in range(shots)])
            res = E.run_single_path(eng, st, circ, shots, chi, k, 2, uniforms=u)
        if export:
            for s in sampled:
                samples[s] = {"outcomes": res["outcomes"][s].copy(), "p0s": res["p0s"][s].copy(),
                              "F": float(res["F"][s]), "state": st.export(int(res["ids"][s]))}
        st.release(res["ids"])
        return res

    for w in range(warmup):
        one_step(10_000 + w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        one_step(s, export=(s == steps - 1 and not timing))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = None
    if timing:
        eng.timing(True)
        eng.timing_stats(reset=True)
        one_step(steps, export=True)
        torch.cuda.synchronize()
        stats = eng.timing_stats(reset=True)
        eng.timing(False)
    topo = st.topo
    st.close()
    eng.close()
    return dt, stats, samples, topo


def tree_precision_vs_fp64(workload: str, samples: dict):
    """Sampled complex64 tree shots against the complex128 tree path replaying
    their outcomes: every p_0 and the state-fidelity error from the FP64
    overlap of the exported states."""
    shots = sorted(samples)
    outs = np.stack([samples[s]["outcomes"] for s in shots])
    _, _, ref, topo = run_gpu_tree("c128", len(shots), 1, 0, False, workload,
                                   sampled=range(len(shots)), outcomes=outs)
    dp, fe = [], []
    for i, s in enumerate(shots):
        a, b = samples[s]["state"], ref[i]["state"]
        ov = tree_overlap(topo, a, b)
        na, nb = tree_overlap(topo, a, a).real, tree_overlap(topo, b, b).real
        fe.append(float(abs(1 - abs(ov) ** 2 / (na * nb))))
        dp.append(float(np.max(np.abs(samples[s]["p0s"] - ref[i]["p0s"]))))
    return {"reference": "GPU FP64 tree path (complex128) replaying the outcomes",
            "shots": shots, "max_abs_probability_error": max(dp),
            "state_fidelity_error": max(fe),
            "targets": {"max_abs_probability_error": 1e-6, "state_fidelity_error": 1e-6}}


def cpu_baseline(rounds: int, rounds_multi: int):
    """The oracle timed in this process on a bounded sample of one shot (first
    rounds plus the final compression), scaled to a whole shot: 10 rounds and
    the final compression (all rounds cost the same: the oracle's bond dims
    are fixed).  The value is single-threaded (BLAS limited to one thread);
    the same sample on every BLAS thread the process has is given beside it."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from inputs import circuits as C

    _, prm = C.workload(WORKLOAD)
    total_rounds = prm["depth"] // prm["layers_per_round"]

    def rate(t_rounds, t_final, r):
        return 1.0 / (t_rounds / r * total_rounds + t_final)

    with threadpool_limits(limits=1, user_api="blas"):
        t1, f1 = _oracle_shot_sample(rounds)
    threads = sum(i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas")
    tm, fm = _oracle_shot_sample(rounds_multi)
    return {"value": round(rate(t1, f1, rounds), 6), "unit": "shots/s", "cores": 1,
            "kind": "oracle",
            "sample": f"first {rounds} of {total_rounds} rounds (compression + 4 measurements "
                      f"each, {t1:.1f} s) and the final compression ({f1:.1f} s) of one shot, "
                      f"one BLAS thread; shot time = {total_rounds}/{rounds} x rounds + final",
            "all_threads": {"value": round(rate(tm, fm, rounds_multi), 6), "unit": "shots/s",
                            "cores": int(threads or 1),
                            "sample": f"first {rounds_multi} rounds ({tm:.1f} s) and the final "
                                      f"compression ({fm:.1f} s), one process, "
                                      f"{int(threads or 1)} BLAS threads"}}


def copy_calibration(nbytes: int = 1 << 30, reps: int = 5):
    """A plain copy kernel of known size: `nbytes` read and written per launch."""
    import torch
    from paper_2609_26516_amd import capi
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream().cuda_stream
    capi.dcs_test_copy(src.data_ptr(), dst.data_ptr(), nbytes, 1, stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    capi.dcs_test_copy(src.data_ptr(), dst.data_ptr(), nbytes, reps, stream)
    b.record()
    torch.cuda.synchronize()
    if not bool(torch.equal(src, dst)):
        raise RuntimeError("copy kernel produced wrong data")
    ms = a.elapsed_time(b) / reps
    return {"copy_bytes_per_launch": nbytes, "launches": reps + 1, "avg_ms": round(ms, 4),
            "GB_per_s_read_plus_write": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shots", type=int, default=256)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--cpu-rounds", type=int, default=1,
                    help="measurement rounds of the single-threaded oracle sample")
    ap.add_argument("--cpu-rounds-multi", type=int, default=2,
                    help="measurement rounds of the all-threads oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the (untimed) complex128 replay of sampled shots")
    ap.add_argument("--workload", default="sp40",
                    choices=sorted(SINGLE_PATH) + sorted(MULTI_PATH) + sorted(LARGE_CHI)
                    + sorted(TREE))
    ap.add_argument("--graphs", action="store_true",
                    help="replay recurring compression steps from HIP graphs (no per-kernel timing)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--no-tune", action="store_true",
                    help="fixed 64x64 contraction tiles instead of the online autotuner")
    ap.add_argument("--save-tiles", default=None, help="write the tuned tile table (JSON) here")
    args = ap.parse_args()
    TUNE["enabled"] = not args.no_tune
    TUNE["save"] = args.save_tiles
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(independent shots would shard across GPUs without communication)",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        print(json.dumps(copy_calibration()))
        return
    if args.workload in LARGE_CHI:
        wl = LARGE_CHI[args.workload]
        dt, dt64, stats, cmp = run_large_chi(wl, args.steps, args.warmup, not args.graphs,
                                             graphs=args.graphs)
        out = {"metric": "shots/s (split-BF16 form, chi=1024), FP64 path beside it",
               "value": round(args.steps / dt, 5), "unit": "shots/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": round(1e3 * dt / args.steps, 1), "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3",
               "data": "synthetic: seeded Haar brickwork dynamic circuit",
               "config": {"workload": wl, "shots_per_step": 1, "graphs": args.graphs},
               "roofline": roofline(stats, "bf16x3", names={
                   "qr": "qrt_q1_kernel + qrt_v_kernel + qrl_wpart_kernel + qrl_update_kernel (m > 512), "
                         "qrs_* / qr_left_kernel (m <= 512)",
                   "gemm_nn": "gemm_bf16x3_kernel<0, 0>", "gemm_nt": "gemm_bf16x3_kernel<0, 1>",
                   "gemm_cn": "gemm_bf16x3_kernel<2, 0>", "gemm_jt": "gemm_bf16x3_kernel<3, 1>"})
               if stats else None,
               "fp64_path": {"value": round(1 / dt64, 5), "unit": "shots/s", "dtype": "c128",
                             "steps": 1, "warmup": 0,
                             "note": "one replay shot on a fresh engine (tile tuning included)"},
               "precision_vs_fp64": cmp}
        print(json.dumps(out))
        return
    if args.workload in TREE:
        wl = TREE[args.workload]
        shots = args.shots if args.shots != 256 else 64
        dt, stats, samples, _ = run_gpu_tree("c64", shots, args.steps, args.warmup, True, wl,
                                             sampled=(0, shots - 1))
        out = {"metric": "shots/s (tree tensor network [1,3,9,27], chi=32, FP32-MFMA form)",
               "value": round(shots * args.steps / dt, 4), "unit": "shots/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": round(1e3 * dt / args.steps, 2), "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "c64",
               "data": "synthetic: seeded Haar brickwork dynamic circuit",
               "config": {"workload": wl, "shots_per_step": shots, "tree": [1, 3, 9, 27],
                          "chi": 32},
               "roofline": roofline(stats, "c64", names={
                   "gemm_nn": "gemm_kernel (tree contractions, A B)",
                   "gemm_nt": "gemm_kernel (tree contractions, A B^T)",
                   "gemm_cn": "gemm_kernel (tree contractions, A^H B)",
                   "gemm_jt": "gemm_kernel (tree contractions, conj(A) B^T)",
                   "qr": "qr_left_kernel / qrl_* (node QR)",
                   "other": "permute_kernel (leg transpositions)"}),
               "precision_vs_fp64": None if args.no_precision
               else tree_precision_vs_fp64(wl, samples)}
        if not args.no_fp64:
            dt64, _, _, _ = run_gpu_tree("c128", shots, args.fp64_steps, args.warmup, False, wl)
            out["fp64_path"] = {"value": round(shots * args.fp64_steps / dt64, 4),
                                "unit": "shots/s", "steps": args.fp64_steps,
                                "warmup": args.warmup, "dtype": "c128"}
        print(json.dumps(out))
        return
    if args.workload in MULTI_PATH:
        wl = MULTI_PATH[args.workload]
        dt, stats, info = run_gpu_multipath("c64", args.steps, args.warmup, True, wl)
        out = {"metric": "multi-path runs/s (grouped FP32-MFMA form, uneven chi 32..256, M=64)",
               "value": round(args.steps / dt, 5), "unit": "runs/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": round(1e3 * dt / args.steps, 2), "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "c64",
               "data": "synthetic: seeded Haar brickwork dynamic circuit",
               "config": {"workload": wl, **info}, "roofline": roofline(stats, "c64")}
        if not args.no_fp64:
            dt64, _, _ = run_gpu_multipath("c128", args.fp64_steps, args.warmup, False, wl)
            out["fp64_path"] = {"value": round(args.fp64_steps / dt64, 5), "unit": "runs/s",
                                "steps": args.fp64_steps, "warmup": args.warmup,
                                "dtype": "c128"}
        print(json.dumps(out))
        return
    if args.workload != "sp40":
        wl = SINGLE_PATH[args.workload]
        dt, stats, fids, _ = run_gpu("c64", args.shots, args.steps, args.warmup,
                                     not args.graphs, wl, graphs=args.graphs)
        out = {"metric": "shots/s (batched FP32-MFMA form)", "value": round(args.shots * args.steps / dt, 4),
               "unit": "shots/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": round(1e3 * dt / args.steps, 2), "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "c64",
               "data": "synthetic: seeded Haar brickwork dynamic circuit",
               "config": {"workload": wl, "shots_per_step": args.shots, "graphs": args.graphs},
               "roofline": roofline(stats, "c64") if stats else None,
               "mean_fidelity_estimate": round(float(np.mean(fids)), 6)}
        if not args.no_fp64:
            dt64, _, _, _ = run_gpu("c128", args.shots, args.fp64_steps, args.warmup, False, wl)
            out["fp64_path"] = {"value": round(args.shots * args.fp64_steps / dt64, 4),
                                "unit": "shots/s", "steps": args.fp64_steps,
                                "warmup": args.warmup, "dtype": "c128"}
        print(json.dumps(out))
        return
    sampled = (0, args.shots - 1)
    dt, stats, fids, samples = run_gpu("c64", args.shots, args.steps, args.warmup, timing=True,
                                       sampled=sampled)
    value = args.shots * args.steps / dt
    out = {
        "metric": "shots/s (batched FP32-MFMA form, chi=256), FP64 path beside it",
        "value": round(value, 4), "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic: seeded Haar brickwork dynamic circuit",
        "config": {"workload": "n40_depth20_chi256_4meas_per_2layers_single_path",
                   "shots_per_step": args.shots, "n_qubits": 40, "depth": 20, "chi": 256,
                   "sweeps": 2, "precision": "complex64 contractions, FP64 QR/norms"},
        "roofline": roofline(stats, "c64", counters=args.shots == 256),
        "mean_fidelity_estimate": round(float(np.mean(fids)), 6),
    }
    out["roofline"]["measured_on"] = ("one instrumented step after the timed ones "
                                      "(HIP events around every launch)")
    if not args.no_precision:
        out["precision_vs_fp64"] = precision_vs_fp64(WORKLOAD, samples)
    if not args.no_fp64:
        dt64, _, _, _ = run_gpu("c128", args.shots, args.fp64_steps, args.warmup, timing=False)
        out["fp64_path"] = {"value": round(args.shots * args.fp64_steps / dt64, 4),
                            "unit": "shots/s", "steps": args.fp64_steps, "warmup": args.warmup,
                            "dtype": "c128"}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_rounds, args.cpu_rounds_multi)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
