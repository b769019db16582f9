"""Drivers of the paper's validation studies, run on the library (Sec. V).

* path distributions of the multi-path strategy (Alg. 2) for teleportation
  (Sec. V-A, four paths; eight with Bob's qubit measured) and the dynamic GHZ
  preparation (Sec. V-B, 2^r equiprobable paths);
* the total variation distance between the single-path strategy's empirical
  path frequencies over N runs (Alg. 1) and the multi-path probabilities, as a
  function of N, mean and spread over repetitions (the single-path panels of
  the teleportation and GHZ figures);
* the GHZ distance when at most M branches are kept, without and with
  renormalisation of the kept probabilities (the branch-cap panel);
* wall time and state memory of the multi-path GHZ run against the number of
  qubits (the scaling figure);
* fidelity, runtime and state memory against depth for seeded random dynamic
  circuits (distant gate pairs, measured subsets, parity-conditioned gates),
  single path over several runs and multi path with a branch cap, for each
  bond cap (Sec. V-C, MPS columns of its figure and table).

Every tensor operation goes through engine.py and libdcs.so on the GPU; this
module only groups shots, counts paths and forms distances.

    python -m paper_2609_26516_amd.validation [--study teleport|ghz|cap|scaling|random]

prints one JSON line per study.
"""
from __future__ import annotations

import argparse
import json
import time
from collections import Counter
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

Path = Tuple[int, ...]


def tvd(p: Dict[Path, float], q: Dict[Path, float]) -> float:
    """Total variation distance 1/2 sum |p - q| over the union of the paths
    (a path missing from one side has probability 0 there)."""
    keys = set(p) | set(q)
    return 0.5 * float(sum(abs(p.get(k, 0.0) - q.get(k, 0.0)) for k in keys))


def frequencies(paths: Sequence[Path]) -> Dict[Path, float]:
    """Empirical distribution of a list of outcome tuples."""
    n = len(paths)
    if n == 0:
        return {}
    return {k: c / n for k, c in Counter(paths).items()}


def tvd_curve(paths: Sequence[Path], exact: Dict[Path, float], ns: Sequence[int],
              reps: int) -> List[Dict]:
    """The runs are split into `reps` consecutive groups of max(ns); for each N
    the first N runs of every group give one empirical distribution and one
    distance to `exact`.  Returns mean, sample standard deviation and the
    per-repetition distances for every N."""
    nmax = max(ns)
    if len(paths) < nmax * reps:
        raise ValueError("need max(ns) * reps runs")
    out = []
    for n in ns:
        d = [tvd(frequencies(paths[r * nmax:r * nmax + n]), exact) for r in range(reps)]
        out.append({"N": int(n), "tvd_mean": float(np.mean(d)),
                    "tvd_sd": float(np.std(d, ddof=1)) if reps > 1 else 0.0,
                    "tvd": [float(x) for x in d]})
    return out


def _max_paths(circ) -> int:
    """Upper bound on the live branches of an uncapped multi-path run: 2^r for
    the dynamic GHZ circuit (its resets have one possible outcome), else two
    per measurement."""
    r = circ.meta.get("r") if circ.meta else None
    return 2 ** int(r) if r is not None else 2 ** circ.n_measurements()


def _state(eng, circ, precision: str, chi: int, capacity: int, init_seed: int):
    from .engine import State
    return State(eng, precision, circ.n_qubits, capacity, chi, 4, [chi], init_seed)


def path_distribution(eng, circ, chi: int, k: int, n_sweeps: int = 2, precision: str = "c128",
                      max_branches: Optional[int] = None, capacity: Optional[int] = None,
                      init_seed: int = 7) -> Dict:
    """Multi-path run: {path: p} of the kept branches, the dropped mass and
    the path-weighted fidelity."""
    from .engine import run_multi_path
    live = _max_paths(circ) if max_branches is None else min(_max_paths(circ), max_branches)
    cap = capacity or 2 * live + 2   # a measurement holds parents and new children
    st = _state(eng, circ, precision, chi, cap, init_seed)
    try:
        res = run_multi_path(eng, st, circ, chi, k, n_sweeps, max_branches=max_branches)
    finally:
        st.close()
    return {"p": {tuple(int(m) for m in b["path"]): float(b["p"]) for b in res["branches"]},
            "dropped": float(res["dropped"]), "F_mp": float(res["F_mp"])}


def single_path_runs(eng, circ, runs: int, chi: int, k: int, n_sweeps: int = 2,
                     precision: str = "c128", seed: int = 1, init_seed: int = 7) -> List[Path]:
    """Outcome tuples of `runs` independent single-path runs, advanced in one
    batch; run s draws its outcomes from the seeded uniforms of shot s."""
    from inputs.randomness import shot_uniforms
    from .engine import run_single_path
    nm = circ.n_measurements()
    u = np.stack([shot_uniforms(seed, s, nm) for s in range(runs)]) if nm else None
    st = _state(eng, circ, precision, chi, runs, init_seed)
    try:
        res = run_single_path(eng, st, circ, runs, chi, k, n_sweeps, uniforms=u)
    finally:
        st.close()
    return [tuple(int(m) for m in row) for row in res["outcomes"]]


def tvd_vs_shots(eng, circ, ns: Sequence[int], reps: int, chi: int, k: int, n_sweeps: int = 2,
                 precision: str = "c128", seed: int = 1) -> Dict:
    """Single-path distance to the multi-path distribution against the number
    of runs N (one batch of max(ns) * reps runs)."""
    exact = path_distribution(eng, circ, chi, k, n_sweeps, precision)["p"]
    paths = single_path_runs(eng, circ, max(ns) * reps, chi, k, n_sweeps, precision, seed)
    return {"exact": {"".join(map(str, key)): v for key, v in sorted(exact.items())},
            "curve": tvd_curve(paths, exact, ns, reps)}


def ghz_tvd_vs_cap(eng, n: int, caps: Iterable[int], chi: int = 4, k: int = 25,
                   n_sweeps: int = 2, precision: str = "c128") -> Dict:
    """Distance of the capped multi-path GHZ distribution to the uncapped one,
    raw (dropped mass missing) and with the kept probabilities renormalised."""
    from inputs.circuits import ghz_dynamic
    circ = ghz_dynamic(n)
    exact = path_distribution(eng, circ, chi, k, n_sweeps, precision)["p"]
    rows = []
    for m in caps:
        r = path_distribution(eng, circ, chi, k, n_sweeps, precision, max_branches=int(m))
        kept = r["p"]
        tot = sum(kept.values())
        rows.append({"M": int(m), "kept": len(kept), "dropped": r["dropped"],
                     "tvd_raw": tvd(kept, exact),
                     "tvd_renormalised": tvd({p: v / tot for p, v in kept.items()}, exact)})
    return {"n": n, "paths": len(exact), "rows": rows}


def ghz_scaling(eng, ns: Sequence[int], chi: int = 4, k: int = 25, n_sweeps: int = 2,
                precision: str = "c128", repeats: int = 3) -> List[Dict]:
    """Wall time (median of `repeats` runs, host driver included) and state
    buffer size of the uncapped multi-path GHZ run for each n."""
    import torch
    from inputs.circuits import ghz_dynamic
    from .engine import run_multi_path
    rows = []
    for n in ns:
        circ = ghz_dynamic(n)
        cap = 2 * _max_paths(circ) + 2
        st = _state(eng, circ, precision, chi, cap, 7)
        times = []
        try:
            for _ in range(repeats):
                st.reset()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = run_multi_path(eng, st, circ, chi, k, n_sweeps)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            rows.append({"n": int(n), "paths": len(res["branches"]),
                         "seconds": float(np.median(times)), "state_bytes": int(st.nbytes),
                         "slots": int(cap)})
        finally:
            st.close()
    return rows


def random_circuit_study(eng, n: int, depths: Sequence[int], chis: Sequence[int],
                         circuits: int = 3, runs: int = 10, max_branches: int = 8, k: int = 20,
                         n_sweeps: int = 2, precision: str = "c128", seed: int = 1,
                         mpo_bond_max: int = 16) -> List[Dict]:
    """For each depth, bond cap and seeded circuit (inputs.circuits.random_dynamic
    with seed c = 0..circuits-1): `runs` single-path runs in one batch (their
    mean fidelity estimate, Alg. 1) and one multi-path run capped at
    `max_branches` (probability-weighted fidelity, Alg. 2).  Rows give mean
    and standard deviation over the circuits, the wall time of the batch and
    of the multi-path run, and the state memory in use (one slot per run; the
    slots the multi-path run needs)."""
    import torch
    from inputs.circuits import random_dynamic
    from inputs.randomness import shot_uniforms
    from .engine import State, run_multi_path, run_single_path
    rows = []
    for depth in depths:
        for chi in chis:
            f_sp, f_mp, t_sp, t_mp, m_sp, m_mp = [], [], [], [], [], []
            for c in range(circuits):
                circ = random_dynamic(n, depth, c)
                nm = circ.n_measurements()
                u = (np.stack([shot_uniforms(seed, s, nm) for s in range(runs)]) if nm
                     else None)
                st = State(eng, precision, n, runs, chi, mpo_bond_max, [chi], 7 + c)
                try:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    res = run_single_path(eng, st, circ, runs, chi, k, n_sweeps, uniforms=u)
                    torch.cuda.synchronize()
                    t_sp.append(time.perf_counter() - t0)
                    f_sp.append(float(np.mean(res["F"])))
                    m_sp.append(st.nbytes / runs)
                finally:
                    st.close()
                cap = 2 * max_branches + 2
                st = State(eng, precision, n, cap, chi, mpo_bond_max, [chi], 7 + c)
                try:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    res = run_multi_path(eng, st, circ, chi, k, n_sweeps,
                                         max_branches=max_branches)
                    torch.cuda.synchronize()
                    t_mp.append(time.perf_counter() - t0)
                    f_mp.append(float(res["F_mp"]))
                    m_mp.append(st.nbytes)
                finally:
                    st.close()
            sd = (lambda x: float(np.std(x, ddof=1)) if len(x) > 1 else 0.0)  # noqa: E731
            rows.append({"depth": int(depth), "chi": int(chi),
                         "F_sp": float(np.mean(f_sp)), "F_sp_sd": sd(f_sp),
                         "F_mp": float(np.mean(f_mp)), "F_mp_sd": sd(f_mp),
                         "seconds_sp": float(np.mean(t_sp)), "seconds_mp": float(np.mean(t_mp)),
                         "bytes_per_run_sp": float(np.mean(m_sp)),
                         "bytes_mp": float(np.mean(m_mp)), "F_sp_each": f_sp,
                         "F_mp_each": f_mp})
    return rows


def main(argv: Optional[Sequence[str]] = None) -> None:
    from inputs.circuits import ghz_dynamic, teleportation
    from .engine import Engine
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--study", choices=["teleport", "ghz", "cap", "scaling", "random", "all"],
                    default="all")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--precision", default="c128")
    args = ap.parse_args(argv)
    eng = Engine(0)
    ns = [1, 2, 4, 8, 16, 32]
    try:
        if args.study in ("teleport", "all"):
            for fm in (False, True):
                r = tvd_vs_shots(eng, teleportation(fm), ns, args.reps, 2, 20,
                                 precision=args.precision)
                print(json.dumps({"study": "teleport" + ("_bob" if fm else ""), **r}))
        if args.study in ("ghz", "all"):
            for n in (5, 9, 13):
                r = tvd_vs_shots(eng, ghz_dynamic(n), ns + [64, 128], args.reps, 4, 25,
                                 precision=args.precision)
                print(json.dumps({"study": f"ghz{n}_single_path", **r}))
        if args.study in ("cap", "all"):
            for n in (11, 13, 15, 17):
                print(json.dumps({"study": "ghz_cap",
                                  **ghz_tvd_vs_cap(eng, n, [1, 4, 16, 64, 256],
                                                   precision=args.precision)}))
        if args.study in ("scaling", "all"):
            print(json.dumps({"study": "ghz_scaling",
                              "rows": ghz_scaling(eng, [5, 7, 9, 11, 13, 15, 17],
                                                  precision=args.precision)}))
        if args.study in ("random", "all"):
            print(json.dumps({"study": "random_dynamic_n27",
                              "rows": random_circuit_study(eng, 27, range(2, 9), [8, 16, 32],
                                                           precision=args.precision)}))
    finally:
        eng.close()


if __name__ == "__main__":
    main()
