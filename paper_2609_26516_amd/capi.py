"""ctypes binding of libdcs.so: the C functions of include/dcs.h under the same
names, with argument marshalling only (numpy arrays for host arrays, integers
for device pointers and hipStream_t handles).  Every non-zero status raises
DcsError carrying the library's message.  There is no fallback: if the
library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_longlong, c_size_t, c_void_p

import numpy as np
# PyTorch provides the device memory and streams; loading it first makes
# libdcs.so bind to the same HIP runtime (both carry libamdhip64.so.7), so the
# process holds exactly one runtime whatever the caller imported first.
import torch  # noqa: F401

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdcs.so")

DCS_OK, DCS_EINVAL, DCS_EQUBITS, DCS_EZEROPROB = 0, -1, -2, -3
DCS_ENONLOCAL = DCS_EQUBITS   # former name
DCS_ECAPACITY, DCS_ENOMEM, DCS_EHIP, DCS_ESTATE, DCS_ENUMERIC = -4, -5, -6, -7, -8
DCS_C128, DCS_C64, DCS_BF16X3 = 0, 1, 2
STATUS_NAMES = {0: "DCS_OK", -1: "DCS_EINVAL", -2: "DCS_EQUBITS", -3: "DCS_EZEROPROB",
                -4: "DCS_ECAPACITY", -5: "DCS_ENOMEM", -6: "DCS_EHIP", -7: "DCS_ESTATE",
                -8: "DCS_ENUMERIC"}
EXPORTED = [
    "dcs_last_error", "dcs_version", "dcs_ctx_create", "dcs_ctx_destroy", "dcs_ctx_set_timing",
    "dcs_ctx_timing", "dcs_ctx_set_graphs", "dcs_ctx_set_tuning", "dcs_ctx_tuning_save",
    "dcs_ctx_tuning_load", "dcs_state_bytes", "dcs_state_create", "dcs_state_destroy",
    "dcs_state_set_init", "dcs_state_set_warm_start", "dcs_branch_init_zero", "dcs_branch_set_chi", "dcs_branch_release",
    "dcs_branch_dims", "dcs_chunk_compile", "dcs_gate_rank", "dcs_chunk_bonds", "dcs_chunk_export", "dcs_chunk_destroy",
    "dcs_compress_step", "dcs_measure_prob", "dcs_measure_sample_collapse", "dcs_collapse", "dcs_topk_by_weight", "dcs_prune_adaptive",
    "dcs_overlap", "dcs_overlap_noalloc", "dcs_export_mps", "dcs_import_mps",
    "dcs_tree_n_nodes", "dcs_tree_state_bytes", "dcs_tree_create", "dcs_tree_destroy",
    "dcs_tree_set_init", "dcs_tree_branch_init_zero", "dcs_tree_branch_set_chi",
    "dcs_tree_branch_release", "dcs_tree_chunk_compile", "dcs_tchunk_destroy", "dcs_tchunk_bonds",
    "dcs_tree_chunk_scratch", "dcs_tree_compress_step", "dcs_tree_measure_prob",
    "dcs_tree_collapse", "dcs_tree_export",
]
EXPORTED_TESTING = ["dcs_test_gemm", "dcs_test_mpo", "dcs_test_qr", "dcs_test_copy",
                    "dcs_test_permute", "dcs_test_permute_dev", "dcs_test_gemm_gate",
                    "dcs_test_permute_plan"]


class DcsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2609_26516_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)
_P = c_void_p
_IP = POINTER(c_int)
_DP = POINTER(c_double)

_SIGS = {
    "dcs_last_error": (ctypes.c_char_p, []),
    "dcs_version": (c_int, []),
    "dcs_ctx_create": (c_int, [POINTER(c_void_p), c_int]),
    "dcs_ctx_destroy": (c_int, [_P]),
    "dcs_ctx_set_timing": (c_int, [_P, c_int]),
    "dcs_ctx_set_graphs": (c_int, [_P, c_int]),
    "dcs_ctx_set_tuning": (c_int, [_P, c_int, c_int]),
    "dcs_ctx_tuning_save": (c_int, [_P, ctypes.c_char_p]),
    "dcs_ctx_tuning_load": (c_int, [_P, ctypes.c_char_p]),
    "dcs_ctx_timing": (c_int, [_P, POINTER(c_longlong), _DP, _DP, _DP, c_int]),
    "dcs_state_bytes": (c_int, [c_int, c_int, c_int, c_int, c_int, c_int, POINTER(c_size_t)]),
    "dcs_state_create": (c_int, [_P, POINTER(c_void_p), c_int, c_int, c_int, c_int, c_int, c_int,
                                 _P, c_size_t, _P]),
    "dcs_state_destroy": (c_int, [_P]),
    "dcs_state_set_init": (c_int, [_P, c_int, _DP, _P]),
    "dcs_branch_init_zero": (c_int, [_P, c_int, _IP, _IP, _P]),
    "dcs_branch_set_chi": (c_int, [_P, c_int, _IP, _IP]),
    "dcs_branch_release": (c_int, [_P, c_int, _IP]),
    "dcs_branch_dims": (c_int, [_P, c_int, _IP]),
    "dcs_chunk_compile": (c_int, [_P, POINTER(c_void_p), c_int, c_int, _IP, _IP, _DP]),
    "dcs_chunk_bonds": (c_int, [_P, _IP]),
    "dcs_gate_rank": (c_int, [_DP, _IP]),
    "dcs_chunk_export": (c_int, [_P, _DP, c_size_t]),
    "dcs_chunk_destroy": (c_int, [_P]),
    "dcs_state_set_warm_start": (c_int, [_P, c_int, c_double]),
    "dcs_compress_step": (c_int, [_P, c_int, _IP, POINTER(c_void_p), c_int, _DP, _P]),
    "dcs_measure_prob": (c_int, [_P, c_int, _IP, _IP, _DP, _P]),
    "dcs_measure_sample_collapse": (c_int, [_P, c_int, _IP, _IP, _P, c_double, _P, _P, _P]),
    "dcs_collapse": (c_int, [_P, c_int, _IP, _IP, _IP, _IP, c_double, _DP, _P]),
    "dcs_topk_by_weight": (c_int, [c_int, _DP, c_int, _IP, _IP, _DP]),
    "dcs_prune_adaptive": (c_int, [c_int, _DP, c_int, c_double, c_double, _IP, _IP, _DP]),
    "dcs_overlap": (c_int, [_P, c_int, c_int, _DP, _P]),
    "dcs_overlap_noalloc": (c_int, [_P, c_int, c_int, _P, _P]),
    "dcs_export_mps": (c_int, [_P, c_int, _DP, c_size_t, _IP, _P]),
    "dcs_import_mps": (c_int, [_P, c_int, c_int, _DP, _IP, _P]),
    "dcs_tree_n_nodes": (c_int, [_IP, c_int, _IP]),
    "dcs_tree_state_bytes": (c_int, [c_int, c_int, _IP, c_int, c_int, c_int, c_size_t, c_int,
                                     POINTER(c_size_t)]),
    "dcs_tree_create": (c_int, [_P, POINTER(c_void_p), c_int, c_int, _IP, c_int, c_int, c_int,
                                c_size_t, c_int, _P, c_size_t, _P]),
    "dcs_tree_destroy": (c_int, [_P]),
    "dcs_tree_set_init": (c_int, [_P, c_int, _DP, _P]),
    "dcs_tree_branch_init_zero": (c_int, [_P, c_int, _IP, _IP, _P]),
    "dcs_tree_branch_set_chi": (c_int, [_P, c_int, _IP, _IP]),
    "dcs_tree_branch_release": (c_int, [_P, c_int, _IP]),
    "dcs_tree_chunk_compile": (c_int, [_P, POINTER(c_void_p), c_int, _IP, c_int, _IP, _IP, _DP]),
    "dcs_tchunk_destroy": (c_int, [_P]),
    "dcs_tchunk_bonds": (c_int, [_P, _IP, c_int]),
    "dcs_tree_chunk_scratch": (c_int, [_P, c_int, c_int, POINTER(c_size_t)]),
    "dcs_tree_compress_step": (c_int, [_P, c_int, _IP, POINTER(c_void_p), c_int, _DP, _P]),
    "dcs_tree_measure_prob": (c_int, [_P, c_int, _IP, _IP, _DP, _P]),
    "dcs_tree_collapse": (c_int, [_P, c_int, _IP, _IP, _IP, _IP, c_double, _DP, _P]),
    "dcs_tree_export": (c_int, [_P, c_int, _DP, c_size_t, _IP, _P]),
    "dcs_test_gemm": (c_int, [c_int] * 11 + [_DP, _DP, _DP, _P]),
    "dcs_test_mpo": (c_int, [c_int] * 6 + [_DP, _DP, _DP, _P]),
    "dcs_test_qr": (c_int, [c_int] * 6 + [_DP, _DP, _DP, _P]),
    "dcs_test_copy": (c_int, [_P, _P, ctypes.c_size_t, c_int, _P]),
    "dcs_test_permute": (c_int, [c_int] * 3 + [_IP, _IP] + [c_int] * 3 + [_DP, _DP, _P]),
    "dcs_test_gemm_gate": (c_int, [c_int] * 8 + [_DP, _DP, _DP, _DP, _P]),
    "dcs_test_permute_plan": (c_int, [c_int, _IP, _IP, c_int, _IP, c_int, _IP]),
    "dcs_test_permute_dev": (c_int, [c_int] * 3 + [_IP, _IP] + [c_int] * 3 + [_P, _P, c_int, _P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(rc: int) -> None:
    if rc != DCS_OK:
        raise DcsError(rc, _lib.dcs_last_error().decode())


def _ints(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1))


def _dbl(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(_IP)


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def dcs_last_error() -> str:
    return _lib.dcs_last_error().decode()


def dcs_version() -> int:
    return _lib.dcs_version()


def dcs_ctx_create(device: int) -> int:
    h = c_void_p()
    _check(_lib.dcs_ctx_create(ctypes.byref(h), device))
    return h.value


def dcs_ctx_destroy(ctx: int) -> None:
    _check(_lib.dcs_ctx_destroy(ctx))


def dcs_ctx_set_tuning(ctx: int, enabled: bool, reps: int = 3) -> None:
    _check(_lib.dcs_ctx_set_tuning(ctx, 1 if enabled else 0, reps))


def dcs_ctx_tuning_save(ctx: int, path: str) -> None:
    _check(_lib.dcs_ctx_tuning_save(ctx, path.encode()))


def dcs_ctx_tuning_load(ctx: int, path: str) -> None:
    _check(_lib.dcs_ctx_tuning_load(ctx, path.encode()))


def dcs_ctx_set_graphs(ctx: int, enabled: bool) -> None:
    _check(_lib.dcs_ctx_set_graphs(ctx, 1 if enabled else 0))


def dcs_ctx_set_timing(ctx: int, enabled: bool) -> None:
    _check(_lib.dcs_ctx_set_timing(ctx, 1 if enabled else 0))


TIMING_CLASSES = ["gemm_nn", "gemm_nt", "gemm_cn", "gemm_jt", "gate_operator", "qr", "measure",
                  "other"]


def dcs_ctx_timing(ctx: int, reset: bool = False):
    k = len(TIMING_CLASSES)
    launches = (c_longlong * k)()
    ms, flops, byts = (c_double * k)(), (c_double * k)(), (c_double * k)()
    _check(_lib.dcs_ctx_timing(ctx, launches, ms, flops, byts, 1 if reset else 0))
    return list(launches), list(ms), list(flops), list(byts)


def dcs_state_bytes(precision, n_qubits, capacity, chi_max, mpo_bond_max, n_init_slots) -> int:
    out = c_size_t()
    _check(_lib.dcs_state_bytes(precision, n_qubits, capacity, chi_max, mpo_bond_max,
                                n_init_slots, ctypes.byref(out)))
    return out.value


def dcs_state_create(ctx, precision, n_qubits, capacity, chi_max, mpo_bond_max, n_init_slots,
                     d_buffer: int, nbytes: int, stream: int) -> int:
    h = c_void_p()
    _check(_lib.dcs_state_create(ctx, ctypes.byref(h), precision, n_qubits, capacity, chi_max,
                                 mpo_bond_max, n_init_slots, d_buffer, nbytes, stream))
    return h.value


def dcs_state_destroy(st: int) -> None:
    _check(_lib.dcs_state_destroy(st))


def dcs_state_set_init(st: int, chi_cap: int, gauss: np.ndarray, stream: int) -> None:
    g = np.ascontiguousarray(gauss, dtype=np.complex128).view(np.float64)
    _check(_lib.dcs_state_set_init(st, chi_cap, _dp(g), stream))


def dcs_branch_init_zero(st, ids, chi_caps, stream) -> None:
    i, c = _ints(ids), _ints(chi_caps)
    _check(_lib.dcs_branch_init_zero(st, len(i), _ip(i), _ip(c), stream))


def dcs_branch_set_chi(st, ids, chi_caps) -> None:
    i, c = _ints(ids), _ints(chi_caps)
    _check(_lib.dcs_branch_set_chi(st, len(i), _ip(i), _ip(c)))


def dcs_branch_release(st, ids) -> None:
    i = _ints(ids)
    _check(_lib.dcs_branch_release(st, len(i), _ip(i)))


def dcs_branch_dims(st, bid, n_qubits) -> np.ndarray:
    out = np.zeros(n_qubits + 1, dtype=np.int32)
    _check(_lib.dcs_branch_dims(st, bid, _ip(out)))
    return out


def dcs_chunk_compile(ctx, n_qubits, q0, q1, mats: np.ndarray) -> int:
    a, b = _ints(q0), _ints(q1)
    m = np.ascontiguousarray(mats, dtype=np.complex128).view(np.float64)
    h = c_void_p()
    _check(_lib.dcs_chunk_compile(ctx, ctypes.byref(h), n_qubits, len(a), _ip(a), _ip(b), _dp(m)))
    return h.value


def dcs_chunk_bonds(ch, n_qubits) -> np.ndarray:
    out = np.zeros(n_qubits + 1, dtype=np.int32)
    _check(_lib.dcs_chunk_bonds(ch, _ip(out)))
    return out


def dcs_chunk_export(ch, n_qubits):
    """The compiled operator as a list of W_j[w_j, 2, 2, w_j+1] arrays."""
    w = dcs_chunk_bonds(ch, n_qubits)
    sizes = [int(w[j]) * 4 * int(w[j + 1]) for j in range(n_qubits)]
    buf = np.zeros(2 * sum(sizes))
    _check(_lib.dcs_chunk_export(ch, _dp(buf), buf.size))
    z = buf.view(np.complex128)
    out, o = [], 0
    for j, sz in enumerate(sizes):
        out.append(z[o:o + sz].reshape(int(w[j]), 2, 2, int(w[j + 1])).copy())
        o += sz
    return out


def dcs_gate_rank(mat) -> int:
    m = np.ascontiguousarray(np.asarray(mat, dtype=np.complex128).reshape(16)).view(np.float64)
    r = c_int()
    _check(_lib.dcs_gate_rank(_dp(m), ctypes.byref(r)))
    return r.value


def dcs_chunk_destroy(ch) -> None:
    _check(_lib.dcs_chunk_destroy(ch))


def dcs_state_set_warm_start(st, enabled: bool, eta: float = 0.0) -> None:
    _check(_lib.dcs_state_set_warm_start(st, 1 if enabled else 0, float(eta)))


def dcs_compress_step(st, ids, chunks, n_sweeps, stream) -> np.ndarray:
    i = _ints(ids)
    arr = (c_void_p * len(i))(*chunks)
    fid = np.zeros(len(i), dtype=np.float64)
    _check(_lib.dcs_compress_step(st, len(i), _ip(i), arr, n_sweeps, _dp(fid), stream))
    return fid


def dcs_measure_prob(st, ids, qubits, stream) -> np.ndarray:
    i, q = _ints(ids), _ints(qubits)
    p0 = np.zeros(len(i), dtype=np.float64)
    _check(_lib.dcs_measure_prob(st, len(i), _ip(i), _ip(q), _dp(p0), stream))
    return p0


def dcs_measure_sample_collapse(st, ids, qubits, u_dev: int, eps: float, outcome_dev: int,
                                pm_dev: int, stream) -> None:
    """Device pointers: u_dev (float64[n]), outcome_dev (int32[n]), pm_dev
    (float64[n]); nothing is synchronised."""
    i, q = _ints(ids), _ints(qubits)
    _check(_lib.dcs_measure_sample_collapse(st, len(i), _ip(i), _ip(q), u_dev, eps, outcome_dev,
                                            pm_dev, stream))


def dcs_collapse(st, src_ids, qubits, outcomes, dst_ids, eps, stream) -> np.ndarray:
    s, q, o, d = _ints(src_ids), _ints(qubits), _ints(outcomes), _ints(dst_ids)
    pm = np.zeros(len(s), dtype=np.float64)
    _check(_lib.dcs_collapse(st, len(s), _ip(s), _ip(q), _ip(o), _ip(d), eps, _dp(pm), stream))
    return pm


def dcs_topk_by_weight(weights, k):
    w = _dbl(weights)
    keep = np.zeros(max(1, min(len(w), k)), dtype=np.int32)
    nk = c_int()
    disc = c_double()
    _check(_lib.dcs_topk_by_weight(len(w), _dp(w), k, _ip(keep), ctypes.byref(nk),
                                   ctypes.byref(disc)))
    return keep[:nk.value].copy(), disc.value


def dcs_prune_adaptive(weights, k_max, mass_tol=0.0, rel_min=0.0):
    w = _dbl(weights)
    keep = np.zeros(max(1, min(len(w), k_max)), dtype=np.int32)
    nk = c_int()
    disc = c_double()
    _check(_lib.dcs_prune_adaptive(len(w), _dp(w), k_max, mass_tol, rel_min, _ip(keep),
                                   ctypes.byref(nk), ctypes.byref(disc)))
    return keep[:nk.value].copy(), disc.value


def dcs_overlap(st: int, id_a: int, id_b: int, stream: int = 0) -> complex:
    out = np.zeros(2)
    _check(_lib.dcs_overlap(st, id_a, id_b, _dp(out), stream))
    return complex(out[0], out[1])


def dcs_overlap_noalloc(st: int, id_a: int, id_b: int, out_dev: int, stream: int = 0) -> None:
    """<a|b> written to device memory out_dev (2 doubles) without allocation
    or host synchronisation."""
    _check(_lib.dcs_overlap_noalloc(st, id_a, id_b, out_dev, stream))


def dcs_export_mps(st, bid, n_qubits, chi_max, stream):
    dims = np.zeros(n_qubits + 1, dtype=np.int32)
    cap = 2 * sum(2 * min(chi_max, 2 ** j, 2 ** (n_qubits - j))
                  * min(chi_max, 2 ** (j + 1), 2 ** (n_qubits - j - 1)) for j in range(n_qubits))
    buf = np.zeros(cap, dtype=np.float64)
    _check(_lib.dcs_export_mps(st, bid, _dp(buf), cap, _ip(dims), stream))
    out, o = [], 0
    flat = buf.view(np.complex128)
    for j in range(n_qubits):
        e = int(dims[j]) * 2 * int(dims[j + 1])
        out.append(flat[o:o + e].reshape(int(dims[j]), 2, int(dims[j + 1])).copy())
        o += e
    return out


def dcs_import_mps(st, bid, chi_cap, sites, stream) -> None:
    dims = _ints([sites[0].shape[0]] + [a.shape[2] for a in sites])
    flat = np.concatenate([np.ascontiguousarray(a, dtype=np.complex128).reshape(-1)
                           for a in sites]).view(np.float64)
    _check(_lib.dcs_import_mps(st, bid, chi_cap, _dp(flat), _ip(dims), stream))


# --- tree tensor network -------------------------------------------------------

def dcs_tree_n_nodes(levels) -> int:
    lv = _ints(levels)
    out = c_int()
    _check(_lib.dcs_tree_n_nodes(_ip(lv), len(lv), ctypes.byref(out)))
    return out.value


def dcs_tree_state_bytes(precision, levels, capacity, chi_max, mpo_bond_max, scratch_elems,
                         n_init_slots) -> int:
    lv = _ints(levels)
    out = c_size_t()
    _check(_lib.dcs_tree_state_bytes(precision, len(lv), _ip(lv), capacity, chi_max, mpo_bond_max,
                                     scratch_elems, n_init_slots, ctypes.byref(out)))
    return out.value


def dcs_tree_create(ctx, precision, levels, capacity, chi_max, mpo_bond_max, scratch_elems,
                    n_init_slots, d_buffer: int, nbytes: int, stream: int) -> int:
    lv = _ints(levels)
    h = c_void_p()
    _check(_lib.dcs_tree_create(ctx, ctypes.byref(h), precision, len(lv), _ip(lv), capacity,
                                chi_max, mpo_bond_max, scratch_elems, n_init_slots, d_buffer,
                                nbytes, stream))
    return h.value


def dcs_tree_destroy(t: int) -> None:
    _check(_lib.dcs_tree_destroy(t))


def dcs_tree_set_init(t: int, chi_cap: int, gauss: np.ndarray, stream: int) -> None:
    g = np.ascontiguousarray(gauss, dtype=np.complex128).view(np.float64)
    _check(_lib.dcs_tree_set_init(t, chi_cap, _dp(g), stream))


def dcs_tree_branch_init_zero(t, ids, chi_caps, stream) -> None:
    a, c = _ints(ids), _ints(chi_caps)
    _check(_lib.dcs_tree_branch_init_zero(t, len(a), _ip(a), _ip(c), stream))


def dcs_tree_branch_set_chi(t, ids, chi_caps) -> None:
    a, c = _ints(ids), _ints(chi_caps)
    _check(_lib.dcs_tree_branch_set_chi(t, len(a), _ip(a), _ip(c)))


def dcs_tree_branch_release(t, ids) -> None:
    a = _ints(ids)
    _check(_lib.dcs_tree_branch_release(t, len(a), _ip(a)))


def dcs_tree_chunk_compile(ctx, levels, q0, q1, mats: np.ndarray) -> int:
    lv, a, b = _ints(levels), _ints(q0), _ints(q1)
    m = np.ascontiguousarray(mats, dtype=np.complex128).view(np.float64)
    h = c_void_p()
    _check(_lib.dcs_tree_chunk_compile(ctx, ctypes.byref(h), len(lv), _ip(lv), len(a), _ip(a),
                                       _ip(b), _dp(m)))
    return h.value


def dcs_tchunk_destroy(ch) -> None:
    _check(_lib.dcs_tchunk_destroy(ch))


def dcs_tchunk_bonds(ch, n_nodes) -> np.ndarray:
    w = np.zeros(n_nodes, dtype=np.int32)
    _check(_lib.dcs_tchunk_bonds(ch, _ip(w), n_nodes))
    return w


def dcs_tree_chunk_scratch(ch, chi_bra, chi_ket) -> int:
    out = c_size_t()
    _check(_lib.dcs_tree_chunk_scratch(ch, chi_bra, chi_ket, ctypes.byref(out)))
    return out.value


def dcs_tree_compress_step(t, ids, chunks, n_sweeps, stream) -> np.ndarray:
    a = _ints(ids)
    arr = (c_void_p * len(a))(*chunks)
    f = np.zeros(len(a))
    _check(_lib.dcs_tree_compress_step(t, len(a), _ip(a), arr, n_sweeps, _dp(f), stream))
    return f


def dcs_tree_measure_prob(t, ids, qubits, stream) -> np.ndarray:
    a, q = _ints(ids), _ints(qubits)
    p = np.zeros(len(a))
    _check(_lib.dcs_tree_measure_prob(t, len(a), _ip(a), _ip(q), _dp(p), stream))
    return p


def dcs_tree_collapse(t, src_ids, qubits, outcomes, dst_ids, eps, stream) -> np.ndarray:
    a, q, m, d = _ints(src_ids), _ints(qubits), _ints(outcomes), _ints(dst_ids)
    pm = np.zeros(len(a))
    _check(_lib.dcs_tree_collapse(t, len(a), _ip(a), _ip(q), _ip(m), _ip(d), eps, _dp(pm), stream))
    return pm


def dcs_tree_export(t, bid, shapes_of, n_nodes, cap_elems, stream):
    """Node tensors of a branch; shapes_of(dims) gives each node's shape from
    the edge dims the library reports."""
    dims = np.zeros(n_nodes, dtype=np.int32)
    buf = np.zeros(2 * cap_elems, dtype=np.float64)
    _check(_lib.dcs_tree_export(t, bid, _dp(buf), len(buf), _ip(dims), stream))
    flat = buf.view(np.complex128)
    out, o = [], 0
    for shp in shapes_of([int(x) for x in dims]):
        e = int(np.prod(shp))
        out.append(flat[o:o + e].reshape(shp).copy())
        o += e
    return out


# --- kernel-level test entry points (include/dcs_testing.h) -----------------

def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def dcs_test_gemm(ta, tb, tc, tacc, opa, opb, a, b, stream=0, variant=0) -> np.ndarray:
    """a: (batch, rows, cols) as stored; b likewise; returns (batch, M, N)."""
    a, b = _c128(a), _c128(b)
    batch = a.shape[0]
    m = a.shape[2] if opa == 2 else a.shape[1]
    k = a.shape[1] if opa == 2 else a.shape[2]
    n = b.shape[1] if opb == 1 else b.shape[2]
    c = np.zeros((batch, m, n), dtype=np.complex128)
    _check(_lib.dcs_test_gemm(ta, tb, tc, tacc, opa, opb, m, n, k, batch, variant,
                              _dp(a.view(np.float64)), _dp(b.view(np.float64)),
                              _dp(c.view(np.float64)), stream))
    return c


def dcs_test_mpo(ct, direction, d0, d1, wl, wr, x, w, stream=0) -> np.ndarray:
    x, w = _c128(x), _c128(w)
    out = np.zeros(d0 * d1 * 2 * (wr if direction == 0 else wl), dtype=np.complex128)
    _check(_lib.dcs_test_mpo(ct, direction, d0, d1, wl, wr, _dp(x.view(np.float64)),
                             _dp(w.view(np.float64)), _dp(out.view(np.float64)), stream))
    return out


def dcs_test_qr(ct_in, ct_out, m, n, mode, variant, f, stream=0):
    f = _c128(f)
    q = np.zeros(m * n, dtype=np.complex128)
    nrm = np.zeros(1)
    _check(_lib.dcs_test_qr(ct_in, ct_out, m, n, mode, int(variant),
                            _dp(f.view(np.float64)), _dp(q.view(np.float64)), _dp(nrm), stream))
    return q, float(nrm[0])


def dcs_test_copy(src: int, dst: int, nbytes: int, reps: int = 1, stream: int = 0) -> None:
    _check(_lib.dcs_test_copy(src, dst, nbytes, reps, stream))


def dcs_test_permute(ct_in, ct_out, x, perm, conj=False, variant=0, stream=0) -> np.ndarray:
    """x: (batch, *dims) complex; returns (batch, *dims[perm]) complex128."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    batch, dims = x.shape[0], [int(d) for d in x.shape[1:]]
    perm = [int(p) for p in perm]
    out = np.zeros((batch, *[dims[p] for p in perm]), dtype=np.complex128)
    d = (ctypes.c_int * len(dims))(*dims)
    p = (ctypes.c_int * len(perm))(*perm)
    _check(_lib.dcs_test_permute(ct_in, ct_out, len(dims), d, p, int(bool(conj)), batch,
                                 int(variant), _dp(x.view(np.float64).reshape(-1)),
                                 _dp(out.view(np.float64).reshape(-1)), stream))
    return out


def dcs_test_permute_dev(ct_in, ct_out, dims, perm, src: int, dst: int, conj=False, batch=1,
                         variant=0, reps=1, stream=0) -> None:
    """Device-buffer form of dcs_test_permute (no synchronisation)."""
    dims = [int(d) for d in dims]
    perm = [int(p) for p in perm]
    d = (ctypes.c_int * len(dims))(*dims)
    p = (ctypes.c_int * len(perm))(*perm)
    _check(_lib.dcs_test_permute_dev(ct_in, ct_out, len(dims), d, p, int(bool(conj)), batch,
                                     int(variant), src, dst, reps, stream))


def dcs_test_gemm_gate(ct, direction, a, b, w, variant=0, stream=0) -> np.ndarray:
    """a: (M, K); b: (K, N) for direction 0, (N, K) for 1; w: (wl, 2, 2, wr).
    Returns the operator-applied product, flat."""
    a, b, w = _c128(a), _c128(b), _c128(w)
    m, k = a.shape
    n = b.shape[1] if direction == 0 else b.shape[0]
    wl, wr = w.shape[0], w.shape[3]
    nc = (m // wl) * 2 * wr * (n // 2) if direction == 0 else wl * (m // 2) * 2 * (n // wr)
    c = np.zeros(nc, dtype=np.complex128)
    _check(_lib.dcs_test_gemm_gate(ct, direction, m, n, k, wl, wr, int(variant),
                                   _dp(a.view(np.float64)), _dp(b.view(np.float64)),
                                   _dp(w.view(np.float64)), _dp(c.view(np.float64)), stream))
    return c


def dcs_test_permute_plan(dims, perm, esize=8):
    """The tiled transposition kernel's plan (host only): a dict, or None when
    the tiled kernel does not take the transposition."""
    dims = [int(d) for d in dims]
    perm = [int(p) for p in perm]
    d = (ctypes.c_int * len(dims))(*dims)
    p = (ctypes.c_int * len(perm))(*perm)
    out = (ctypes.c_int * 512)()
    planned = ctypes.c_int(0)
    _check(_lib.dcs_test_permute_plan(len(dims), d, p, esize, out, 512, ctypes.byref(planned)))
    if not planned.value:
        return None
    v = list(out)
    keys = ["pi", "pc", "pa", "po", "pitch", "tiles", "ept", "ni", "nc", "na", "nr"]
    plan = dict(zip(keys, v[:11]))
    pos = 11

    def take(n):
        nonlocal pos
        r = v[pos:pos + n]
        pos += n
        return r
    ni, nc, na, nr = plan["ni"], plan["nc"], plan["na"], plan["nr"]
    plan.update(i_ext=take(ni), i_lds=take(ni), c_ext=take(nc), c_in=take(nc), c_lds=take(nc),
                a_ext=take(na), a_out=take(na), r_ext=take(nr), r_in=take(nr), r_out=take(nr))
    return plan
