"""Plausible mistakes planted in the oracle (on the CPU, by monkeypatching)
must be caught by the independent checks used as pins."""
import numpy as np
import pytest

from inputs import circuits as C
from inputs.randomness import bra_init_gaussians
from oracle import mps as M
from oracle import statevector as SV


def _exact_regime_error(n=6, seed=3):
    return max(_exact_regime_error_s(n, 1, seed), _exact_regime_error_s(n, 2, seed))


def _exact_regime_error_s(n, s, seed):
    rng = np.random.default_rng(seed)
    chi = 2 ** (n // 2)
    ops = []
    for layer in range(3):
        for q in range(layer % 2, n - 1, 2):
            ops.append(((q, q + 1), C.haar_unitary(rng, 4)))
        ops.append(((int(rng.integers(n)),), C.haar_unitary(rng, 2)))
    psi = [rng.standard_normal(a.shape) + 1j * rng.standard_normal(a.shape)
           for a in M.zero_state(n, chi)]
    psi[0] = psi[0] / np.sqrt(M.norm_sq(psi))
    new, f, _ = M.compress(psi, M.chunk_mpo(n, ops),
                           M.generic_bra(bra_init_gaussians(n, chi, seed)), s)
    sv = M.to_statevector(psi)
    for qubits, mat in ops:
        sv = SV.apply_gate(sv, n, qubits, mat)
    v = M.to_statevector(new)
    return max(abs(abs(np.vdot(sv, v)) ** 2 - 1), abs(f - 1))


def _measure_error(n=5, seed=4):
    rng = np.random.default_rng(seed)
    psi = [rng.standard_normal(a.shape) + 1j * rng.standard_normal(a.shape)
           for a in M.zero_state(n, 4)]
    psi[0] = psi[0] / np.sqrt(M.norm_sq(psi))
    sv = M.to_statevector(psi)
    err = 0.0
    for q in range(n):
        n0, n1 = M.outcome_norms(psi, q)
        s0, s1 = SV.outcome_norms(sv, n, q)
        err = max(err, abs(n0 - s0), abs(n1 - s1))
        post = M.to_statevector(M.collapse(psi, q, 1, n1))
        err = max(err, np.max(np.abs(post - SV.project(sv, n, q, 1, s1))))
    return err


def test_unmodified_oracle_passes():
    assert _exact_regime_error() < 1e-12
    assert _measure_error() < 1e-12


def test_dropped_conjugate_in_left_environment(monkeypatch):
    def bad(lenv, bra, ket, w):
        x = np.einsum("awx,xty->awty", lenv, ket)
        x = np.einsum("awty,wstv->asvy", x, w)
        return np.einsum("asc,asvy->cvy", bra, x)
    monkeypatch.setattr(M, "left_env_step", bad)
    assert _exact_regime_error() > 1e-3


def test_swapped_physical_legs_of_gate_operator(monkeypatch):
    def bad(lenv, ket, w, renv):
        x = np.einsum("awx,xty->awty", lenv, ket)
        x = np.einsum("awty,wtsv->asvy", x, w)         # in/out legs exchanged
        return np.einsum("asvy,cvy->asc", x, renv)
    monkeypatch.setattr(M, "site_tensor", bad)
    assert _exact_regime_error() > 1e-3


def test_transposed_gate_split(monkeypatch):
    good = M.split_two_qubit

    def bad(mat, cutoff=M.SPLIT_CUTOFF):
        return good(mat.T, cutoff)
    monkeypatch.setattr(M, "split_two_qubit", bad)
    assert _exact_regime_error() > 1e-3


def test_wrong_collapse_scale(monkeypatch):
    def bad(mps, q, m, norm_m):
        out = [a.copy() for a in mps]
        out[q][:, 1 - m, :] = 0.0
        out[q][:, m, :] /= norm_m
        return out
    monkeypatch.setattr(M, "collapse", bad)
    assert _measure_error() > 1e-3


def test_projector_on_wrong_site(monkeypatch):
    good = M.outcome_norms

    def bad(mps, q):
        return good(mps, (q + 1) % len(mps))
    monkeypatch.setattr(M, "outcome_norms", bad)
    assert _measure_error() > 1e-3


@pytest.mark.parametrize("wrong_order", [True])
def test_layer_product_in_wrong_time_order(monkeypatch, wrong_order):
    good_layers = M.asap_layers

    def bad(ops):
        return list(reversed(good_layers(ops)))
    monkeypatch.setattr(M, "asap_layers", bad)
    assert _exact_regime_error() > 1e-3
