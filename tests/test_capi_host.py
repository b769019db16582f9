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
        capi.dcs_chunk_compile(0, 4, [0], [2], C.CNOT_01.reshape(-1))
    assert e.value.code == capi.DCS_ENONLOCAL
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
