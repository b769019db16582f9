"""The allocation-free overlap entry point (fixed device scratch) against the
existing dcs_overlap, through the C ABI: two calls in a row, the second on
smaller states (the scratch keeps the first call's contents), then a state
whose bonds exceed the fixed scratch."""
import numpy as np
import pytest

from inputs import circuits as C
from inputs.randomness import shot_uniforms

pytestmark = pytest.mark.gpu


def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_26516_amd import capi
    from paper_2609_26516_amd import engine as E
    return torch, capi, E


def _two_shots(E, eng, prec, n, chi, depth):
    circ, prm = C.workload("cfg1_n10_chi16", n=n, depth=depth, chi=chi)
    k = C.segment_max(circ) + 1
    nm = circ.n_measurements()
    u = np.stack([shot_uniforms(prm["seed"], s, nm) for s in range(2)])
    st = E.State(eng, prec, n, 4, chi, 4, [chi], prm["init_seed"])
    r = E.run_single_path(eng, st, circ, 2, chi, k, 2, uniforms=u)
    return st, [int(i) for i in r["ids"]]


def _compare(torch, capi, eng, st, ids, tol):
    out = torch.full((4,), 7.0, dtype=torch.float64, device="cuda")
    for a in ids:
        for b in ids:
            ref = capi.dcs_overlap(st.h, a, b, eng.stream())
            capi.dcs_overlap_noalloc(st.h, a, b, out.data_ptr(), eng.stream())
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            assert got[2] == 7.0 and got[3] == 7.0          # nothing written past the result
            assert abs(complex(got[0], got[1]) - ref) <= tol * max(1.0, abs(ref)), (a, b, got, ref)
            if a == b:
                assert abs(ref - 1.0) < 1e-5                  # normalised states


def test_noalloc_overlap_matches_dcs_overlap_twice():
    torch, capi, E = _setup()
    eng = E.Engine(0)
    # first call: 12 qubits, bond cap 64, complex64
    st, ids = _two_shots(E, eng, "c64", 12, 64, 8)
    _compare(torch, capi, eng, st, ids, 1e-12)
    st.close()
    # second call: smaller states (6 qubits, bond cap 4, complex128)
    st, ids = _two_shots(E, eng, "c128", 6, 4, 6)
    _compare(torch, capi, eng, st, ids, 1e-13)
    st.close()
    eng.close()


def test_noalloc_overlap_rejects_bonds_above_the_scratch():
    torch, capi, E = _setup()
    eng = E.Engine(0)
    n, chi = 18, 512
    st = E.State(eng, "c64", n, 2, chi, 4, [chi], 3)
    dims = [min(chi, 2 ** b, 2 ** (n - b)) for b in range(n + 1)]
    rng = np.random.default_rng(4)
    sites = [rng.standard_normal((dims[j], 2, dims[j + 1])) + 0j for j in range(n)]
    capi.dcs_import_mps(st.h, 0, chi, sites, eng.stream())
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    with pytest.raises(capi.DcsError) as e:
        capi.dcs_overlap_noalloc(st.h, 0, 0, out.data_ptr(), eng.stream())
    assert e.value.code == capi.DCS_ENOMEM
    assert "256" in str(e.value)
    st.close()
    eng.close()
