"""Autotuned contraction tile shapes: a run that tunes online gives the same
bits as a run with tuning off (every tile shape sums each output over K in
the same order), and the decided table survives a save/load round trip."""
import json

import numpy as np
import pytest

from inputs import circuits as C
from inputs.randomness import shot_uniforms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_26516_amd import engine
    return engine


def _run(E, prec, tuning, load=None, save=None, repeats=2):
    circ, prm = C.workload("cfg4_n24_chi64_x1024", n=12, depth=8, chi=32)
    n, chi = prm["n"], prm["chi"]
    k = C.segment_max(circ) + 1
    shots = 8
    u = np.stack([shot_uniforms(prm["seed"], s, circ.n_measurements()) for s in range(shots)])
    eng = E.Engine(0)
    eng.tuning(tuning, 2)
    if load:
        eng.load_tuning(load)
    st = E.State(eng, prec, n, shots, chi, 4, [chi], prm["init_seed"])
    out = []
    for _ in range(repeats):
        r = E.run_single_path(eng, st, circ, shots, chi, k, 2, uniforms=u)
        out.append((r["p0s"].copy(), r["F"].copy(), [st.export(int(i)) for i in r["ids"]]))
        st.release(r["ids"])
    if save:
        eng.save_tuning(save)
    st.close()
    eng.close()
    return out


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_tuned_run_bit_identical(E, prec, tmp_path):
    path = str(tmp_path / "tiles.json")
    base = _run(E, prec, False, repeats=1)[0]
    tuned = _run(E, prec, True, save=path)
    table = json.load(open(path))
    assert table["format"] == "dcs-gemm-tiles-1"
    assert len(table["entries"]) > 0
    for e in table["entries"]:
        assert 0 <= e["best"] < 4 and len(e["key"]) == 10
    loaded = _run(E, prec, False, load=path, repeats=1)
    for p0, f, mps in tuned + loaded:
        np.testing.assert_array_equal(p0, base[0])
        np.testing.assert_array_equal(f, base[1])
        for a, b in zip(mps, base[2]):
            for x, y in zip(a, b):
                np.testing.assert_array_equal(x, y)


def test_bad_table_rejected(E, tmp_path):
    from paper_2609_26516_amd import capi
    bad = tmp_path / "bad.json"
    bad.write_text('{"format": "something-else"}')
    eng = E.Engine(0)
    try:
        with pytest.raises(capi.DcsError):
            eng.load_tuning(str(bad))
        with pytest.raises(capi.DcsError):
            eng.tuning(True, 0)
    finally:
        eng.close()
