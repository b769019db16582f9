"""Compression steps replayed from captured HIP graphs give bit-identical
results to eager launches.  Several runs share one state, with eager
measurement and collapse work and host synchronisation between the replays,
and every run is compared with an eager reference run."""
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


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("name,over,shots", [
    ("cfg1_n10_chi16", {}, 1),
    ("cfg4_n24_chi64_x1024", dict(n=12, depth=8, chi=16), 4),
])
def test_graph_replay_matches_eager(E, prec, name, over, shots):
    circ, prm = C.workload(name, **over)
    n, chi = prm["n"], prm["chi"]
    k = C.segment_max(circ) + 1
    u = np.stack([shot_uniforms(prm["seed"], s, circ.n_measurements()) for s in range(shots)])

    def run(graphs, repeats):
        eng = E.Engine(0)
        eng.graphs(graphs)
        st = E.State(eng, prec, n, shots, chi, 4, [chi], prm["init_seed"])
        out = []
        for _ in range(repeats):
            r = E.run_single_path(eng, st, circ, shots, chi, k, 2, uniforms=u)
            out.append((r, [st.export(int(i)) for i in r["ids"]]))
            st.release(r["ids"])
        st.close()
        eng.close()
        return out

    eager = run(False, 1)[0]
    for r, mps in run(True, 4):
        np.testing.assert_array_equal(r["outcomes"], eager[0]["outcomes"])
        np.testing.assert_array_equal(r["p0s"], eager[0]["p0s"])
        np.testing.assert_array_equal(r["F"], eager[0]["F"])
        for a, b in zip(mps, eager[1]):
            for x, y in zip(a, b):
                np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_graph_replay_distant_gates_and_warm_start(E, prec):
    """Chunks of gates on distant pairs (operator bonds up to 16, chunks closed
    at the cap) with the warm-start guess: graph replays equal the eager run
    bit for bit."""
    circ = C.random_dynamic(10, 4, 3)
    n, chi, shots = 10, 8, 3
    u = np.stack([shot_uniforms(5, s, circ.n_measurements()) for s in range(shots)])

    def run(graphs, repeats):
        eng = E.Engine(0)
        eng.graphs(graphs)
        st = E.State(eng, prec, n, shots, chi, 16, [chi], 9)
        st.warm_start(0.05)
        out = []
        for _ in range(repeats):
            r = E.run_single_path(eng, st, circ, shots, chi, 20, 2, uniforms=u)
            out.append((r, [st.export(int(i)) for i in r["ids"]]))
            st.release(r["ids"])
        st.close()
        eng.close()
        return out

    eager = run(False, 1)[0]
    for r, mps in run(True, 3):
        np.testing.assert_array_equal(r["outcomes"], eager[0]["outcomes"])
        np.testing.assert_array_equal(r["F"], eager[0]["F"])
        for a, b in zip(mps, eager[1]):
            for x, y in zip(a, b):
                np.testing.assert_array_equal(x, y)
