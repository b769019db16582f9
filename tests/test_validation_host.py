"""Host-side pieces of the validation drivers: distances, frequencies and the
grouping of runs into repetitions, checked on hand-worked cases."""
import numpy as np

from inputs import circuits as C
from paper_2609_26516_amd import validation as V


def test_tvd_hand_cases():
    assert V.tvd({(0,): 1.0}, {(0,): 1.0}) == 0.0
    assert V.tvd({(0,): 1.0}, {(1,): 1.0}) == 1.0
    # disjoint mass counts once per side
    assert abs(V.tvd({(0, 0): 0.5, (0, 1): 0.5}, {(0, 0): 0.25, (1, 1): 0.75}) - 0.75) < 1e-15
    # GHZ cap: M of 2^r equiprobable paths kept, raw and renormalised
    r, m = 5, 8
    exact = {(i,): 2.0 ** -r for i in range(2 ** r)}
    kept = {(i,): 2.0 ** -r for i in range(m)}
    assert abs(V.tvd(kept, exact) - 0.5 * (1 - m * 2.0 ** -r)) < 1e-15
    ren = {k: v / sum(kept.values()) for k, v in kept.items()}
    assert abs(V.tvd(ren, exact) - (1 - m * 2.0 ** -r)) < 1e-15


def test_frequencies_and_curve():
    paths = [(0, 1), (0, 1), (1, 0), (0, 1)]
    f = V.frequencies(paths)
    assert f == {(0, 1): 0.75, (1, 0): 0.25}
    assert V.frequencies([]) == {}
    exact = {(0, 1): 0.5, (1, 0): 0.5}
    # two repetitions of up to 2 runs: groups [(0,1),(0,1)] and [(1,0),(0,1)]
    c = V.tvd_curve(paths, exact, [1, 2], 2)
    assert c[0]["N"] == 1 and c[0]["tvd"] == [0.5, 0.5]
    assert c[1]["tvd"] == [0.5, 0.0]
    assert abs(c[1]["tvd_sd"] - np.std([0.5, 0.0], ddof=1)) < 1e-15


def test_max_paths_bounds():
    assert V._max_paths(C.teleportation(False)) == 4
    assert V._max_paths(C.teleportation(True)) == 8
    assert V._max_paths(C.ghz_dynamic(9)) == 16      # resets add no paths
