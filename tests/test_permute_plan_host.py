"""Host-side check of the tiled transposition kernel's planner (no GPU): the
plan's index maps, composed as the kernel composes them (input run and tile
tables into LDS, LDS into output runs), reproduce the transposition for the
leg orders of the tree contractions and for random ragged shapes, every
output element written once."""
import numpy as np
import pytest

capi = pytest.importorskip("paper_2609_26516_amd.capi")


def _table(n, ext, w):
    """Entry x of a group table: sum over its legs (fastest first) of
    coordinate times weight."""
    x = np.arange(n)
    v = np.zeros(n, dtype=np.int64)
    for e, ww in zip(ext, w):
        v += (x % e) * ww
        x = x // e
    return v


def _check_plan(dims, perm, esize):
    plan = capi.dcs_test_permute_plan(dims, perm, esize)
    total = int(np.prod(dims))
    ref = np.arange(total).reshape(dims).transpose(perm).reshape(-1)   # input index of output o
    if plan is None:
        return False
    pi, pc, pa, po, pitch = plan["pi"], plan["pc"], plan["pa"], plan["po"], plan["pitch"]
    n = pa * po
    assert n == pc * pi and n <= 256 * plan["ept"]
    assert pi <= 64 and po <= 64 and pa <= 256 and pc <= 256
    assert pa * pitch * esize <= 48 * 1024
    t_i = _table(pi, plan["i_ext"], plan["i_lds"])
    c_in = _table(pc, plan["c_ext"], plan["c_in"])
    c_lds = _table(pc, plan["c_ext"], plan["c_lds"])
    a_out = _table(pa, plan["a_ext"], plan["a_out"])
    tiles = plan["tiles"]
    t_in = _table(tiles, plan["r_ext"], plan["r_in"])
    t_out = _table(tiles, plan["r_ext"], plan["r_out"])
    e = np.arange(n)
    c, i = e // pi, e % pi
    a, b = e // po, e % po
    read_off = c_in[c] + i                 # input offset within the tile
    read_pos = t_i[i] + c_lds[c]           # LDS slot it lands in
    write_pos = a * pitch + b              # LDS slot each output element takes
    write_off = a_out[a] + b               # output offset within the tile
    assert len(np.unique(read_pos)) == n
    assert np.array_equal(np.sort(read_pos), np.sort(write_pos))
    lds = np.full(pa * pitch, -1, dtype=np.int64)
    out = np.full(total, -1, dtype=np.int64)
    written = np.zeros(total, dtype=np.int64)
    for t in range(tiles):
        src = t_in[t] + read_off
        assert src.min() >= 0 and src.max() < total
        lds[read_pos] = src
        dst = t_out[t] + write_off
        assert dst.min() >= 0 and dst.max() < total
        out[dst] = lds[write_pos]
        np.add.at(written, dst, 1)
    assert np.all(written == 1)
    np.testing.assert_array_equal(out, ref)
    return True


# (input dims, output leg order) of the largest transpositions of the tree
# [1, 3, 9, 27] at bond cap 32 with operator legs of 4
TREE = [
    ([8, 8, 4, 4, 32, 4, 32], [0, 2, 4, 6, 1, 5, 3]),
    ([8, 8, 4, 1024], [3, 1, 0, 2]),
    ([8, 4, 64, 128], [2, 3, 0, 1]),
    ([32, 32, 8, 8, 4], [0, 2, 3, 4, 1]),
    ([32, 4, 32, 32], [2, 3, 0, 1]),
    ([8, 32, 512], [0, 2, 1]),
]


@pytest.mark.parametrize("esize", [8, 16])
@pytest.mark.parametrize("case", TREE)
def test_plan_tree_transpositions(case, esize):
    dims, perm = case
    assert _check_plan(dims, perm, esize)


def test_plan_random_shapes():
    rng = np.random.default_rng(3)
    choices = [1, 2, 3, 4, 5, 7, 8, 16, 31, 32, 33, 64, 100]
    planned = 0
    for _ in range(150):
        rank = int(rng.integers(1, 7))
        dims = [int(rng.choice(choices)) for _ in range(rank)]
        while np.prod(dims) > 40000:
            dims[int(np.argmax(dims))] //= 2
        perm = [int(p) for p in rng.permutation(rank)]
        for esize in (8, 16):
            planned += _check_plan(dims, perm, esize)
    assert planned > 200
