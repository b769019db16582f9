"""Kernel-level checks of the contraction, gate-operator and QR kernels
against plain numpy references (FP64), through include/dcs_testing.h."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

F32, F64 = 0, 1
OPN, OPT, OPC, OPJ = 0, 1, 2, 3


@pytest.fixture(scope="module")
def capi():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_26516_amd import capi as c
    return c


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


COMBOS = [
    (F64, F64, F64, F64, OPN, OPN), (F64, F64, F64, F64, OPN, OPT),
    (F64, F64, F64, F64, OPC, OPN), (F64, F64, F64, F64, OPJ, OPT),
    (F32, F32, F32, F32, OPN, OPN), (F32, F32, F32, F32, OPN, OPT),
    (F32, F32, F32, F32, OPC, OPN), (F32, F32, F32, F32, OPJ, OPT),
    (F64, F32, F64, F64, OPN, OPN), (F32, F64, F64, F64, OPC, OPN),
    (F32, F64, F64, F64, OPN, OPT), (F32, F64, F64, F64, OPJ, OPT),
    (F32, F32, F64, F64, OPC, OPN), (F32, F32, F64, F64, OPJ, OPT),
]


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("combo", COMBOS)
@pytest.mark.parametrize("mnk", [(1, 1, 1), (16, 16, 4), (64, 64, 16), (70, 130, 37),
                                 (200, 96, 257), (300, 260, 40)])
def test_gemm(capi, combo, mnk, variant):
    ta, tb, tc, tacc, opa, opb = combo
    if variant == 4 and tacc != F32:
        pytest.skip("the 128 x 128 tile exists for FP32 accumulation only")
    m, n, k = mnk
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    batch = 3
    a = _rand(rng, batch, k, m) if opa == OPC else _rand(rng, batch, m, k)
    b = _rand(rng, batch, n, k) if opb == OPT else _rand(rng, batch, k, n)
    if ta == F32:
        a = a.astype(np.complex64).astype(np.complex128)
    if tb == F32:
        b = b.astype(np.complex64).astype(np.complex128)
    c = capi.dcs_test_gemm(ta, tb, tc, tacc, opa, opb, a, b, variant=variant)
    A = {OPN: a, OPC: np.conj(np.swapaxes(a, 1, 2)), OPJ: np.conj(a)}[opa]
    B = {OPN: b, OPT: np.swapaxes(b, 1, 2)}[opb]
    ref = A @ B
    # rounding bound ~ K u max|a||b|; inputs are O(1), so scale by K
    u = 1.2e-16 if (tacc == F64 and tc == F64) else 6e-8
    tol = 8 * u * k * 2
    err = np.max(np.abs(c - ref))
    assert err < tol, (err, tol)


BF16X3 = 2


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("ops", [(OPN, OPN), (OPN, OPT), (OPC, OPN), (OPJ, OPT)])
@pytest.mark.parametrize("mnk", [(1, 1, 1), (16, 16, 32), (64, 64, 64), (70, 130, 37),
                                 (200, 96, 257), (33, 150, 1000)])
def test_gemm_bf16x3(capi, ops, mnk, variant):
    """Split-BF16 products: x = hi + lo + d with |x - hi| <= 2^-9 |x| and
    |d| <= 2^-18 |x|, so each real product carries at most ~3 * 2^-18 |x y|
    (the dropped lo*lo term and the two d terms), plus FP32 accumulation.
    Plain BF16 (error ~2^-9) fails this bound by orders of magnitude."""
    opa, opb = ops
    m, n, k = mnk
    rng = np.random.default_rng(m * 5 + n * 11 + k)
    batch = 2
    a = _rand(rng, batch, k, m) if opa == OPC else _rand(rng, batch, m, k)
    b = _rand(rng, batch, n, k) if opb == OPT else _rand(rng, batch, k, n)
    a = a.astype(np.complex64).astype(np.complex128)
    b = b.astype(np.complex64).astype(np.complex128)
    c = capi.dcs_test_gemm(F32, F32, F32, BF16X3, opa, opb, a, b, variant=variant)
    A = {OPN: a, OPC: np.conj(np.swapaxes(a, 1, 2)), OPJ: np.conj(a)}[opa]
    B = {OPN: b, OPT: np.swapaxes(b, 1, 2)}[opb]
    ref = A @ B
    absA = np.abs(A.real) + np.abs(A.imag)
    absB = np.abs(B.real) + np.abs(B.imag)
    S = absA @ absB                       # sum_k of |real products|
    bound = (4 * 2.0 ** -18 + 2 * (k + 2) * 2.0 ** -24) * S + 1e-30
    err = np.abs(c - ref)
    assert np.all(err <= bound), float(np.max(err / bound))
    if k >= 32:
        # far more accurate than single BF16 rounding of the operands
        assert np.max(err / S) < 2.0 ** -14


def test_bf16x3_tile_shapes_bit_identical(capi):
    rng = np.random.default_rng(9)
    a = _rand(rng, 2, 150, 300).astype(np.complex64).astype(np.complex128)
    b = _rand(rng, 2, 300, 90).astype(np.complex64).astype(np.complex128)
    ref = capi.dcs_test_gemm(F32, F32, F32, BF16X3, OPN, OPN, a, b, variant=0)
    for v in (1, 2, 3):
        np.testing.assert_array_equal(
            capi.dcs_test_gemm(F32, F32, F32, BF16X3, OPN, OPN, a, b, variant=v), ref)


@pytest.mark.parametrize("ct", [F32, F64])
@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("d0,d1,wl,wr", [(1, 2, 1, 4), (5, 7, 4, 4), (33, 300, 4, 1),
                                         (9, 11, 16, 4), (3, 70, 2, 16)])
def test_gate_operator(capi, ct, direction, d0, d1, wl, wr):
    rng = np.random.default_rng(d0 * 31 + d1 + wl * 5 + wr)
    w = _rand(rng, wl, 2, 2, wr)
    if direction == 0:
        x = _rand(rng, d0, wl, 2, d1)
        ref = np.einsum("awty,wstv->asvy", x, w)
    else:
        x = _rand(rng, d0, 2, d1, wr)
        ref = np.einsum("xtcv,wstv->wxsc", x, w)
    if ct == F32:
        x = x.astype(np.complex64).astype(np.complex128)
        w = w.astype(np.complex64).astype(np.complex128)
        ref = (np.einsum("awty,wstv->asvy", x, w) if direction == 0
               else np.einsum("xtcv,wstv->wxsc", x, w))
    out = capi.dcs_test_mpo(ct, direction, d0, d1, wl, wr, x.reshape(-1), w.reshape(-1))
    tol = 1e-12 if ct == F64 else 1e-5
    assert np.max(np.abs(out - ref.reshape(-1))) < tol * np.sqrt(wl * wr * 4)


@pytest.mark.parametrize("use_lds", [0, 1, 2, 4, 5, 6, 7])
@pytest.mark.parametrize("m,n", [(2, 1), (4, 2), (8, 8), (32, 16), (64, 32), (128, 64),
                                 (128, 128), (130, 65),
                                 (512, 256), (34, 17), (100, 100), (512, 512), (511, 257),
                                 (129, 17), (300, 300)])
def test_qr_full_rank(capi, use_lds, m, n):
    rng = np.random.default_rng(m + n)
    f = _rand(rng, m, n)
    q, nrm2 = capi.dcs_test_qr(F64, F64, m, n, 0, use_lds, f.reshape(-1))
    q = q.reshape(m, n)
    qn, _ = np.linalg.qr(f)
    assert abs(nrm2 - np.sum(np.abs(f) ** 2)) < 1e-10 * nrm2
    np.testing.assert_allclose(q.conj().T @ q, np.eye(n), atol=1e-12)
    # same Householder convention as LAPACK: Q agrees element-wise
    assert np.max(np.abs(q - qn)) < 1e-10
    # LQ mode on the conjugate transpose layout
    g = f.conj().T.copy()                                  # n x m
    ql, _ = capi.dcs_test_qr(F64, F64, m, n, 1, use_lds, g.reshape(-1))
    ql = ql.reshape(n, m)
    np.testing.assert_allclose(ql @ ql.conj().T, np.eye(n), atol=1e-12)
    assert np.max(np.abs(ql - qn.conj().T)) < 1e-10


@pytest.mark.parametrize("variant", [0, 2, 3, 4, 5, 6, 7])
def test_qr_rank_deficient_and_normalise(capi, variant):
    rng = np.random.default_rng(1)
    m, n = 64, 32
    f = _rand(rng, m, 3) @ _rand(rng, 3, n)                  # rank 3
    f[:, 5] = 0
    q, _ = capi.dcs_test_qr(F64, F64, m, n, 0, variant, f.reshape(-1))
    q = q.reshape(m, n)
    np.testing.assert_allclose(q.conj().T @ q, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(q @ (q.conj().T @ f), f, atol=1e-11)
    # mode 2: F / |F|
    t, nrm2 = capi.dcs_test_qr(F32, F32, 10, 3, 2, variant if variant in (2, 4, 5) else 0,
                               f[:10, :3].reshape(-1))
    ref = f[:10, :3] / np.linalg.norm(f[:10, :3])
    assert np.max(np.abs(t.reshape(10, 3) - ref)) < 1e-6
    # exactly zero matrix: Q is the leading identity columns
    z, _ = capi.dcs_test_qr(F64, F64, 6, 3, 0, variant, np.zeros(18, complex))
    np.testing.assert_allclose(z.reshape(6, 3), np.eye(6)[:, :3], atol=0)


@pytest.mark.parametrize("variant", [0, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("tiny", [1e-120, 1e-170, 1e-250])
@pytest.mark.parametrize("m,n", [(256, 128), (128, 64)])
def test_qr_tiny_noise_columns(capi, mode, tiny, variant, m, n):
    """Rank-deficient local tensors carry noise far below the FP64 square
    range; the factorisation must stay finite and orthonormal."""
    rng = np.random.default_rng(int(-np.log10(tiny)))
    f = _rand(rng, m, 2) @ _rand(rng, 2, n) + tiny * _rand(rng, m, n)
    f[:, 7] *= tiny
    if mode == 0:
        q, _ = capi.dcs_test_qr(F64, F64, m, n, 0, variant, f.reshape(-1))
        q = q.reshape(m, n)
        gram = q.conj().T @ q
        rec = q @ (q.conj().T @ f)
        target = f
    else:
        g = f.conj().T.copy()
        q, _ = capi.dcs_test_qr(F64, F64, m, n, 1, variant, g.reshape(-1))
        q = q.reshape(n, m)
        gram = q @ q.conj().T
        rec = (g @ q.conj().T) @ q
        target = g
    assert np.all(np.isfinite(q))
    np.testing.assert_allclose(gram, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(rec, target, atol=1e-12)


@pytest.mark.parametrize("m,n", [(64, 32), (513, 200), (600, 300), (1024, 512), (1030, 515),
                                 (1500, 700), (2048, 37), (2048, 1024)])
def test_qr_large_matches_lapack(capi, m, n):
    """Multi-kernel path for more than 512 rows (16-column panels factored
    over 256-row chunks, strip updates over 256-row chunks): same reflectors
    as LAPACK, so Q agrees element-wise, in both the QR and the LQ layout."""
    rng = np.random.default_rng(m * 3 + n)
    f = _rand(rng, m, n)
    qn, _ = np.linalg.qr(f)
    q, nrm2 = capi.dcs_test_qr(F64, F64, m, n, 0, 3, f.reshape(-1))
    q = q.reshape(m, n)
    assert abs(nrm2 - np.sum(np.abs(f) ** 2)) < 1e-10 * nrm2
    assert np.max(np.abs(q.conj().T @ q - np.eye(n))) < 1e-12
    assert np.max(np.abs(q - qn)) < 1e-10
    g = f.conj().T.copy()
    ql, _ = capi.dcs_test_qr(F64, F64, m, n, 1, 3, g.reshape(-1))
    assert np.max(np.abs(ql.reshape(n, m) - qn.conj().T)) < 1e-10
    # complex64 storage in and out, FP64 inside
    q32, _ = capi.dcs_test_qr(F32, F32, m, n, 0, 3, f.astype(np.complex64).reshape(-1))
    assert np.max(np.abs(q32.reshape(m, n) - qn)) < 1e-5


@pytest.mark.parametrize("mode", [0, 1])
def test_qr_large_tiny_noise_columns(capi, mode):
    """Panels the chunked Cholesky QR does not take (a column of noise far
    below the FP64 square range, an exactly rank-deficient block) on the
    multi-kernel path with several row chunks: finite and orthonormal."""
    rng = np.random.default_rng(17 + mode)
    m, n = 1100, 300
    f = _rand(rng, m, 2) @ _rand(rng, 2, n) + 1e-170 * _rand(rng, m, n)
    f[:, 7] *= 1e-170
    f[:, 40] = 0
    if mode == 0:
        q, _ = capi.dcs_test_qr(F64, F64, m, n, 0, 3, f.reshape(-1))
        q = q.reshape(m, n)
        gram, rec, target = q.conj().T @ q, q @ (q.conj().T @ f), f
    else:
        g = f.conj().T.copy()
        q, _ = capi.dcs_test_qr(F64, F64, m, n, 1, 3, g.reshape(-1))
        q = q.reshape(n, m)
        gram, rec, target = q @ q.conj().T, (g @ q.conj().T) @ q, g
    assert np.all(np.isfinite(q))
    np.testing.assert_allclose(gram, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(rec, target, atol=1e-12)


def test_tile_shapes_bit_identical(capi):
    """Every tile shape accumulates each output over K in the same order."""
    rng = np.random.default_rng(5)
    a = _rand(rng, 2, 150, 300).astype(np.complex64).astype(np.complex128)
    b = _rand(rng, 2, 300, 90).astype(np.complex64).astype(np.complex128)
    ref = capi.dcs_test_gemm(F32, F32, F32, F32, OPN, OPN, a, b, variant=0)
    for v in (1, 2, 3):
        np.testing.assert_array_equal(capi.dcs_test_gemm(F32, F32, F32, F32, OPN, OPN, a, b,
                                                         variant=v), ref)


def test_copy_kernel(capi):
    import torch
    src = torch.arange(1 << 20, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    capi.dcs_test_copy(src.data_ptr(), dst.data_ptr(), 4 << 20, 2,
                       torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def _perm_ref(x, perm, conj, ct_out):
    """Definition of the batched transposition: item b's legs reordered."""
    y = np.transpose(x, [0] + [p + 1 for p in perm])
    if conj:
        y = np.conj(y)
    if ct_out == F32:
        y = y.astype(np.complex64)
    return y.astype(np.complex128)


# Leg transpositions of the tree contraction executor (the kind that move a
# bond leg to the end or bring shared legs together), and ragged ones.
PERM_CASES = [
    ((8, 32, 32, 4), (1, 2, 0, 3)),          # middle legs outward
    ((32, 32, 8, 8, 4), (3, 0, 1, 4, 2)),
    ((1024, 8, 4, 8), (0, 3, 2, 1)),
    ((64, 128), (1, 0)),                     # plain matrix transpose
    ((512, 32), (1, 0)),
    ((8, 1024, 32), (0, 2, 1)),
    ((33, 31, 5), (2, 0, 1)),                # no power-of-two leg
    ((7, 3, 100, 2), (3, 2, 1, 0)),
    ((2, 2, 2, 2, 2, 2, 2, 2), (7, 0, 6, 1, 5, 2, 4, 3)),
    ((67, 129), (1, 0)),                     # prime-ish extents larger than a run
    ((5, 1, 7, 1), (3, 2, 1, 0)),            # unit legs
    ((300,), (0,)),                          # rank 1: a copy
]


@pytest.mark.parametrize("cts", [(F32, F32), (F64, F64), (F32, F64), (F64, F32)])
@pytest.mark.parametrize("case", PERM_CASES)
def test_permute(capi, case, cts):
    """Every kernel of the leg transposition against its definition, bit for
    bit (a copy with a storage conversion; the tiled kernel only where it
    takes the transposition)."""
    dims, perm = case
    rng = np.random.default_rng(sum(dims) + 7 * len(dims))
    for batch, conj in ((1, False), (3, True)):
        x = _rand(rng, batch, *dims)
        if cts[0] == F32:
            x = x.astype(np.complex64).astype(np.complex128)
        ref = _perm_ref(x, perm, conj, cts[1])
        for variant in (0, 1, 2):
            try:
                y = capi.dcs_test_permute(cts[0], cts[1], x, perm, conj, variant)
            except RuntimeError as e:
                assert variant == 2 and "tiled kernel does not take" in str(e)
                continue
            np.testing.assert_array_equal(y, ref, err_msg=f"variant {variant}")


def test_permute_tiled_takes_tree_shapes(capi):
    """The tiled kernel takes the transpositions of bond legs with extents of
    powers of two (the tree's), and random ragged ones agree with the
    definition."""
    rng = np.random.default_rng(11)
    for dims, perm in PERM_CASES[:6]:
        x = _rand(rng, 2, *dims).astype(np.complex64).astype(np.complex128)
        y = capi.dcs_test_permute(F32, F32, x, perm, False, 2)
        np.testing.assert_array_equal(y, _perm_ref(x, perm, False, F32))
    choices = [1, 2, 3, 4, 5, 7, 8, 16, 31, 32, 33, 64]
    for _ in range(40):
        rank = int(rng.integers(2, 7))
        dims = [int(rng.choice(choices)) for _ in range(rank)]
        while np.prod(dims) > 200000:
            dims[int(np.argmax(dims))] //= 2
        perm = [int(p) for p in rng.permutation(rank)]
        x = _rand(rng, 2, *dims)
        for variant in (0, 2):
            try:
                y = capi.dcs_test_permute(F64, F64, x, perm, True, variant)
            except RuntimeError as e:
                assert variant == 2 and "tiled kernel does not take" in str(e)
                continue
            np.testing.assert_array_equal(y, _perm_ref(x, perm, True, F64),
                                          err_msg=f"{dims} {perm} variant {variant}")


@pytest.mark.parametrize("variant", [0, 1, 4])
@pytest.mark.parametrize("n,k", [(1, 3), (64, 40), (70, 33), (256, 130), (300, 64)])
def test_gemm_hermitian_mode(capi, variant, n, k):
    """Measurement transfers A^H (E A) and conj(A) (A G^T)^T: in the Hermitian
    mode only the tiles on and below the diagonal are computed; they equal the
    full product's, and every tile above the diagonal is exactly the conjugate
    transpose of its mirror."""
    rng = np.random.default_rng(n * 7 + k + variant)
    tile = {0: 64, 1: 32, 4: 128}[variant]
    a = _rand(rng, 2, k, n).astype(np.complex64).astype(np.complex128)   # stored K x M
    e = _rand(rng, 2, k, k)
    e = e + e.conj().transpose(0, 2, 1)
    ea = e @ a                                                           # E A, K x N
    cases = [((F32, F32, F64, F64), OPC, OPN, a, a, a.conj().transpose(0, 2, 1) @ a),
             ((F32, F64, F64, F64), OPC, OPN, a, ea, a.conj().transpose(0, 2, 1) @ ea)]
    if variant == 4:   # the 128 x 128 tile exists for FP32 accumulation only
        cases = [((F32, F32, F32, F32), OPC, OPN, a, a, a.conj().transpose(0, 2, 1) @ a)]
    i, j = np.indices((n, n))
    below = (i // tile) > (j // tile)
    on_or_below = (i // tile) >= (j // tile)
    for types, opa, opb, x, y, ref in cases:
        full = capi.dcs_test_gemm(*types, opa, opb, x, y, variant=variant).reshape(2, n, n)
        herm = capi.dcs_test_gemm(*types, opa, opb, x, y, variant=variant | 16).reshape(2, n, n)
        tol = 1e-12 if types[3] == F64 else 1e-4
        assert np.max(np.abs(herm - ref)) <= tol * max(1.0, np.max(np.abs(ref)))
        for b in range(2):
            np.testing.assert_array_equal(herm[b][on_or_below], full[b][on_or_below])
            np.testing.assert_array_equal(herm[b][below.T], herm[b].conj().T[below.T])


def test_permute_tree_full_size(capi):
    """The largest leg transposition of the 27-qubit tree workload at its real
    size (4.2 million elements per item: a node tensor with two operator legs),
    tiled kernel and the kernel the library picks, against the definition."""
    dims = [8, 8, 4, 4, 32, 4, 32]               # input legs, row-major
    perm = [0, 2, 4, 6, 1, 5, 3]                 # output leg k = input leg perm[k]
    rng = np.random.default_rng(27)
    x = (_rand(rng, 1, *dims)).astype(np.complex64).astype(np.complex128)
    ref = _perm_ref(x, perm, False, F32)
    for variant in (0, 2):
        y = capi.dcs_test_permute(F32, F32, x, perm, False, variant)
        np.testing.assert_array_equal(y, ref)


@pytest.mark.parametrize("ct", [F32, F64])
@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("d0,d1,k,wl,wr", [(3, 5, 7, 1, 4), (16, 32, 40, 4, 4), (33, 70, 65, 4, 1),
                                           (9, 40, 16, 2, 4), (70, 33, 130, 4, 2),
                                           (64, 64, 256, 4, 4)])
def test_gemm_gate_epilogue(capi, ct, direction, d0, d1, k, wl, wr):
    """The contraction with the gate operator applied in its epilogue (on the
    matrix cores) against the product followed by the operator, for every
    tile shape, and bit-identical across tile shapes."""
    rng = np.random.default_rng(d0 * 13 + d1 * 7 + k + wl * 3 + wr + direction)
    w = _rand(rng, wl, 2, 2, wr)
    if direction == 0:
        a, b = _rand(rng, d0 * wl, k), _rand(rng, k, 2 * d1)
    else:
        a, b = _rand(rng, 2 * d0, k), _rand(rng, d1 * wr, k)
    if ct == F32:
        a, b, w = (z.astype(np.complex64).astype(np.complex128) for z in (a, b, w))
    if direction == 0:
        ref = np.einsum("awty,wstv->asvy", (a @ b).reshape(d0, wl, 2, d1), w).reshape(-1)
    else:
        ref = np.einsum("xtcv,wstv->wxsc", (a @ b.T).reshape(d0, 2, d1, wr), w).reshape(-1)
    scale = np.max(np.abs(ref))
    tol = 1e-12 if ct == F64 else 2e-5
    first = None
    for variant in ([0, 1, 2, 3, 4] if ct == F32 else [0, 1, 2, 3]):
        out = capi.dcs_test_gemm_gate(ct, direction, a, b, w, variant)
        assert np.max(np.abs(out - ref)) <= tol * scale, f"variant {variant}"
        if first is None:
            first = out
        else:
            np.testing.assert_array_equal(out, first, err_msg=f"variant {variant}")
