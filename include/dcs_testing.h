/*
 * dcs_testing.h -- kernel-level entry points of libdcs.so for unit tests.
 *
 * Each call runs one internal kernel of the compression step on host data
 * (complex128 interleaved in, complex128 interleaved out), allocating and
 * freeing its own device buffers, and synchronises `stream` (hipStream_t).
 * Storage types: 0 complex64, 1 complex128.  They exist so the contraction,
 * gate-operator and QR kernels can be checked one by one against plain
 * references; the simulation path does not use them.  Status codes as in
 * dcs.h.
 */
#ifndef DCS_TESTING_H
#define DCS_TESTING_H

#ifdef __cplusplus
extern "C" {
#endif

/* C[b] = op(A[b]) op(B[b]) for b < batch.  opa: 0 N (A stored M x K),
 * 2 C (conjugate transpose, A stored K x M), 3 J (conjugate, stored M x K);
 * opb: 0 N (B stored K x N), 1 T (B stored N x K).  Items are contiguous:
 * A[b] at b * M * K, B[b] at b * K * N, C[b] at b * M * N.  ta/tb/tc are the
 * storage types of A, B, C and tacc the accumulation type (1 = FP64 MFMA,
 * 0 = FP32 MFMA, 2 = split-BF16 products on BF16 MFMA with FP32 accumulation,
 * complex64 storage only); only the combinations the library uses are available
 * (DCS_EINVAL otherwise).  variant: output tile shape 0 64x64, 1 32x32,
 * 2 128x64, 3 64x128, 4 128x128 (FP32 accumulation only); plus 16 for the
 * Hermitian mode of the measurement transfers (M = N, square tiles, not the
 * split-BF16 form): only the tiles on and below the diagonal are computed and
 * those below it also write their conjugate transpose above it, so C is
 * exactly Hermitian when the product is Hermitian. */
int dcs_test_gemm(int ta, int tb, int tc, int tacc, int opa, int opb, int M, int N, int K,
                  int batch, int variant, const double *A, const double *B, double *C,
                  void *stream);

/* Contraction with the gate operator applied in its epilogue (the fused
 * form of the compression step, operator bonds wl, wr in {1, 2, 4}), one
 * item, storage and accumulation type ct (0 complex64 / FP32, 1 complex128 /
 * FP64).  dir 0 (moving right): X1 = A B (A M x K, B K x N row-major, M =
 * d0 wl, N = 2 d1, X1[a][wl][t][y]) -> C = X2[a][s][wr][y] (d0 x 2 x wr x
 * d1).  dir 1 (moving left): Y1 = A B^T (A M x K, B stored N x K, M = 2 d0,
 * N = d1 wr, Y1[x][t][c][wr]) -> C = Y2[wl][x][s][c] (wl x d0 x 2 x d1).
 * W[wl][s][t][wr] as for dcs_test_mpo; variant: tile shape as for
 * dcs_test_gemm (128 x 128 for complex64 only). */
int dcs_test_gemm_gate(int ct, int dir, int M, int N, int K, int wl, int wr, int variant,
                       const double *A, const double *B, const double *W, double *C,
                       void *stream);

/* Gate-operator application.  dir 0: in X1[d0][wl][2][d1] -> out
 * X2[d0][2][wr][d1]; dir 1: in Y1[d0][2][d1][wr] -> out Y2[wl][d0][2][d1];
 * w = W[wl][2][2][wr]. */
int dcs_test_mpo(int ct, int dir, int d0, int d1, int wl, int wr, const double *in,
                 const double *w, double *out, void *stream);

/* FP64 Householder QR of one matrix.  mode 0: F is m x n row-major, Q (m x n)
 * returned; mode 1: F is n x m row-major, Q^H of QR(F^H) (n x m) returned;
 * mode 2: F / |F| returned.  *nrm2_out = |F|^2.  variant: 0 unblocked with the
 * matrix in global memory, 1 unblocked in LDS when it fits, 2 blocked
 * (16-column panels in LDS, FP64 MFMA updates; m <= 512), 3 large-matrix
 * multi-kernel path (modes 0 and 1, m <= 2048), 4 left-looking form of the
 * blocked variant (the one compression steps use; m <= 512), 5 the same in
 * two launches (factorisation, then one workgroup per 16-column block of Q),
 * as used for batches that do not fill the chip, 6 variant 4 with two-wave
 * workgroups for m <= 128 (as used for batches of more than 512 such
 * matrices; larger m as variant 4), 7 the spread path (modes 0 and 1,
 * n <= m <= 512: one workgroup per 16-column panel, trailing updates and Q
 * blocks over many workgroups, as used for small batches of large matrices). */
int dcs_test_qr(int ct_in, int ct_out, int m, int n, int mode, int variant, const double *F,
                double *Q, double *nrm2_out, void *stream);

/* Device-to-device copy of `bytes` (a multiple of 16; both pointers device
 * memory, 16-byte aligned) from src to dst, `reps` times, enqueued on the
 * stream without synchronisation: `bytes` read and `bytes` written per launch.
 * Reference point that converts the profiler's HBM byte counters. */
int dcs_test_copy(const void *src, void *dst, size_t bytes, int reps, void *stream);

/* Batched transposition with optional conjugation and storage conversion.
 * `in` holds `batch` items, each a row-major tensor of `rank` legs with
 * extents dims[0..rank); item b of `out` is item b of `in` with its legs in
 * the order perm (output leg k = input leg perm[k]), conjugated when conj.
 * variant: 0 the kernel the library picks, 1 the element-wise kernel, 2 the
 * LDS-tiled kernel (DCS_EINVAL where it does not take the transposition).
 * rank <= 12, batch * prod(dims) <= 2^28. */
int dcs_test_permute(int ct_in, int ct_out, int rank, const int *dims, const int *perm, int conj,
                     int batch, int variant, const double *in, double *out, void *stream);

/* Host only (no device call): the tiled kernel's plan for the transposition
 * of dcs_test_permute with elements of esize bytes (8 or 16).  *planned = 1
 * with the plan in out (pi, pc, pa, po, pitch, tiles, elements per thread,
 * ni, nc, na, nr, then the leg descriptors: I extents and LDS weights, C
 * extents, input strides and LDS weights, A extents and output strides, the
 * tile-indexing legs' extents, input strides and output strides), or 0 when
 * the tiled kernel does not take the transposition.  For checking the
 * planner's index maps on the host. */
int dcs_test_permute_plan(int rank, const int *dims, const int *perm, int esize, int *out,
                          int out_len, int *planned);

/* The same transposition on device buffers (`in`: batch items of the input
 * storage type, `out`: batch items of the output type, both device memory),
 * `reps` times, enqueued on the stream without synchronisation.  For timing
 * the kernels on the transpositions of a workload. */
int dcs_test_permute_dev(int ct_in, int ct_out, int rank, const int *dims, const int *perm,
                         int conj, int batch, int variant, const void *in, void *out, int reps,
                         void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DCS_TESTING_H */
