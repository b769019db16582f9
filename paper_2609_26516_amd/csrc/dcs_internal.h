// Internal declarations shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dcs {

// Storage type of a complex operand.
enum CType { CT_F32 = 0, CT_F64 = 1 };

// Operand transformation in a GEMM C = op(A) op(B):
//   N  as stored (A: M x K row-major, B: K x N row-major)
//   T  transposed (B only: stored N x K)
//   C  conjugate transpose (A only: stored K x M)
//   J  conjugate, not transposed (A only: stored M x K)
enum GemmOp { OP_N = 0, OP_T = 1, OP_C = 2, OP_J = 3 };

// One batched operand: item b lives at base + idx(b) * stride bytes, where
// idx(b) = ids[b] (slot addressing) or b (call-local addressing).
struct Operand {
  const void* base;
  long long stride;
  int by_slot;
  int pad_;
};

struct GemmGroup {
  Operand a, b, c;
  const int* ids;
  int M, N, K, lda, ldb, ldc;
  int batch;
  int tiles_n, tiles_per_item;
  int tile_begin;
  // gate operator applied in the epilogue (GEMM_EPI_*): W[wl][s][t][wr]
  // per batch item, call-locally addressed
  Operand w;
  int wl, wr;
  // Hermitian product (M = N, square tiles, no epilogue): only the tiles on
  // and below the diagonal are computed, tiles_per_item = T (T + 1) / 2 for
  // T tile rows; each tile below the diagonal also writes its conjugate
  // transpose above it
  int herm, pad_;
};

constexpr int GEMM_MAX_GROUPS = 16;
// Epilogues: none (C = op(A) op(B)), or the gate operator of a site applied
// to the product before it is stored (the product itself is never written):
//   RIGHT  product X1[a][wl][t][y] (M = dl wl, N = 2 kr, columns (t, y)) ->
//          C = X2[a][s][wr][y], ldc = kr
//   LEFT   product Y1[x][t][c][wr] (M = 2 kl, N = dr wr) ->
//          C = Y2[wl][x][s][c], ldc = dr
// for operator bonds wl, wr <= GEMM_EPI_WMAX.
enum { GEMM_EPI_NONE = 0, GEMM_EPI_RIGHT = 1, GEMM_EPI_LEFT = 2 };
constexpr int GEMM_EPI_WMAX = 4;
struct GemmArgs {
  GemmGroup g[GEMM_MAX_GROUPS];
  int ngroups;
  int total_tiles;
  int epi;   // one epilogue for every group of a launch
};

// Tile shapes of the GEMM kernel (output tile BM x BN per workgroup).
enum GemmVariant { GEMM_64x64 = 0, GEMM_32x32 = 1, GEMM_128x64 = 2, GEMM_64x128 = 3, GEMM_128x128 = 4 };
constexpr int GEMM_VARIANTS = 5;
// Tile shapes available for an accumulation type: 128 x 128 only for FP32
// accumulation (its FP64 accumulators would not fit the registers).
inline int gemm_variants(int tacc) { return tacc == CT_F32 ? 5 : 4; }
void gemm_tile_shape(int variant, int* bm, int* bn);
// Accumulation mode of a GEMM besides the storage types: split-BF16 products
// (three BF16 MFMA products per real product, FP32 accumulation) over
// complex64 operands.
constexpr int ACC_BF16X3 = 2;
hipError_t launch_gemm_bf16x3(int opa, int opb, int variant, const GemmArgs& args, hipStream_t s);
hipError_t launch_gemm(int ta, int tb, int tc, int tacc, int opa, int opb, int variant,
                       const GemmArgs& args, hipStream_t s);

// Gate-operator application (one batch item per branch).
//   dir 0 (moving right):  X1[a][wl][t][y] -> X2[a][s][wr][y]
//   dir 1 (moving left):   Y1[x][t][c][wr] -> Y2[wl][x][s][c]
// W[wl][s][t][wr] (complex, path precision), addressed call-locally.
struct MpoGroup {
  Operand in, out, w;
  const int* ids;
  int d0, d1;      // dir 0: (chi_l bra, chi_r ket); dir 1: (chi_l ket, chi_r bra)
  int wl, wr;
  int batch;
  int blk_per_item;
  int blk_begin;
};
constexpr int MPO_MAX_GROUPS = 16;
struct MpoArgs {
  MpoGroup g[MPO_MAX_GROUPS];
  int ngroups;
  int total_blocks;
};
hipError_t launch_mpo(int ct, int dir, const MpoArgs& args, hipStream_t s);

// FP64 Householder QR / LQ of the environment tensor (one workgroup per
// branch).  mode 0: F is m x n row-major (m >= n), Q (m x n) written in the
// same layout.  mode 1: F is n x m row-major (n <= m), QR of F^H, Q^H (n x m)
// written.  mode 2: no factorisation, T = F / |F| written in F's layout.
// In every mode |F|^2 is written to nrm2 (FP64, slot- or call-addressed).
struct QrGroup {
  Operand f, q, ws, nrm2;
  const int* ids;
  int m, n, mode;
  int batch;
  int blk_begin;
};
constexpr int QR_MAX_GROUPS = 16;
struct QrArgs {
  QrGroup g[QR_MAX_GROUPS];
  int ngroups;
  int total_blocks;
  int use_lds;     // factor in LDS (all groups fit) instead of the global workspace
};
hipError_t launch_qr(int ct_in, int ct_out, const QrArgs& args, size_t lds_bytes, hipStream_t s);
size_t qr_lds_limit();
// Blocked variant (16-column panels in LDS, FP64 MFMA updates) for m <=
// qr_blocked_max_rows(); the workspace of each item holds m*n + 256*ceil(n/16)
// complex128 values, row-major working matrix first.
hipError_t launch_qr_blocked(int ct_in, int ct_out, const QrArgs& args, int m_max, hipStream_t s);
int qr_blocked_max_rows();
// Left-looking form of the blocked variant (modes 0-2, m >= n, same limits and
// workspace): each panel is updated from the stored V of the earlier panels
// just before it is factored, and Q is formed 16 columns at a time.  split:
// two launches, the factorisations, then one workgroup per 16-column block of
// each Q (for batches too small to fill the chip).  Matrices of at most 128
// rows run with 256 threads each, or 128 when there are more than 512 of
// them; threads = 128 or 256 forces that width (tests), 0 chooses.
hipError_t launch_qr_left(int ct_in, int ct_out, const QrArgs& args, int m_max, bool split,
                          hipStream_t s, int threads = 0);
// Largest number of matrices for which the runtime splits the left-looking QR.
int qr_split_max_items();
// Multi-kernel variant for qr_blocked_max_rows() < m <= qr_large_max_rows()
// (modes 0 and 1): panels factored by one workgroup per matrix, trailing
// updates and the backward Q accumulation spread over 16-column strips.  The
// workspace of each item holds qr_large_ws_elems(m, n) complex128 values.
hipError_t launch_qr_large(int ct_in, int ct_out, const QrArgs& args, hipStream_t s);
// Spread variant for small batches of matrices of at most qr_spread_max_rows()
// rows (modes 0 and 1): one workgroup per matrix factors each 16-column panel
// (Cholesky QR and Householder reconstruction where the panel allows it),
// the trailing updates and the Q blocks are spread over many workgroups.  The
// workspace of each item holds qr_large_ws_elems(m, n) complex128 values.
hipError_t launch_qr_spread(int ct_in, int ct_out, const QrArgs& args, hipStream_t s);
int qr_spread_max_rows();
// Largest number of matrices for which the runtime takes the spread path.
int qr_spread_max_items();
// The Q blocks of the left-looking kernel alone (one workgroup per 16-column
// block of each Q) from the explicit V (m x n) and the T factors after it at
// each item's workspace.
hipError_t launch_qr_qblocks(int ct_in, int ct_out, const QrArgs& args, int m_max, hipStream_t s);
int qr_large_max_rows();
size_t qr_large_ws_elems(int m, int n);

// n_m = Re sum_{a,b} conj(A[a][m][b]) Z[a][m][b] for m = 0, 1 (FP64), one
// workgroup per branch; Z = A when z.base is null.
struct NormGroup {
  Operand a, z, out;
  const int* ids;
  int dl, dr;
  int batch;
  int blk_begin;
};
constexpr int NORM_MAX_GROUPS = 16;
struct NormArgs {
  NormGroup g[NORM_MAX_GROUPS];
  int ngroups;
  int total_blocks;
};
hipError_t launch_norms(int ct_a, int ct_z, const NormArgs& args, hipStream_t s);

// Collapse site tensor A[dl][2][dr]: slice 1-m zeroed, slice m scaled by the
// FP64 factor `scale` (= 1/sqrt(n_m)).
// dst[a][s][b] (dl x 2 x dr) = src[a][s][b] where a < kl and b < kr (src is
// kl x 2 x kr), else 0, plus eta * init[a][s][b] when init.base is set: the
// ket embedded in the bra's bond dims with seeded completion, or (eta = 0,
// equal dims) a batched copy.  One launch per site, item b at slot ids[b].
struct EmbedArgs {
  Operand dst, src, init;
  const int* ids;
  int dl, dr, kl, kr;
  int batch;
  double eta;
};
hipError_t launch_embed(int ct, const EmbedArgs& args, hipStream_t s);

struct CollapseItem {
  void* a;
  double scale;
  int dl, dr, m;
  int pad_;
};
hipError_t launch_collapse(int ct, const CollapseItem* items_dev, int n_items, int max_elems,
                           hipStream_t s);

// Device-side sampling and collapse of site tensor A[dl][2][dr]: with
// (n_0, n_1) = norms[2k], [2k + 1] and u = u[idx], outcome m = (u >= p_0),
// switched to the other outcome if p_m <= eps; slice 1-m zeroed, slice m
// scaled by 1/sqrt(n_m) (FP64); outcome[idx] = m, pm[idx] = p_m (pm NaN and
// outcome -1, tensor untouched, when n_0 + n_1 is not positive and finite).
struct SampleItem {
  void* a;
  int dl, dr, k, idx;
};
hipError_t launch_sample_collapse(int ct, const SampleItem* items_dev, int n_items, int max_elems,
                                  const double* norms, const double* u, double eps, int* outcome,
                                  double* pm, hipStream_t s);

// Batched transposition: output element o (row-major over dims[0..rank))
// reads input element sum_k c_k in_stride[k] (c the output coordinates),
// conjugated when conj, converted between the storage types of the launch.
constexpr int PERMUTE_MAX_RANK = 12;
struct PermuteArgs {
  Operand in, out;
  const int* ids;
  int rank, conj, batch, pad_;
  long long total;
  int dims[PERMUTE_MAX_RANK];
  long long in_stride[PERMUTE_MAX_RANK];
};
// variant: PERMUTE_AUTO picks the kernel, PERMUTE_ELEMENTWISE and
// PERMUTE_TILED force one (the tiled kernel returns hipErrorInvalidValue for
// a transposition it cannot tile).
enum { PERMUTE_AUTO = 0, PERMUTE_ELEMENTWISE = 1, PERMUTE_TILED = 2 };
hipError_t launch_permute(int ct_in, int ct_out, const PermuteArgs& a, hipStream_t s,
                          int variant = PERMUTE_AUTO);
// The tiled kernel's plan for a transposition (host only, for tests): pi, pc,
// pa, po, pitch, tiles, elements per thread, ni, nc, na, nr, then the leg
// descriptors (I: extents, LDS weights; C: extents, input strides, LDS
// weights; A: extents, output strides; rest: extents, input strides, output
// strides).  False when the tiled kernel does not take the transposition or
// out_len is too small.
bool permute_tile_plan(const PermuteArgs& a, int esize, int* out, int out_len);

// Sum of the split-K partial products of a contraction (complex128):
// out[item][e] = sum_{s < parts} part[item][s * mn + e] for e < mn, the
// parts added in order s = 0, 1, ...
struct KsumArgs {
  Operand part, out;
  const int* ids;
  int parts, mn, batch, pad_;
};
hipError_t launch_ksum(const KsumArgs& a, hipStream_t s);

// Writes (1, 0), (0, 0) as two complex words at each listed address.
hipError_t launch_fill_unit(int ct, void* const* ptrs_dev, int n, hipStream_t s);

}  // namespace dcs
