// Host-side pieces of the runtime shared by the MPS entry points
// (runtime.cpp, which defines them) and the tree-tensor-network entry points
// (tree.cpp): status reporting, the batched GEMM / QR / transposition
// launchers with their timing and tile tuning, and the two-qubit gate split.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <new>
#include <string>
#include <vector>

#include "dcs.h"
#include "dcs_internal.h"

namespace dcs {
namespace rt {

// Sets the thread-local message of dcs_last_error and returns `code`.
int fail(int code, const std::string& msg);

// Entry points return a status and never let a C++ exception cross the C ABI.
template <typename F>
int guarded(F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail(DCS_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(DCS_EINVAL, "internal error");
  }
}

// One batched GEMM C = op(A) op(B) (see GemmGroup) or QR job (see QrGroup).
struct GemmJob {
  Operand a, b, c;
  const int* ids;
  int M, N, K, lda, ldb, ldc, batch;
  // gate operator applied in the epilogue (GEMM_EPI_*, see GemmArgs)
  int epi = GEMM_EPI_NONE;
  Operand w = Operand{nullptr, 0, 0, 0};
  int wl = 0, wr = 0;
  // the product is Hermitian (M = N): computed on and below the diagonal
  // where the tile shape is square, and mirrored
  int herm = 0;
};
struct QrJob {
  Operand f, q, ws, nrm2;
  const int* ids;
  int m, n, mode, batch;
};

// Timing classes of dcs_ctx_set_timing; CLS_BY_FORM files a GEMM under the
// class of its operand form (0-3).
enum { CLS_BY_FORM = -1, CLS_QR = 5, CLS_MEAS = 6, CLS_OTHER = 7 };

int gemm(dcs_ctx* ctx, int ta, int tb, int tc, int tacc, int opa, int opb,
         const std::vector<GemmJob>& jobs, hipStream_t s, int cls);
int qr(dcs_ctx* ctx, int ct_in, int ct_out, const std::vector<QrJob>& jobs, hipStream_t s);
int permute(dcs_ctx* ctx, int ct_in, int ct_out, const PermuteArgs& a, hipStream_t s);
int ksum(dcs_ctx* ctx, const KsumArgs& a, hipStream_t s, int cls);
// Resolves pending tile-shape trials (after the stream has been synchronised).
void tune_sync(dcs_ctx* ctx);
int ctx_device(const dcs_ctx* ctx);

// complex128 workspace elements of one QR job of an m x n matrix.
size_t qr_job_ws_elems(int m, int n, int mode);

// Operator-Schmidt split of a two-qubit gate (16 complex128, row-major, basis
// |q0 q1>): G[(s0 s1), (t0 t1)] = sum_w left[s0][t0][w] right[w][s1][t1],
// r terms (singular values above 1e-14 of the largest).
struct GateSplit {
  int r = 0;
  std::vector<std::complex<double>> left;    // [s][t][w]
  std::vector<std::complex<double>> right;   // [w][s][t]
};
GateSplit split_gate(dcs_ctx* ctx, const double* mat);

inline Operand local(const void* base, long long stride) {
  Operand o;
  o.base = base;
  o.stride = stride;
  o.by_slot = 0;
  o.pad_ = 0;
  return o;
}

}  // namespace rt
}  // namespace dcs
