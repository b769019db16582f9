// Batched transposition of complex tensors, with optional conjugation and
// conversion between complex64 and complex128 storage: the data movement
// between the contractions of the tree tensor network, whose operands are
// brought into the row-major matrix layouts the GEMM kernels take.
//
// Output element o (row-major over the output dims) reads the input at
// sum_k c_k in_stride[k], c the output coordinates.  One grid row per batch
// item, items addressed through the slot-id table or call-locally.
#include "dcs_internal.h"
#include <algorithm>

#include "kernel_util.h"

namespace dcs {
namespace {

template <int CTI, int CTO>
__global__ __launch_bounds__(256) void permute_kernel(const PermuteArgs a) {
  using TI = typename St<CTI>::T;
  using TO = typename St<CTO>::T;
  const int item = blockIdx.y;
  const TI* __restrict__ src = reinterpret_cast<const TI*>(item_ptr(a.in, a.ids, item));
  TO* __restrict__ dst = reinterpret_cast<TO*>(const_cast<char*>(item_ptr(a.out, a.ids, item)));
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x; o < a.total; o += step) {
    long long rem = o, off = 0;
    for (int k = a.rank - 1; k >= 0; --k) {
      const long long d = a.dims[k];
      const long long c = rem % d;
      rem /= d;
      off += c * a.in_stride[k];
    }
    const TI v = src[off];
    TO w;
    w.x = v.x;
    w.y = a.conj ? -v.y : v.y;
    dst[o] = w;
  }
}

}  // namespace

hipError_t launch_permute(int ct_in, int ct_out, const PermuteArgs& a, hipStream_t s) {
  if (a.batch <= 0 || a.total <= 0) return hipSuccess;
  if (a.rank < 1 || a.rank > PERMUTE_MAX_RANK || a.batch > 65535) return hipErrorInvalidValue;
  const long long blocks = (a.total + 255) / 256;
  const dim3 grid((unsigned)std::min<long long>(blocks, 4096), (unsigned)a.batch), blk(256);
#define DCS_PERM(I, O)                                                      \
  if (ct_in == I && ct_out == O) {                                          \
    hipLaunchKernelGGL((permute_kernel<I, O>), grid, blk, 0, s, a);         \
    return hipGetLastError();                                               \
  }
  DCS_PERM(CT_F32, CT_F32)
  DCS_PERM(CT_F64, CT_F64)
  DCS_PERM(CT_F32, CT_F64)
  DCS_PERM(CT_F64, CT_F32)
#undef DCS_PERM
  return hipErrorInvalidValue;
}

}  // namespace dcs
