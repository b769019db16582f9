// Site tensor embedded in larger bond dims with an optional multiple of a
// second tensor added (the warm-start guess of a compression step), or a
// plain batched copy of site tensors between slot regions.
#include "dcs_internal.h"
#include "kernel_util.h"

namespace dcs {
namespace {

constexpr int NT = 256;

template <int CT>
__global__ __launch_bounds__(NT) void embed_kernel(const EmbedArgs a) {
  using T = typename St<CT>::T;
  const int item = blockIdx.y;
  const long long idx = (long long)blockIdx.x * NT + threadIdx.x;
  const long long tot = (long long)a.dl * 2 * a.dr;
  if (idx >= tot) return;
  const int b = (int)(idx % a.dr), sa = (int)(idx / a.dr);   // sa = 2 a + s
  const int al = sa >> 1, s = sa & 1;
  T* dst = reinterpret_cast<T*>(const_cast<char*>(item_ptr(a.dst, a.ids, item)));
  double re = 0.0, im = 0.0;
  if (al < a.kl && b < a.kr) {
    const T* src = reinterpret_cast<const T*>(item_ptr(a.src, a.ids, item));
    const T v = src[((long long)al * 2 + s) * a.kr + b];
    re = v.x;
    im = v.y;
  }
  if (a.init.base) {
    const T* ini = reinterpret_cast<const T*>(item_ptr(a.init, a.ids, item));
    const T u = ini[idx];
    re += a.eta * (double)u.x;
    im += a.eta * (double)u.y;
  }
  T o;
  o.x = re;
  o.y = im;
  dst[idx] = o;
}

}  // namespace

hipError_t launch_embed(int ct, const EmbedArgs& args, hipStream_t s) {
  const long long tot = (long long)args.dl * 2 * args.dr;
  if (args.batch <= 0 || tot <= 0) return hipSuccess;
  if (args.kl < 0 || args.kr < 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((tot + NT - 1) / NT), args.batch), blk(NT);
  if (ct == CT_F32)
    hipLaunchKernelGGL((embed_kernel<CT_F32>), grid, blk, 0, s, args);
  else
    hipLaunchKernelGGL((embed_kernel<CT_F64>), grid, blk, 0, s, args);
  return hipGetLastError();
}

}  // namespace dcs
