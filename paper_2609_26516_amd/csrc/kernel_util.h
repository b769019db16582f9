// Device helpers shared by the non-GEMM kernels: storage types, operand
// addressing, complex arithmetic, scaled sums of squares and reductions.
#pragma once

#include <utility>

#include "dcs_internal.h"

namespace dcs {
namespace {

// f(std::integral_constant<int, k>) for k = 0 .. N-1, expanded at compile time
template <typename Fn, int... K>
__device__ __forceinline__ void static_for_impl(Fn&& f, std::integer_sequence<int, K...>) {
  (f(std::integral_constant<int, K>{}), ...);
}
template <int N, typename Fn>
__device__ __forceinline__ void static_for(Fn&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <int CT>
struct St;
template <>
struct St<CT_F32> {
  using T = float2;
  using R = float;
};
template <>
struct St<CT_F64> {
  using T = double2;
  using R = double;
};

__device__ __forceinline__ const char* item_ptr(const Operand& o, const int* ids, int b) {
  const long long idx = o.by_slot ? ids[b] : b;
  return static_cast<const char*>(o.base) + idx * o.stride;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// conj(a) * b
__device__ __forceinline__ double2 cdotc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over a 256-thread block; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  return scratch[0] + scratch[1] + scratch[2] + scratch[3];
}

// Running (scale, sum of squares) pair: the represented value is
// scale^2 * ssq, accumulated without squaring anything tiny or huge.
__device__ __forceinline__ void ssq_add(double& sc, double& q, double x) {
  x = fabs(x);
  if (x > 0.0) {
    if (sc < x) {
      const double r = sc / x;
      q = 1.0 + q * r * r;
      sc = x;
    } else {
      const double r = x / sc;
      q += r * r;
    }
  }
}

__device__ __forceinline__ void ssq_merge(double& sc, double& q, double sc2, double q2) {
  if (sc2 > sc) {
    const double r = sc / sc2;
    q = q2 + q * r * r;
    sc = sc2;
  } else if (sc2 > 0.0) {
    const double r = sc2 / sc;
    q += q2 * r * r;
  }
}

// Merge of (scale, ssq) over a 256-thread block; every thread gets the result.
__device__ __forceinline__ void block_ssq(double& sc, double& q, double* scratch) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double s2 = __shfl_xor(sc, o, 64), q2 = __shfl_xor(q, o, 64);
    ssq_merge(sc, q, s2, q2);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    scratch[2 * wave] = sc;
    scratch[2 * wave + 1] = q;
  }
  __syncthreads();
  sc = scratch[0];
  q = scratch[1];
  for (int w = 1; w < 4; ++w) ssq_merge(sc, q, scratch[2 * w], scratch[2 * w + 1]);
}

// 1 / d by Smith's scaling (no overflow or underflow of |d|^2).
__device__ __forceinline__ double2 crecip(double2 d) {
  if (fabs(d.x) >= fabs(d.y)) {
    const double r = d.y / d.x, den = d.x + d.y * r;
    return make_double2(1.0 / den, -r / den);
  }
  const double r = d.x / d.y, den = d.x * r + d.y;
  return make_double2(r / den, -1.0 / den);
}

template <int GROUPS, typename G>
__device__ __forceinline__ int find_group(const G* g, int ngroups, int blk) {
  int gi = 0;
  while (gi + 1 < ngroups && blk >= g[gi + 1].blk_begin) ++gi;
  return gi;
}

template <typename TI>
__device__ __forceinline__ double2 to_d2(TI v) {
  return make_double2((double)v.x, (double)v.y);
}

typedef double v4d_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4d_t mfma64(double a, double b, v4d_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// complex accumulate (cr, ci) += (ar + i ai)(br + i bi) on one 16x16x4 step
__device__ __forceinline__ void cmma(double ar, double ai, double br, double bi, v4d_t& cr,
                                     v4d_t& ci) {
  cr = mfma64(ar, br, cr);
  cr = mfma64(-ai, bi, cr);
  ci = mfma64(ar, bi, ci);
  ci = mfma64(ai, br, ci);
}

// Complex accumulation with three real MFMA products per step (Gauss):
// p1 += ar br, p2 += ai bi, p3 += (ar + ai)(br + bi); then re = p1 - p2,
// im = p3 - p1 - p2.  One product fewer than cmma per step, normwise error
// of the same order in FP64.
struct CAcc3 {
  v4d_t p1, p2, p3;
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      p1[r] = 0.0;
      p2[r] = 0.0;
      p3[r] = 0.0;
    }
  }
  __device__ __forceinline__ void add(double ar, double ai, double br, double bi) {
    p1 = mfma64(ar, br, p1);
    p2 = mfma64(ai, bi, p2);
    p3 = mfma64(ar + ai, br + bi, p3);
  }
  __device__ __forceinline__ double re(int r) const { return p1[r] - p2[r]; }
  __device__ __forceinline__ double im(int r) const { return p3[r] - p1[r] - p2[r]; }
};

__device__ __forceinline__ void zero4(v4d_t& a) {
  a[0] = 0;
  a[1] = 0;
  a[2] = 0;
  a[3] = 0;
}

// Wave-wide sum of a double without LDS round trips: four DPP steps (lane
// xor 1, xor 2, half-row mirror, row mirror) leave every lane of a 16-lane
// row with the same row sum, then the four row sums are read with readlane
// and added in a fixed order.  The result is identical in every lane.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffull), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffull), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_d<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v);   // row_half_mirror
  v += dpp_d<0x140>(v);   // row_mirror
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
__device__ __forceinline__ double wave_max_dpp(double v) {
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  v = fmax(v, dpp_d<0x140>(v));
  return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

// Wave sums of N independent doubles, the DPP stages interleaved across the
// values; every lane gets every total (same order as wave_sum_dpp).
template <int N>
__device__ __forceinline__ void wave_sums_dpp(double (&v)[N]) {
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_d<0xB1>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_d<0x4E>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_d<0x141>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] += dpp_d<0x140>(v[q]);
#pragma unroll
  for (int q = 0; q < N; ++q)
    v[q] = (readlane_d(v[q], 0) + readlane_d(v[q], 16)) + (readlane_d(v[q], 32) + readlane_d(v[q], 48));
}

// (sum, max) over NW waves with the DPP wave reduction; every thread gets
// both, summed over the waves in a fixed order.
template <int NW>
__device__ __forceinline__ void block_sum_max_dpp(double& sm, double& mx, double* scratch) {
  sm = wave_sum_dpp(sm);
  mx = wave_max_dpp(mx);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    scratch[2 * wave] = sm;
    scratch[2 * wave + 1] = mx;
  }
  __syncthreads();
  sm = 0.0;
  mx = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    sm += scratch[2 * w];
    mx = fmax(mx, scratch[2 * w + 1]);
  }
}

// Block-wide (sum, max) over NW waves; every thread gets both.
template <int NW>
__device__ __forceinline__ void block_sum_max(double& sm, double& mx, double* scratch) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    sm += __shfl_xor(sm, o, 64);
    mx = fmax(mx, __shfl_xor(mx, o, 64));
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    scratch[2 * wave] = sm;
    scratch[2 * wave + 1] = mx;
  }
  __syncthreads();
  sm = 0.0;
  mx = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    sm += scratch[2 * w];
    mx = fmax(mx, scratch[2 * w + 1]);
  }
}

}  // namespace
}  // namespace dcs
