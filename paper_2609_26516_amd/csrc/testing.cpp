// Kernel-level test entry points (include/dcs_testing.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dcs.h"
#include "dcs_internal.h"
#include "dcs_testing.h"

using namespace dcs;

namespace dcs {
int testing_fail(int code, const std::string& msg);
}

namespace {

// Entry points return a status and never let a C++ exception (a failed host
// allocation inside a std container, say) cross the C ABI.
template <typename F>
int guarded(F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return testing_fail(DCS_ENOMEM, "host allocation failed");
  } catch (...) {
    return testing_fail(DCS_EINVAL, "internal error");
  }
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

size_t csz(int ct) { return ct == CT_F32 ? 8 : 16; }

std::vector<char> pack(int ct, const double* src, size_t count) {
  std::vector<char> out(count * csz(ct));
  for (size_t i = 0; i < count; ++i) {
    if (ct == CT_F32) {
      reinterpret_cast<float2*>(out.data())[i] = make_float2((float)src[2 * i], (float)src[2 * i + 1]);
    } else {
      reinterpret_cast<double2*>(out.data())[i] = make_double2(src[2 * i], src[2 * i + 1]);
    }
  }
  return out;
}

void unpack(int ct, const std::vector<char>& in, double* dst, size_t count) {
  for (size_t i = 0; i < count; ++i) {
    if (ct == CT_F32) {
      const float2 v = reinterpret_cast<const float2*>(in.data())[i];
      dst[2 * i] = v.x;
      dst[2 * i + 1] = v.y;
    } else {
      const double2 v = reinterpret_cast<const double2*>(in.data())[i];
      dst[2 * i] = v.x;
      dst[2 * i + 1] = v.y;
    }
  }
}

#define T_HIP(expr)                                                                           \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return testing_fail(DCS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

int upload(int ct, const double* src, size_t count, DevBuf& b, hipStream_t s) {
  std::vector<char> h = pack(ct, src, count);
  T_HIP(hipMalloc(&b.p, std::max<size_t>(h.size(), 256)));
  T_HIP(hipMemcpyAsync(b.p, h.data(), h.size(), hipMemcpyHostToDevice, s));
  T_HIP(hipStreamSynchronize(s));
  return DCS_OK;
}

Operand op_of(const void* p, long long stride) {
  Operand o;
  o.base = p;
  o.stride = stride;
  o.by_slot = 0;
  o.pad_ = 0;
  return o;
}

// Plain device-to-device copy: one 16-byte load and store per thread and
// iteration, grid-stride.  Reference point for the HBM byte counters.
__global__ void __launch_bounds__(256) copy16_kernel(const int4* __restrict__ src,
                                                     int4* __restrict__ dst, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
}

// Arguments of a batched transposition of row-major items `dims` into leg
// order `perm`, item b at base + b * (item bytes); DCS_OK or the error.
int permute_args(int ct_in, int ct_out, int rank, const int* dims, const int* perm, int conj,
                 int batch, int variant, PermuteArgs* a) {
  if (rank < 1 || rank > PERMUTE_MAX_RANK || batch < 1 || batch > 65535 || !dims || !perm ||
      variant < 0 || variant > 2 || ct_in < 0 || ct_in > 1 || ct_out < 0 || ct_out > 1)
    return testing_fail(DCS_EINVAL, "bad permute test arguments");
  long long total = 1;
  std::vector<long long> stride(rank, 1);
  std::vector<int> seen(rank, 0);
  for (int k = rank - 1; k >= 0; --k) {
    if (dims[k] < 1) return testing_fail(DCS_EINVAL, "permute test: leg extents must be positive");
    stride[k] = total;
    total *= dims[k];
    if (total > (1LL << 28)) return testing_fail(DCS_EINVAL, "permute test: too large");
  }
  for (int k = 0; k < rank; ++k)
    if (perm[k] < 0 || perm[k] >= rank || seen[perm[k]]++)
      return testing_fail(DCS_EINVAL, "permute test: perm is not a permutation");
  if (total * batch > (1LL << 28)) return testing_fail(DCS_EINVAL, "permute test: too large");
  std::memset(a, 0, sizeof(*a));
  a->in = op_of(nullptr, total * (long long)csz(ct_in));
  a->out = op_of(nullptr, total * (long long)csz(ct_out));
  a->ids = nullptr;
  a->rank = rank;
  a->conj = conj ? 1 : 0;
  a->batch = batch;
  a->total = total;
  for (int k = 0; k < rank; ++k) {
    a->dims[k] = dims[perm[k]];
    a->in_stride[k] = stride[perm[k]];
  }
  return DCS_OK;
}

int run_permute(int ct_in, int ct_out, const PermuteArgs& a, int variant, hipStream_t s) {
  const hipError_t e = launch_permute(ct_in, ct_out, a, s, variant);
  if (e == hipErrorInvalidValue && variant == PERMUTE_TILED)
    return testing_fail(DCS_EINVAL, "permute test: the tiled kernel does not take this transposition");
  T_HIP(e);
  return DCS_OK;
}

}  // namespace

extern "C" {

int dcs_test_copy(const void* src, void* dst, size_t bytes, int reps, void* stream) {
  return guarded([&]() -> int {
    if (!src || !dst || bytes % 16 != 0 || reps < 1 || reps > 1000)
      return testing_fail(DCS_EINVAL, "bad copy test arguments");
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
      return testing_fail(DCS_EINVAL, "copy buffers must be 16-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t n16 = bytes / 16;
    const int blocks = (int)std::min<size_t>(8192, (n16 + 255) / 256 + (n16 == 0));
    for (int r = 0; r < reps; ++r) {
      hipLaunchKernelGGL(copy16_kernel, dim3(blocks), dim3(256), 0, s,
                         static_cast<const int4*>(src), static_cast<int4*>(dst), n16);
      T_HIP(hipGetLastError());
    }
    return DCS_OK;
  });
}

int dcs_test_gemm(int ta, int tb, int tc, int tacc, int opa, int opb, int M, int N, int K,
                  int batch, int variant, const double* A, const double* B, double* C,
                  void* stream) {
  return guarded([&]() -> int {
    if (M < 1 || N < 1 || K < 1 || batch < 1 || !A || !B || !C)
      return testing_fail(DCS_EINVAL, "bad gemm test arguments");
    if ((opa != OP_N && opa != OP_C && opa != OP_J) || (opb != OP_N && opb != OP_T))
      return testing_fail(DCS_EINVAL, "bad op");
    const bool herm = (variant & 16) != 0;
    variant &= ~16;
    if (variant < 0 || variant >= GEMM_VARIANTS) return testing_fail(DCS_EINVAL, "bad tile shape");
    int bm = 64, bn = 64;
    gemm_tile_shape(variant, &bm, &bn);
    if (herm && (M != N || bm != bn))
      return testing_fail(DCS_EINVAL, "the Hermitian mode takes M = N and a square tile");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf da, db, dc;
    const size_t na = (size_t)M * K * batch, nb = (size_t)K * N * batch, nc = (size_t)M * N * batch;
    int rc = upload(ta, A, na, da, s);
    if (rc) return rc;
    rc = upload(tb, B, nb, db, s);
    if (rc) return rc;
    T_HIP(hipMalloc(&dc.p, nc * csz(tc)));
    GemmArgs args;
    std::memset(&args, 0, sizeof(args));
    GemmGroup& g = args.g[0];
    g.a = op_of(da.p, (long long)M * K * csz(ta));
    g.b = op_of(db.p, (long long)K * N * csz(tb));
    g.c = op_of(dc.p, (long long)M * N * csz(tc));
    g.ids = nullptr;
    g.M = M;
    g.N = N;
    g.K = K;
    g.lda = (opa == OP_C) ? M : K;
    g.ldb = (opb == OP_T) ? K : N;
    g.ldc = N;
    g.batch = batch;
    g.tiles_n = (N + bn - 1) / bn;
    g.tiles_per_item = ((M + bm - 1) / bm) * g.tiles_n;
    if (herm) {
      if (tacc == ACC_BF16X3) return testing_fail(DCS_EINVAL, "no Hermitian mode in the split-BF16 form");
      g.herm = 1;
      g.tiles_per_item = g.tiles_n * (g.tiles_n + 1) / 2;
    }
    g.tile_begin = 0;
    args.ngroups = 1;
    args.total_tiles = g.tiles_per_item * batch;
    hipError_t e = launch_gemm(ta, tb, tc, tacc, opa, opb, variant, args, s);
    if (e == hipErrorInvalidValue) return testing_fail(DCS_EINVAL, "type/op combination not built");
    T_HIP(e);
    std::vector<char> h(nc * csz(tc));
    T_HIP(hipMemcpyAsync(h.data(), dc.p, h.size(), hipMemcpyDeviceToHost, s));
    T_HIP(hipStreamSynchronize(s));
    unpack(tc, h, C, nc);
    return DCS_OK;
  });
}

int dcs_test_mpo(int ct, int dir, int d0, int d1, int wl, int wr, const double* in,
                 const double* w, double* out, void* stream) {
  return guarded([&]() -> int {
    if (d0 < 1 || d1 < 1 || wl < 1 || wr < 1 || wl > 16 || wr > 16 || !in || !w || !out)
      return testing_fail(DCS_EINVAL, "bad mpo test arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf di, dw, dout;
    const size_t nin = (size_t)d0 * d1 * 2 * (dir == 0 ? wl : wr);
    const size_t nout = (size_t)d0 * d1 * 2 * (dir == 0 ? wr : wl);
    int rc = upload(ct, in, nin, di, s);
    if (rc) return rc;
    rc = upload(ct, w, (size_t)wl * 4 * wr, dw, s);
    if (rc) return rc;
    T_HIP(hipMalloc(&dout.p, nout * csz(ct)));
    MpoArgs args;
    std::memset(&args, 0, sizeof(args));
    MpoGroup& g = args.g[0];
    g.in = op_of(di.p, 0);
    g.out = op_of(dout.p, 0);
    g.w = op_of(dw.p, 0);
    g.ids = nullptr;
    g.d0 = d0;
    g.d1 = d1;
    g.wl = wl;
    g.wr = wr;
    g.batch = 1;
    g.blk_per_item = (int)(((long long)d0 * d1 + 255) / 256);
    g.blk_begin = 0;
    args.ngroups = 1;
    args.total_blocks = g.blk_per_item;
    T_HIP(launch_mpo(ct, dir, args, s));
    std::vector<char> h(nout * csz(ct));
    T_HIP(hipMemcpyAsync(h.data(), dout.p, h.size(), hipMemcpyDeviceToHost, s));
    T_HIP(hipStreamSynchronize(s));
    unpack(ct, h, out, nout);
    return DCS_OK;
  });
}

int dcs_test_qr(int ct_in, int ct_out, int m, int n, int mode, int use_lds, const double* F,
                double* Q, double* nrm2_out, void* stream) {
  return guarded([&]() -> int {
    if (m < 1 || n < 1 || n > 1024 || (mode != 2 && m < n) || mode < 0 || mode > 2 || !F || !Q ||
        !nrm2_out)
      return testing_fail(DCS_EINVAL, "bad qr test arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf df, dq, dws, dn;
    const size_t mn = (size_t)m * n;
    int rc = upload(ct_in, F, mn, df, s);
    if (rc) return rc;
    T_HIP(hipMalloc(&dq.p, mn * csz(ct_out)));
    T_HIP(hipMalloc(&dws.p, std::max(mn + ((size_t)n / 16 + 2) * 256, qr_large_ws_elems(m, n)) * 16));
    T_HIP(hipMalloc(&dn.p, 256));
    QrArgs args;
    std::memset(&args, 0, sizeof(args));
    QrGroup& g = args.g[0];
    g.f = op_of(df.p, 0);
    g.q = op_of(dq.p, 0);
    g.ws = op_of(dws.p, 0);
    g.nrm2 = op_of(dn.p, 0);
    g.ids = nullptr;
    g.m = m;
    g.n = n;
    g.mode = mode;
    g.batch = 1;
    g.blk_begin = 0;
    args.ngroups = 1;
    args.total_blocks = 1;
    const size_t lds = mn * 16;
    if (use_lds == 7) {   // spread variant (small batches)
      if (mode == 2 || m > qr_spread_max_rows() || m < n)
        return testing_fail(DCS_EINVAL, "the spread QR takes modes 0/1 and n <= m <= 512");
      T_HIP(launch_qr_spread(ct_in, ct_out, args, s));
    } else if (use_lds == 3) {   // large-matrix variant
      if (mode == 2 || m > qr_large_max_rows())
        return testing_fail(DCS_EINVAL, "the large-matrix QR takes modes 0/1 and m <= 2048");
      T_HIP(launch_qr_large(ct_in, ct_out, args, s));
    } else if (use_lds == 2 || use_lds == 4 || use_lds == 5 || use_lds == 6) {
      // blocked: right-looking, left-looking, left-looking split, left-looking
      // with two-wave workgroups for up to 128 rows
      if (m > qr_blocked_max_rows()) return testing_fail(DCS_EINVAL, "too many rows for the blocked QR");
      args.use_lds = 1;
      if (use_lds == 2)
        T_HIP(launch_qr_blocked(ct_in, ct_out, args, m, s));
      else
        T_HIP(launch_qr_left(ct_in, ct_out, args, m, use_lds == 5, s, use_lds == 6 ? 128 : 0));
    } else {
      args.use_lds = (use_lds && mode != 2 && lds <= qr_lds_limit()) ? 1 : 0;
      T_HIP(launch_qr(ct_in, ct_out, args, args.use_lds ? lds : 0, s));
    }
    std::vector<char> h(mn * csz(ct_out));
    T_HIP(hipMemcpyAsync(h.data(), dq.p, h.size(), hipMemcpyDeviceToHost, s));
    T_HIP(hipMemcpyAsync(nrm2_out, dn.p, sizeof(double), hipMemcpyDeviceToHost, s));
    T_HIP(hipStreamSynchronize(s));
    unpack(ct_out, h, Q, mn);
    return DCS_OK;
  });
}

int dcs_test_gemm_gate(int ct, int dir, int M, int N, int K, int wl, int wr, int variant,
                       const double* A, const double* B, const double* W, double* C,
                       void* stream) {
  return guarded([&]() -> int {
    auto pow2 = [](int w) { return w >= 1 && w <= GEMM_EPI_WMAX && (w & (w - 1)) == 0; };
    if (M < 1 || N < 1 || K < 1 || !A || !B || !W || !C || (ct != CT_F32 && ct != CT_F64) ||
        (dir != 0 && dir != 1) || !pow2(wl) || !pow2(wr) || variant < 0 || variant >= GEMM_VARIANTS ||
        (ct == CT_F64 && variant == GEMM_128x128))
      return testing_fail(DCS_EINVAL, "bad gate-epilogue test arguments");
    if (dir == 0 ? (M % wl != 0 || N % 2 != 0) : (M % 2 != 0 || N % wr != 0))
      return testing_fail(DCS_EINVAL, "gate-epilogue test: shape does not hold whole groups");
    int bm = 64, bn = 64;
    gemm_tile_shape(variant, &bm, &bn);
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf da, db, dw, dc;
    // output: d0 x 2 x wr x d1 (M = d0 wl, N = 2 d1) or wl x d0 x 2 x d1 (M = 2 d0, N = d1 wr)
    const size_t na = (size_t)M * K, nb = (size_t)K * N, nw = (size_t)wl * 4 * wr;
    const size_t nc = dir == 0 ? (size_t)(M / wl) * 2 * wr * (N / 2) : (size_t)wl * (M / 2) * 2 * (N / wr);
    int rc = upload(ct, A, na, da, s);
    if (rc) return rc;
    rc = upload(ct, B, nb, db, s);
    if (rc) return rc;
    rc = upload(ct, W, nw, dw, s);
    if (rc) return rc;
    T_HIP(hipMalloc(&dc.p, nc * csz(ct)));
    GemmArgs args;
    std::memset(&args, 0, sizeof(args));
    GemmGroup& g = args.g[0];
    g.a = op_of(da.p, 0);
    g.b = op_of(db.p, 0);
    g.c = op_of(dc.p, 0);
    g.w = op_of(dw.p, 0);
    g.ids = nullptr;
    g.M = M;
    g.N = N;
    g.K = K;
    g.lda = K;
    g.ldb = dir == 0 ? N : K;
    g.ldc = dir == 0 ? N / 2 : N / wr;
    g.batch = 1;
    g.wl = wl;
    g.wr = wr;
    g.tiles_n = dir == 0 ? (N / 2 + bn / 2 - 1) / (bn / 2) : (N + bn - 1) / bn;
    g.tiles_per_item = ((M + bm - 1) / bm) * g.tiles_n;
    args.ngroups = 1;
    args.total_tiles = g.tiles_per_item;
    args.epi = dir == 0 ? GEMM_EPI_RIGHT : GEMM_EPI_LEFT;
    T_HIP(launch_gemm(ct, ct, ct, ct, OP_N, dir == 0 ? OP_N : OP_T, variant, args, s));
    std::vector<char> h(nc * csz(ct));
    T_HIP(hipMemcpyAsync(h.data(), dc.p, h.size(), hipMemcpyDeviceToHost, s));
    T_HIP(hipStreamSynchronize(s));
    unpack(ct, h, C, nc);
    return DCS_OK;
  });
}

int dcs_test_permute(int ct_in, int ct_out, int rank, const int* dims, const int* perm, int conj,
                     int batch, int variant, const double* in, double* out, void* stream) {
  return guarded([&]() -> int {
    PermuteArgs a;
    int rc = permute_args(ct_in, ct_out, rank, dims, perm, conj, batch, variant, &a);
    if (rc) return rc;
    if (!in || !out) return testing_fail(DCS_EINVAL, "bad permute test arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf di, dout;
    const size_t count = (size_t)a.total * batch;
    rc = upload(ct_in, in, count, di, s);
    if (rc) return rc;
    T_HIP(hipMalloc(&dout.p, std::max<size_t>(count * csz(ct_out), 256)));
    a.in.base = di.p;
    a.out.base = dout.p;
    rc = run_permute(ct_in, ct_out, a, variant, s);
    if (rc) return rc;
    std::vector<char> h(count * csz(ct_out));
    T_HIP(hipMemcpyAsync(h.data(), dout.p, h.size(), hipMemcpyDeviceToHost, s));
    T_HIP(hipStreamSynchronize(s));
    unpack(ct_out, h, out, count);
    return DCS_OK;
  });
}

int dcs_test_permute_plan(int rank, const int* dims, const int* perm, int esize, int* out,
                          int out_len, int* planned) {
  return guarded([&]() -> int {
    if ((esize != 8 && esize != 16) || !out || !planned || out_len < 0)
      return testing_fail(DCS_EINVAL, "bad permute plan arguments");
    PermuteArgs a;
    const int ct = esize == 8 ? CT_F32 : CT_F64;
    int rc = permute_args(ct, ct, rank, dims, perm, 0, 1, 0, &a);
    if (rc) return rc;
    *planned = permute_tile_plan(a, esize, out, out_len) ? 1 : 0;
    return DCS_OK;
  });
}

int dcs_test_permute_dev(int ct_in, int ct_out, int rank, const int* dims, const int* perm,
                         int conj, int batch, int variant, const void* in, void* out, int reps,
                         void* stream) {
  return guarded([&]() -> int {
    PermuteArgs a;
    int rc = permute_args(ct_in, ct_out, rank, dims, perm, conj, batch, variant, &a);
    if (rc) return rc;
    if (!in || !out || reps < 1 || reps > 1000)
      return testing_fail(DCS_EINVAL, "bad permute test arguments");
    a.in.base = in;
    a.out.base = out;
    for (int r = 0; r < reps; ++r) {
      rc = run_permute(ct_in, ct_out, a, variant, static_cast<hipStream_t>(stream));
      if (rc) return rc;
    }
    return DCS_OK;
  });
}

}  // extern "C"
