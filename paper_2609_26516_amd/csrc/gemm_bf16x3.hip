// Split-BF16 ("bf16x3") complex GEMM on CDNA4 BF16 matrix cores.
//
// Operands and result are complex64.  Every FP32 component x is split into a
// BF16 pair x = hi + lo + O(2^-17 |x|), hi = bf16(x) and lo = bf16(x - hi),
// both rounded to nearest even (v_cvt_pk_bf16_f32).  A real product then
// takes three BF16 MFMA products with FP32 accumulation,
//   x y ~ hi(x) hi(y) + hi(x) lo(y) + lo(x) hi(y),
// dropping lo(x) lo(y) (relative size 2^-16), and a complex product takes
// four real ones (Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br): twelve
// v_mfma_f32_16x16x32_bf16 per 16x16 output block and 32-deep K step.
//
// Tiling as in the FP32 / FP64 kernel: a 256-thread workgroup (2x2 waves)
// per BM x BN output tile, K in steps of 32.  The split happens once per
// element while a K tile is staged into LDS; LDS holds four BF16 planes per
// operand (re hi, re lo, im hi, im lo) in [row][k] order with rows padded to
// 80 bytes, so each lane's 8 consecutive k values (one MFMA operand) are one
// conflict-free 16-byte read.  The next K tile is fetched into registers
// while the current one is multiplied; workgroup ids are remapped per XCD.
// The accumulation order of an output element does not depend on the tile
// shape, so all shapes give bit-identical results.
#include "dcs_internal.h"

namespace dcs {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int BK = 32, NT = 256, SK = BK + 8;   // SK: padded LDS row (bf16 units)

__device__ __forceinline__ int xcd_remap(int bid, int total) {
  const int q = total >> 3, r = total & 7;
  const int x = bid & 7, i = bid >> 3;
  return x * q + min(x, r) + i;
}

__device__ __forceinline__ const char* item_ptr(const Operand& o, const int* ids, int b) {
  const long long idx = o.by_slot ? ids[b] : b;
  return static_cast<const char*>(o.base) + idx * o.stride;
}

__device__ __forceinline__ unsigned pack2(float a, float b) {
  bf2 v;
  v[0] = (__bf16)a;
  v[1] = (__bf16)b;
  return __builtin_bit_cast(unsigned, v);
}

// (a, b) -> packed hi pair and packed lo pair (element a in the low half)
__device__ __forceinline__ void split2(float a, float b, unsigned& hi, unsigned& lo) {
  hi = pack2(a, b);
  const float ha = __uint_as_float(hi << 16), hb = __uint_as_float(hi & 0xffff0000u);
  lo = pack2(a - ha, b - hb);
}

__device__ __forceinline__ v4f mma(const bf8& a, const bf8& b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf8 neg8(bf8 x) {
  u4 u = __builtin_bit_cast(u4, x);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf8, u);
}

// Staging of one operand tile: R rows (M or N) x BK k values.
//   KMAJOR: stored row-major with k contiguous (A as N / J, B as T);
//           each thread loads E consecutive k of one row.
//   otherwise stored with rows contiguous (A as C, B as N); each thread loads
//           E/2 consecutive rows at two consecutive k, so k pairs pack into
//           one 32-bit LDS word.
template <int R, bool KMAJOR, bool CONJ>
struct Stage {
  static constexpr int E = R * BK / NT;
  float re[E], im[E];

  // vec: rows of X start on 16 bytes; a thread's run inside the matrix is then
  // read 16 bytes (two elements) at a time
  __device__ __forceinline__ void load(const float2* __restrict__ X, long long ld, int r0,
                                       int rmax, int k0, int kmax, int tid, bool vec) {
    if constexpr (KMAJOR) {
      constexpr int TPR = BK / E;
      const int row = r0 + tid / TPR, kq = k0 + (tid % TPR) * E;
      if constexpr (E % 2 == 0) {
        if (vec && row < rmax && kq + E <= kmax) {
          const float4* q = reinterpret_cast<const float4*>(X + (long long)row * ld + kq);
#pragma unroll
          for (int u = 0; u < E / 2; ++u) {
            const float4 v = q[u];
            re[2 * u] = v.x;
            im[2 * u] = CONJ ? -v.y : v.y;
            re[2 * u + 1] = v.z;
            im[2 * u + 1] = CONJ ? -v.w : v.w;
          }
          return;
        }
      }
#pragma unroll
      for (int u = 0; u < E; ++u) {
        float2 v = make_float2(0.f, 0.f);
        if (row < rmax && kq + u < kmax) v = X[(long long)row * ld + kq + u];
        re[u] = v.x;
        im[u] = CONJ ? -v.y : v.y;
      }
    } else {
      constexpr int H = E / 2, TPK = R / H;   // TPK threads per k pair
      const int kp = tid / TPK, rq = r0 + (tid % TPK) * H;
      if constexpr (H % 2 == 0) {
        if (vec && rq + H <= rmax && k0 + 2 * kp + 1 < kmax) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const float4* q = reinterpret_cast<const float4*>(X + (long long)(k0 + 2 * kp + h) * ld + rq);
#pragma unroll
            for (int u = 0; u < H / 2; ++u) {
              const float4 v = q[u];
              re[h * H + 2 * u] = v.x;
              im[h * H + 2 * u] = CONJ ? -v.y : v.y;
              re[h * H + 2 * u + 1] = v.z;
              im[h * H + 2 * u + 1] = CONJ ? -v.w : v.w;
            }
          }
          return;
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int k = k0 + 2 * kp + h;
#pragma unroll
        for (int u = 0; u < H; ++u) {
          float2 v = make_float2(0.f, 0.f);
          if (rq + u < rmax && k < kmax) v = X[(long long)k * ld + rq + u];
          re[h * H + u] = v.x;
          im[h * H + u] = CONJ ? -v.y : v.y;
        }
      }
    }
  }

  // planes: [0] re hi, [1] re lo, [2] im hi, [3] im lo; each R x SK bf16
  __device__ __forceinline__ void store(__bf16* s, int tid) const {
    unsigned* w = reinterpret_cast<unsigned*>(s);
    constexpr int PW = R * SK / 2;   // plane size in 32-bit words
    if constexpr (KMAJOR) {
      constexpr int TPR = BK / E;
      const int row = tid / TPR, kq = (tid % TPR) * E;
      const int base = (row * SK + kq) / 2;
#pragma unroll
      for (int u = 0; u < E; u += 2) {
        unsigned h, l;
        split2(re[u], re[u + 1], h, l);
        w[base + u / 2] = h;
        w[PW + base + u / 2] = l;
        split2(im[u], im[u + 1], h, l);
        w[2 * PW + base + u / 2] = h;
        w[3 * PW + base + u / 2] = l;
      }
    } else {
      constexpr int H = E / 2, TPK = R / H;
      const int kp = tid / TPK, rq = (tid % TPK) * H;
#pragma unroll
      for (int u = 0; u < H; ++u) {
        const int base = ((rq + u) * SK + 2 * kp) / 2;
        unsigned h, l;
        split2(re[u], re[H + u], h, l);
        w[base] = h;
        w[PW + base] = l;
        split2(im[u], im[H + u], h, l);
        w[2 * PW + base] = h;
        w[3 * PW + base] = l;
      }
    }
  }
};

template <int OPA, int OPB, int BM, int BN>
__global__ __launch_bounds__(NT) void gemm_bf16x3_kernel(const GemmArgs args) {
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  __shared__ __attribute__((aligned(16))) __bf16 sA[4 * BM * SK];
  __shared__ __attribute__((aligned(16))) __bf16 sB[4 * BN * SK];

  const int tile = xcd_remap(blockIdx.x, args.total_tiles);
  int gi = 0;
  while (gi + 1 < args.ngroups && tile >= args.g[gi + 1].tile_begin) ++gi;
  const GemmGroup& G = args.g[gi];
  const int local = tile - G.tile_begin;
  const int item = local / G.tiles_per_item;
  const int t = local - item * G.tiles_per_item;
  const int m0 = (t / G.tiles_n) * BM;
  const int n0 = (t % G.tiles_n) * BN;
  const int M = G.M, N = G.N, K = G.K;

  const float2* __restrict__ A = reinterpret_cast<const float2*>(item_ptr(G.a, G.ids, item));
  const float2* __restrict__ B = reinterpret_cast<const float2*>(item_ptr(G.b, G.ids, item));
  float2* __restrict__ C = reinterpret_cast<float2*>(const_cast<char*>(item_ptr(G.c, G.ids, item)));
  const bool vec_a = G.lda % 2 == 0 && (reinterpret_cast<unsigned long long>(A) & 15) == 0;
  const bool vec_b = G.ldb % 2 == 0 && (reinterpret_cast<unsigned long long>(B) & 15) == 0;

  const int tid = threadIdx.x;
  Stage<BM, OPA == OP_N || OPA == OP_J, OPA == OP_C || OPA == OP_J> sa;
  Stage<BN, OPB == OP_T, false> sb;

  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  const int li = lane & 15, lk = lane >> 4;

  v4f cr[FM][FN], ci[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        cr[i][j][r] = 0.f;
        ci[i][j][r] = 0.f;
      }

  const int nk = (K + BK - 1) / BK;
  if (nk > 0) {
    sa.load(A, G.lda, m0, M, 0, K, tid, vec_a);
    sb.load(B, G.ldb, n0, N, 0, K, tid, vec_b);
  }
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
    sa.store(sA, tid);
    sb.store(sB, tid);
    __syncthreads();
    if (kt + 1 < nk) {
      sa.load(A, G.lda, m0, M, (kt + 1) * BK, K, tid, vec_a);
      sb.load(B, G.ldb, n0, N, (kt + 1) * BK, K, tid, vec_b);
    }
    bf8 y[FN][4];
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int p = 0; p < 4; ++p)
        y[j][p] = *reinterpret_cast<const bf8*>(&sB[p * BN * SK + (wn + j * 16 + li) * SK + 8 * lk]);
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      bf8 x[4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
        x[p] = *reinterpret_cast<const bf8*>(&sA[p * BM * SK + (wm + i * 16 + li) * SK + 8 * lk]);
      const bf8 nxh = neg8(x[2]), nxl = neg8(x[3]);
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        // real part: Ar Br - Ai Bi
        cr[i][j] = mma(x[0], y[j][0], cr[i][j]);
        cr[i][j] = mma(x[0], y[j][1], cr[i][j]);
        cr[i][j] = mma(x[1], y[j][0], cr[i][j]);
        cr[i][j] = mma(nxh, y[j][2], cr[i][j]);
        cr[i][j] = mma(nxh, y[j][3], cr[i][j]);
        cr[i][j] = mma(nxl, y[j][2], cr[i][j]);
        // imaginary part: Ar Bi + Ai Br
        ci[i][j] = mma(x[0], y[j][2], ci[i][j]);
        ci[i][j] = mma(x[0], y[j][3], ci[i][j]);
        ci[i][j] = mma(x[1], y[j][2], ci[i][j]);
        ci[i][j] = mma(x[2], y[j][0], ci[i][j]);
        ci[i][j] = mma(x[2], y[j][1], ci[i][j]);
        ci[i][j] = mma(x[3], y[j][0], ci[i][j]);
      }
    }
  }

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn + j * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + 4 * lk + r;
        if (row < M && col < N) C[(long long)row * G.ldc + col] = make_float2(cr[i][j][r], ci[i][j][r]);
      }
    }
}

template <int OPA, int OPB>
hipError_t run(int variant, const GemmArgs& args, hipStream_t s) {
  if (args.total_tiles <= 0) return hipSuccess;
  const dim3 grid(args.total_tiles), blk(NT);
  switch (variant) {
    case GEMM_64x64:
      hipLaunchKernelGGL((gemm_bf16x3_kernel<OPA, OPB, 64, 64>), grid, blk, 0, s, args);
      break;
    case GEMM_32x32:
      hipLaunchKernelGGL((gemm_bf16x3_kernel<OPA, OPB, 32, 32>), grid, blk, 0, s, args);
      break;
    case GEMM_128x64:
      hipLaunchKernelGGL((gemm_bf16x3_kernel<OPA, OPB, 128, 64>), grid, blk, 0, s, args);
      break;
    case GEMM_64x128:
      hipLaunchKernelGGL((gemm_bf16x3_kernel<OPA, OPB, 64, 128>), grid, blk, 0, s, args);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_bf16x3(int opa, int opb, int variant, const GemmArgs& args,
                              hipStream_t s) {
  if (opa == OP_N && opb == OP_N) return run<OP_N, OP_N>(variant, args, s);
  if (opa == OP_N && opb == OP_T) return run<OP_N, OP_T>(variant, args, s);
  if (opa == OP_C && opb == OP_N) return run<OP_C, OP_N>(variant, args, s);
  if (opa == OP_J && opb == OP_T) return run<OP_J, OP_T>(variant, args, s);
  return hipErrorInvalidValue;
}

}  // namespace dcs
