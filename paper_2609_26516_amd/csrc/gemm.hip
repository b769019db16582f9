// Batched / grouped complex GEMM on CDNA4 matrix cores.
//
// C = op(A) op(B) for complex operands stored interleaved (re, im), with the
// complex product taken as three real MFMA products per 16x16 block (Gauss:
// P1 += Ar Br, P2 += Ai Bi, P3 += (Ar + Ai)(Br + Bi), then Cr = P1 - P2,
// Ci = P3 - P1 - P2; normwise error of the same order as four products).  FP32 operands use
// v_mfma_f32_16x16x4_f32 (FP32 accumulation), FP64 operands
// v_mfma_f64_16x16x4_f64.  Mixed storage (e.g. complex64 site tensors against
// a complex128 environment) is converted while staging into LDS.
//
// Tiling: one 256-thread workgroup (4 wave64 in a 2x2 grid) per BM x BN
// output tile; each wave owns a (BM/2) x (BN/2) quadrant made of 16x16 MFMA
// blocks with real and imaginary accumulators.  K advances in steps of 8
// complex columns through LDS held as split real / imaginary planes in
// [k][m] order, so the 16 lanes of an MFMA operand row read consecutive
// words.  The next K tile is fetched into registers while the current one is
// multiplied and then stored into the second of two LDS stages, one barrier
// per K step.  Workgroup ids are remapped so consecutive tiles (same batch
// item, shared operands) land on the same XCD / L2.  Tile shapes: 64x64,
// 32x32, 128x64, 64x128 (chosen per shape class by the runtime's autotuner);
// every shape accumulates each output element over K in the same order, so
// they give bit-identical results.
//
// Every group of a launch is a batch of equal-shape problems; item b of a
// group addresses its operands through the slot-id table or its call-local
// index, with stride 0 for an operand shared by all items.
#include "dcs_internal.h"

namespace dcs {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

// Operand layout of both 16x16x4 forms: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16].  Result: lane l, item r holds D[row][l % 16] with
// row = 4 (l / 16) + r for FP32 and row = l / 16 + 4 r for FP64.
template <typename R>
struct Mfma;
template <>
struct Mfma<float> {
  using V = v4f;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};
template <>
struct Mfma<double> {
  using V = v4d;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};

template <int CT>
struct Store;
template <>
struct Store<CT_F32> {
  using T = float2;
};
template <>
struct Store<CT_F64> {
  using T = double2;
};

// K step of 8 complex columns: two LDS stages of a 64x64 tile stay small
// enough (17 KB in FP32, 35 KB in FP64) that registers, not LDS, bound the
// workgroups per CU; the MFMAs take k in ascending groups of 4, so results do
// not depend on the step
constexpr int NT = 256, PAD = 4;
template <typename R>
constexpr int gemm_bk() { return 8; }


__device__ __forceinline__ int xcd_remap(int bid, int total) {
  const int q = total >> 3, r = total & 7;
  const int x = bid & 7, i = bid >> 3;
  return x * q + min(x, r) + i;
}

__device__ __forceinline__ const char* item_ptr(const Operand& o, const int* ids, int b) {
  const long long idx = o.by_slot ? ids[b] : b;
  return static_cast<const char*>(o.base) + idx * o.stride;
}

// Occupancy target given to the compiler, in waves per SIMD: the workgroups
// per CU that the tile's LDS stages allow (160 KB per CU; one wave per SIMD
// each), capped by what the tile's registers fit into 512 without spilling
// (FP32 64x64: 5; FP64 64x64, 96 accumulator registers: 3; FP64 128x64, 192:
// one).  Without it the compiler spends registers freely (an FP64 64x64 tile
// took more than 256 and ran one wave per SIMD).
template <typename R, int BM, int BN>
constexpr int gemm_min_blocks() {
  const int lds = (int)((160 * 1024) / (2 * 2 * gemm_bk<R>() * ((BM + PAD) + (BN + PAD)) * sizeof(R)));
  const int regs = sizeof(R) == 8 ? (BM * BN <= 32 * 32 ? 4 : BM * BN <= 64 * 64 ? 3 : 1)
                                   : (BM * BN <= 32 * 32 ? 4 : BM * BN <= 64 * 64 ? 5
                                                            : BM * BN <= 128 * 64 ? 3 : 2);
  const int n = lds < regs ? lds : regs;
  return n < 1 ? 1 : n;
}

template <int TA, int TB, int TC, typename R, int OPA, int OPB, int BM, int BN, int EPI>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(gemm_min_blocks<R, BM, BN>(), 8)))
void gemm_kernel(const GemmArgs args) {
  static_assert(EPI != GEMM_EPI_RIGHT || OPB == OP_N, "the right epilogue maps B's columns");
  using CA = typename Store<TA>::T;
  using CB = typename Store<TB>::T;
  using CC = typename Store<TC>::T;
  using V = typename Mfma<R>::V;
  constexpr int BK = gemm_bk<R>();
  constexpr int TPK = NT / BK;       // threads per k row when a row is staged along m / n
  constexpr int EA = BM * BK / NT;   // A elements staged per thread
  constexpr int EB = BN * BK / NT;   // B elements staged per thread
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  static_assert(EA >= 1 && EB >= 1 && BK % EA == 0 && BK % EB == 0, "staging map");

  // two LDS stages: the next K tile is stored while the current one is read;
  // the epilogue's half tile of the product (rows) reuses the same memory
  // once the K loop is done
  constexpr int EH = EPI == GEMM_EPI_NONE ? 1 : BM / 2;
  constexpr int EW = EPI == GEMM_EPI_NONE ? 1 : BN + 1;
  constexpr size_t SA = sizeof(R) * 2 * BK * (BM + PAD), SB = sizeof(R) * 2 * BK * (BN + PAD);
  constexpr size_t SC = sizeof(R) * EH * EW;
  constexpr size_t SMEM = (2 * SA + 2 * SB) > 2 * SC ? (2 * SA + 2 * SB) : 2 * SC;
  __shared__ __attribute__((aligned(16))) char smem[SMEM];
  R(*sA_r)[BK][BM + PAD] = reinterpret_cast<R(*)[BK][BM + PAD]>(smem);
  R(*sA_i)[BK][BM + PAD] = reinterpret_cast<R(*)[BK][BM + PAD]>(smem + SA);
  R(*sB_r)[BK][BN + PAD] = reinterpret_cast<R(*)[BK][BN + PAD]>(smem + 2 * SA);
  R(*sB_i)[BK][BN + PAD] = reinterpret_cast<R(*)[BK][BN + PAD]>(smem + 2 * SA + SB);
  R(*sC_r)[EW] = reinterpret_cast<R(*)[EW]>(smem);
  R(*sC_i)[EW] = reinterpret_cast<R(*)[EW]>(smem + SC);
  // the item's gate operator (epilogue)
  __shared__ CC sW[EPI == GEMM_EPI_NONE ? 1 : GEMM_EPI_WMAX * 4 * GEMM_EPI_WMAX];
  int stage = 0;

  const int tile = xcd_remap(blockIdx.x, args.total_tiles);
  int gi = 0;
  while (gi + 1 < args.ngroups && tile >= args.g[gi + 1].tile_begin) ++gi;
  const GemmGroup& G = args.g[gi];
  const int local = tile - G.tile_begin;
  const int item = local / G.tiles_per_item;
  const int t = local - item * G.tiles_per_item;
  int tm = t / G.tiles_n, tn = t % G.tiles_n;
  if (EPI == GEMM_EPI_NONE && G.herm) {   // t = tm (tm + 1) / 2 + tn, tn <= tm
    tm = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
    while ((tm + 1) * (tm + 2) / 2 <= t) ++tm;
    while (tm * (tm + 1) / 2 > t) --tm;
    tn = t - tm * (tm + 1) / 2;
  }
  const int m0 = tm * BM;
  // right epilogue: tile columns (t, y) for y in [n0, n0 + BN / 2), t = 0, 1
  const int n0 = tn * (EPI == GEMM_EPI_RIGHT ? BN / 2 : BN);
  const bool mirror = EPI == GEMM_EPI_NONE && G.herm && tn != tm;   // uniform
  const int M = G.M, N = G.N, K = G.K;
  const int lda = G.lda, ldb = G.ldb, ldc = G.ldc;

  const CA* __restrict__ A = reinterpret_cast<const CA*>(item_ptr(G.a, G.ids, item));
  const CB* __restrict__ B = reinterpret_cast<const CB*>(item_ptr(G.b, G.ids, item));
  CC* __restrict__ C = reinterpret_cast<CC*>(const_cast<char*>(item_ptr(G.c, G.ids, item)));

  const int tid = threadIdx.x;
  R ar[EA], ai[EA], br[EB], bi[EB];
  // complex64 operands whose rows start on 16 bytes are staged two elements
  // (16 bytes) per load where a thread's run lies inside the matrix
  constexpr bool PA = sizeof(CA) == 8 && EA % 2 == 0, PB = sizeof(CB) == 8 && EB % 2 == 0;
  const bool vec_a = PA && lda % 2 == 0 && (reinterpret_cast<unsigned long long>(A) & 15) == 0;
  const bool vec_b = PB && EPI != GEMM_EPI_RIGHT && ldb % 2 == 0 &&
                     (reinterpret_cast<unsigned long long>(B) & 15) == 0;
  if constexpr (EPI != GEMM_EPI_NONE) {   // visible after the first barrier
    const CC* __restrict__ W = reinterpret_cast<const CC*>(item_ptr(G.w, nullptr, item));
    const int nw = G.wl * 4 * G.wr;
    for (int i = tid; i < nw; i += NT) sW[i] = W[i];
  }

  auto load_a = [&](int k0) {
    if constexpr (OPA == OP_N || OPA == OP_J) {   // stored M x K: EA consecutive k
      constexpr int TPR = BK / EA;
      const int row = tid / TPR, kq = (tid % TPR) * EA;
      const int m = m0 + row;
      if constexpr (PA) {
        if (vec_a && m < M && k0 + kq + EA <= K) {
          const float4* q = reinterpret_cast<const float4*>(A + (long long)m * lda + k0 + kq);
#pragma unroll
          for (int u = 0; u < EA / 2; ++u) {
            const float4 v = q[u];
            ar[2 * u] = v.x;
            ai[2 * u] = (OPA == OP_J) ? -v.y : v.y;
            ar[2 * u + 1] = v.z;
            ai[2 * u + 1] = (OPA == OP_J) ? -v.w : v.w;
          }
          return;
        }
      }
#pragma unroll
      for (int u = 0; u < EA; ++u) {
        const int k = k0 + kq + u;
        R re = 0, im = 0;
        if (m < M && k < K) {
          const CA v = A[(long long)m * lda + k];
          re = v.x;
          im = v.y;
        }
        ar[u] = re;
        ai[u] = (OPA == OP_J) ? -im : im;
      }
    } else {  // OP_C: stored K x M, conjugated; EA consecutive m
      const int kr = tid / TPK, mq = (tid % TPK) * EA;
      const int k = k0 + kr;
      if constexpr (PA) {
        if (vec_a && k < K && m0 + mq + EA <= M) {
          const float4* q = reinterpret_cast<const float4*>(A + (long long)k * lda + m0 + mq);
#pragma unroll
          for (int u = 0; u < EA / 2; ++u) {
            const float4 v = q[u];
            ar[2 * u] = v.x;
            ai[2 * u] = -v.y;
            ar[2 * u + 1] = v.z;
            ai[2 * u + 1] = -v.w;
          }
          return;
        }
      }
#pragma unroll
      for (int u = 0; u < EA; ++u) {
        const int m = m0 + mq + u;
        R re = 0, im = 0;
        if (m < M && k < K) {
          const CA v = A[(long long)k * lda + m];
          re = v.x;
          im = v.y;
        }
        ar[u] = re;
        ai[u] = -im;
      }
    }
  };
  auto store_a = [&]() {
    if constexpr (OPA == OP_N || OPA == OP_J) {
      constexpr int TPR = BK / EA;
      const int row = tid / TPR, kq = (tid % TPR) * EA;
#pragma unroll
      for (int u = 0; u < EA; ++u) {
        sA_r[stage][kq + u][row] = ar[u];
        sA_i[stage][kq + u][row] = ai[u];
      }
    } else {
      const int kr = tid / TPK, mq = (tid % TPK) * EA;
#pragma unroll
      for (int u = 0; u < EA; ++u) {
        sA_r[stage][kr][mq + u] = ar[u];
        sA_i[stage][kr][mq + u] = ai[u];
      }
    }
  };
  auto load_b = [&](int k0) {
    if constexpr (OPB == OP_N) {  // stored K x N: EB consecutive n
      const int kr = tid / TPK, nq = (tid % TPK) * EB;
      const int k = k0 + kr;
      if constexpr (PB && EPI != GEMM_EPI_RIGHT) {
        if (vec_b && k < K && n0 + nq + EB <= N) {
          const float4* q = reinterpret_cast<const float4*>(B + (long long)k * ldb + n0 + nq);
#pragma unroll
          for (int u = 0; u < EB / 2; ++u) {
            const float4 v = q[u];
            br[2 * u] = v.x;
            bi[2 * u] = v.y;
            br[2 * u + 1] = v.z;
            bi[2 * u + 1] = v.w;
          }
          return;
        }
      }
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        int n = n0 + nq + u;
        bool inb = n < N;
        if constexpr (EPI == GEMM_EPI_RIGHT) {   // column (t, y) of the stored (t, y) pairs
          const int cl = nq + u, half = N / 2, y = n0 + cl % (BN / 2);
          n = (cl / (BN / 2)) * half + y;
          inb = y < half;
        }
        R re = 0, im = 0;
        if (inb && k < K) {
          const CB v = B[(long long)k * ldb + n];
          re = v.x;
          im = v.y;
        }
        br[u] = re;
        bi[u] = im;
      }
    } else {  // OP_T: stored N x K: EB consecutive k
      constexpr int TPR = BK / EB;
      const int nr = tid / TPR, kq = (tid % TPR) * EB;
      const int n = n0 + nr;
      if constexpr (PB) {
        if (vec_b && n < N && k0 + kq + EB <= K) {
          const float4* q = reinterpret_cast<const float4*>(B + (long long)n * ldb + k0 + kq);
#pragma unroll
          for (int u = 0; u < EB / 2; ++u) {
            const float4 v = q[u];
            br[2 * u] = v.x;
            bi[2 * u] = v.y;
            br[2 * u + 1] = v.z;
            bi[2 * u + 1] = v.w;
          }
          return;
        }
      }
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        const int k = k0 + kq + u;
        R re = 0, im = 0;
        if (n < N && k < K) {
          const CB v = B[(long long)n * ldb + k];
          re = v.x;
          im = v.y;
        }
        br[u] = re;
        bi[u] = im;
      }
    }
  };
  auto store_b = [&]() {
    if constexpr (OPB == OP_N) {
      const int kr = tid / TPK, nq = (tid % TPK) * EB;
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        sB_r[stage][kr][nq + u] = br[u];
        sB_i[stage][kr][nq + u] = bi[u];
      }
    } else {
      constexpr int TPR = BK / EB;
      const int nr = tid / TPR, kq = (tid % TPR) * EB;
#pragma unroll
      for (int u = 0; u < EB; ++u) {
        sB_r[stage][kq + u][nr] = br[u];
        sB_i[stage][kq + u][nr] = bi[u];
      }
    }
  };

  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  const int li = lane & 15, lk = lane >> 4;

  // three real products per complex block (Gauss): p1 = Ar Br, p2 = Ai Bi,
  // p3 = (Ar + Ai)(Br + Bi); Cr = p1 - p2, Ci = p3 - p1 - p2
  V p1[FM][FN], p2[FM][FN], p3[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        p1[i][j][r] = 0;
        p2[i][j][r] = 0;
        p3[i][j][r] = 0;
      }

  const int nk = (K + BK - 1) / BK;
  if (nk > 0) {
    load_a(0);
    load_b(0);
    store_a();
    store_b();
    __syncthreads();
  }
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) {
      load_a((kt + 1) * BK);
      load_b((kt + 1) * BK);
    }
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + lk;
      R xr[FM], xi[FM], xs[FM], yr[FN], yi[FN], ys[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        xr[i] = sA_r[stage][kr][wm + i * 16 + li];
        xi[i] = sA_i[stage][kr][wm + i * 16 + li];
        xs[i] = xr[i] + xi[i];
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        yr[j] = sB_r[stage][kr][wn + j * 16 + li];
        yi[j] = sB_i[stage][kr][wn + j * 16 + li];
        ys[j] = yr[j] + yi[j];
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          p1[i][j] = Mfma<R>::mma(xr[i], yr[j], p1[i][j]);
          p2[i][j] = Mfma<R>::mma(xi[i], yi[j], p2[i][j]);
          p3[i][j] = Mfma<R>::mma(xs[i], ys[j], p3[i][j]);
        }
    }
    if (kt + 1 < nk) {
      stage ^= 1;   // the other stage was last read before the previous barrier
      store_a();
      store_b();
    }
    __syncthreads();
  }

  if constexpr (EPI == GEMM_EPI_NONE) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int col = n0 + wn + j * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm + i * 16 + Mfma<R>::row(lk, r);
          if (row < M && col < N) {
            CC v;
            v.x = p1[i][j][r] - p2[i][j][r];
            v.y = p3[i][j][r] - p1[i][j][r] - p2[i][j][r];
            C[(long long)row * ldc + col] = v;
            if (mirror) {
              v.y = -v.y;
              C[(long long)col * ldc + row] = v;
            }
          }
        }
      }
  } else {
    // The product tile goes through LDS half by half (rows); every thread then
    // applies the gate operator to whole (row group, column group) blocks, in
    // the order of the stand-alone operator kernels.
    constexpr int W4 = GEMM_EPI_WMAX;
    const int wl = G.wl, wr = G.wr;
    // A operand: W_real[li][4 kk + lk], row li = output (j, c'), column
    // 4 kk + lk = input (k = (4 kk + lk) / 2, c = lk & 1); W is in LDS since
    // the K loop's first barrier
    R wa[4];
    {
      int j, cp;
      if constexpr (sizeof(R) == 4) {
        j = li >> 1;
        cp = li & 1;
      } else {
        j = li & 7;
        cp = li >> 3;
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int k = 2 * kk + (lk >> 1), c = lk & 1;
        CC w;
        w.x = 0;
        w.y = 0;
        if constexpr (EPI == GEMM_EPI_RIGHT) {
          const int wli = k >> 1, t = k & 1, sp = j / W4, o = j % W4;
          if (wli < wl && o < wr) w = sW[((wli * 2 + sp) * 2 + t) * wr + o];
        } else {
          const int t = k / W4, o = k % W4, l = j >> 1, sp = j & 1;
          if (o < wr && l < wl) w = sW[((l * 2 + sp) * 2 + t) * wr + o];
        }
        // y = w x: re(y) = re w re x - im w im x, im(y) = im w re x + re w im x
        wa[kk] = cp == 0 ? (c == 0 ? w.x : -w.y) : (c == 0 ? w.y : w.x);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      __syncthreads();   // the K loop's (or the previous half's) LDS reads are done
      if ((wave >> 1) == h) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = i * 16 + Mfma<R>::row(lk, r), col = wn + j * 16 + li;
              sC_r[row][col] = p1[i][j][r] - p2[i][j][r];
              sC_i[row][col] = p3[i][j][r] - p1[i][j][r] - p2[i][j][r];
            }
      }
      __syncthreads();
      const int mh = m0 + h * (BM / 2);
      // The operator as one real 16 x 16 matrix on the matrix cores: item n
      // (a row group and a column) has 8 complex inputs x_k and 8 complex
      // outputs y_j = sum_k W_jk x_k; as reals, row jrow(j, c') of the
      // product is component c' of y_j and row 2k + c of the input component
      // c of x_k.  16 items per product, 4 MFMA k-steps.
      //   RIGHT  k = 2 wl_i + t, j = 4 sp + o: W[wl_i][sp][t][o]
      //          x_k = X1[a][wl_i][t][y], y_j to X2[a][sp][o][y]
      //   LEFT   k = 4 t + o,   j = 2 l + sp: W[l][sp][t][o]
      //          x_k = Y1[x][t][c][o], y_j to Y2[l][x][sp][c]
      // The output rows are ordered so that a lane holds whole complex
      // outputs: 2 j + c' for the FP32 layout (rows 4 lk + r), 8 c' + j for
      // the FP64 layout (rows lk + 4 r).
      const int nitems = EPI == GEMM_EPI_RIGHT ? ((BM / 2) / wl) * (BN / 2) : (BM / 4) * (BN / wr);
      for (int blk0 = wave * 16; blk0 < nitems; blk0 += 4 * 16) {
        const int item = blk0 + li;
        bool valid = item < nitems;
        int ra = 0, rb = 0, cbase = 0;   // LDS row base / column base of the item, and its output place
        long long obase = 0;
        if constexpr (EPI == GEMM_EPI_RIGHT) {
          constexpr int HB = BN / 2;
          const int yl = item % HB, al = item / HB;
          const int a = mh / wl + al, y = n0 + yl;
          valid = valid && a < M / wl && y < N / 2;
          ra = al * wl;
          cbase = yl;
          obase = (long long)a * 2 * wr * ldc + y;
          rb = HB;
        } else {
          const int nc = BN / wr;
          const int cl = item % nc, xl = item / nc;
          const int x = mh / 2 + xl, c = n0 / wr + cl;
          valid = valid && x < M / 2 && c < N / wr;
          ra = xl * 2;
          cbase = cl * wr;
          obase = (long long)x * 2 * ldc + c;
        }
        // B operand: input row 4 kk + lk = component (lk & 1) of x_k,
        // k = 2 kk + (lk >> 1)
        R acc_v[4];
        V acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = 0;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = 2 * kk + (lk >> 1);
          int row, col;
          bool in;
          if constexpr (EPI == GEMM_EPI_RIGHT) {
            const int wli = k >> 1, t = k & 1;
            in = valid && wli < wl;
            row = ra + wli;
            col = t * rb + cbase;
          } else {
            const int t = k / W4, o = k % W4;
            in = valid && o < wr;
            row = ra + t;
            col = cbase + o;
          }
          const R xv = !in ? R(0) : ((lk & 1) ? sC_i[row][col] : sC_r[row][col]);
          acc = Mfma<R>::mma(wa[kk], xv, acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) acc_v[r] = acc[r];
        if (valid) {
          // the two complex outputs of this lane: (j, re at slot r0, im at slot r1)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            int j, r0, r1;
            if constexpr (sizeof(R) == 4) {   // rows 4 lk + r: 2 j + c'
              j = 2 * lk + q;
              r0 = 2 * q;
              r1 = 2 * q + 1;
            } else {                          // rows lk + 4 r: 8 c' + j
              j = lk + 4 * q;
              r0 = q;
              r1 = q + 2;
            }
            CC v;
            v.x = acc_v[r0];
            v.y = acc_v[r1];
            if constexpr (EPI == GEMM_EPI_RIGHT) {
              const int sp = j / W4, o = j % W4;
              if (o < wr) C[obase + (long long)(sp * wr + o) * ldc] = v;
            } else {
              const int l = j >> 1, sp = j & 1;
              if (l < wl) C[obase + ((long long)l * (M / 2) * 2 + sp) * ldc] = v;
            }
          }
        }
      }
    }
  }
}

template <int TA, int TB, int TC, typename R, int OPA, int OPB, int EPI = GEMM_EPI_NONE>
hipError_t run(int variant, const GemmArgs& args, hipStream_t s) {
  if (args.total_tiles <= 0) return hipSuccess;
  const dim3 grid(args.total_tiles), blk(NT);
  switch (variant) {
    case GEMM_64x64:
      hipLaunchKernelGGL((gemm_kernel<TA, TB, TC, R, OPA, OPB, 64, 64, EPI>), grid, blk, 0, s, args);
      break;
    case GEMM_32x32:
      hipLaunchKernelGGL((gemm_kernel<TA, TB, TC, R, OPA, OPB, 32, 32, EPI>), grid, blk, 0, s, args);
      break;
    case GEMM_128x64:
      hipLaunchKernelGGL((gemm_kernel<TA, TB, TC, R, OPA, OPB, 128, 64, EPI>), grid, blk, 0, s, args);
      break;
    case GEMM_64x128:
      hipLaunchKernelGGL((gemm_kernel<TA, TB, TC, R, OPA, OPB, 64, 128, EPI>), grid, blk, 0, s, args);
      break;
    case GEMM_128x128:
      if constexpr (sizeof(R) == 4) {
        hipLaunchKernelGGL((gemm_kernel<TA, TB, TC, R, OPA, OPB, 128, 128, EPI>), grid, blk, 0, s, args);
        break;
      }
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

void gemm_tile_shape(int variant, int* bm, int* bn) {
  switch (variant) {
    case GEMM_32x32:
      *bm = 32;
      *bn = 32;
      return;
    case GEMM_128x64:
      *bm = 128;
      *bn = 64;
      return;
    case GEMM_64x128:
      *bm = 64;
      *bn = 128;
      return;
    case GEMM_128x128:
      *bm = 128;
      *bn = 128;
      return;
    default:
      *bm = 64;
      *bn = 64;
  }
}

hipError_t launch_gemm(int ta, int tb, int tc, int tacc, int opa, int opb, int variant,
                       const GemmArgs& args, hipStream_t s) {
  if (tacc == ACC_BF16X3)
    return (ta == CT_F32 && tb == CT_F32 && tc == CT_F32 && args.epi == GEMM_EPI_NONE)
               ? launch_gemm_bf16x3(opa, opb, variant, args, s)
               : hipErrorInvalidValue;
  if (args.epi != GEMM_EPI_NONE) {   // gate operator in the epilogue
    for (int g = 0; g < args.ngroups; ++g)
      if (args.g[g].wl < 1 || args.g[g].wl > GEMM_EPI_WMAX || args.g[g].wr < 1 ||
          args.g[g].wr > GEMM_EPI_WMAX)
        return hipErrorInvalidValue;
    const bool same = ta == tb && tb == tc && tacc == ta;
    if (same && args.epi == GEMM_EPI_RIGHT && opa == OP_N && opb == OP_N)
      return ta == CT_F32 ? run<CT_F32, CT_F32, CT_F32, float, OP_N, OP_N, GEMM_EPI_RIGHT>(variant, args, s)
                          : run<CT_F64, CT_F64, CT_F64, double, OP_N, OP_N, GEMM_EPI_RIGHT>(variant, args, s);
    if (same && args.epi == GEMM_EPI_LEFT && opa == OP_N && opb == OP_T)
      return ta == CT_F32 ? run<CT_F32, CT_F32, CT_F32, float, OP_N, OP_T, GEMM_EPI_LEFT>(variant, args, s)
                          : run<CT_F64, CT_F64, CT_F64, double, OP_N, OP_T, GEMM_EPI_LEFT>(variant, args, s);
    return hipErrorInvalidValue;
  }
#define DCS_GEMM_CASE(TA, TB, TC, R, OA, OB)                                             \
  if (ta == TA && tb == TB && tc == TC && tacc == (sizeof(R) == 8 ? CT_F64 : CT_F32) && \
      opa == OA && opb == OB)                                                            \
    return run<TA, TB, TC, R, OA, OB>(variant, args, s);
  // compression-step contractions in path precision
  DCS_GEMM_CASE(CT_F64, CT_F64, CT_F64, double, OP_N, OP_N)
  DCS_GEMM_CASE(CT_F64, CT_F64, CT_F64, double, OP_N, OP_T)
  DCS_GEMM_CASE(CT_F64, CT_F64, CT_F64, double, OP_C, OP_N)
  DCS_GEMM_CASE(CT_F64, CT_F64, CT_F64, double, OP_J, OP_T)
  DCS_GEMM_CASE(CT_F32, CT_F32, CT_F32, float, OP_N, OP_N)
  DCS_GEMM_CASE(CT_F32, CT_F32, CT_F32, float, OP_N, OP_T)
  DCS_GEMM_CASE(CT_F32, CT_F32, CT_F32, float, OP_C, OP_N)
  DCS_GEMM_CASE(CT_F32, CT_F32, CT_F32, float, OP_J, OP_T)
  // FP64 measurement contractions over complex64 site tensors
  DCS_GEMM_CASE(CT_F64, CT_F32, CT_F64, double, OP_N, OP_N)
  DCS_GEMM_CASE(CT_F32, CT_F64, CT_F64, double, OP_C, OP_N)
  DCS_GEMM_CASE(CT_F32, CT_F64, CT_F64, double, OP_N, OP_T)
  DCS_GEMM_CASE(CT_F32, CT_F64, CT_F64, double, OP_J, OP_T)
  DCS_GEMM_CASE(CT_F32, CT_F32, CT_F64, double, OP_C, OP_N)
  DCS_GEMM_CASE(CT_F32, CT_F32, CT_F64, double, OP_J, OP_T)
#undef DCS_GEMM_CASE
  return hipErrorInvalidValue;
}

}  // namespace dcs
