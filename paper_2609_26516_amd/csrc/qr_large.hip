// FP64 Householder QR with explicit thin Q for local matrices of more than
// 512 rows (bond caps above 256), where one workgroup per matrix would leave
// the chip idle and the panel no longer fits in LDS, and the spread path for
// small batches of smaller matrices.  Same reflectors as the other QR kernels
// (LAPACK convention: v_k = 1, beta = -sign(Re alpha) |x|,
// tau = ((beta - Re alpha) / beta, -Im alpha / beta), tau = 0 for a zero
// column), blocked in panels of 16 columns with the compact WY form
// H_p ... H_{p+15} = I - V T V^H:
//   qrl_load   F (mode 0) or F^H (mode 1) -> FP64 working matrix A (m x n,
//              row-major), |F|^2 partial sums per chunk
//   qrt_* (m > 512) / qrs_panel (m <= 512)
//              A[p:, p:p+16] factored by Cholesky QR and Householder
//              reconstruction (qr_cholpanel.h), or column by column where
//              the panel does not allow it, by one 512-thread workgroup per
//              256-row chunk (m > 512) or per matrix (m <= 512); writes the
//              explicit V (unit diagonal) and T
//   qrl_wpart  W = V^H A[p:, c:] in parts over (16-column strip, 256-row
//   qrl_update chunk) tiles on FP64 MFMA, then A[p:, c:] -= V X W with
//              X = T^H, every chunk summing its strip's parts in one order
// After the last panel A is reset to [I; 0] and the panels are applied in
// reverse order with X = T, which leaves the thin Q = H_0 ... H_{n-1} [I; 0]
// in A; qrl_store writes Q (mode 0) or Q^H (mode 1) in the output precision.
#include "dcs_internal.h"
#include "kernel_util.h"
#include "qr_panel.h"
#include "qr_cholpanel.h"

namespace dcs {
namespace {


constexpr int QRL_CHUNKS = 64;   // load / store / fill work units per matrix

struct QrlItem {
  const QrGroup* g;
  int item;
};

__device__ __forceinline__ QrlItem qrl_item(const QrArgs& args, int flat) {
  const int gi = find_group<QR_MAX_GROUPS>(args.g, args.ngroups, flat);
  return {&args.g[gi], flat - args.g[gi].blk_begin};
}

__device__ __forceinline__ double2* qrl_ws(const QrlItem& it) {
  return reinterpret_cast<double2*>(const_cast<char*>(item_ptr(it.g->ws, it.g->ids, it.item)));
}

// workspace: A (m n), V (m n), T factors (16 (n + 16)), |F|^2 chunk partials,
// then the W parts of the strip updates
__device__ __forceinline__ double* qrl_partials(double2* ws, int m, int n) {
  return reinterpret_cast<double*>(ws + 2LL * m * n + 16LL * (n + 16));
}

template <int CTI>
__global__ __launch_bounds__(256) void qrl_load_kernel(const QrArgs args) {
  using TI = typename St<CTI>::T;
  __shared__ double s_red[4];
  const QrlItem it = qrl_item(args, blockIdx.y);
  const int m = it.g->m, n = it.g->n, mode = it.g->mode;
  const TI* __restrict__ F = reinterpret_cast<const TI*>(item_ptr(it.g->f, it.g->ids, it.item));
  double2* A = qrl_ws(it);
  const long long mn = (long long)m * n;
  const long long per = (mn + QRL_CHUNKS - 1) / QRL_CHUNKS;
  const long long e0 = per * blockIdx.x, e1 = min(mn, e0 + per);
  double part = 0.0;
  for (long long idx = e0 + threadIdx.x; idx < e1; idx += 256) {
    double2 v;
    if (mode == 0) {
      v = to_d2(F[idx]);
    } else {   // A[i][j] = conj(F[j][i]), F stored n x m
      const long long i = idx / n, j = idx % n;
      v = cconj(to_d2(F[j * m + i]));
    }
    part += v.x * v.x + v.y * v.y;
    A[idx] = v;
  }
  part = block_sum(part, s_red);
  if (threadIdx.x == 0) qrl_partials(A, m, n)[blockIdx.x] = part;
}

// A[p:, c0:c0+16] -= V X (V^H A[p:, c0:c0+16]) with X = T^H (conj_t) or T,
// in two launches over (16-column strip, QRL_CH-row chunk) tiles so the chip
// has many waves in flight: qrl_wpart writes each chunk's W = V^H A part,
// qrl_update sums the parts of its strip in chunk order (the same sum in
// every chunk of the strip), forms X W and updates its rows.
constexpr int QRL_CH = 256;   // rows per chunk (four waves of 64)

__device__ __forceinline__ double2* qrl_wparts(double2* ws, int m, int n) {
  return reinterpret_cast<double2*>(qrl_partials(ws, m, n) + QRL_CHUNKS);
}

// Scratch of the split panel factorisation (after the W parts): G1 and G2
// parts of up to QRT_MAXCH row chunks, a copy of Q1's top block, and the
// fallback flag (its real part).
constexpr int QRT_CH = 256;                          // rows per chunk workgroup
constexpr int QRT_MAXCH = 2048 / QRT_CH;
constexpr int QRT_SCRATCH = 2 * QRT_MAXCH * 256 + 256 + 16;
__device__ __forceinline__ double2* qrt_scratch(double2* ws, int m, int n) {
  const long long parts = (long long)((n + 15) / 16) * ((m + QRL_CH - 1) / QRL_CH) * 256;
  return qrl_wparts(ws, m, n) + parts;
}

template <int NB>
__global__ __launch_bounds__(256) void qrl_wpart_kernel(const QrArgs args, int p, int c_off) {
  __shared__ double2 sW[4][256];
  const QrlItem it = qrl_item(args, blockIdx.z);
  const int m = it.g->m, n = it.g->n;
  const int c0 = p + c_off + 16 * blockIdx.x;
  const int mp = m - p;
  if (p >= n || c0 >= n || (int)blockIdx.y * QRL_CH >= mp) return;
  double2* A = qrl_ws(it);
  const double2* V = A + (long long)m * n;
  const int nbk = min(NB, n - p);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int col = c0 + li;
  const bool col_ok = col < n;
  const int r0 = blockIdx.y * QRL_CH + wave * 64, r1 = min(mp, r0 + 64);
  const double2 zero = make_double2(0.0, 0.0);
  CAcc3 w;
  w.zero();
  double2 vv[16], bb[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int i = r0 + 4 * u + lk;
    const bool ok = i < r1;
    vv[u] = (ok && li < nbk) ? V[(long long)(p + i) * n + p + li] : zero;
    bb[u] = (ok && col_ok) ? A[(long long)(p + i) * n + col] : zero;
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) w.add(vv[u].x, -vv[u].y, bb[u].x, bb[u].y);
#pragma unroll
  for (int t = 0; t < 4; ++t) sW[wave][(lk + 4 * t) * 16 + li] = make_double2(w.re(t), w.im(t));
  __syncthreads();
  const int e = threadIdx.x;
  double2 sum = sW[0][e];
#pragma unroll
  for (int w = 1; w < 4; ++w) {
    sum.x += sW[w][e].x;
    sum.y += sW[w][e].y;
  }
  const int nchunk = (mp + QRL_CH - 1) / QRL_CH;
  qrl_wparts(A, m, n)[((long long)blockIdx.x * nchunk + blockIdx.y) * 256 + e] = sum;
}

// In the forward pass (c_off = NB) the strip-0 workgroups, which update the
// next panel's columns, also leave that panel's G1 part of their rows (those
// below the next panel's first row) in the split panel's scratch.
template <int NB>
__global__ __launch_bounds__(256) void qrl_update_kernel(const QrArgs args, int p, int c_off,
                                                         int conj_t) {
  __shared__ double2 sW[256];
  __shared__ double2 sG[4 * 256];
  const QrlItem it = qrl_item(args, blockIdx.z);
  const int m = it.g->m, n = it.g->n;
  const int c0 = p + c_off + 16 * blockIdx.x;
  const int mp = m - p;
  if (p >= n || c0 >= n || (int)blockIdx.y * QRL_CH >= mp) return;
  double2* A = qrl_ws(it);
  const double2* V = A + (long long)m * n;
  const double2* T = V + (long long)m * n + (long long)(p / NB) * NB * NB;
  const int nbk = min(NB, n - p);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int col = c0 + li;
  const bool col_ok = col < n;
  const double2 zero = make_double2(0.0, 0.0);
  {
    const int nchunk = (mp + QRL_CH - 1) / QRL_CH;
    const double2* parts = qrl_wparts(A, m, n) + (long long)blockIdx.x * nchunk * 256;
    const int e = threadIdx.x;
    double2 sum = parts[e];
    for (int c = 1; c < nchunk; ++c) {
      sum.x += parts[c * 256 + e].x;
      sum.y += parts[c * 256 + e].y;
    }
    sW[e] = sum;
  }
  __syncthreads();
  v4d_t wr, wi;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const double2 w = sW[(lk + 4 * t) * 16 + li];
    wr[t] = w.x;
    wi[t] = w.y;
  }
  // W2 = X W (result item t = row lk + 4t = the B operand of k-step t)
  CAcc3 x2;
  x2.zero();
#pragma unroll
  for (int t = 0; t < NB / 4; ++t) {
    const int s = 4 * t + lk;
    double2 x = zero;
    if (li < nbk && s < nbk) {
      if (conj_t) {
        const double2 tt = T[s * NB + li];
        x = make_double2(tt.x, -tt.y);
      } else {
        x = T[li * NB + s];
      }
    }
    x2.add(x.x, x.y, wr[t], wi[t]);
  }
  double xr[4], xi[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    xr[t] = x2.re(t);
    xi[t] = x2.im(t);
  }
  // this wave's 64 rows: A -= V W2, four 16-row blocks
  const int r0 = blockIdx.y * QRL_CH + wave * 64, r1 = min(mp, r0 + 64);
  double2 av[4][4];
  double2 vv[4][NB / 4];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int rb = r0 + 16 * h;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = rb + lk + 4 * t;
      av[h][t] = (i < r1 && col_ok) ? A[(long long)(p + i) * n + col] : zero;
    }
#pragma unroll
    for (int t = 0; t < NB / 4; ++t) {
      const int i = rb + li, sref = 4 * t + lk;
      vv[h][t] = (i < r1 && sref < nbk) ? V[(long long)(p + i) * n + p + sref] : zero;
    }
  }
  const bool gram = c_off == NB && blockIdx.x == 0;   // uniform
  CAcc3 g;
  g.zero();
  bool z = false;
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    CAcc3 e;   // V W2 for this block
    e.zero();
#pragma unroll
    for (int t = 0; t < NB / 4; ++t) e.add(vv[h][t].x, vv[h][t].y, xr[t], xi[t]);
    double2 nv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = r0 + 16 * h + lk + 4 * t;
      nv[t] = make_double2(av[h][t].x - e.re(t), av[h][t].y - e.im(t));
      if (col_ok && i < r1) A[(long long)(p + i) * n + col] = nv[t];
    }
    if (gram) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = r0 + 16 * h + lk + 4 * t;
        const bool in = col_ok && i >= NB && i < r1;
        const double2 a = in ? nv[t] : zero;
        z = z || (in && a.x == 0.0 && a.y == 0.0);
        g.add(a.x, -a.y, a.x, a.y);
      }
    }
  }
  if (gram) {
    const bool anyz = __ballot(z) != 0ull;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      sG[wave * 256 + (lk + 4 * r) * 16 + li] =
          make_double2(g.re(r), lane == 0 && r == 0 ? (anyz ? 1.0 : 0.0) : g.im(r));
    __syncthreads();
    const int e = threadIdx.x;
    double2 sum = sG[e];
#pragma unroll
    for (int w = 1; w < 4; ++w) sum = make_double2(sum.x + sG[w * 256 + e].x, sum.y + sG[w * 256 + e].y);
    qrt_scratch(A, m, n)[blockIdx.y * 256 + e] = sum;
  }
}

__global__ __launch_bounds__(256) void qrl_fill_kernel(const QrArgs args) {
  const QrlItem it = qrl_item(args, blockIdx.y);
  const int m = it.g->m, n = it.g->n;
  double2* A = qrl_ws(it);
  const long long mn = (long long)m * n;
  const long long per = (mn + QRL_CHUNKS - 1) / QRL_CHUNKS;
  const long long e0 = per * blockIdx.x, e1 = min(mn, e0 + per);
  for (long long idx = e0 + threadIdx.x; idx < e1; idx += 256)
    A[idx] = make_double2((idx / n == idx % n) ? 1.0 : 0.0, 0.0);
}

template <int CTO>
__global__ __launch_bounds__(256) void qrl_store_kernel(const QrArgs args) {
  using TO = typename St<CTO>::T;
  const QrlItem it = qrl_item(args, blockIdx.y);
  const int m = it.g->m, n = it.g->n, mode = it.g->mode;
  const double2* A = qrl_ws(it);
  TO* Q = reinterpret_cast<TO*>(const_cast<char*>(item_ptr(it.g->q, it.g->ids, it.item)));
  const long long mn = (long long)m * n;
  const long long per = (mn + QRL_CHUNKS - 1) / QRL_CHUNKS;
  const long long e0 = per * blockIdx.x, e1 = min(mn, e0 + per);
  for (long long idx = e0 + threadIdx.x; idx < e1; idx += 256) {
    double2 v;
    if (mode == 0) {
      v = A[idx];
    } else {   // Q^H: out[j][i] = conj(A[i][j]), out stored n x m
      const long long j = idx / m, i = idx % m;
      v = cconj(A[i * n + j]);
    }
    TO o;
    o.x = v.x;
    o.y = v.y;
    Q[idx] = o;
  }
}


// Spread path for small batches of matrices of at most 512 rows: the panels
// are factored by one 512-thread workgroup per matrix (Cholesky QR and
// Householder reconstruction where the panel allows it, else column by
// column), the trailing updates run over 16-column strips with one workgroup
// per strip and matrix, and Q is formed by the blocked kernel's Q-block
// launch from the explicit V and T in the workspace.  The workspace is the
// large path's.
constexpr int QRS_NW = 8, QRS_MAXB = 4;   // 512 threads, rows in 16-row blocks
constexpr size_t QRS_LDS = (size_t)512 * QB * sizeof(double2) + (size_t)QRS_NW * 256 * sizeof(double2);

// The panel at column p of one matrix, by the whole 512-thread workgroup; P
// (512 x 16 panel rows) and Wp (8 areas of 256) in LDS.  Uniform early exit
// when p >= n.
__device__ __forceinline__ void spread_panel(const QrlItem& it, int p, double2* P, double2* Wp) {
  PanelSmem2<QRS_NW, QB>& psm = *reinterpret_cast<PanelSmem2<QRS_NW, QB>*>(P);
  const int m = it.g->m, n = it.g->n;
  if (p >= n) return;
  double2* A = qrl_ws(it);
  double2* V = A + (long long)m * n;
  double2* Tg = V + (long long)m * n;
  const int mp = m - p, nbk = min(QB, n - p), k = p / QB;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), li = lane & 15, lk = lane >> 4;
  const double2 zero = make_double2(0.0, 0.0);

  if (p == 0 && tid == 0) {   // |F|^2 from the chunk partials, in a fixed order
    const double* part = qrl_partials(A, m, n);
    double s = 0.0;
    for (int c = 0; c < QRL_CHUNKS; ++c) s += part[c];
    *reinterpret_cast<double*>(const_cast<char*>(item_ptr(it.g->nrm2, it.g->ids, it.item))) = s;
  }
  double2 a[QRS_MAXB][4];   // rows 16 beta + 4t + lk, column p + li
#pragma unroll
  for (int b = 0; b < QRS_MAXB; ++b) {
    const int beta = wave + QRS_NW * b;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int row = 16 * beta + 4 * t + lk;
      a[b][t] = (beta >= k && row < m && li < nbk) ? A[(long long)row * n + p + li] : zero;
    }
  }
  bool chol = false;
  if (mp > nbk) {
    chol = panel_cholqr<QRS_NW, QRS_MAXB>(a, m, k, mp, nbk, P, Wp);
  } else {
#pragma unroll
    for (int b = 0; b < QRS_MAXB; ++b) {
      const int beta = wave + QRS_NW * b;
      if (beta >= k && 16 * beta < m) {
#pragma unroll
        for (int t = 0; t < 4; ++t) P[pidx(16 * (beta - k) + 4 * t + lk, li)] = a[b][t];
      }
    }
    __syncthreads();
  }
  if (!chol) {
    double2 ar[1][QB];
#pragma unroll
    for (int c = 0; c < QB; ++c) ar[0][c] = tid < mp ? P[pidx(tid, c)] : zero;
    factor_panel2<1, QB, 512>(ar, mp, nbk, psm, Wp);
#pragma unroll
    for (int c = 0; c < QB; ++c) {
      const bool in = tid < mp && c < nbk;
      P[pidx(tid, c)] = !in ? zero : (tid > c ? ar[0][c] : make_double2(tid == c ? 1.0 : 0.0, 0.0));
    }
  }
  __syncthreads();
  if (tid < mp) {
#pragma unroll
    for (int c = 0; c < QB; ++c)
      if (c < nbk) V[(long long)(p + tid) * n + p + c] = P[pidx(tid, c)];
  }
  if (tid < QB * QB) Tg[(long long)k * QB * QB + tid] = Wp[tid];
}

__global__ __launch_bounds__(512, 1) void qrs_panel_kernel(const QrArgs args, int p) {
  extern __shared__ __attribute__((aligned(16))) double2 qrs_dyn[];
  spread_panel(qrl_item(args, blockIdx.x), p, qrs_dyn, qrs_dyn + 512 * QB);
}

// Trailing update of the spread path, one 512-thread workgroup per (16-column
// strip, matrix): A[p:, c0:c0+16] -= V T^H (V^H A[p:, c0:c0+16]).  Wave w
// takes panel rows 64w .. 64w + 63 (at most 512 rows); the waves' parts of
// W = V^H A are summed through LDS in a fixed order.
// The workgroup of strip 0, whose columns are the next panel's, then factors
// that panel (look-ahead): its latency overlaps the other strips' updates,
// and the next update launch finds V and T in place.
__global__ __launch_bounds__(512, 1) void qrs_update_kernel(const QrArgs args, int p) {
  extern __shared__ __attribute__((aligned(16))) double2 qrs_dyn[];
  double2 (*sW)[256] = reinterpret_cast<double2 (*)[256]>(qrs_dyn + 512 * QB);
  const QrlItem it = qrl_item(args, blockIdx.y);
  const int m = it.g->m, n = it.g->n;
  const int c0 = p + QB + 16 * blockIdx.x;
  if (p >= n || c0 >= n) return;   // uniform over the workgroup
  double2* A = qrl_ws(it);
  const double2* V = A + (long long)m * n;
  const double2* T = V + (long long)m * n + (long long)(p / QB) * QB * QB;
  const int mp = m - p, nbk = min(QB, n - p);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), li = lane & 15, lk = lane >> 4;
  const int col = c0 + li;
  const bool col_ok = col < n;
  const int r0 = 64 * wave, r1 = min(mp, r0 + 64);
  const double2 zero = make_double2(0.0, 0.0);
  // this wave's rows of the strip (row r0 + 16h + 4t + lk) and its part of W
  double2 av[4][4];
  CAcc3 w;
  w.zero();
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    double2 vw[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = r0 + 16 * h + 4 * t + lk;
      av[h][t] = (i < r1 && col_ok) ? A[(long long)(p + i) * n + col] : zero;
      vw[t] = (i < r1 && li < nbk) ? V[(long long)(p + i) * n + p + li] : zero;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) w.add(vw[t].x, -vw[t].y, av[h][t].x, av[h][t].y);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) sW[wave][(lk + 4 * r) * 16 + li] = make_double2(w.re(r), w.im(r));
  __syncthreads();
  if (tid < 256) {
    double2 sum = sW[0][tid];
#pragma unroll
    for (int u = 1; u < QRS_NW; ++u) {
      sum.x += sW[u][tid].x;
      sum.y += sW[u][tid].y;
    }
    sW[0][tid] = sum;
  }
  __syncthreads();
  v4d_t wr, wi;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const double2 x = sW[0][(lk + 4 * t) * 16 + li];
    wr[t] = x.x;
    wi[t] = x.y;
  }
  // W2 = T^H W (item t = row lk + 4t = the B operand of k-step t)
  CAcc3 x2;
  x2.zero();
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int sr = 4 * t + lk;
    double2 x = zero;
    if (li < nbk && sr < nbk) {
      const double2 tt = T[sr * QB + li];
      x = make_double2(tt.x, -tt.y);
    }
    x2.add(x.x, x.y, wr[t], wi[t]);
  }
  double x2r[4], x2i[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    x2r[t] = x2.re(t);
    x2i[t] = x2.im(t);
  }
  // A -= V W2, block by block
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int rb = r0 + 16 * h;
    if (rb >= r1) break;   // uniform over the wave
    CAcc3 e;
    e.zero();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = rb + li, sr = 4 * t + lk;
      const double2 v = (i < r1 && sr < nbk) ? V[(long long)(p + i) * n + p + sr] : zero;
      e.add(v.x, v.y, x2r[t], x2i[t]);
    }
    if (col_ok) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = rb + lk + 4 * t;
        if (i < r1)
          A[(long long)(p + i) * n + col] = make_double2(av[h][t].x - e.re(t), av[h][t].y - e.im(t));
      }
    }
  }
  if (blockIdx.x == 0) {   // the next panel (columns c0 .. c0 + 15, just updated)
    __threadfence_block();
    __syncthreads();
    spread_panel(it, c0, qrs_dyn, qrs_dyn + 512 * QB);
  }
}

// Column-by-column factorisation of the panel rows of A (512 < m <= 2048
// rows, four rows per thread of a 512-thread workgroup), for panels the
// Cholesky QR does not take: writes V (unit diagonal) and T.  sP (16 QB
// values) and sWp (8 x 256) are its LDS scratch.
constexpr int QRT_RP = 4;   // rows per thread (2048 rows)

__device__ __noinline__ void tall_fallback(const double2* A, double2* V, double2* Tg, int p, int n,
                                           int mp, int nbk, int k, double2* sP, double2* sWp) {
  static_assert(sizeof(PanelSmem2<QRS_NW, QB>) <= 16 * QB * sizeof(double2), "fallback scratch fits");
  PanelSmem2<QRS_NW, QB>& psm = *reinterpret_cast<PanelSmem2<QRS_NW, QB>*>(sP);
  const int tid = threadIdx.x;
  const double2 zero = make_double2(0.0, 0.0);
  double2 a[QRT_RP][QB];
#pragma unroll
  for (int r = 0; r < QRT_RP; ++r) {
    const int i = tid + r * 512;
#pragma unroll
    for (int c = 0; c < QB; ++c)
      a[r][c] = (i < mp && c < nbk) ? A[(long long)(p + i) * n + p + c] : zero;
  }
  factor_panel2<QRT_RP, QB, 512>(a, mp, nbk, psm, sWp);
#pragma unroll
  for (int r = 0; r < QRT_RP; ++r) {
    const int i = tid + r * 512;
    if (i < mp) {
#pragma unroll
      for (int c = 0; c < QB; ++c) {
        if (c < nbk) {
          const double2 v = (i < c) ? zero : (i == c ? make_double2(1.0, 0.0) : a[r][c]);
          V[(long long)(p + i) * n + p + c] = v;
        }
      }
    }
  }
  if (tid < QB * QB) Tg[(long long)k * QB * QB + tid] = sWp[tid];
}

// Panel factorisation for 512 < m <= 2048 rows: Cholesky QR twice and
// Householder reconstruction (qr_cholpanel.h) with the row work of each
// 16-column panel spread over one 512-thread workgroup per 256-row chunk
// (block c of the chunk to wave c mod 8):
//   G1 parts   one per row chunk (exact-zero flag in Im G[0][0]): for the
//              first panel from qrt_gram, for the others from the strip-0
//              workgroups of the previous panel's update, which have just
//              written those columns
//   qrt_q1     every workgroup sums the parts in chunk order and forms
//              R1^{-1} (identical in all of them); Q1 = A R1^{-1} into the V
//              area, its top block also to the scratch, G2 parts
//   qrt_v      every workgroup sums the G2 parts and runs the
//              reconstruction on the top block (identical in all of them);
//              V = Q1 M in place, V's top block and T from chunk 0
// A panel the Cholesky QR does not take (an exact zero, a small pivot, a
// squared norm out of range, no rows below the diagonal block) is factored
// column by column by the chunk-0 workgroup of qrt_v (tall_fallback); qrt_q1
// passes its decision on through the flag in the scratch.
struct QrtCtx {
  double2 *A, *V, *Tg, *sc;
  int m, n, mp, nbk, k, nblk, nch;
  bool live;   // this workgroup's chunk holds rows of the panel
};

__device__ __forceinline__ QrtCtx qrt_ctx(const QrArgs& args, int p) {
  const QrlItem it = qrl_item(args, blockIdx.y);
  QrtCtx c;
  c.m = it.g->m;
  c.n = it.g->n;
  c.A = qrl_ws(it);
  c.V = c.A + (long long)c.m * c.n;
  c.Tg = c.V + (long long)c.m * c.n;
  c.sc = qrt_scratch(c.A, c.m, c.n);
  c.mp = c.m - p;
  c.nbk = min(QB, c.n - p);
  c.k = p / QB;
  c.nblk = (c.mp + 15) / 16;
  c.nch = (c.mp + QRT_CH - 1) / QRT_CH;
  c.live = p < c.n && (int)blockIdx.x < c.nch;
  return c;
}

// Sums the waves' 16 x 16 parts in sWp (8 x 256) into part 0 of sWp, then
// writes it to dst (256 values).
__device__ __forceinline__ void qrt_reduce_store(double2* sWp, double2* dst, int tid) {
  __syncthreads();
  if (tid < 256) {
    double2 s = sWp[tid];
#pragma unroll
    for (int w = 1; w < 8; ++w) s = make_double2(s.x + sWp[w * 256 + tid].x, s.y + sWp[w * 256 + tid].y);
    dst[tid] = s;
  }
}

// Loads the chunk parts src[0 .. nch) into sWp as eight parts (zeros beyond
// nch).
__device__ __forceinline__ void qrt_load_parts(double2* sWp, const double2* src, int nch, int tid) {
  for (int e = tid; e < 8 * 256; e += 512)
    sWp[e] = (e >> 8) < nch ? src[e] : make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(512, 1) void qrt_gram_kernel(const QrArgs args, int p) {
  __shared__ __attribute__((aligned(16))) double2 sWp[8 * 256];
  const QrtCtx c = qrt_ctx(args, p);
  if (!c.live) return;
  if (p == 0 && blockIdx.x == 0 && threadIdx.x == 0) {   // |F|^2 from the load's chunk sums
    const QrlItem it = qrl_item(args, blockIdx.y);
    const double* part = qrl_partials(c.A, c.m, c.n);
    double s = 0.0;
    for (int q = 0; q < QRL_CHUNKS; ++q) s += part[q];
    *reinterpret_cast<double*>(const_cast<char*>(item_ptr(it.g->nrm2, it.g->ids, it.item))) = s;
  }
  if (c.mp <= c.nbk) return;   // column by column
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const double2 zero = make_double2(0.0, 0.0);
  const int b0 = blockIdx.x * (QRT_CH / 16), b1 = min(c.nblk, b0 + QRT_CH / 16);
  CAcc3 g;
  g.zero();
  bool z = false;
  for (int b = b0 + wave; b < b1; b += 8) {
    double2 a4[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = 16 * b + 4 * t + lk;
      const bool in = i < c.mp && li < c.nbk;
      a4[t] = in ? c.A[(long long)(p + i) * c.n + p + li] : zero;
      z = z || (in && a4[t].x == 0.0 && a4[t].y == 0.0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) g.add(a4[t].x, -a4[t].y, a4[t].x, a4[t].y);
  }
  const bool anyz = __ballot(z) != 0ull;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    sWp[wave * 256 + (lk + 4 * r) * 16 + li] =
        make_double2(g.re(r), lane == 0 && r == 0 ? (anyz ? 1.0 : 0.0) : g.im(r));
  qrt_reduce_store(sWp, c.sc + blockIdx.x * 256, tid);
}

__global__ __launch_bounds__(512, 1) void qrt_q1_kernel(const QrArgs args, int p) {
  __shared__ __attribute__((aligned(16))) double2 sWp[8 * 256];
  const QrtCtx c = qrt_ctx(args, p);
  if (!c.live) return;
  double2* flag = c.sc + QRT_SCRATCH - 16;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const double2 zero = make_double2(0.0, 0.0);
  if (c.mp <= c.nbk) {   // no rows below the diagonal block: column by column
    if (blockIdx.x == 0 && tid == 0) *flag = make_double2(1.0, 0.0);
    return;
  }
  // G1 parts: one per chunk of qrt_gram (first panel) or of the previous
  // panel's update (its rows start 16 above)
  const int nparts = p == 0 ? c.nch : (c.mp + QB + QRL_CH - 1) / QRL_CH;
  qrt_load_parts(sWp, c.sc, nparts, tid);
  __syncthreads();
  if (wave == 0) panel_first_pass<8>(sWp, c.nbk);
  __syncthreads();
  const bool ok = sWp[16].x == 0.0;
  if (blockIdx.x == 0 && tid == 0) *flag = make_double2(ok ? 0.0 : 1.0, 0.0);
  if (!ok) return;
  double2 xb[4];   // X1[lk + 4s][li], the B operand of k-step s
#pragma unroll
  for (int s = 0; s < 4; ++s) xb[s] = sWp[(lk + 4 * s) * 16 + li];
  __syncthreads();   // X1 read everywhere before the parts are rewritten
  const int b0 = blockIdx.x * (QRT_CH / 16), b1 = min(c.nblk, b0 + QRT_CH / 16);
  double2* qtop = c.sc + 2 * QRT_MAXCH * 256;
  CAcc3 g2;
  g2.zero();
  for (int b = b0 + wave; b < b1; b += 8) {
    CAcc3 q;
    q.zero();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int i = 16 * b + li, col = 4 * s + lk;
      const double2 av = (i < c.mp && col < c.nbk) ? c.A[(long long)(p + i) * c.n + p + col] : zero;
      q.add(av.x, av.y, xb[s].x, xb[s].y);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * b + lk + 4 * r;
      const double2 qv = make_double2(q.re(r), q.im(r));
      if (i < c.mp && li < c.nbk) c.V[(long long)(p + i) * c.n + p + li] = qv;
      if (b == 0) qtop[pidx(lk + 4 * r, li)] = qv;
      g2.add(qv.x, -qv.y, qv.x, qv.y);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
    sWp[wave * 256 + (lk + 4 * r) * 16 + li] = make_double2(g2.re(r), g2.im(r));
  qrt_reduce_store(sWp, c.sc + (QRT_MAXCH + blockIdx.x) * 256, tid);
}

__global__ __launch_bounds__(512, 1) void qrt_v_kernel(const QrArgs args, int p) {
  __shared__ __attribute__((aligned(16))) double2 sP[16 * QB];
  __shared__ __attribute__((aligned(16))) double2 sWp[8 * 256];
  const QrtCtx c = qrt_ctx(args, p);
  if (!c.live) return;
  const double2* flag = c.sc + QRT_SCRATCH - 16;
  if (flag->x != 0.0) {   // the first pass did not take the panel
    if (blockIdx.x == 0) tall_fallback(c.A, c.V, c.Tg, p, c.n, c.mp, c.nbk, c.k, sP, sWp);
    return;
  }
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const double2 zero = make_double2(0.0, 0.0);
  qrt_load_parts(sWp, c.sc + QRT_MAXCH * 256, c.nch, tid);
  const double2* qtop = c.sc + 2 * QRT_MAXCH * 256;
  if (tid < 256) sP[tid] = qtop[tid];
  __syncthreads();
  if (wave == 0) panel_second_pass<8>(sP, sWp, c.nbk, c.mp);
  __syncthreads();
  if (sWp[16].x != 0.0) {   // identical in every workgroup
    if (blockIdx.x == 0) {
      __syncthreads();   // the flag read everywhere before the LDS is reused
      tall_fallback(c.A, c.V, c.Tg, p, c.n, c.mp, c.nbk, c.k, sP, sWp);
    }
    return;
  }
  double2 mb[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) mb[s] = sWp[256 + (lk + 4 * s) * 16 + li];
  const int b0 = blockIdx.x * (QRT_CH / 16), b1 = min(c.nblk, b0 + QRT_CH / 16);
  for (int b = b0 + wave; b < b1; b += 8) {
    if (b == 0) continue;
    CAcc3 y;
    y.zero();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int i = 16 * b + li, col = 4 * s + lk;
      const double2 av = (i < c.mp && col < c.nbk) ? c.V[(long long)(p + i) * c.n + p + col] : zero;
      y.add(av.x, av.y, mb[s].x, mb[s].y);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * b + lk + 4 * r;
      if (i < c.mp && li < c.nbk) c.V[(long long)(p + i) * c.n + p + li] = make_double2(y.re(r), y.im(r));
    }
  }
  if (blockIdx.x == 0) {
    if (wave == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = lk + 4 * r;
        if (i < c.mp && li < c.nbk) c.V[(long long)(p + i) * c.n + p + li] = sP[pidx(i, li)];
      }
    }
    if (tid < QB * QB) c.Tg[(long long)c.k * QB * QB + tid] = sWp[tid];
  }
}

template <int CTI, int CTO>
hipError_t run_tall(QrArgs args, int items, int m_max, int n_max, hipStream_t s) {
  const dim3 chunks(QRL_CHUNKS, items);
  hipLaunchKernelGGL((qrl_load_kernel<CTI>), chunks, dim3(256), 0, s, args);
  const dim3 pch((m_max + QRT_CH - 1) / QRT_CH, items);
  hipLaunchKernelGGL(qrt_gram_kernel, pch, dim3(512), 0, s, args, 0);
  for (int p = 0; p < n_max; p += QB) {
    hipLaunchKernelGGL(qrt_q1_kernel, pch, dim3(512), 0, s, args, p);
    hipLaunchKernelGGL(qrt_v_kernel, pch, dim3(512), 0, s, args, p);
    const int strips = (n_max - p - QB + 15) / 16;
    if (strips > 0) {
      const dim3 grid(strips, (m_max - p + QRL_CH - 1) / QRL_CH, items);
      hipLaunchKernelGGL((qrl_wpart_kernel<QB>), grid, dim3(256), 0, s, args, p, QB);
      hipLaunchKernelGGL((qrl_update_kernel<QB>), grid, dim3(256), 0, s, args, p, QB, 1);
    }
  }
  hipLaunchKernelGGL(qrl_fill_kernel, chunks, dim3(256), 0, s, args);
  for (int p = ((n_max - 1) / QB) * QB; p >= 0; p -= QB) {
    const dim3 grid((n_max - p + 15) / 16, (m_max - p + QRL_CH - 1) / QRL_CH, items);
    hipLaunchKernelGGL((qrl_wpart_kernel<QB>), grid, dim3(256), 0, s, args, p, 0);
    hipLaunchKernelGGL((qrl_update_kernel<QB>), grid, dim3(256), 0, s, args, p, 0, 0);
  }
  hipLaunchKernelGGL((qrl_store_kernel<CTO>), chunks, dim3(256), 0, s, args);
  return hipGetLastError();
}

template <int CTI>
hipError_t run_spread(QrArgs args, int items, int m_max, int n_max, hipStream_t s) {
  static hipError_t attr1 = hipFuncSetAttribute(reinterpret_cast<const void*>(&qrs_panel_kernel),
                                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                                (int)QRS_LDS);
  static hipError_t attr2 = hipFuncSetAttribute(reinterpret_cast<const void*>(&qrs_update_kernel),
                                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                                (int)QRS_LDS);
  if (attr1 != hipSuccess) return attr1;
  if (attr2 != hipSuccess) return attr2;
  const dim3 chunks(QRL_CHUNKS, items);
  hipLaunchKernelGGL((qrl_load_kernel<CTI>), chunks, dim3(256), 0, s, args);
  hipLaunchKernelGGL(qrs_panel_kernel, dim3(items), dim3(512), QRS_LDS, s, args, 0);
  for (int p = 0; p + QB < n_max; p += QB)   // update by panel p, factor panel p + 16
    hipLaunchKernelGGL(qrs_update_kernel, dim3((n_max - p - QB + 15) / 16, items), dim3(512), QRS_LDS,
                       s, args, p);
  return hipGetLastError();
}

}  // namespace

int qr_large_max_rows() { return 2048; }

size_t qr_large_ws_elems(int m, int n) {
  const size_t parts = (((size_t)n + 15) / 16) * (((size_t)m + QRL_CH - 1) / QRL_CH) * 256;
  return 2 * (size_t)m * n + 16 * ((size_t)n + 16) + QRL_CHUNKS / 2 + parts + QRT_SCRATCH + 1;
}

hipError_t launch_qr_large(int ct_in, int ct_out, const QrArgs& args_in, hipStream_t s) {
  QrArgs args = args_in;
  int items = 0, m_max = 0, n_max = 0;
  for (int g = 0; g < args.ngroups; ++g) {
    if (args.g[g].mode == 2 || args.g[g].m < args.g[g].n) return hipErrorInvalidValue;
    args.g[g].blk_begin = items;
    items += args.g[g].batch;
    m_max = max(m_max, args.g[g].m);
    n_max = max(n_max, args.g[g].n);
  }
  if (items == 0) return hipSuccess;
  if (m_max > qr_large_max_rows()) return hipErrorInvalidValue;
#define DCS_QRL(I, O)            \
  if (ct_in == I && ct_out == O) \
    return run_tall<I, O>(args, items, m_max, n_max, s);
  DCS_QRL(CT_F32, CT_F32)
  DCS_QRL(CT_F64, CT_F64)
  DCS_QRL(CT_F64, CT_F32)
#undef DCS_QRL
  return hipErrorInvalidValue;
}

int qr_spread_max_rows() { return 512; }
int qr_spread_max_items() { return 96; }

hipError_t launch_qr_spread(int ct_in, int ct_out, const QrArgs& args_in, hipStream_t s) {
  QrArgs args = args_in;
  int items = 0, m_max = 0, n_max = 0;
  for (int g = 0; g < args.ngroups; ++g) {
    if (args.g[g].mode == 2 || args.g[g].m < args.g[g].n) return hipErrorInvalidValue;
    args.g[g].blk_begin = items;
    items += args.g[g].batch;
    m_max = max(m_max, args.g[g].m);
    n_max = max(n_max, args.g[g].n);
  }
  if (items == 0) return hipSuccess;
  if (m_max > qr_spread_max_rows()) return hipErrorInvalidValue;
  hipError_t e = ct_in == CT_F32   ? run_spread<CT_F32>(args, items, m_max, n_max, s)
                 : ct_in == CT_F64 ? run_spread<CT_F64>(args, items, m_max, n_max, s)
                                   : hipErrorInvalidValue;
  if (e != hipSuccess) return e;
  // Q from V and T: the blocked kernel's Q blocks read V at the workspace
  // start and T after it, so each group's workspace is taken m n further on
  QrArgs qa = args;
  for (int g = 0; g < qa.ngroups; ++g)
    qa.g[g].ws.base = static_cast<const char*>(qa.g[g].ws.base) +
                      (size_t)qa.g[g].m * qa.g[g].n * sizeof(double2);
  return launch_qr_qblocks(ct_in, ct_out, qa, m_max, s);
}

}  // namespace dcs
