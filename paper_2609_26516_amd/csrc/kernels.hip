// Non-GEMM kernels of the compression step and the dynamic operations:
// layered gate-operator application, FP64 Householder QR / LQ of the local
// tensor (gauge shift), outcome norms for the measurement probability, and
// the collapse of a site tensor.
#include "dcs_internal.h"
#include <cstring>
#include "kernel_util.h"
#include "qr_panel.h"
#include "qr_cholpanel.h"

namespace dcs {
namespace {

constexpr int NT = 256;

// ---------------------------------------------------------------------------
// Gate-operator application.  WMAX bounds the operator bond dims so the
// per-thread inputs stay in registers (loops fully unrolled, predicated).

template <int CT, int WMAX>
__global__ __launch_bounds__(NT) void mpo_right_kernel(const MpoArgs args) {
  // X1[a][wl][t][y] -> X2[a][s][wr][y]
  using T = typename St<CT>::T;
  using R = typename St<CT>::R;
  __shared__ T sW[WMAX * 4 * WMAX];
  const int gi = find_group<MPO_MAX_GROUPS>(args.g, args.ngroups, blockIdx.x);
  const MpoGroup& G = args.g[gi];
  const int local = blockIdx.x - G.blk_begin;
  const int item = local / G.blk_per_item;
  const int sub = local - item * G.blk_per_item;
  const int wl = G.wl, wr = G.wr, d0 = G.d0, d1 = G.d1;
  const T* __restrict__ X1 = reinterpret_cast<const T*>(item_ptr(G.in, G.ids, item));
  T* __restrict__ X2 = reinterpret_cast<T*>(const_cast<char*>(item_ptr(G.out, G.ids, item)));
  const T* __restrict__ W = reinterpret_cast<const T*>(item_ptr(G.w, G.ids, item));
  const int nw = wl * 4 * wr;
  for (int i = threadIdx.x; i < nw; i += NT) sW[i] = W[i];
  __syncthreads();
  const long long idx = (long long)sub * NT + threadIdx.x;
  if (idx >= (long long)d0 * d1) return;
  const int a = (int)(idx / d1), y = (int)(idx % d1);
  R xr[2 * WMAX], xi[2 * WMAX];
#pragma unroll
  for (int k = 0; k < 2 * WMAX; ++k) {
    xr[k] = 0;
    xi[k] = 0;
    if (k < 2 * wl) {   // k = wl_i * 2 + t
      const T v = X1[((long long)a * 2 * wl + k) * d1 + y];
      xr[k] = v.x;
      xi[k] = v.y;
    }
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int o = 0; o < WMAX; ++o) {
      if (o < wr) {
        R accr = 0, acci = 0;
#pragma unroll
        for (int k = 0; k < 2 * WMAX; ++k) {
          if (k < 2 * wl) {
            const int wli = k >> 1, t = k & 1;
            const T w = sW[((wli * 2 + s) * 2 + t) * wr + o];
            accr += w.x * xr[k] - w.y * xi[k];
            acci += w.x * xi[k] + w.y * xr[k];
          }
        }
        T out;
        out.x = accr;
        out.y = acci;
        X2[(((long long)a * 2 + s) * wr + o) * d1 + y] = out;
      }
    }
  }
}

template <int CT, int WMAX>
__global__ __launch_bounds__(NT) void mpo_left_kernel(const MpoArgs args) {
  // Y1[x][t][c][wr] -> Y2[wl][x][s][c]
  using T = typename St<CT>::T;
  using R = typename St<CT>::R;
  __shared__ T sW[WMAX * 4 * WMAX];
  const int gi = find_group<MPO_MAX_GROUPS>(args.g, args.ngroups, blockIdx.x);
  const MpoGroup& G = args.g[gi];
  const int local = blockIdx.x - G.blk_begin;
  const int item = local / G.blk_per_item;
  const int sub = local - item * G.blk_per_item;
  const int wl = G.wl, wr = G.wr, d0 = G.d0, d1 = G.d1;
  const T* __restrict__ Y1 = reinterpret_cast<const T*>(item_ptr(G.in, G.ids, item));
  T* __restrict__ Y2 = reinterpret_cast<T*>(const_cast<char*>(item_ptr(G.out, G.ids, item)));
  const T* __restrict__ W = reinterpret_cast<const T*>(item_ptr(G.w, G.ids, item));
  const int nw = wl * 4 * wr;
  for (int i = threadIdx.x; i < nw; i += NT) sW[i] = W[i];
  __syncthreads();
  const long long idx = (long long)sub * NT + threadIdx.x;
  if (idx >= (long long)d0 * d1) return;
  const int x = (int)(idx / d1), c = (int)(idx % d1);
  R yr[2 * WMAX], yi[2 * WMAX];
#pragma unroll
  for (int k = 0; k < 2 * WMAX; ++k) {   // k = t * WMAX + wr_i
    yr[k] = 0;
    yi[k] = 0;
    const int t = k / WMAX, o = k % WMAX;
    if (o < wr) {
      const T v = Y1[(((long long)x * 2 + t) * d1 + c) * wr + o];
      yr[k] = v.x;
      yi[k] = v.y;
    }
  }
#pragma unroll
  for (int l = 0; l < WMAX; ++l) {
    if (l < wl) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        R accr = 0, acci = 0;
#pragma unroll
        for (int k = 0; k < 2 * WMAX; ++k) {
          const int t = k / WMAX, o = k % WMAX;
          if (o < wr) {
            const T w = sW[((l * 2 + s) * 2 + t) * wr + o];
            accr += w.x * yr[k] - w.y * yi[k];
            acci += w.x * yi[k] + w.y * yr[k];
          }
        }
        T out;
        out.x = accr;
        out.y = acci;
        Y2[(((long long)l * d0 + x) * 2 + s) * d1 + c] = out;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 Householder QR in the LAPACK convention (zgeqr2 reflectors
// H_k = I - tau_k v v^H, v_k = 1, beta = -sign(Re alpha) |(alpha, x)|,
// tau = ((beta - Re alpha) / beta, -Im alpha / beta), v = x / (alpha - beta);
// tau = 0 when x = 0 and alpha is real), then the thin Q = H_0 ... H_{n-1}
// [I; 0] accumulated backwards (zung2r).  The m x n working matrix is held
// column-major either in LDS or in the branch's global workspace.


template <int CTI, int CTO>
__global__ __launch_bounds__(NT) void qr_kernel(const QrArgs args) {
  using TI = typename St<CTI>::T;
  using TO = typename St<CTO>::T;
  extern __shared__ double2 dyn_lds[];
  __shared__ double2 s_tau[1024];
  __shared__ double s_red[8];
  __shared__ double2 s_bc[2];

  const int gi = find_group<QR_MAX_GROUPS>(args.g, args.ngroups, blockIdx.x);
  const QrGroup& G = args.g[gi];
  const int item = blockIdx.x - G.blk_begin;
  const int m = G.m, n = G.n, mode = G.mode;
  const TI* __restrict__ F = reinterpret_cast<const TI*>(item_ptr(G.f, G.ids, item));
  TO* __restrict__ Q = reinterpret_cast<TO*>(const_cast<char*>(item_ptr(G.q, G.ids, item)));
  double* nrm = reinterpret_cast<double*>(const_cast<char*>(item_ptr(G.nrm2, G.ids, item)));
  double2* W = args.use_lds
                   ? dyn_lds
                   : reinterpret_cast<double2*>(const_cast<char*>(item_ptr(G.ws, G.ids, item)));
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const long long mn = (long long)m * n;

  // load (column-major working copy of T, or of T^H in mode 1) and |F|^2
  double part = 0;
  if (mode == 0) {
    for (long long idx = tid; idx < mn; idx += NT) {
      const double2 v = to_d2(F[idx]);
      part += v.x * v.x + v.y * v.y;
      const int i = (int)(idx / n), j = (int)(idx % n);
      W[i + (long long)j * m] = v;
    }
  } else if (mode == 1) {
    for (long long idx = tid; idx < mn; idx += NT) {
      const double2 v = to_d2(F[idx]);
      part += v.x * v.x + v.y * v.y;
      W[idx] = cconj(v);   // F is n x m row-major: F[j][i] -> W[i + j m]
    }
  } else {
    for (long long idx = tid; idx < mn; idx += NT) {
      const double2 v = to_d2(F[idx]);
      part += v.x * v.x + v.y * v.y;
    }
  }
  const double nu2 = block_sum(part, s_red);
  if (tid == 0) *nrm = nu2;
  if (mode == 2) {
    const double sc = nu2 > 0 ? 1.0 / sqrt(nu2) : 0.0;
    for (long long idx = tid; idx < mn; idx += NT) {
      const double2 v = to_d2(F[idx]);
      TO o;
      o.x = v.x * sc;
      o.y = v.y * sc;
      Q[idx] = o;
    }
    return;
  }
  __syncthreads();

  // factorisation
  for (int k = 0; k < n; ++k) {
    double2* colk = W + (long long)k * m;
    // scaled sum of squares of x = column k below the diagonal (no underflow
    // for the tiny entries rank-deficient local tensors carry)
    double sc = 0.0, q = 0.0;
    for (int i = k + 1 + tid; i < m; i += NT) {
      const double2 v = colk[i];
      ssq_add(sc, q, v.x);
      ssq_add(sc, q, v.y);
    }
    block_ssq(sc, q, s_red);
    if (tid == 0) {
      const double2 alpha = colk[k];
      double2 tau = make_double2(0.0, 0.0), scal = make_double2(1.0, 0.0);
      if (!(sc == 0.0 && alpha.y == 0.0)) {
        double sa = sc, qa = q;
        ssq_add(sa, qa, alpha.x);
        ssq_add(sa, qa, alpha.y);
        const double nrm_all = sa * sqrt(qa);
        if (nrm_all > 1e-280) {
          const double beta = alpha.x >= 0.0 ? -nrm_all : nrm_all;
          tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
          scal = crecip(make_double2(alpha.x - beta, alpha.y));   // 1 / (alpha - beta)
          colk[k] = make_double2(beta, 0.0);
        }
      }
      s_tau[k] = tau;
      s_bc[0] = tau;
      s_bc[1] = scal;
    }
    __syncthreads();
    const double2 tau = s_bc[0], scal = s_bc[1];
    if (tau.x == 0.0 && tau.y == 0.0) {
      __syncthreads();
      continue;
    }
    for (int i = k + 1 + tid; i < m; i += NT) colk[i] = cmul(colk[i], scal);
    __syncthreads();
    const double2 ctau = cconj(tau);
    for (int j = k + 1 + wave; j < n; j += 4) {
      double2* colj = W + (long long)j * m;
      double sr = 0, si = 0;
      for (int i = k + lane; i < m; i += 64) {
        const double2 v = (i == k) ? make_double2(1.0, 0.0) : colk[i];
        const double2 w = cdotc(v, colj[i]);
        sr += w.x;
        si += w.y;
      }
      sr = wave_sum(sr);
      si = wave_sum(si);
      const double2 c = cmul(ctau, make_double2(sr, si));
      for (int i = k + lane; i < m; i += 64) {
        const double2 v = (i == k) ? make_double2(1.0, 0.0) : colk[i];
        const double2 u = cmul(v, c);
        colj[i] = make_double2(colj[i].x - u.x, colj[i].y - u.y);
      }
    }
    __syncthreads();
  }

  // thin Q, accumulated backwards
  for (int k = n - 1; k >= 0; --k) {
    const double2 tau = s_tau[k];
    double2* colk = W + (long long)k * m;
    if (k < n - 1 && !(tau.x == 0.0 && tau.y == 0.0)) {
      for (int j = k + 1 + wave; j < n; j += 4) {
        double2* colj = W + (long long)j * m;
        double sr = 0, si = 0;
        for (int i = k + lane; i < m; i += 64) {
          const double2 v = (i == k) ? make_double2(1.0, 0.0) : colk[i];
          const double2 w = cdotc(v, colj[i]);
          sr += w.x;
          si += w.y;
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        const double2 c = cmul(tau, make_double2(sr, si));
        for (int i = k + lane; i < m; i += 64) {
          const double2 v = (i == k) ? make_double2(1.0, 0.0) : colk[i];
          const double2 u = cmul(v, c);
          colj[i] = make_double2(colj[i].x - u.x, colj[i].y - u.y);
        }
      }
    }
    __syncthreads();
    for (int i = tid; i < m; i += NT) {
      if (i < k) {
        colk[i] = make_double2(0.0, 0.0);
      } else if (i == k) {
        colk[i] = make_double2(1.0 - tau.x, -tau.y);
      } else {
        const double2 v = colk[i];
        colk[i] = make_double2(-(tau.x * v.x - tau.y * v.y), -(tau.x * v.y + tau.y * v.x));
      }
    }
    __syncthreads();
  }

  // write Q (mode 0, m x n row-major) or Q^H (mode 1, n x m row-major)
  if (mode == 0) {
    for (long long idx = tid; idx < mn; idx += NT) {
      const int i = (int)(idx / n), j = (int)(idx % n);
      const double2 v = W[i + (long long)j * m];
      TO o;
      o.x = v.x;
      o.y = v.y;
      Q[idx] = o;
    }
  } else {
    for (long long idx = tid; idx < mn; idx += NT) {
      const double2 v = W[idx];
      TO o;
      o.x = v.x;
      o.y = -v.y;
      Q[idx] = o;
    }
  }
}

// ---------------------------------------------------------------------------
// Blocked FP64 Householder QR with explicit thin Q (same reflectors as the
// unblocked kernel above), one workgroup per matrix of at most 512 rows; the
// m x n working matrix is row-major in the branch's global workspace.  Per
// 16-column panel:
//   * the panel rows go to registers, one row per thread, and are factored
//     there (factor_panel: one workgroup reduction round per column; the T
//     factor of the compact WY form H_p ... H_{p+15} = I - V T V^H from the
//     Gram entries gathered in the same rounds);
//   * V goes to LDS (rows swizzled against bank conflicts) and every wave
//     copies the rows it owns into registers in the two MFMA operand layouts
//     it needs;
//   * the trailing columns are updated 16 at a time by the whole workgroup:
//     each wave loads its rows of the strip once, forms its part of
//     W = V^H A on FP64 MFMA (v_mfma_f64_16x16x4), the parts are summed
//     through LDS in a fixed order, W2 = T^H W, and each wave writes its rows
//     of A - V W2 from the same registers: one read and one write of the
//     trailing matrix per panel.
// Q is then accumulated backwards panel by panel in place, the same way with
// X = T, after the panel's own columns [I; 0] - V (T V1^H).

// Reflector r of the panel at local row i; the panel in LDS is explicit (0
// above the diagonal, 1 on it, 0 in unused columns and rows).
__device__ __forceinline__ double2 pv(const double2* P, int i, int r) { return P[pidx(i, r)]; }

// NTQ threads per workgroup: 512 (8 waves, one workgroup per CU) for up to
// 512 rows, 256 (4 waves, two per CU) for up to 128 rows; wave w owns rows
// [w rw, (w + 1) rw) below the panel top, at most MAXB blocks of 16.
// Dynamic LDS: the panel's V for up to PROWS rows (also holding the panel
// factorisation scratch before V is written), then one W part per wave
// (also holding T while the panel is factored).
template <int NTQ>
struct QrShape {
  static constexpr int NW = NTQ / 64;
  static constexpr int MAXB = NTQ == 512 ? 4 : 2;
  static constexpr int PROWS = NTQ == 512 ? 512 : 128;
  static constexpr size_t P_BYTES = (size_t)PROWS * QB * sizeof(double2);
  static constexpr size_t LDS_BYTES = P_BYTES + (size_t)NW * 256 * sizeof(double2);
  static_assert(sizeof(PanelSmem<NW, QB>) <= P_BYTES, "factorisation scratch fits the panel area");
  // left-looking variant: 16-row blocks per wave, V_j^T areas in the panel area
  static constexpr int QLB = (NTQ == 512 ? 32 : 8) / NW;
  static_assert((size_t)NW * QLB * 256 * sizeof(double2) <= P_BYTES, "V_j^T areas fit");
  static_assert(sizeof(PanelSmem2<NW, QB>) <= P_BYTES, "factorisation scratch fits");
};

// Columns c_begin..n-1 of rows p + [r0, r1) of A: A -= V X (V^H A) with
// X[li][4t + lk] = xv[t] (T^H or T), strips of 16 columns.  Both V operands
// come from the panel in LDS; the waves' W parts are summed through Wp in a
// fixed order.  Every thread of the workgroup takes part.
template <int NTQ>
__device__ __forceinline__ void update_strips(double2* __restrict__ A, int n, int p, int mp,
                                              int nbk, int r0, int r1, int c_begin,
                                              const double2* P, const double2 (&xv)[4],
                                              double2* Wp) {
  constexpr int NW = QrShape<NTQ>::NW, MAXB = QrShape<NTQ>::MAXB;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const double2 zero = make_double2(0.0, 0.0);
  for (int c0 = c_begin; c0 < n; c0 += 16) {
    const int col = c0 + li;
    const bool ok = col < n;
    // row r0 + lk of the strip; the other rows are wave-uniform offsets
    double2* __restrict__ Arow = A + (long long)(p + r0 + lk) * n + col;
    double2 a[MAXB][4];
#pragma unroll
    for (int b = 0; b < MAXB; ++b)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = r0 + 16 * b + lk + 4 * t;
        a[b][t] = (i < r1 && ok) ? Arow[(16 * b + 4 * t) * n] : zero;
      }
    CAcc3 w;
    w.zero();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double2 v = pv(P, r0 + 16 * b + 4 * t + lk, li);   // A operand conj(V[i][li])
        w.add(v.x, -v.y, a[b][t].x, a[b][t].y);
      }
      __builtin_amdgcn_sched_barrier(0);   // keep the LDS operand reads block by block
    }
    v4d_t wr, wi;
#pragma unroll
    for (int r = 0; r < 4; ++r) Wp[wave * 256 + (lk + 4 * r) * 16 + li] = make_double2(w.re(r), w.im(r));
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = (lk + 4 * r) * 16 + li;
      double2 sum = Wp[e];
#pragma unroll
      for (int w = 1; w < NW; ++w) {
        sum.x += Wp[w * 256 + e].x;
        sum.y += Wp[w * 256 + e].y;
      }
      wr[r] = sum.x;
      wi[r] = sum.y;
    }
    __syncthreads();   // every wave has its W before the next strip's parts
    // W2 = X W (result item t = row lk + 4t = the B operand of k-step t)
    CAcc3 x2;
    x2.zero();
#pragma unroll
    for (int t = 0; t < 4; ++t) x2.add(xv[t].x, xv[t].y, wr[t], wi[t]);
    double x2r[4], x2i[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      x2r[t] = x2.re(t);
      x2i[t] = x2.im(t);
    }
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      CAcc3 e;   // V W2 for this block
      e.zero();
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double2 v = pv(P, r0 + 16 * b + li, 4 * t + lk);   // A operand V[i][4t + lk]
        e.add(v.x, v.y, x2r[t], x2i[t]);
      }
      __builtin_amdgcn_sched_barrier(0);
      if (ok) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = r0 + 16 * b + lk + 4 * t;
          if (i < r1)
            Arow[(16 * b + 4 * t) * n] = make_double2(a[b][t].x - e.re(t), a[b][t].y - e.im(t));
        }
      }
    }
  }
}

template <int CTI, int CTO, int NTQ>
__global__ __launch_bounds__(NTQ, NTQ == 256 ? 2 : 1) void qr_blocked_kernel(const QrArgs args) {
  using Shape = QrShape<NTQ>;
  constexpr int NW = Shape::NW;
  using TI = typename St<CTI>::T;
  using TO = typename St<CTO>::T;
  extern __shared__ __attribute__((aligned(16))) double2 dyn[];
  PanelSmem<NW, QB>& psm = *reinterpret_cast<PanelSmem<NW, QB>*>(dyn);
  double* s_red = reinterpret_cast<double*>(dyn);       // start of the kernel only
  double2* P = dyn;
  double2* Wp = dyn + Shape::P_BYTES / sizeof(double2);
  double2* sT = Wp;                                     // while a panel is factored

  const int gi = find_group<QR_MAX_GROUPS>(args.g, args.ngroups, blockIdx.x);
  const QrGroup& G = args.g[gi];
  const int item = blockIdx.x - G.blk_begin;
  const int m = G.m, n = G.n, mode = G.mode;
  const TI* __restrict__ F = reinterpret_cast<const TI*>(item_ptr(G.f, G.ids, item));
  TO* __restrict__ Q = reinterpret_cast<TO*>(const_cast<char*>(item_ptr(G.q, G.ids, item)));
  double* nrm = reinterpret_cast<double*>(const_cast<char*>(item_ptr(G.nrm2, G.ids, item)));
  double2* A = reinterpret_cast<double2*>(const_cast<char*>(item_ptr(G.ws, G.ids, item)));
  double2* Tg = A + (long long)m * n;       // T factor of every panel
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const long long mn = (long long)m * n;

  // load the row-major working matrix (T, or T^H in mode 1) and |F|^2
  double part = 0;
  if (mode == 0) {
    for (long long idx = tid; idx < mn; idx += NTQ) {
      const double2 v = to_d2(F[idx]);
      part += v.x * v.x + v.y * v.y;
      A[idx] = v;
    }
  } else if (mode == 1) {
    for (long long idx = tid; idx < mn; idx += NTQ) {   // F is n x m: F[j][i]
      const double2 v = to_d2(F[idx]);
      part += v.x * v.x + v.y * v.y;
      const int j = (int)(idx / m), i = (int)(idx % m);
      A[(long long)i * n + j] = cconj(v);
    }
  } else {
    for (long long idx = tid; idx < mn; idx += NTQ) {
      const double2 v = to_d2(F[idx]);
      part += v.x * v.x + v.y * v.y;
    }
  }
  double nu2 = part, nu_mx = 0.0;
  block_sum_max<NW>(nu2, nu_mx, s_red);
  if (tid == 0) *nrm = nu2;
  if (mode == 2) {
    const double sc = nu2 > 0 ? 1.0 / sqrt(nu2) : 0.0;
    for (long long idx = tid; idx < mn; idx += NTQ) {
      const double2 v = to_d2(F[idx]);
      TO o;
      o.x = v.x * sc;
      o.y = v.y * sc;
      Q[idx] = o;
    }
    return;
  }
  __syncthreads();

  const int li = lane & 15, lk = lane >> 4;
  const int npan = (n + QB - 1) / QB;
  for (int pi = 0; pi < npan; ++pi) {
    const int p = pi * QB, nbk = min(QB, n - p), mp = m - p;
    const int rw = ((mp + 16 * NW - 1) / (16 * NW)) * 16;
    const int r0 = wave * rw, r1 = min(mp, r0 + rw);
    double2 a[1][QB];
#pragma unroll
    for (int c = 0; c < QB; ++c)
      a[0][c] = (tid < mp && c < nbk) ? A[(long long)(p + tid) * n + p + c] : make_double2(0.0, 0.0);
    factor_panel<1, QB, NTQ>(a, mp, nbk, psm, sT);
    // explicit V to LDS (over the factorisation scratch), the panel to the
    // workspace for the Q accumulation, T to the workspace and X = T^H to
    // registers
    if (tid < Shape::PROWS) {
#pragma unroll
      for (int c = 0; c < QB; ++c) {
        const bool in = tid < mp && c < nbk;
        P[pidx(tid, c)] = !in ? make_double2(0.0, 0.0)
                              : (tid < c ? make_double2(0.0, 0.0)
                                         : (tid == c ? make_double2(1.0, 0.0) : a[0][c]));
        if (in) A[(long long)(p + tid) * n + p + c] = a[0][c];
      }
    }
    if (tid < QB * QB) Tg[(long long)pi * QB * QB + tid] = sT[tid];
    double2 xv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) xv[t] = cconj(sT[(4 * t + lk) * QB + li]);
    __syncthreads();
    update_strips<NTQ>(A, n, p, mp, nbk, r0, r1, p + nbk, P, xv, Wp);
    __syncthreads();
  }

  // explicit thin Q, panels in reverse order (in place)
  for (int pi = npan - 1; pi >= 0; --pi) {
    const int p = pi * QB, nbk = min(QB, n - p), mp = m - p;
    const int rw = ((mp + 16 * NW - 1) / (16 * NW)) * 16;
    const int r0 = wave * rw, r1 = min(mp, r0 + rw);
    for (int e = tid; e < Shape::PROWS * QB; e += NTQ) {   // explicit V
      const int i = e / QB, c = e % QB;
      double2 v = make_double2(0.0, 0.0);
      if (i < mp && c < nbk)
        v = i > c ? A[(long long)(p + i) * n + p + c] : make_double2(i == c ? 1.0 : 0.0, 0.0);
      P[pidx(i, c)] = v;
    }
    double2 xv[4];   // X = T: xv[t] = T[li][4t + lk]
#pragma unroll
    for (int t = 0; t < 4; ++t) xv[t] = Tg[(long long)pi * QB * QB + li * QB + 4 * t + lk];
    __syncthreads();
    // the panel's own columns: [I; 0] - V (T V1^H), V1 the top nbk x nbk block
    {
      v4d_t sr, si;
      zero4(sr);
      zero4(si);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int s2 = 4 * t + lk;
        const double2 b = pv(P, li, s2);   // V1[li][s2] -> conj for B
        cmma(xv[t].x, xv[t].y, b.x, -b.y, sr, si);
      }
      // S = T V1^H in registers (item t: row lk + 4t, col li)
      for (int rb = wave * 16; rb < mp; rb += 16 * NW) {
        v4d_t dr, di;
        zero4(dr);
        zero4(di);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const double2 v = pv(P, rb + li, 4 * t + lk);
          cmma(v.x, v.y, sr[t], si[t], dr, di);
        }
        if (li < nbk) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int i = rb + lk + 4 * t;
            if (i < mp)
              A[(long long)(p + i) * n + p + li] =
                  make_double2((i == li ? 1.0 : 0.0) - dr[t], -di[t]);
          }
        }
      }
    }
    for (int e = tid; e < p * nbk; e += NTQ) {   // rows above the panel
      const int i = e / nbk, c = e % nbk;
      A[(long long)i * n + p + c] = make_double2(0.0, 0.0);
    }
    update_strips<NTQ>(A, n, p, mp, nbk, r0, r1, p + nbk, P, xv, Wp);
    __syncthreads();
  }

  // write Q (mode 0) or Q^H (mode 1)
  if (mode == 0) {
    for (long long idx = tid; idx < mn; idx += NTQ) {
      const double2 v = A[idx];
      TO o;
      o.x = v.x;
      o.y = v.y;
      Q[idx] = o;
    }
  } else {
    for (long long idx = tid; idx < mn; idx += NTQ) {   // out[j][i] = conj(A[i][j])
      const int j = (int)(idx / m), i = (int)(idx % m);
      const double2 v = A[(long long)i * n + j];
      TO o;
      o.x = v.x;
      o.y = -v.y;
      Q[idx] = o;
    }
  }
}

// ---------------------------------------------------------------------------
// Left-looking variant of the blocked QR (same reflectors, same LDS budget).
// Only Q is wanted, so the working matrix is never kept: panel k is read
// from F, brought up to date by applying H_0^H, ..., H_{k-1}^H (the block
// reflectors of the panels before it) and factored; then block k of Q,
// H_0 H_1 ... H_k [0; I; 0], is formed from its identity columns by applying
// H_k, ..., H_0 and written out.  Both loops apply one panel's reflector to
// 16 columns held in registers, and each such step streams only that panel's
// explicit V (rows p_j .. m-1) from the workspace: HBM traffic per step is a
// read of V_j, where the right-looking form reads and writes the trailing
// matrix once per panel in both the factorisation and the Q accumulation.
// The next step's V is loaded while the current step runs.
//
// Rows are dealt to the waves in 16-row blocks, block beta to wave beta mod NW,
// so the rows below a panel top stay spread over every wave.  Each wave keeps
// V_j of its blocks in registers in the layout of the W = V^H a product and a
// transposed copy in its own LDS area for E = V W2 (the panel area of the
// factorisation, which is idle while the steps run).

// Raw buffer accesses: an offset at or past the end of the range reads zero
// and writes nothing, so guarded loads need no branches (which would make the
// compiler wait for every load in flight before using any of them).
typedef unsigned int qrl_u2 __attribute__((ext_vector_type(2)));
typedef unsigned int qrl_u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t qrl_rsrc(const void* p, long long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}
// Byte offset = voff + soff; callers keep soff = 0 so that the whole offset
// takes part in the bounds check, and a lane that must not access memory
// passes voff = the range size.
__device__ __forceinline__ double2 qrl_load(__amdgpu_buffer_rsrc_t r, int voff, int soff,
                                            const double2*) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
__device__ __forceinline__ double2 qrl_load(__amdgpu_buffer_rsrc_t r, int voff, int soff,
                                            const float2*) {
  const float2 f =
      __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  return make_double2(f.x, f.y);
}
__device__ __forceinline__ void qrl_store(__amdgpu_buffer_rsrc_t r, int voff, int soff, double2 v,
                                          double2*) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(qrl_u4, v), r, voff, soff, 0);
}
__device__ __forceinline__ void qrl_store(__amdgpu_buffer_rsrc_t r, int voff, int soff, double2 v,
                                          float2*) {
  const float2 f = make_float2((float)v.x, (float)v.y);
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(qrl_u2, f), r, voff, soff, 0);
}

// One step on the 16 columns in a: FACT: a <- H_j^H a (X = T^H), otherwise
// a <- H_j a (X = T), H_j = I - V_j T_j V_j^H.  On entry v holds V_j; on exit it
// holds V_jn (zero if jn < 0).  In FACT mode block j of a is not updated:
// after this step those rows only hold R, which is not wanted.  The waves'
// parts of W = V_j^H a are summed in two stages: wave w adds up entries
// [w E, (w + 1) E) of all parts (E = 256 / NW) and leaves the sums in place
// in its own part, from where every wave then reads its entries.
template <int NTQ, bool FACT>
__device__ __forceinline__ void qrl_step(double2 (&a)[QrShape<NTQ>::QLB][4],
                                         double2 (&v)[QrShape<NTQ>::QLB][4],
                                         __amdgpu_buffer_rsrc_t rV,
                                         const double2* __restrict__ Tg, int m, int n, int j,
                                         int jn, bool first, double2* VT, double2* Wp) {
  constexpr int NW = QrShape<NTQ>::NW, MAXB = QrShape<NTQ>::QLB, EPW = 256 / NW;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  // X of this step (needed after the W sum)
  double2 xv[4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
    xv[t] = FACT ? cconj(Tg[(long long)j * 256 + (4 * t + lk) * 16 + li])
                 : Tg[(long long)j * 256 + li * 16 + 4 * t + lk];
  // this wave's part of W = V_j^H a (first step of a Q block: a = [0; I; 0]
  // is zero outside block j)
  CAcc3 w;
  w.zero();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int beta = wave + NW * b;
    if (beta >= j && 16 * beta < m && (!first || beta == j)) {
#pragma unroll
      for (int t = 0; t < 4; ++t) w.add(v[b][t].x, -v[b][t].y, a[b][t].x, a[b][t].y);
    }
  }
  __syncthreads();   // every wave has read the sums of the previous step
  double2* Wq = Wp + wave * 256;
#pragma unroll
  for (int r = 0; r < 4; ++r) Wq[(lk + 4 * r) * 16 + li] = make_double2(w.re(r), w.im(r));
  double2* Vt = VT + wave * (MAXB * 256);
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int beta = wave + NW * b;
    if (beta >= j && 16 * beta < m) {
#pragma unroll
      for (int t = 0; t < 4; ++t) Vt[b * 256 + pidx(4 * t + lk, li)] = v[b][t];
    }
  }
  {   // V of the next step, in flight during the rest of this one; rows at
      // or past m fall outside the range and read zero
    const int oob = m * n * 16, loff = (lk * n + li) * 16;
    const bool cok = jn >= 0 && 16 * jn + li < n;
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int beta = wave + NW * b;
      const bool bact = beta >= jn && 16 * beta < m;   // uniform
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r0 = 16 * beta + 4 * t;
        // branch-free select of the offset (branches around the loads would
        // make the compiler wait for all of them before the W sum)
        const int msk = -(int)(bact && cok);
        v[b][t] = qrl_load(rV, oob + ((loff + (r0 * n + 16 * jn) * 16 - oob) & msk), 0,
                           (const double2*)nullptr);
      }
    }
  }
  __syncthreads();
  if constexpr (EPW <= 64) {
    if (lane < EPW) {
      const int e = wave * EPW + lane;
      double2 x[NW];
#pragma unroll
      for (int u = 0; u < NW; ++u) x[u] = Wp[u * 256 + e];
      double2 sum = x[0];
#pragma unroll
      for (int u = 1; u < NW; ++u) {
        sum.x += x[u].x;
        sum.y += x[u].y;
      }
      Wp[wave * 256 + e] = sum;
    }
  } else {   // fewer than 4 waves: each wave sums EPW / 64 entries per lane
#pragma unroll
    for (int e0 = 0; e0 < EPW; e0 += 64) {
      const int e = wave * EPW + e0 + lane;
      double2 x[NW];
#pragma unroll
      for (int u = 0; u < NW; ++u) x[u] = Wp[u * 256 + e];
      double2 sum = x[0];
#pragma unroll
      for (int u = 1; u < NW; ++u) {
        sum.x += x[u].x;
        sum.y += x[u].y;
      }
      Wp[wave * 256 + e] = sum;
    }
  }
  __syncthreads();
  double wr[4], wi[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = (lk + 4 * r) * 16 + li;
    const double2 x = Wp[(e / EPW) * 256 + e];
    wr[r] = x.x;
    wi[r] = x.y;
  }
  CAcc3 x2;   // W2 = X W
  x2.zero();
#pragma unroll
  for (int t = 0; t < 4; ++t) x2.add(xv[t].x, xv[t].y, wr[t], wi[t]);
  double x2r[4], x2i[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    x2r[t] = x2.re(t);
    x2i[t] = x2.im(t);
  }
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int beta = wave + NW * b;
    if (beta >= j + (FACT ? 1 : 0) && 16 * beta < m) {
      CAcc3 e;   // rows of this block of V_j W2
      e.zero();
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double2 vt = Vt[b * 256 + pidx(li, 4 * t + lk)];   // V_j[16 beta + li][4t + lk]
        e.add(vt.x, vt.y, x2r[t], x2i[t]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        a[b][r] = make_double2(a[b][r].x - e.re(r), a[b][r].y - e.im(r));
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int CTI, int CTO, int NTQ>
__global__ __launch_bounds__(NTQ, NTQ == 512 ? 1 : 2) void qr_left_kernel(const QrArgs args, int part) {
  using Shape = QrShape<NTQ>;
  constexpr int NW = Shape::NW, MAXB = Shape::QLB;
  using TI = typename St<CTI>::T;
  using TO = typename St<CTO>::T;
  extern __shared__ __attribute__((aligned(16))) double2 dyn[];
  PanelSmem2<NW, QB>& psm = *reinterpret_cast<PanelSmem2<NW, QB>*>(dyn);
  double* s_red = reinterpret_cast<double*>(dyn);
  double2* P = dyn;   // panel rows to factor, or the waves' V_j^T areas
  double2* Wp = dyn + Shape::P_BYTES / sizeof(double2);
  double2* sT = Wp;   // while a panel is factored

  const int gi = find_group<QR_MAX_GROUPS>(args.g, args.ngroups, blockIdx.x);
  const QrGroup& G = args.g[gi];
  // part 0: whole QR; part 1: factorisation only (V, T to the workspace);
  // part 2: one block of Q per workgroup from the stored V, T
  const int npan = (G.n + QB - 1) / QB;
  const int local = blockIdx.x - G.blk_begin;
  const int item = part == 2 ? local / npan : local;
  const int m = G.m, n = G.n, mode = G.mode;
  const TI* __restrict__ F = reinterpret_cast<const TI*>(item_ptr(G.f, G.ids, item));
  TO* __restrict__ Q = reinterpret_cast<TO*>(const_cast<char*>(item_ptr(G.q, G.ids, item)));
  double* nrm = reinterpret_cast<double*>(const_cast<char*>(item_ptr(G.nrm2, G.ids, item)));
  double2* Vw = reinterpret_cast<double2*>(const_cast<char*>(item_ptr(G.ws, G.ids, item)));
  double2* Tg = Vw + (long long)m * n;   // T factor of every panel
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform block ownership
  const int li = lane & 15, lk = lane >> 4;
  const double2 zero = make_double2(0.0, 0.0);
  const long long mn = (long long)m * n;

  if (part == 2) {   // block kq of Q: H_0 ... H_kq applied to its identity columns
    const int k = local - item * npan, p = k * QB, nbk = min(QB, n - p);
    const __amdgpu_buffer_rsrc_t rQ = qrl_rsrc(Q, mn * (long long)sizeof(TO));
    const __amdgpu_buffer_rsrc_t rV = qrl_rsrc(Vw, mn * 16);
    const int oobQ = (int)(mn * sizeof(TO)), oobV = (int)(mn * 16);
    const int loffQ = (mode == 0 ? lk * n + li : li * m + lk) * (int)sizeof(TO);
    const int loffV = (lk * n + li) * 16;
    double2 a[MAXB][4], v[MAXB][4];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int beta = wave + NW * b;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r0 = 16 * beta + 4 * t;
        a[b][t] = make_double2(r0 + lk == p + li && li < nbk ? 1.0 : 0.0, 0.0);
        const int msk = -(int)(beta >= k && 16 * beta < m && li < nbk);   // rows past m: out of range
        v[b][t] = qrl_load(rV, oobV + ((loffV + (r0 * n + p) * 16 - oobV) & msk), 0,
                           (const double2*)nullptr);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
#pragma unroll 1
    for (int j = k; j >= 0; --j) qrl_step<NTQ, false>(a, v, rV, Tg, m, n, j, j - 1, j == k, P, Wp);
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int beta = wave + NW * b;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r0 = 16 * beta + 4 * t;
        const bool in = lk < m - r0 && li < nbk;
        const int sQ = (mode == 0 ? r0 * n + p : p * m + r0) * (int)sizeof(TO);
        const double2 o = make_double2(a[b][t].x, mode == 0 ? a[b][t].y : -a[b][t].y);
        qrl_store(rQ, in ? loffQ + sQ : oobQ, 0, o, (TO*)nullptr);
      }
    }
    return;
  }

  if (mode == 2) {   // T = F / |F|
    double part = 0;
    for (long long idx = tid; idx < mn; idx += NTQ) {
      const double2 u = to_d2(F[idx]);
      part += u.x * u.x + u.y * u.y;
    }
    double nu2 = part, nu_mx = 0.0;
    block_sum_max<NW>(nu2, nu_mx, s_red);
    if (tid == 0) *nrm = nu2;
    const double sc = nu2 > 0 ? 1.0 / sqrt(nu2) : 0.0;
    for (long long idx = tid; idx < mn; idx += NTQ) {
      const double2 u = to_d2(F[idx]);
      TO o;
      o.x = u.x * sc;
      o.y = u.y * sc;
      Q[idx] = o;
    }
    return;
  }

  const __amdgpu_buffer_rsrc_t rF = qrl_rsrc(F, mn * (long long)sizeof(TI));
  const __amdgpu_buffer_rsrc_t rQ = qrl_rsrc(Q, mn * (long long)sizeof(TO));
  const __amdgpu_buffer_rsrc_t rV = qrl_rsrc(Vw, mn * 16);
  const int oobF = (int)(mn * sizeof(TI)), oobQ = (int)(mn * sizeof(TO)), oobV = (int)(mn * 16);
  double nsq = 0;   // |F|^2, each entry is read once
  double2 a[MAXB][4], v[MAXB][4];
#pragma unroll 1
  for (int k = 0; k < npan; ++k) {
    const int p = k * QB, nbk = min(QB, n - p), mp = m - p;
    // lane-dependent offsets are formed anew for each panel (the empty asm
    // keeps them from being hoisted and held across the loop)
    int tl = threadIdx.x;
    asm volatile("" : "+v"(tl));
    const int li = tl & 15, lk = (tl & 63) >> 4;
    const int loffV = (lk * n + li) * 16;
    // per-lane parts of the byte offsets of row r0 + lk, column c0 + li (r0, c0 uniform)
    const int loffF = (mode == 0 ? lk * n + li : li * m + lk) * (int)sizeof(TI);
    const int loffQ = (mode == 0 ? lk * n + li : li * m + lk) * (int)sizeof(TO);
    // columns p .. p+15 of A (= F, or F^H in mode 1), and V_0
    // (for k > 0 in the whole QR, v holds V_0 here, loaded by the last step
    // of the previous Q block)
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int beta = wave + NW * b;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r0 = 16 * beta + 4 * t;
        const bool in = lk < m - r0 && li < nbk;
        const int sF = (mode == 0 ? r0 * n + p : p * m + r0) * (int)sizeof(TI);
        double2 u = qrl_load(rF, in ? loffF + sF : oobF, 0, (const TI*)nullptr);
        if (mode != 0) u.y = -u.y;
        nsq += u.x * u.x + u.y * u.y;
        a[b][t] = u;
        if (part == 1 && k > 0) {   // V_0 (rows past m: out of range)
          const int msk = -(int)(16 * beta < m && li < n);
          v[b][t] = qrl_load(rV, oobV + ((loffV + r0 * n * 16 - oobV) & msk), 0,
                             (const double2*)nullptr);
        }
      }
    }
#pragma unroll 1
    for (int j = 0; j < k; ++j)
      qrl_step<NTQ, true>(a, v, rV, Tg, m, n, j, j + 1 < k ? j + 1 : -1, false, P, Wp);

    // factor the panel: by Cholesky QR and Householder reconstruction where
    // the panel allows it, else column by column (rows p.. to LDS, one row
    // per thread)
    __syncthreads();
    bool chol = false;
    if (mp > nbk) {
      chol = panel_cholqr<NW, MAXB>(a, m, k, mp, nbk, P, Wp);
    } else {
#pragma unroll
      for (int b = 0; b < MAXB; ++b) {
        const int beta = wave + NW * b;
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
      factor_panel2<1, QB, NTQ>(ar, mp, nbk, psm, sT);
      // explicit V_k (rows p.., zero past m) to LDS
      if (tid < Shape::PROWS) {
#pragma unroll
        for (int c = 0; c < QB; ++c) {
          const bool in = tid < mp && c < nbk;
          P[pidx(tid, c)] = !in ? zero : (tid > c ? ar[0][c] : make_double2(tid == c ? 1.0 : 0.0, 0.0));
        }
      }
    }
    __syncthreads();
    // V_k and T_k to the workspace
    if (tid < mp) {
#pragma unroll
      for (int c = 0; c < QB; ++c)
        if (c < nbk) Vw[(long long)(p + tid) * n + p + c] = P[pidx(tid, c)];
    }
    if constexpr (NTQ >= QB * QB) {
      if (tid < QB * QB) Tg[(long long)k * QB * QB + tid] = sT[tid];
    } else {
      for (int e = tid; e < QB * QB; e += NTQ) Tg[(long long)k * QB * QB + e] = sT[e];
    }
    __threadfence_block();
    __syncthreads();
    if (part == 1) continue;

    // block k of Q
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int beta = wave + NW * b;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int row = 16 * beta + 4 * t + lk;
        a[b][t] = make_double2(row == p + li && li < nbk ? 1.0 : 0.0, 0.0);
        v[b][t] = beta >= k && 16 * beta < m ? P[pidx(16 * (beta - k) + 4 * t + lk, li)] : zero;
      }
    }
    // nothing in flight on entry to the loop, so the compiler can count the
    // loads of each step exactly (the last step loads V_0 for the next
    // panel's updates)
    __builtin_amdgcn_s_waitcnt(0);
#pragma unroll 1
    for (int j = k; j >= 0; --j)
      qrl_step<NTQ, false>(a, v, rV, Tg, m, n, j, j > 0 ? j - 1 : (k + 1 < npan ? 0 : -1), j == k,
                           P, Wp);
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int beta = wave + NW * b;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r0 = 16 * beta + 4 * t;
        const bool in = lk < m - r0 && li < nbk;
        const int sQ = (mode == 0 ? r0 * n + p : p * m + r0) * (int)sizeof(TO);
        const double2 o = make_double2(a[b][t].x, mode == 0 ? a[b][t].y : -a[b][t].y);
        qrl_store(rQ, in ? loffQ + sQ : oobQ, 0, o, (TO*)nullptr);
      }
    }
  }
  double nu2 = nsq, nu_mx = 0.0;
  block_sum_max<NW>(nu2, nu_mx, s_red);
  if (tid == 0) *nrm = nu2;
}

// ---------------------------------------------------------------------------
// Outcome norms n_m = Re sum conj(A[a][m][b]) Z[a][m][b], FP64 accumulation.

template <int CTA, int CTZ>
__global__ __launch_bounds__(NT) void norms_kernel(const NormArgs args) {
  using TA = typename St<CTA>::T;
  using TZ = typename St<CTZ>::T;
  __shared__ double s_red[4];
  const int gi = find_group<NORM_MAX_GROUPS>(args.g, args.ngroups, blockIdx.x);
  const NormGroup& G = args.g[gi];
  const int item = blockIdx.x - G.blk_begin;
  const TA* __restrict__ A = reinterpret_cast<const TA*>(item_ptr(G.a, G.ids, item));
  const TZ* __restrict__ Z = G.z.base ? reinterpret_cast<const TZ*>(item_ptr(G.z, G.ids, item))
                                      : reinterpret_cast<const TZ*>(A);
  double* out = reinterpret_cast<double*>(const_cast<char*>(item_ptr(G.out, G.ids, item)));
  const int dl = G.dl, dr = G.dr;
  const long long tot = (long long)dl * 2 * dr;
  double p0 = 0, p1 = 0;
  for (long long idx = threadIdx.x; idx < tot; idx += NT) {
    const double2 a = to_d2(A[idx]);
    const double2 z = to_d2(Z[idx]);
    const double v = a.x * z.x + a.y * z.y;
    const int s = (int)((idx / dr) & 1);
    if (s == 0)
      p0 += v;
    else
      p1 += v;
  }
  p0 = block_sum(p0, s_red);
  p1 = block_sum(p1, s_red);
  if (threadIdx.x == 0) {
    out[0] = p0;
    out[1] = p1;
  }
}

// ---------------------------------------------------------------------------

template <int CT>
__global__ __launch_bounds__(NT) void collapse_kernel(const CollapseItem* items) {
  using T = typename St<CT>::T;
  const CollapseItem it = items[blockIdx.y];
  const long long idx = (long long)blockIdx.x * NT + threadIdx.x;
  const long long tot = (long long)it.dl * it.dr;
  if (idx >= tot) return;
  const int a = (int)(idx / it.dr), b = (int)(idx % it.dr);
  T* A = reinterpret_cast<T*>(it.a);
  const double sc = it.scale;
  T& keep = A[((long long)a * 2 + it.m) * it.dr + b];
  T& drop = A[((long long)a * 2 + (1 - it.m)) * it.dr + b];
  T k = keep;
  k.x = (double)k.x * sc;
  k.y = (double)k.y * sc;
  keep = k;
  T z;
  z.x = 0;
  z.y = 0;
  drop = z;
}

// Sampling and collapse on the device: every block derives the outcome from
// the same FP64 norms and uniform, so all blocks of an item agree.
template <int CT>
__global__ __launch_bounds__(NT) void sample_collapse_kernel(const SampleItem* items,
                                                             const double* norms, const double* u,
                                                             double eps, int* outcome, double* pm) {
  using T = typename St<CT>::T;
  const SampleItem it = items[blockIdx.y];
  const double n0 = norms[2 * it.k], n1 = norms[2 * it.k + 1];
  const double tot = n0 + n1;
  const bool ok = tot > 0.0 && isfinite(tot);
  int m = (ok && u[it.idx] >= n0 / tot) ? 1 : 0;
  if (ok && !((m ? n1 : n0) / tot > eps)) m = 1 - m;
  const double nm = m ? n1 : n0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    outcome[it.idx] = ok ? m : -1;
    pm[it.idx] = ok ? nm / tot : __builtin_nan("");
  }
  if (!ok) return;
  const long long idx = (long long)blockIdx.x * NT + threadIdx.x;
  const long long total = (long long)it.dl * it.dr;
  if (idx >= total) return;
  const int a = (int)(idx / it.dr), b = (int)(idx % it.dr);
  T* A = reinterpret_cast<T*>(it.a);
  const double sc = 1.0 / sqrt(nm);
  T& keep = A[((long long)a * 2 + m) * it.dr + b];
  T& drop = A[((long long)a * 2 + (1 - m)) * it.dr + b];
  T k = keep;
  k.x = (double)k.x * sc;
  k.y = (double)k.y * sc;
  keep = k;
  T z;
  z.x = 0;
  z.y = 0;
  drop = z;
}

// Writes the complex pair (1, 0) at each listed address: the 1 x 2 x 1 site
// tensor of |0>, or a 1 x 1 x 1 boundary environment (its second word is
// alignment padding).
template <int CT>
__global__ void fill_unit_kernel(void* const* ptrs, int n) {
  using T = typename St<CT>::T;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T one, zero;
  one.x = 1;
  one.y = 0;
  zero.x = 0;
  zero.y = 0;
  T* p = reinterpret_cast<T*>(ptrs[i]);
  p[0] = one;
  p[1] = zero;
}

}  // namespace

hipError_t launch_mpo(int ct, int dir, const MpoArgs& args, hipStream_t s) {
  if (args.total_blocks <= 0) return hipSuccess;
  int wmax = 1;
  for (int i = 0; i < args.ngroups; ++i) wmax = max(wmax, max(args.g[i].wl, args.g[i].wr));
  const dim3 grid(args.total_blocks), blk(NT);
#define DCS_MPO(CT, DIR, WM)                                                      \
  if (ct == CT && dir == DIR && wmax <= WM) {                                     \
    if (DIR == 0)                                                                 \
      hipLaunchKernelGGL((mpo_right_kernel<CT, WM>), grid, blk, 0, s, args);      \
    else                                                                          \
      hipLaunchKernelGGL((mpo_left_kernel<CT, WM>), grid, blk, 0, s, args);       \
    return hipGetLastError();                                                     \
  }
  DCS_MPO(CT_F32, 0, 4)
  DCS_MPO(CT_F32, 0, 16)
  DCS_MPO(CT_F32, 1, 4)
  DCS_MPO(CT_F32, 1, 16)
  DCS_MPO(CT_F64, 0, 4)
  DCS_MPO(CT_F64, 0, 16)
  DCS_MPO(CT_F64, 1, 4)
  DCS_MPO(CT_F64, 1, 16)
#undef DCS_MPO
  return hipErrorInvalidValue;
}

size_t qr_lds_limit() {
  // dynamic LDS for the working matrix next to the static arrays (16.1 KB),
  // within the 64 KB a workgroup gets without an opt-in
  return 64 * 1024 - 17 * 1024;
}

size_t qr_blocked_lds(int m) {
  return m <= 128 ? QrShape<256>::LDS_BYTES : QrShape<512>::LDS_BYTES;
}
int qr_blocked_max_rows() { return 512; }
// about 5/8 of the MI355X's 256 CUs
int qr_split_max_items() { return 160; }

hipError_t launch_qr_blocked(int ct_in, int ct_out, const QrArgs& args, int m_max, hipStream_t s) {
  if (args.total_blocks <= 0) return hipSuccess;
  const size_t lds = qr_blocked_lds(m_max);
  const bool small = m_max <= 128;
  const dim3 grid(args.total_blocks), blk(small ? 256 : 512);
#define DCS_QRB(I, O, T)                                                                    \
  if (ct_in == I && ct_out == O && (T == 256) == small) {                                  \
    static hipError_t attr = hipFuncSetAttribute(                                          \
        reinterpret_cast<const void*>(&qr_blocked_kernel<I, O, T>),                         \
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)qr_blocked_lds(512));              \
    if (lds > 48 * 1024 && attr != hipSuccess) return attr;                                 \
    hipLaunchKernelGGL((qr_blocked_kernel<I, O, T>), grid, blk, lds, s, args);              \
    return hipGetLastError();                                                               \
  }
  DCS_QRB(CT_F32, CT_F32, 512)
  DCS_QRB(CT_F64, CT_F64, 512)
  DCS_QRB(CT_F64, CT_F32, 512)
  DCS_QRB(CT_F32, CT_F32, 256)
  DCS_QRB(CT_F64, CT_F64, 256)
  DCS_QRB(CT_F64, CT_F32, 256)
#undef DCS_QRB
  return hipErrorInvalidValue;
}

namespace {
hipError_t launch_left(int ct_in, int ct_out, const QrArgs& args, int m_max, bool split,
                       bool qblocks_only, hipStream_t s, int threads) {
  if (args.total_blocks <= 0) return hipSuccess;
  // up to 128 rows: four waves per matrix (two matrices per CU), or, when
  // there are more matrices than that fits on the chip at once, two waves
  // per matrix so that four matrices (40 KB of LDS each) share a CU; the
  // per-column latency of the factorisation, not the arithmetic, bounds
  // these small QRs
  const int ntq = m_max > 128 ? 512
                  : (threads == 128 || threads == 256) ? threads
                  : (args.total_blocks > 2 * 256 ? 128 : 256);
  const size_t lds = ntq == 512 ? QrShape<512>::LDS_BYTES
                                : ntq == 256 ? QrShape<256>::LDS_BYTES : QrShape<128>::LDS_BYTES;
  const dim3 blk(ntq);
  // split: the factorisations first (one workgroup per matrix), then every
  // 16-column block of every Q in its own workgroup
  QrArgs qa;
  std::memset(&qa, 0, sizeof(qa));
  if (split) {
    for (int g = 0; g < args.ngroups; ++g) {
      if (args.g[g].mode == 2) continue;
      QrGroup& d = qa.g[qa.ngroups++];
      d = args.g[g];
      d.blk_begin = qa.total_blocks;
      qa.total_blocks += d.batch * ((d.n + QB - 1) / QB);
    }
  }
#define DCS_QRL(I, O, T)                                                                    \
  if (ct_in == I && ct_out == O && T == ntq) {                                             \
    static hipError_t attr = hipFuncSetAttribute(                                          \
        reinterpret_cast<const void*>(&qr_left_kernel<I, O, T>),                            \
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)QrShape<T>::LDS_BYTES);            \
    if (lds > 48 * 1024 && attr != hipSuccess) return attr;                                 \
    if (!qblocks_only)                                                                      \
      hipLaunchKernelGGL((qr_left_kernel<I, O, T>), dim3(args.total_blocks), blk, lds, s,   \
                         args, split ? 1 : 0);                                              \
    if (split && qa.total_blocks > 0)                                                       \
      hipLaunchKernelGGL((qr_left_kernel<I, O, T>), dim3(qa.total_blocks), blk, lds, s, qa, 2); \
    return hipGetLastError();                                                               \
  }
  DCS_QRL(CT_F32, CT_F32, 512)
  DCS_QRL(CT_F64, CT_F64, 512)
  DCS_QRL(CT_F64, CT_F32, 512)
  DCS_QRL(CT_F32, CT_F32, 256)
  DCS_QRL(CT_F64, CT_F64, 256)
  DCS_QRL(CT_F64, CT_F32, 256)
  DCS_QRL(CT_F32, CT_F32, 128)
  DCS_QRL(CT_F64, CT_F64, 128)
  DCS_QRL(CT_F64, CT_F32, 128)
#undef DCS_QRL
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_qr_left(int ct_in, int ct_out, const QrArgs& args, int m_max, bool split,
                          hipStream_t s, int threads) {
  return launch_left(ct_in, ct_out, args, m_max, split, false, s, threads);
}

hipError_t launch_qr_qblocks(int ct_in, int ct_out, const QrArgs& args, int m_max, hipStream_t s) {
  QrArgs a = args;
  int blocks = 0;
  for (int g = 0; g < a.ngroups; ++g) {
    a.g[g].blk_begin = blocks;
    blocks += a.g[g].batch;
  }
  a.total_blocks = blocks;
  a.use_lds = 1;
  return launch_left(ct_in, ct_out, a, m_max, true, true, s, 0);
}

hipError_t launch_qr(int ct_in, int ct_out, const QrArgs& args, size_t lds_bytes, hipStream_t s) {
  if (args.total_blocks <= 0) return hipSuccess;
  if (!args.use_lds) lds_bytes = 0;
  const dim3 grid(args.total_blocks), blk(NT);
#define DCS_QR(I, O)                                                                        \
  if (ct_in == I && ct_out == O) {                                                          \
    static hipError_t attr = hipFuncSetAttribute(                                          \
        reinterpret_cast<const void*>(&qr_kernel<I, O>),                                    \
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)qr_lds_limit());                   \
    if (lds_bytes > 0 && attr != hipSuccess) return attr;                                   \
    hipLaunchKernelGGL((qr_kernel<I, O>), grid, blk, lds_bytes, s, args);                   \
    return hipGetLastError();                                                               \
  }
  DCS_QR(CT_F32, CT_F32)
  DCS_QR(CT_F64, CT_F64)
  DCS_QR(CT_F64, CT_F32)
#undef DCS_QR
  return hipErrorInvalidValue;
}

hipError_t launch_norms(int ct_a, int ct_z, const NormArgs& args, hipStream_t s) {
  if (args.total_blocks <= 0) return hipSuccess;
  const dim3 grid(args.total_blocks), blk(NT);
  if (ct_a == CT_F32 && ct_z == CT_F32)
    hipLaunchKernelGGL((norms_kernel<CT_F32, CT_F32>), grid, blk, 0, s, args);
  else if (ct_a == CT_F32 && ct_z == CT_F64)
    hipLaunchKernelGGL((norms_kernel<CT_F32, CT_F64>), grid, blk, 0, s, args);
  else if (ct_a == CT_F64 && ct_z == CT_F64)
    hipLaunchKernelGGL((norms_kernel<CT_F64, CT_F64>), grid, blk, 0, s, args);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_collapse(int ct, const CollapseItem* items_dev, int n_items, int max_elems,
                           hipStream_t s) {
  if (n_items <= 0 || max_elems <= 0) return hipSuccess;
  const dim3 grid((max_elems + NT - 1) / NT, n_items), blk(NT);
  if (ct == CT_F32)
    hipLaunchKernelGGL((collapse_kernel<CT_F32>), grid, blk, 0, s, items_dev);
  else
    hipLaunchKernelGGL((collapse_kernel<CT_F64>), grid, blk, 0, s, items_dev);
  return hipGetLastError();
}

hipError_t launch_sample_collapse(int ct, const SampleItem* items_dev, int n_items, int max_elems,
                                  const double* norms, const double* u, double eps, int* outcome,
                                  double* pm, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const dim3 grid((max(max_elems, 1) + NT - 1) / NT, n_items), blk(NT);
  if (ct == CT_F32)
    hipLaunchKernelGGL((sample_collapse_kernel<CT_F32>), grid, blk, 0, s, items_dev, norms, u, eps,
                       outcome, pm);
  else
    hipLaunchKernelGGL((sample_collapse_kernel<CT_F64>), grid, blk, 0, s, items_dev, norms, u, eps,
                       outcome, pm);
  return hipGetLastError();
}

hipError_t launch_fill_unit(int ct, void* const* ptrs_dev, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((n + 127) / 128), blk(128);
  if (ct == CT_F32)
    hipLaunchKernelGGL((fill_unit_kernel<CT_F32>), grid, blk, 0, s, ptrs_dev, n);
  else
    hipLaunchKernelGGL((fill_unit_kernel<CT_F64>), grid, blk, 0, s, ptrs_dev, n);
  return hipGetLastError();
}

}  // namespace dcs
