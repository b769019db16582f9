// Householder factorisation of one QR panel held in registers, shared by the
// blocked (m <= 512) and the large-matrix QR kernels.
//
// Thread tid of an NT-thread workgroup holds panel rows tid + r NT (r < RP),
// columns 0..NB-1, in a[r][.].  Reflectors follow LAPACK (zlarfg): v_k = 1,
// beta = -sign(Re alpha) |(alpha, x)|, tau = ((beta - Re alpha) / beta,
// -Im alpha / beta), v = x / (alpha - beta), tau = 0 when x = 0 and alpha is
// real or the column norm is below 1e-280 (then v = e_k exactly).  Column kk
// takes one reduction round over the workgroup: with x the entries below the
// diagonal and v = [1; scal x],
//   |x|^2, max|x|,  p_c = x^H a_c (c > kk),  q_c = v_c^H x (c < kk)
// are reduced together (DPP within lane quads, quad partials through LDS, a
// group of lanes per value, DPP again); then one wave forms the reflector,
// v^H a_c = a[kk][c] + conj(scal) p_c, the Gram entry
// v_c^H v = conj(v_c[kk]) + scal q_c of the zlarft recurrence
// T[j][kk] = -tau_kk T[j][j:kk] G[j:kk][kk], T[kk][kk] = tau_kk, and the
// update coefficients, which every thread then applies to its rows.  Squares
// are summed directly unless max|x| leaves [1e-140, 1e140], where a scaled
// second pass keeps them representable.
#pragma once

#include "kernel_util.h"

namespace dcs {
namespace {

template <int NW, int NB>
struct PanelSmem {
  double q[2 * NB][NW * 16];   // quad partials per reduced value
  double fin[2 * NB];          // reduced values
  double mx[NW];
  double red[2 * NW];
  double2 row[NB];             // row kk of the panel
  double2 cc[NB];              // conj(tau) v^H a_c of the columns c > kk
  double2 scal;                // v = [1; scal x]
};

// On return a holds R on and above the diagonal (the diagonal entry itself is
// not needed and left as is) and v below it; sT (NB x NB, row-major, LDS)
// holds T.  Every thread of the workgroup must call it; ends with a barrier.
template <int RP, int NB, int NT>
__device__ __forceinline__ void factor_panel(double2 (&a)[RP][NB], int mp, int nbk,
                                             PanelSmem<NT / 64, NB>& sm, double2* sT) {
  constexpr int NW = NT / 64;
  constexpr int NV = 2 * NB;                       // |x|^2 + NB-1 complex values + spare
  constexpr int NQ = NW * 16;
  constexpr int LPV = (NT / NV) >= 16 ? 16 : 8;    // lanes per value in stage 2
  static_assert(NV * LPV <= NT, "stage 2 needs LPV lanes per reduced value");
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (tid < NB * NB) sT[tid] = make_double2(0.0, 0.0);

  static_for<NB>([&](auto kc) {
    constexpr int kk = decltype(kc)::value;
    if (kk >= nbk) return;   // uniform over the workgroup
    // reduced values: slots 2j, 2j+1 = value j (j < NB-1: column c = j for
    // c < kk, c = j + 1 for c > kk), slot 2NB-2 = |x|^2; partial sums built
    // and quad-reduced in chunks of NVC slots to bound register use
    constexpr int NVC = NV < 16 ? NV : 16;
    double mx = 0.0;
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int i = tid + r * NT;
      if (i > kk && i < mp) {
        const double2 xi = a[r][kk];
        mx = fmax(mx, fmax(fabs(xi.x), fabs(xi.y)));
      }
    }
    mx = wave_max_dpp(mx);
    __syncthreads();   // readers of the previous round are done
    if (tid == kk) {   // row kk: alpha, R entries (c > kk) and v_c[kk] (c < kk)
#pragma unroll
      for (int c = 0; c < NB; ++c) sm.row[c] = a[0][c];
    }
#pragma unroll
    for (int q0 = 0; q0 < NV; q0 += NVC) {
      double x[NVC];
#pragma unroll
      for (int q = 0; q < NVC; ++q) x[q] = 0.0;
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        const int i = tid + r * NT;
        if (i > kk && i < mp) {
          const double2 xi = a[r][kk];
#pragma unroll
          for (int c = 0; c < NB; ++c) {
            if (c == kk) continue;
            const int j = c < kk ? c : c - 1;
            if (2 * j < q0 || 2 * j >= q0 + NVC) continue;
            // c > kk: p_c = x^H a_c; c < kk: q_c = v_c^H x (a holds v_c)
            const double2 w = (c > kk) ? cdotc(xi, a[r][c]) : cdotc(a[r][c], xi);
            x[2 * j - q0] += w.x;
            x[2 * j + 1 - q0] += w.y;
          }
          if (2 * NB - 2 >= q0 && 2 * NB - 2 < q0 + NVC) x[2 * NB - 2 - q0] += xi.x * xi.x + xi.y * xi.y;
        }
      }
#pragma unroll
      for (int q = 0; q < NVC; ++q) x[q] += dpp_d<0xB1>(x[q]);
#pragma unroll
      for (int q = 0; q < NVC; ++q) x[q] += dpp_d<0x4E>(x[q]);
      if ((lane & 3) == 0) {
#pragma unroll
        for (int q = 0; q < NVC; ++q)
          if (q0 + q < NV) sm.q[q0 + q][wave * 16 + (lane >> 2)] = x[q];
      }
    }
    if (lane == 0) sm.mx[wave] = mx;
    __syncthreads();
    if (tid < NV * LPV) {
      const int q = tid / LPV, sub = tid % LPV;
      double v = 0.0;
#pragma unroll
      for (int u = 0; u < NQ / LPV; ++u) v += sm.q[q][sub * (NQ / LPV) + u];
      v += dpp_d<0xB1>(v);
      v += dpp_d<0x4E>(v);
      v += dpp_d<0x141>(v);
      if (LPV == 16) v += dpp_d<0x140>(v);
      if (sub == 0) sm.fin[q] = v;
    }
    __syncthreads();
    double mxa = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) mxa = fmax(mxa, sm.mx[w]);
    double sc = 0.0, qn = 0.0;
    if (mxa > 0.0 && (mxa < 1e-140 || mxa > 1e140)) {
      // squares leave the safe range: scaled second pass (rare, uniform)
      double sm2 = 0.0, dummy = 0.0;
      const double inv = 1.0 / mxa;
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        const int i = tid + r * NT;
        if (i > kk && i < mp) {
          const double2 v = a[r][kk];
          sm2 += (v.x * inv) * (v.x * inv) + (v.y * inv) * (v.y * inv);
        }
      }
      block_sum_max_dpp<NW>(sm2, dummy, sm.red);
      sc = mxa;
      qn = sm2;
    } else if (mxa > 0.0) {
      sc = 1.0;
      qn = sm.fin[2 * NB - 2];
    }
    // the reflector, the update coefficients and the T column: wave 0 only
    if (wave == 0) {
      const double2 alpha = sm.row[kk];
      double2 tau = make_double2(0.0, 0.0), scal = make_double2(0.0, 0.0);
      if (!(sc == 0.0 && alpha.y == 0.0)) {
        double sa = sc, qa = qn;
        ssq_add(sa, qa, alpha.x);
        ssq_add(sa, qa, alpha.y);
        const double nrm_all = sa * sqrt(qa);
        if (nrm_all > 1e-280) {
          const double beta = alpha.x >= 0.0 ? -nrm_all : nrm_all;
          tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
          scal = crecip(make_double2(alpha.x - beta, alpha.y));
        }
      }
      // v^H a_c (c > kk) and the Gram entry v_c^H v (c < kk)
      auto dval = [&](int c) {
        const int slot = 2 * (c < kk ? c : c - 1);
        const double2 pq = make_double2(sm.fin[slot], sm.fin[slot + 1]);
        const double2 rc = sm.row[c];
        if (c > kk) {
          const double2 u = cmul(cconj(scal), pq);
          return make_double2(rc.x + u.x, rc.y + u.y);
        }
        const double2 u = cmul(scal, pq);
        return make_double2(rc.x + u.x, -rc.y + u.y);
      };
      if (lane < NB && lane > kk && lane < nbk) sm.cc[lane] = cmul(cconj(tau), dval(lane));
      if (lane < kk) {   // T[j][kk] = -tau T[j][j:kk] G[j:kk][kk]
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          if (t >= lane && t < kk) {
            const double2 u = cmul(sT[lane * NB + t], dval(t));
            acc.x += u.x;
            acc.y += u.y;
          }
        }
        const double2 u = cmul(tau, acc);
        sT[lane * NB + kk] = make_double2(-u.x, -u.y);
      } else if (lane == kk) {
        sT[kk * NB + kk] = tau;
        sm.scal = scal;
      }
    }
    __syncthreads();
    const double2 scal = sm.scal;
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int i = tid + r * NT;
      if (i > kk && i < mp) a[r][kk] = cmul(a[r][kk], scal);
    }
    // a_c -= v conj(tau) (v^H a_c) for the remaining panel columns
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c > kk && c < nbk) {
        const double2 cc = sm.cc[c];
#pragma unroll
        for (int r = 0; r < RP; ++r) {
          const int i = tid + r * NT;
          if (i >= kk && i < mp) {
            const double2 v = (i == kk) ? make_double2(1.0, 0.0) : a[r][kk];
            const double2 u = cmul(v, cc);
            a[r][c] = make_double2(a[r][c].x - u.x, a[r][c].y - u.y);
          }
        }
      }
    }
  });
  __syncthreads();
}

}  // namespace
}  // namespace dcs
