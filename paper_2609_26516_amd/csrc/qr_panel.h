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

// Column kk's reflector from the reduced values fin (slots as in factor_panel)
// and the squared norm sc^2 qn of the entries below the diagonal: tau, the
// scaling of v, the update coefficients cc[c] = conj(tau) v^H a_c (c > kk) and
// column kk of T.  Executed by one wave; lane c handles column c.
template <int NB>
__device__ __forceinline__ void panel_reflector(int kk, int nbk, double sc, double qn,
                                                const double* fin, const double2* row,
                                                double2* cc_out, double2* scal_out,
                                                double2* sT) {
  const int lane = threadIdx.x & 63;
  const double2 alpha = row[kk];
  double2 tau = make_double2(0.0, 0.0), scal = make_double2(0.0, 0.0);
  const double amax = fmax(fabs(alpha.x), fabs(alpha.y));
  // every square representable (the sum of squares of x is in range or zero,
  // |alpha| is in range or zero): direct formulas, one square root and two
  // divisions; otherwise the scaled sums and Smith's reciprocal
  const bool direct = amax < 1e140 && (sc == 1.0 ? true : (sc == 0.0 && (amax == 0.0 || amax > 1e-140)));
  if (direct) {
    if (!(sc == 0.0 && alpha.y == 0.0)) {
      const double nrm_all = sqrt((sc == 1.0 ? qn : 0.0) + alpha.x * alpha.x + alpha.y * alpha.y);
      if (nrm_all > 1e-280) {
        const double beta = alpha.x >= 0.0 ? -nrm_all : nrm_all;
        const double rb = 1.0 / beta;
        tau = make_double2((beta - alpha.x) * rb, -alpha.y * rb);
        const double dx = alpha.x - beta, dy = alpha.y;
        const double id = 1.0 / (dx * dx + dy * dy);   // |alpha - beta| in [|beta|, 2 |beta|]
        scal = make_double2(dx * id, -dy * id);
      }
    }
  } else if (!(sc == 0.0 && alpha.y == 0.0)) {
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
    const double2 pq = make_double2(fin[slot], fin[slot + 1]);
    const double2 rc = row[c];
    if (c > kk) {
      const double2 u = cmul(cconj(scal), pq);
      return make_double2(rc.x + u.x, rc.y + u.y);
    }
    const double2 u = cmul(scal, pq);
    return make_double2(rc.x + u.x, -rc.y + u.y);
  };
  if (lane < NB && lane > kk && lane < nbk) cc_out[lane] = cmul(cconj(tau), dval(lane));
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
    *scal_out = scal;
  }
}

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
    if (wave == 0) panel_reflector<NB>(kk, nbk, sc, qn, sm.fin, sm.row, sm.cc, &sm.scal, sT);
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

// ---------------------------------------------------------------------------
// Variant with two workgroup barriers per column instead of four.  Each wave
// reduces its 32 partial values (the slots of factor_panel, padded to 32) with
// a halving exchange: at lane distances 32 and 16 the permlane swaps hand each
// half of the wave the other half's partials of the values it keeps, inside
// each row of 16 lanes DPP mirrors and a quad swap do the same, and a DPP
// step at distance 1 completes the wave sum of value s in lanes 2s and 2s + 1.  The waves' sums go to LDS, one
// barrier, wave 0 adds them up and forms the reflector, a second barrier, and
// every thread applies it.  The next column's LDS writes cannot disturb the
// readers of this one: those all read before the second barrier.

// panel_reflector with the T column spread over the whole wave: lane c
// forms d_c (v^H a_c for c > kk, the Gram entry v_c^H v for c < kk) once, the
// Gram entries go through LDS (dv, wave-local), and lanes 4j .. 4j + 3 add up
// the four interleaved quarters of T[j][j:kk] d[j:kk] and combine them with
// two DPP steps.  qn is taken as given (read by the caller from a lane).
template <int NB>
__device__ __forceinline__ void panel_reflector2(int kk, int nbk, double sc, double qn,
                                                 const double* fin, const double2* row,
                                                 double2* cc_out, double2* scal_out,
                                                 double2* dv, double2* sT, int lane) {
  const double2 alpha = row[kk];
  double2 tau = make_double2(0.0, 0.0), scal = make_double2(0.0, 0.0);
  const double amax = fmax(fabs(alpha.x), fabs(alpha.y));
  const bool direct = amax < 1e140 && (sc == 1.0 ? true : (sc == 0.0 && (amax == 0.0 || amax > 1e-140)));
  if (direct) {
    if (!(sc == 0.0 && alpha.y == 0.0)) {
      const double nrm_all = sqrt((sc == 1.0 ? qn : 0.0) + alpha.x * alpha.x + alpha.y * alpha.y);
      if (nrm_all > 1e-280) {
        const double beta = alpha.x >= 0.0 ? -nrm_all : nrm_all;
        const double rb = 1.0 / beta;
        tau = make_double2((beta - alpha.x) * rb, -alpha.y * rb);
        const double dx = alpha.x - beta, dy = alpha.y;
        const double id = 1.0 / (dx * dx + dy * dy);   // |alpha - beta| in [|beta|, 2 |beta|]
        scal = make_double2(dx * id, -dy * id);
      }
    }
  } else if (!(sc == 0.0 && alpha.y == 0.0)) {
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
  if (lane < NB && lane != kk) {
    const int c = lane;
    const int slot = 2 * (c < kk ? c : c - 1);
    const double2 pq = make_double2(fin[slot], fin[slot + 1]);
    const double2 rc = row[c];
    if (c > kk) {
      if (c < nbk) {
        const double2 u = cmul(cconj(scal), pq);
        cc_out[c] = cmul(cconj(tau), make_double2(rc.x + u.x, rc.y + u.y));
      }
    } else {
      const double2 u = cmul(scal, pq);
      dv[c] = make_double2(rc.x + u.x, -rc.y + u.y);
    }
  }
  if (kk > 0) {   // T[j][kk] = -tau T[j][j:kk] d[j:kk]
    const int j = lane >> 2, q = lane & 3;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < (NB + 3) / 4; ++u) {
      const int t = q + 4 * u;
      if (t >= j && t < kk) {
        const double2 w = cmul(sT[j * NB + t], dv[t]);
        acc.x += w.x;
        acc.y += w.y;
      }
    }
    acc.x += dpp_d<0xB1>(acc.x);
    acc.y += dpp_d<0xB1>(acc.y);
    acc.x += dpp_d<0x4E>(acc.x);
    acc.y += dpp_d<0x4E>(acc.y);
    if (q == 0 && j < kk) {
      const double2 w = cmul(tau, acc);
      sT[j * NB + kk] = make_double2(-w.x, -w.y);
    }
  }
  if (lane == 0) {
    sT[kk * NB + kk] = tau;
    *scal_out = scal;
  }
}

template <int NW, int NB>
struct PanelSmem2 {
  double part[NW][32];   // per-wave sums of the reduced values
  double fin[32];        // the reduced values (written and read by wave 0)
  double2 dv[NB];        // Gram entries of the T column (wave 0)
  double mx[NW];
  double red[2 * NW];
  double2 row[NB];       // row kk of the panel
  double2 cc[NB];        // conj(tau) v^H a_c of the columns c > kk
  double2 scal;          // v = [1; scal x]
};

// Exchanges a (lanes of one half) with b (lanes of the other half) so that
// afterwards a + b is, in every lane, the sum over the lane pair of the value
// that lane's half keeps: the lower half (by lane distance D = 32 or 16)
// keeps the value of a, the upper half that of b.
template <int D>
__device__ __forceinline__ void half_swap(double& a, double& b) {
  const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
  const unsigned alo = (unsigned)ua, ahi = (unsigned)(ua >> 32);
  const unsigned blo = (unsigned)ub, bhi = (unsigned)(ub >> 32);
  unsigned r0lo, r1lo, r0hi, r1hi;
  if (D == 32) {
    const auto lo = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    r0lo = lo[0]; r1lo = lo[1]; r0hi = hi[0]; r1hi = hi[1];
  } else {
    const auto lo = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    r0lo = lo[0]; r1lo = lo[1]; r0hi = hi[0]; r1hi = hi[1];
  }
  a = __longlong_as_double((long long)(((unsigned long long)r0hi << 32) | r0lo));
  b = __longlong_as_double((long long)(((unsigned long long)r1hi << 32) | r1lo));
}

// Halving step on the M bit of the lane over K value pairs (s, s + K): lanes
// with the M bit set keep s + K, the others s.  The partner lane comes from a
// DPP pattern inside a row of 16 that flips the M bit and keeps every higher
// bit: the row mirror (i <-> 15 - i) for M = 8, the half-row mirror
// (i <-> 7 - i) for M = 4, and the quad swap [2, 3, 0, 1] for M = 2.  Across
// the steps the partners pair disjoint lane sets, so the last step leaves the
// sum over all 16 lanes of the row.
template <int M, int K>
__device__ __forceinline__ void halve_shfl(double (&x)[32], int lane) {
  static_assert(M == 8 || M == 4 || M == 2, "row-local halving steps only");
  constexpr int CTRL = M == 8 ? 0x140 : (M == 4 ? 0x141 : 0x4E);
  const bool up = (lane & M) != 0;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const double send = up ? x[s] : x[s + K];
    const double keep = up ? x[s + K] : x[s];
    x[s] = keep + dpp_d<CTRL>(send);
  }
}

// Wave sums of 32 values; value s ends in lanes 2s and 2s + 1 (returned).
__device__ __forceinline__ double wave_scatter_sum32(double (&x)[32], int lane) {
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    half_swap<32>(x[s], x[s + 16]);
    x[s] += x[s + 16];
  }
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    half_swap<16>(x[s], x[s + 8]);
    x[s] += x[s + 8];
  }
  halve_shfl<8, 4>(x, lane);
  halve_shfl<4, 2>(x, lane);
  halve_shfl<2, 1>(x, lane);
  return x[0] + dpp_d<0xB1>(x[0]);
}

template <int RP, int NB, int NT>
__device__ __forceinline__ void factor_panel2(double2 (&a)[RP][NB], int mp, int nbk,
                                              PanelSmem2<NT / 64, NB>& sm, double2* sT) {
  static_assert(NB <= 16, "at most 32 reduced values");
  constexpr int NW = NT / 64;
  // The thread index passes through an empty asm so that the lane-dependent
  // LDS addresses below are formed here, once per panel, instead of being
  // hoisted into the caller and kept (spilled) across its loops.
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  if constexpr (NT >= NB * NB) {
    if (tid < NB * NB) sT[tid] = make_double2(0.0, 0.0);
  } else {
    for (int e = tid; e < NB * NB; e += NT) sT[e] = make_double2(0.0, 0.0);
  }
  __syncthreads();   // the caller's reads of this LDS are done

  static_for<NB>([&](auto kc) {
    constexpr int kk = decltype(kc)::value;
    if (kk >= nbk) return;   // uniform over the workgroup
    double x[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) x[q] = 0.0;
    double mx = 0.0;
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int i = tid + r * NT;
      if (i > kk && i < mp) {
        const double2 xi = a[r][kk];
        mx = fmax(mx, fmax(fabs(xi.x), fabs(xi.y)));
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          if (c == kk) continue;
          const int j = c < kk ? c : c - 1;
          const double2 w = (c > kk) ? cdotc(xi, a[r][c]) : cdotc(a[r][c], xi);
          x[2 * j] += w.x;
          x[2 * j + 1] += w.y;
        }
        x[2 * NB - 2] += xi.x * xi.x + xi.y * xi.y;
      }
    }
    if (tid == kk) {   // row kk: alpha, R entries (c > kk) and v_c[kk] (c < kk)
#pragma unroll
      for (int c = 0; c < NB; ++c) sm.row[c] = a[0][c];
    }
    const double xs = wave_scatter_sum32(x, lane);
    mx = wave_max_dpp(mx);
    if ((lane & 1) == 0) sm.part[wave][lane >> 1] = xs;
    if (lane == 0) sm.mx[wave] = mx;
    __syncthreads();
    double f = 0.0;   // wave 0, lane s < 32: reduced value s
    if (wave == 0 && lane < 32) {
      f = sm.part[0][lane];
#pragma unroll
      for (int w = 1; w < NW; ++w) f += sm.part[w][lane];
      sm.fin[lane] = f;
    }
    double mxa = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) mxa = fmax(mxa, sm.mx[w]);
    double sc = 0.0, qn = 0.0;
    const bool scaled = mxa > 0.0 && (mxa < 1e-140 || mxa > 1e140);
    if (scaled) {
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
    }
    if (wave == 0) {
      if (!scaled && mxa > 0.0) {
        sc = 1.0;
        qn = readlane_d(f, 2 * NB - 2);
      }
      panel_reflector2<NB>(kk, nbk, sc, qn, sm.fin, sm.row, sm.cc, &sm.scal, sm.dv, sT, lane);
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
