// Panel factorisation of the left-looking QR by Cholesky QR and Householder
// reconstruction, for panels whose columns are well away from linear
// dependence.
//
// The panel A (rows p.. of the 16 panel columns, nbk of them used) is
// orthonormalised twice by Cholesky QR (G = A^H A = R^H R, Q1 = A R^{-1}; the
// same again on Q1: Q = Q1 R2^{-1}), which leaves Q orthonormal to FP64
// rounding when no column is close to the span of the columns before it.
// The Householder form of the panel then follows from Q alone (the
// reconstruction of Ballard, Demmel, Grigori, Jacquelin, Knight, Nguyen,
// "Reconstructing Householder vectors from tall-skinny QR", 2015): the LU
// factorisation without pivoting Q - [S; 0] = Y U, taken column by column
// with s_j = -sign(Re of the j-th pivot entry) -- the sign rule of the
// reflectors, beta = -sign(Re alpha) |(alpha, x)| -- gives V = Y and
// T = -U S Y1^{-H} (Y1 the top 16 x 16 block of Y).  These are the
// reflectors and the T factor of the column-by-column factorisation of A
// itself: A and Q differ by an upper triangular factor with a positive real
// diagonal, which scales every column's (alpha, x) by a positive number and so
// leaves each reflector unchanged.
//
// Work per panel: four 16-column products on the matrix cores (the two Gram
// matrices, Q1 = A R1^{-1} and V = Q1 R2^{-1} U^{-1}), two 16-step
// recurrences on one wave (the first Cholesky factorisation with its inverse,
// the LU with U^{-1} and Y1^{-1}; the second Cholesky factor is I plus half
// the rounding-level deviation of its Gram matrix from I, to first order) and
// five workgroup barriers,
// where the column-by-column form takes two barriers and a reduction over the
// workgroup per column.
//
// The panel is left to the column-by-column factorisation (the caller's
// fallback) when a column has no rows below its diagonal (then the reflector
// of an exactly real pivot is the identity, which the sign rule above does not
// reproduce), when an entry of the panel is exactly zero (structured inputs,
// whose exact zeros the column-by-column form keeps), when a Cholesky pivot
// of a used column is below about 1e-10 of that column's squared norm, or
// when a squared column norm leaves about [1e-200, 1e200].
#pragma once

#include "kernel_util.h"

namespace dcs {
namespace {

// Panels of the blocked QR kernels are 16 columns wide; in LDS a panel is
// row-major with the column index swizzled by the row against bank conflicts.
constexpr int QB = 16;

__device__ __forceinline__ int pidx(int i, int c) { return i * QB + (c ^ (i & 15)); }

// A 16 x 16 matrix on one wave: lane l holds entries (lk + 4r, li), r = 0..3,
// li = l % 16, lk = l / 16 -- the output layout of the 16x16x4 FP64 MFMA.

// Value of lane K of this lane's row of 16 lanes (DPP row_newbcast).
template <int K>
__device__ __forceinline__ double bcol(double v) {
  const unsigned long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, 0x150 + K, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), 0x150 + K, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int K>
__device__ __forceinline__ double2 bcol2(double2 v) {
  return make_double2(bcol<K>(v.x), bcol<K>(v.y));
}

// Value of the lane with the same index in row G of the wave: the permlane
// swaps at distance 16 and 32 pair every row with the others.
template <int G>
__device__ __forceinline__ unsigned brow_u(unsigned u) {
  const auto s1 = __builtin_amdgcn_permlane16_swap(u, u, false, false);   // rows [0 0 2 2], [1 1 3 3]
  const unsigned y = (G & 1) ? s1[1] : s1[0];
  const auto s2 = __builtin_amdgcn_permlane32_swap(y, y, false, false);   // rows [0 1 0 1], [2 3 2 3] of y
  return (G & 2) ? s2[1] : s2[0];
}
template <int G>
__device__ __forceinline__ double brow(double v) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = brow_u<G>((unsigned)b), hi = brow_u<G>((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int G>
__device__ __forceinline__ double2 brow2(double2 v) {
  return make_double2(brow<G>(v.x), brow<G>(v.y));
}

// 1 / sqrt(d) and 1 / d for positive normal d: the hardware estimate refined
// by two Newton steps.
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}
__device__ __forceinline__ double rcp_nr(double d) {
  double y = __builtin_amdgcn_rcp(d);
  y = y * fma(-d, y, 2.0);
  y = y * fma(-d, y, 2.0);
  return y;
}

__device__ __forceinline__ double2 cscale(double2 a, double s) {
  return make_double2(a.x * s, a.y * s);
}
// c ? a : b on the components (a conditional on the vector struct itself is
// lowered through stack memory)
__device__ __forceinline__ double2 csel(bool c, double2 a, double2 b) {
  return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}
// a - b c
__device__ __forceinline__ double2 cfms(double2 a, double2 b, double2 c) {
  return make_double2(fma(-b.y, -c.y, fma(-b.x, c.x, a.x)), fma(-b.x, c.y, fma(-b.y, c.x, a.y)));
}

// The recurrences below run on one wave with the other waves waiting, so
// they are written without branches: lane conditions select multipliers (0
// or the factor), and every lane applies every update.  li and lk are the
// lane's column and row group.

// Right-looking Cholesky factorisation G = R^H R of the Hermitian g, fused
// with the inverse z = R^{-1} (built by the same column operations from the
// identity); columns at or past nbk are identity.  The column of G' below the
// pivot stands in for the conjugate of the pivot row (G' stays Hermitian up to
// rounding).  Returns false when a pivot is below about 1e-10 of its column's
// squared norm (2^-33 by exponents) or a squared norm leaves [2^-664, 2^664]
// (about 1e-200 to 1e200); g and z are then meaningless.
__device__ __forceinline__ bool chol_inv16(double2 (&g)[4], double2 (&z)[4], int nbk, int li,
                                           int lk) {
  // the lane's entry of the diagonal of G, if any (before the updates)
  const double gdiag = (li & 3) != lk ? 0.0
                       : (li >> 2) == 0 ? g[0].x
                       : (li >> 2) == 1 ? g[1].x
                       : (li >> 2) == 2 ? g[2].x : g[3].x;
#pragma unroll
  for (int r = 0; r < 4; ++r) z[r] = make_double2(lk + 4 * r == li ? 1.0 : 0.0, 0.0);
  bool ok = true;
  static_for<16>([&](auto kc) {
    constexpr int k = decltype(kc)::value, kr = k & 3, ks = k >> 2;
    if (k >= nbk) return;   // uniform: identity from here on
    const double dk = readlane_d(g[ks].x, kr * 16 + k);
    const double d0 = readlane_d(gdiag, kr * 16 + k);
    // on the (uniform) sign and exponent bits, in scalar integer code: d0 in
    // [2^-664, 2^664], dk positive and finite with an exponent at most 33
    // below that of d0 (FP64 constants would have to live in vector registers)
    const int ed = (int)((unsigned long long)__double_as_longlong(dk) >> 52);
    const int e0 = (int)((unsigned long long)__double_as_longlong(d0) >> 52);
    ok = ok && e0 >= 1023 - 664 && e0 <= 1023 + 664 && ed >= e0 - 33 && ed < 2047;
    const double dd = ok ? dk : 1.0;
    const double inv = rsqrt_nr(dd);
    const double2 rk = cscale(brow2<kr>(g[ks]), li > k ? inv : 0.0);   // R[k][li], li > k
    // slot r holds rows 4r .. 4r + 3: G' changes only below row k, and Z
    // (upper triangular) only in rows up to k
    static_for<4>([&](auto rc) {
      constexpr int r = decltype(rc)::value;
      if constexpr (4 * r + 3 > k) {
        const double2 ck = cscale(bcol2<k>(g[r]), lk + 4 * r > k ? inv : 0.0);   // conj(R[k][i])
        g[r] = cfms(g[r], ck, rk);
      }
      if constexpr (4 * r <= k) {
        const double2 zk = cscale(bcol2<k>(z[r]), inv);   // Z[i][k]
        const double2 zn = cfms(z[r], zk, rk);
        z[r] = csel(li == k, zk, zn);
      }
    });
  });
  return ok;
}

// Second Cholesky factor of Cholesky QR2, whose Gram matrix is I + E with E
// at rounding level after an accepted first pass: R2 = I + F, F = the strict
// upper triangle of E plus half its diagonal, and R2^{-1} = I - F, both exact
// up to |E|^2.  Returns false (nothing written) when max |E| exceeds 1e-9.
__device__ __forceinline__ bool chol_inv16_near_identity(const double2 (&g)[4], double2 (&z)[4],
                                                         int nbk, int li, int lk) {
  double emax = 0.0;
  double2 f[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = lk + 4 * r;
    const bool used = i < nbk && li < nbk;
    const double2 e = make_double2(used ? g[r].x - (i == li ? 1.0 : 0.0) : 0.0, used ? g[r].y : 0.0);
    emax = fmax(emax, fabs(e.x) + fabs(e.y));
    f[r] = make_double2(i < li ? e.x : (i == li ? 0.5 * e.x : 0.0), i < li ? e.y : 0.0);
  }
  emax = wave_max_dpp(emax);
  if (!(emax <= 1e-9)) return false;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    z[r] = make_double2((lk + 4 * r == li ? 1.0 : 0.0) - f[r].x, -f[r].y);
  return true;
}

// LU factorisation without pivoting of W - S, S = diag(s_k) chosen column by
// column: s_k = -1 if Re w_kk >= 0 else +1, U_kk = w_kk - s_k (|U_kk| >= 1).
// On return w holds U on and above the diagonal and the unit lower factor L
// below it, zu = U^{-1}, zl = L^{-1}, and s_col = s of the lane's column.
// Columns at or past nbk are identity (s = -1).
__device__ __forceinline__ void lu_inv16(double2 (&w)[4], double2 (&zu)[4], double2 (&zl)[4],
                                         double& s_col, int nbk, int li, int lk) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    zu[r] = make_double2(lk + 4 * r == li ? 1.0 : 0.0, 0.0);
    zl[r] = zu[r];
  }
  s_col = -1.0;
  static_for<16>([&](auto kc) {
    constexpr int k = decltype(kc)::value, kr = k & 3, ks = k >> 2;
    if (k >= nbk) return;
    const double ax = readlane_d(w[ks].x, kr * 16 + k), ay = readlane_d(w[ks].y, kr * 16 + k);
    const double sk = ax >= 0.0 ? -1.0 : 1.0;
    s_col = li == k ? sk : s_col;
    const double ux = ax - sk, uy = ay;
    const double den = rcp_nr(ux * ux + uy * uy);
    const double2 iu = make_double2(ux * den, -uy * den);
    const double2 uk = cscale(brow2<kr>(w[ks]), li > k ? 1.0 : 0.0);   // U[k][li], li > k
    const double2 rowzl = brow2<kr>(zl[ks]);                           // row k of L^{-1}
    // slot r holds rows 4r .. 4r + 3: W and L^{-1} (lower triangular) change
    // only from row k down, U^{-1} (upper triangular) only in rows up to k
    static_for<4>([&](auto rc) {
      constexpr int r = decltype(rc)::value;
      const int i = lk + 4 * r;
      if constexpr (4 * r + 3 >= k) {
        const double2 lik = cscale(cmul(bcol2<k>(w[r]), iu), i > k ? 1.0 : 0.0);   // L[i][k]
        const double2 wn = cfms(w[r], lik, uk);
        w[r] = csel(li != k, wn, csel(i > k, lik, csel(i == k, make_double2(ux, uy), w[r])));
        zl[r] = cfms(zl[r], lik, rowzl);
      }
      if constexpr (4 * r <= k) {
        const double2 zuk = cmul(bcol2<k>(zu[r]), iu);   // U^{-1}[i][k]
        const double2 zun = cfms(zu[r], zuk, uk);
        zu[r] = csel(li == k, zuk, zun);
      }
    });
  });
}

// The two one-wave sections of the panel, kept out of line so that their
// recurrences get the registers the caller's loops hold elsewhere; they
// communicate through LDS only.  Called by wave 0.

// G1 (the sum of the NW waves' parts in Wp) -> X1 = R1^{-1} in Wp[0..255]
// (row-major), with a flag in X1[1][0] (below the diagonal): 0 when the
// panel is accepted, 1 when it is left to the column-by-column
// factorisation.  The imaginary part of entry (0, 0) of each part carries
// whether that wave saw an exactly zero entry.
template <int NW>
__device__ __noinline__ void panel_first_pass(
    double2* Wp, int nbk) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  double2 g[4], x[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double2 s = Wp[(lk + 4 * r) * 16 + li];
#pragma unroll
    for (int w = 1; w < NW; ++w) s = make_double2(s.x + Wp[w * 256 + (lk + 4 * r) * 16 + li].x,
                                                  s.y + Wp[w * 256 + (lk + 4 * r) * 16 + li].y);
    g[r] = s;
  }
  const bool noz = readlane_d(g[0].y, 0) < 0.5;
  if (lane == 0) g[0].y = 0.0;
  const bool ok = chol_inv16(g, x, nbk, li, lk) && noz;
  if (lane == 16) x[0] = make_double2(ok ? 0.0 : 1.0, 0.0);
#pragma unroll
  for (int r = 0; r < 4; ++r) Wp[(lk + 4 * r) * 16 + li] = x[r];
}

// G2 (sum of the parts in Wp) and Q1's top block (P rows 0..15) -> T in
// Wp[0..255] (row-major, flag in T[1][0] as above), M = R2^{-1} U^{-1} in
// Wp[256..511] (zero in unused columns), and the top block of V in P rows
// 0..15.
template <int NW>
__device__ __noinline__ void panel_second_pass(
    double2* P, double2* Wp, int nbk, int mp) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const double2 zero = make_double2(0.0, 0.0);
  double2* part0 = Wp;
  double2* part1 = Wp + 256;
  double2 g[4], z2[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double2 s = Wp[(lk + 4 * r) * 16 + li];
#pragma unroll
    for (int w = 1; w < NW; ++w) s = make_double2(s.x + Wp[w * 256 + (lk + 4 * r) * 16 + li].x,
                                                  s.y + Wp[w * 256 + (lk + 4 * r) * 16 + li].y);
    g[r] = s;
  }
  const bool ok =
      chol_inv16_near_identity(g, z2, nbk, li, lk) || chol_inv16(g, z2, nbk, li, lk);
  double2 w[4];   // Q_top = Q1_top R2^{-1}
  {
    CAcc3 q;
    q.zero();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double2 av = P[pidx(li, 4 * s + lk)];
      q.add(av.x, av.y, z2[s].x, z2[s].y);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) w[r] = make_double2(q.re(r), q.im(r));
  }
  double2 zu[4], zl[4];
  double s_col;
  lu_inv16(w, zu, zl, s_col, nbk, li, lk);
  // T = -(U S) L^{-H}
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = lk + 4 * r;
    part0[i * 16 + li] = cscale(w[r], i <= li ? s_col : 0.0);
    part1[i * 16 + li] = zl[r];
  }
  {
    CAcc3 t;
    t.zero();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double2 us = part0[li * 16 + 4 * s + lk];   // (U S)[li][4s + lk]
      const double2 lz = part1[li * 16 + 4 * s + lk];   // L^{-1}[li][4s + lk]
      t.add(us.x, us.y, lz.x, -lz.y);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = lk + 4 * r;
      const double sg = (i < nbk && li < nbk) ? -1.0 : 0.0;
      double2 tv = make_double2(sg * t.re(r), sg * t.im(r));
      if (i == 1 && li == 0) tv = make_double2(ok ? 0.0 : 1.0, 0.0);   // flag (T is upper triangular)
      part0[i * 16 + li] = tv;
    }
  }
  // M = R2^{-1} U^{-1}
#pragma unroll
  for (int r = 0; r < 4; ++r) part1[(lk + 4 * r) * 16 + li] = z2[r];
  {
    CAcc3 mm;
    mm.zero();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double2 zv = part1[li * 16 + 4 * s + lk];   // R2^{-1}[li][4s + lk]
      mm.add(zv.x, zv.y, zu[s].x, zu[s].y);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
      part1[(lk + 4 * r) * 16 + li] = make_double2(li < nbk ? mm.re(r) : 0.0, li < nbk ? mm.im(r) : 0.0);
  }
  // top block of V: L (unit diagonal), zero outside the used rows and columns
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = lk + 4 * r;
    const bool out = li >= nbk || i >= mp;
    const double2 v = make_double2(out ? 0.0 : (i > li ? w[r].x : (i == li ? 1.0 : 0.0)),
                                   out || i <= li ? 0.0 : w[r].y);
    P[pidx(i, li)] = v;
  }
}

// The panel (see above) on a workgroup of NW waves.  a holds the wave's rows
// of A in the step layout (block beta = wave + NW b, b < MAXB, rows
// 16 beta + 4t + lk, column li; zero past row m and column nbk); P holds the
// panel rows (pidx), Wp NW areas of 256 complex values.  Every thread calls
// it; mp > nbk.  Returns true (uniform) with V (explicit, panel-local rows,
// zero in unused columns) in P and T (row-major 16 x 16) in Wp; false with
// the panel rows in P -- A, or Q1 = A R1^{-1}, whose column-by-column
// factorisation has the same reflectors -- for the caller's fallback.  Ends
// with every wave past a barrier after its last read of Wp.
template <int NW, int MAXB>
__device__ __forceinline__ bool panel_cholqr(double2 (&a)[MAXB][4], int m, int k, int mp, int nbk,
                                             double2* P, double2* Wp) {
  static_assert(NW >= 2, "two 256-entry areas of Wp");
  // the thread index passes through an empty asm so that lane-dependent LDS
  // offsets are formed here, once per panel, instead of being hoisted into
  // the caller's loop and held (or spilled) across it
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const double2 zero = make_double2(0.0, 0.0);
  double2* part0 = Wp;         // X1, then T
  double2* part1 = Wp + 256;   // staging, then R2^{-1} U^{-1}

  // rows to P; this wave's part of G1 = A^H A, with the imaginary part of
  // entry (0, 0) replaced by whether the wave saw an exact zero
  {
    CAcc3 g;
    g.zero();
    bool z = false;
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int beta = wave + NW * b;
      if (beta >= k && 16 * beta < m) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          P[pidx(16 * (beta - k) + 4 * t + lk, li)] = a[b][t];
          const int row = 16 * beta + 4 * t + lk;
          z = z || (row < m && li < nbk && a[b][t].x == 0.0 && a[b][t].y == 0.0);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) g.add(a[b][t].x, -a[b][t].y, a[b][t].x, a[b][t].y);
      }
    }
    const bool anyz = __ballot(z) != 0ull;
    double2* q = Wp + wave * 256;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      q[(lk + 4 * r) * 16 + li] =
          make_double2(g.re(r), lane == 0 && r == 0 ? (anyz ? 1.0 : 0.0) : g.im(r));
  }
  __syncthreads();
  if (wave == 0) panel_first_pass<NW>(Wp, nbk);
  __syncthreads();
  if (part0[16].x != 0.0) {
    __syncthreads();   // every wave has read the flag before the fallback reuses Wp
    return false;
  }
  double2 xb[4];   // X1[lk + 4s][li], the B operand of k-step s
#pragma unroll
  for (int s = 0; s < 4; ++s) xb[s] = part0[(lk + 4 * s) * 16 + li];
  __syncthreads();   // X1 read everywhere before the parts are rewritten
  {   // Q1 = A X1 block by block (each wave rewrites only its own rows of P), G2 parts
    CAcc3 g2;
    g2.zero();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int beta = wave + NW * b;
      if (beta >= k && 16 * beta < m) {
        const int r0 = 16 * (beta - k);
        CAcc3 q;
        q.zero();
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const double2 av = P[pidx(r0 + li, 4 * s + lk)];   // A[r0 + li][4s + lk]
          q.add(av.x, av.y, xb[s].x, xb[s].y);
        }
        double2 qv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          qv[r] = make_double2(q.re(r), q.im(r));
          P[pidx(r0 + lk + 4 * r, li)] = qv[r];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) g2.add(qv[t].x, -qv[t].y, qv[t].x, qv[t].y);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
      Wp[wave * 256 + (lk + 4 * r) * 16 + li] = make_double2(g2.re(r), g2.im(r));
  }
  __syncthreads();
  if (wave == 0) panel_second_pass<NW>(P, Wp, nbk, mp);
  __syncthreads();
  if (part0[16].x != 0.0) {
    __syncthreads();
    return false;
  }
  double2 mb[4];   // M[lk + 4s][li]
#pragma unroll
  for (int s = 0; s < 4; ++s) mb[s] = part1[(lk + 4 * s) * 16 + li];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {   // V below the top block = Q1 M
    const int beta = wave + NW * b;
    if (beta > k && 16 * beta < m) {
      const int r0 = 16 * (beta - k);
      CAcc3 y;
      y.zero();
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double2 av = P[pidx(r0 + li, 4 * s + lk)];
        y.add(av.x, av.y, mb[s].x, mb[s].y);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) P[pidx(r0 + lk + 4 * r, li)] = make_double2(y.re(r), y.im(r));
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  return true;
}

}  // namespace
}  // namespace dcs
