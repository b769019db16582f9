// Batched transposition of complex tensors, with optional conjugation and
// conversion between complex64 and complex128 storage: the data movement
// between the contractions of the tree tensor network, whose operands are
// brought into the row-major matrix layouts the GEMM kernels take.
//
// Output element o (row-major over the output dims) reads the input at
// sum_k c_k in_stride[k], c the output coordinates.  One grid row per batch
// item, items addressed through the slot-id table or call-locally.
//
// Two kernels.  The element-wise one decodes every output index and gathers
// its input element: coalesced only where the innermost output leg is also
// contiguous in the input over a long run.  The tiled one moves a sub-block
// through LDS: the legs are split so that a tile holds the input's innermost
// run of at least 256 bytes (read contiguously) times the output's innermost
// run of at least 256 bytes (written contiguously); the remaining legs index
// the tiles.  Inside a tile every address is a sum of two small per-workgroup
// tables (input-run position, output-run position), so the per-element work
// is two table reads and no division.
#include "dcs_internal.h"
#include <algorithm>
#include <cstring>
#include <vector>

#include "kernel_util.h"

namespace dcs {
namespace {

template <int CTI, int CTO>
__global__ __launch_bounds__(256) void permute_kernel(const PermuteArgs a) {
  using TI = typename St<CTI>::T;
  using TO = typename St<CTO>::T;
  const int item = blockIdx.y;
  const TI* __restrict__ src = reinterpret_cast<const TI*>(item_ptr(a.in, a.ids, item));
  TO* __restrict__ dst = reinterpret_cast<TO*>(const_cast<char*>(item_ptr(a.out, a.ids, item)));
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x; o < a.total; o += step) {
    long long rem = o, off = 0;
    for (int k = a.rank - 1; k >= 0; --k) {
      const long long d = a.dims[k];
      const long long c = rem % d;
      rem /= d;
      off += c * a.in_stride[k];
    }
    const TI v = src[off];
    TO w;
    w.x = v.x;
    w.y = a.conj ? -v.y : v.y;
    dst[o] = w;
  }
}

// The same with 32-bit index arithmetic, for tensors whose element count and
// largest input offset stay below 2^31: the per-leg quotient and remainder
// of the output index are 32-bit divisions, where the 64-bit ones of the
// general kernel are long software sequences.
template <int CTI, int CTO>
__global__ __launch_bounds__(256) void permute32_kernel(const PermuteArgs a) {
  using TI = typename St<CTI>::T;
  using TO = typename St<CTO>::T;
  const int item = blockIdx.y;
  const TI* __restrict__ src = reinterpret_cast<const TI*>(item_ptr(a.in, a.ids, item));
  TO* __restrict__ dst = reinterpret_cast<TO*>(const_cast<char*>(item_ptr(a.out, a.ids, item)));
  const unsigned total = (unsigned)a.total, step = gridDim.x * blockDim.x;
  unsigned stride[PERMUTE_MAX_RANK];
#pragma unroll
  for (int k = 0; k < PERMUTE_MAX_RANK; ++k) stride[k] = (unsigned)a.in_stride[k];
  for (unsigned o = blockIdx.x * blockDim.x + threadIdx.x; o < total; o += step) {
    unsigned rem = o, off = 0;
#pragma unroll
    for (int k = PERMUTE_MAX_RANK - 1; k >= 0; --k) {
      if (k < a.rank) {
        const unsigned d = (unsigned)a.dims[k];
        const unsigned q = rem / d;
        off += (rem - q * d) * stride[k];
        rem = q;
      }
    }
    const TI v = src[off];
    TO w;
    w.x = v.x;
    w.y = a.conj ? -v.y : v.y;
    dst[o] = w;
  }
}

// Tiled transposition.  A tile is the set of elements whose legs outside the
// tile are fixed.  Its legs form the input run I (the input's innermost legs,
// contiguous in memory, pi elements), the output run O (the output's
// innermost legs, po elements) and extra legs E that make the tile larger;
// A = (I \ O) + E, C = (O \ I) + E.  An element is (c, i) in read order and
// (a, b) in write order, with b its position in the output run and a, c its
// indices over A and C.  LDS holds the tile as [a][b] with row pitch `pitch`:
//   input offset  = tile_in + c_in(c) + i
//   LDS position  = t_i(i) + c_lds(c)         (= a * pitch + b)
//   output offset = tile_out + a_out(a) + b
// The four tables are built per workgroup from the leg descriptors.
constexpr int PT_MAXG = 12;    // legs per group (I, C, A)
constexpr int PT_MAXR = 24;    // legs indexing the tiles
constexpr int PT_MAXRUN = 64;  // elements of a run (pi, po)
constexpr int PT_MAXTAB = 256; // entries of the C and A tables
struct PermuteTileArgs {
  Operand in, out;
  const int* ids;
  int conj, batch;
  int pi, pc, pa, po, pitch, ni, nc, na, nr;
  unsigned tiles;
  int i_ext[PT_MAXG], i_lds[PT_MAXG];
  int c_ext[PT_MAXG], c_in[PT_MAXG], c_lds[PT_MAXG];
  int a_ext[PT_MAXG], a_out[PT_MAXG];
  int r_ext[PT_MAXR], r_in[PT_MAXR], r_out[PT_MAXR];
};

// Table entry x of a group: sum over its legs (fastest first) of coordinate
// times the leg's weight.
__device__ __forceinline__ int pt_entry(int x, int n, const int* ext, const int* w) {
  int v = 0;
  for (int k = 0; k < n; ++k) {
    const int e = ext[k];
    const int q = x / e;
    v += (x - q * e) * w[k];
    x = q;
  }
  return v;
}

// EPT: elements per thread and tile (pc * pi = pa * po <= 256 * EPT).
template <int CTI, int CTO, int EPT>
__global__ __launch_bounds__(256) void permute_tiled_kernel(const PermuteTileArgs a) {
  using TI = typename St<CTI>::T;
  using TO = typename St<CTO>::T;
  extern __shared__ __align__(16) char pt_dyn[];
  int* t_i = reinterpret_cast<int*>(pt_dyn);
  int* c_in = t_i + PT_MAXRUN;
  int* c_lds = c_in + PT_MAXTAB;
  int* a_out = c_lds + PT_MAXTAB;
  TO* tile = reinterpret_cast<TO*>(a_out + PT_MAXTAB);
  const int tid = threadIdx.x;
  if (tid < a.pi) t_i[tid] = pt_entry(tid, a.ni, a.i_ext, a.i_lds);
  if (tid < a.pc) {
    c_in[tid] = pt_entry(tid, a.nc, a.c_ext, a.c_in);
    c_lds[tid] = pt_entry(tid, a.nc, a.c_ext, a.c_lds);
  }
  if (tid < a.pa) a_out[tid] = pt_entry(tid, a.na, a.a_ext, a.a_out);
  const int item = blockIdx.y;
  const TI* __restrict__ src = reinterpret_cast<const TI*>(item_ptr(a.in, a.ids, item));
  TO* __restrict__ dst = reinterpret_cast<TO*>(const_cast<char*>(item_ptr(a.out, a.ids, item)));
  const int n = a.pc * a.pi;
  // (c, i) and (a, b) of this thread's first element, and the steps of 256
  const int c0 = tid / a.pi, i0 = tid - c0 * a.pi;
  const int dc = 256 / a.pi, di = 256 - dc * a.pi;
  const int a0 = tid / a.po, b0 = tid - a0 * a.po;
  const int da = 256 / a.po, db = 256 - da * a.po;
  __syncthreads();
  for (unsigned t = blockIdx.x; t < a.tiles; t += gridDim.x) {
    int tin = 0, tout = 0;
    unsigned x = t;
    for (int k = 0; k < a.nr; ++k) {
      const unsigned e = (unsigned)a.r_ext[k];
      const unsigned q = x / e;
      const int r = (int)(x - q * e);
      tin += r * a.r_in[k];
      tout += r * a.r_out[k];
      x = q;
    }
    TI v[EPT];
    int pos[EPT];
    {
      int c = c0, i = i0;
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        if (tid + j * 256 < n) {
          v[j] = src[tin + c_in[c] + i];
          pos[j] = t_i[i] + c_lds[c];
        }
        i += di;
        c += dc;
        if (i >= a.pi) {
          i -= a.pi;
          ++c;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      if (tid + j * 256 < n) {
        TO w;
        w.x = v[j].x;
        w.y = a.conj ? -v[j].y : v[j].y;
        tile[pos[j]] = w;
      }
    }
    __syncthreads();
    {
      int ai = a0, b = b0;
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        if (tid + j * 256 < n) dst[tout + a_out[ai] + b] = tile[ai * a.pitch + b];
        b += db;
        ai += da;
        if (b >= a.po) {
          b -= a.po;
          ++ai;
        }
      }
    }
    __syncthreads();
  }
}

// One leg of the planner: extent, input stride, output stride.
struct PLeg {
  long long ext, is, os;
  bool in_o = false, in_i = false, in_e = false;
};

// Splits leg k into (ext / f, strides * f) and (f, strides), the second
// placed after the first; returns the index of the (f) part.
int split_leg(std::vector<PLeg>& L, int k, long long f) {
  PLeg hi = L[k], lo = L[k];
  hi.ext = L[k].ext / f;
  hi.is = L[k].is * f;
  hi.os = L[k].os * f;
  lo.ext = f;
  L[k] = hi;
  L.insert(L.begin() + k + 1, lo);
  return k + 1;
}

// Takes the innermost legs in the order given by `key` (smallest stride
// first) until their product reaches [pmin, pmax], splitting the leg that
// would overshoot by a divisor of its extent.  Marks them with `flag`.
template <typename Key, typename Flag>
long long take_run(std::vector<PLeg>& L, long long pmin, long long pmax, Key key, Flag flag) {
  long long p = 1;
  while (p < pmin) {
    int best = -1;
    for (int k = 0; k < (int)L.size(); ++k)
      if (!flag(L[k]) && (best < 0 || key(L[k]) < key(L[best]))) best = k;
    if (best < 0) break;
    const long long e = L[best].ext;
    if (p * e <= pmax) {
      flag(L[best]) = true;
      p *= e;
      continue;
    }
    long long f = 1;
    for (long long d = 2; d < e && p * d <= pmax; ++d)
      if (e % d == 0) {
        f = d;
        if (p * d >= pmin) break;
      }
    if (f == 1) break;
    const int lo = split_leg(L, best, f);
    flag(L[lo]) = true;
    p *= f;
    break;
  }
  return p;
}

bool plan_tiled(const PermuteArgs& a, int esize, PermuteTileArgs* t, int* ept) {
  std::vector<PLeg> L;
  long long os = 1;
  for (int k = a.rank - 1; k >= 0; --k) {
    if (a.dims[k] > 1) L.insert(L.begin(), PLeg{a.dims[k], a.in_stride[k], os});
    os *= a.dims[k];
  }
  if (L.empty()) return false;
  // the input must be dense: sorted by stride, each stride the product of
  // the extents below it
  {
    std::vector<PLeg> srt = L;
    std::sort(srt.begin(), srt.end(), [](const PLeg& x, const PLeg& y) { return x.is < y.is; });
    long long want = 1;
    for (const PLeg& l : srt) {
      if (l.is != want) return false;
      want *= l.ext;
    }
  }
  const long long pmin = 256 / esize, pmax = 2 * pmin;
  const long long po = take_run(L, pmin, pmax, [](const PLeg& l) { return l.os; },
                                [](PLeg& l) -> bool& { return l.in_o; });
  const long long pi = take_run(L, pmin, pmax, [](const PLeg& l) { return l.is; },
                                [](PLeg& l) -> bool& { return l.in_i; });
  if (po < 2 || pi < 2) return false;
  long long pa = 1, pc = 1;
  for (const PLeg& l : L) {
    if (l.in_i && !l.in_o) pa *= l.ext;
    if (l.in_o && !l.in_i) pc *= l.ext;
  }
  // extra legs E (in neither run), innermost output legs first, fill the tile
  // up to tmax elements: they extend both the read-side index c and the
  // write-side index a
  const long long tmax = esize == 8 ? 2048 : 1024;
  for (;;) {
    int best = -1;
    for (int k = 0; k < (int)L.size(); ++k)
      if (!L[k].in_i && !L[k].in_o && !L[k].in_e && (best < 0 || L[k].os < L[best].os)) best = k;
    if (best < 0) break;
    const long long room = std::min(tmax / (pa * po), (long long)PT_MAXTAB / std::max(pa, pc));
    const long long e = L[best].ext;
    if (e <= room) {
      L[best].in_e = true;
      pa *= e;
      pc *= e;
      continue;
    }
    long long f = 1;
    for (long long d = 2; d <= room && d < e; ++d)
      if (e % d == 0) f = d;
    if (f > 1) {
      const int lo = split_leg(L, best, f);
      L[lo].in_e = true;
      pa *= f;
      pc *= f;
    }
    break;
  }
  if (pa > PT_MAXTAB || pc > PT_MAXTAB || pi > PT_MAXRUN || po > PT_MAXRUN) return false;
  std::memset(t, 0, sizeof(*t));
  // every group's legs fastest first: I and C by input stride, A by output
  // stride
  std::vector<int> by_is(L.size()), by_os(L.size());
  for (int k = 0; k < (int)L.size(); ++k) by_is[k] = by_os[k] = k;
  std::sort(by_is.begin(), by_is.end(), [&](int x, int y) { return L[x].is < L[y].is; });
  std::sort(by_os.begin(), by_os.end(), [&](int x, int y) { return L[x].os < L[y].os; });
  const long long pitch = po % 2 ? po : po + 1;
  const long long n = pa * po;
  int e = n <= 256 ? 1 : n <= 512 ? 2 : n <= 1024 ? 4 : n <= 2048 ? 8 : n <= 4096 ? 16 : 0;
  if (e == 0 || pa * pitch * esize > 48 * 1024) return false;
  // A index over (I \ O) and E
  long long astr = 1;
  std::vector<long long> a_lin(L.size(), 0);
  for (int k : by_os)
    if ((L[k].in_i && !L[k].in_o) || L[k].in_e) {
      if (t->na == PT_MAXG) return false;
      t->a_ext[t->na] = (int)L[k].ext;
      t->a_out[t->na] = (int)L[k].os;
      ++t->na;
      a_lin[k] = astr;
      astr *= L[k].ext;
    }
  for (int k : by_is)
    if (L[k].in_i) {
      if (t->ni == PT_MAXG) return false;
      t->i_ext[t->ni] = (int)L[k].ext;
      t->i_lds[t->ni] = (int)(L[k].in_o ? L[k].os : a_lin[k] * pitch);
      ++t->ni;
    }
  // C index over (O \ I) and E
  for (int k : by_is)
    if ((L[k].in_o && !L[k].in_i) || L[k].in_e) {
      if (t->nc == PT_MAXG) return false;
      t->c_ext[t->nc] = (int)L[k].ext;
      t->c_in[t->nc] = (int)L[k].is;
      t->c_lds[t->nc] = (int)(L[k].in_o ? L[k].os : a_lin[k] * pitch);
      ++t->nc;
    }
  long long tiles = 1;
  for (int k : by_os)
    if (!L[k].in_i && !L[k].in_o && !L[k].in_e) {
      if (t->nr == PT_MAXR) return false;
      t->r_ext[t->nr] = (int)L[k].ext;
      t->r_in[t->nr] = (int)L[k].is;
      t->r_out[t->nr] = (int)L[k].os;
      ++t->nr;
      tiles *= L[k].ext;
    }
  t->in = a.in;
  t->out = a.out;
  t->ids = a.ids;
  t->conj = a.conj;
  t->batch = a.batch;
  t->pi = (int)pi;
  t->pc = (int)pc;
  t->pa = (int)pa;
  t->po = (int)po;
  t->pitch = (int)pitch;
  t->tiles = (unsigned)tiles;
  *ept = e;
  return true;
}

size_t pt_lds_bytes(const PermuteTileArgs& t, int esize) {
  return (size_t)(PT_MAXRUN + 3 * PT_MAXTAB) * sizeof(int) + (size_t)t.pa * t.pitch * esize;
}

template <int I, int O>
hipError_t launch_tiled(const PermuteTileArgs& t, int ept, hipStream_t s) {
  const int esize = (int)sizeof(typename St<O>::T);
  const size_t lds = pt_lds_bytes(t, esize);
  // about 16 workgroups per compute unit over the whole batch
  const unsigned gx = std::max(1u, std::min(t.tiles, (unsigned)((4096 + t.batch - 1) / t.batch)));
  const dim3 grid(gx, (unsigned)t.batch), blk(256);
  switch (ept) {
    case 1: hipLaunchKernelGGL((permute_tiled_kernel<I, O, 1>), grid, blk, lds, s, t); break;
    case 2: hipLaunchKernelGGL((permute_tiled_kernel<I, O, 2>), grid, blk, lds, s, t); break;
    case 4: hipLaunchKernelGGL((permute_tiled_kernel<I, O, 4>), grid, blk, lds, s, t); break;
    case 8: hipLaunchKernelGGL((permute_tiled_kernel<I, O, 8>), grid, blk, lds, s, t); break;
    case 16: hipLaunchKernelGGL((permute_tiled_kernel<I, O, 16>), grid, blk, lds, s, t); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// out[item][e] = sum_{s < parts} part[item][s * mn + e] (complex128), s in
// ascending order.
__global__ __launch_bounds__(256) void ksum_kernel(const KsumArgs a) {
  const int item = blockIdx.y;
  const double2* __restrict__ p = reinterpret_cast<const double2*>(item_ptr(a.part, a.ids, item));
  double2* __restrict__ o = reinterpret_cast<double2*>(const_cast<char*>(item_ptr(a.out, a.ids, item)));
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < a.mn; e += gridDim.x * blockDim.x) {
    double re = 0, im = 0;
    for (int s = 0; s < a.parts; ++s) {
      const double2 v = p[(long long)s * a.mn + e];
      re += v.x;
      im += v.y;
    }
    o[e] = make_double2(re, im);
  }
}

}  // namespace

hipError_t launch_ksum(const KsumArgs& a, hipStream_t s) {
  if (a.batch <= 0 || a.mn <= 0) return hipSuccess;
  if (a.parts < 1 || a.batch > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)std::min(64, (a.mn + 255) / 256), (unsigned)a.batch), blk(256);
  hipLaunchKernelGGL(ksum_kernel, grid, blk, 0, s, a);
  return hipGetLastError();
}

bool permute_tile_plan(const PermuteArgs& a, int esize, int* out, int out_len) {
  PermuteTileArgs t;
  int ept = 0;
  if (!plan_tiled(a, esize, &t, &ept)) return false;
  std::vector<int> v{t.pi, t.pc, t.pa, t.po, t.pitch, (int)t.tiles, ept, t.ni, t.nc, t.na, t.nr};
  v.insert(v.end(), t.i_ext, t.i_ext + t.ni);
  v.insert(v.end(), t.i_lds, t.i_lds + t.ni);
  v.insert(v.end(), t.c_ext, t.c_ext + t.nc);
  v.insert(v.end(), t.c_in, t.c_in + t.nc);
  v.insert(v.end(), t.c_lds, t.c_lds + t.nc);
  v.insert(v.end(), t.a_ext, t.a_ext + t.na);
  v.insert(v.end(), t.a_out, t.a_out + t.na);
  v.insert(v.end(), t.r_ext, t.r_ext + t.nr);
  v.insert(v.end(), t.r_in, t.r_in + t.nr);
  v.insert(v.end(), t.r_out, t.r_out + t.nr);
  if ((int)v.size() > out_len) return false;
  std::copy(v.begin(), v.end(), out);
  return true;
}

hipError_t launch_permute(int ct_in, int ct_out, const PermuteArgs& a, hipStream_t s,
                          int variant) {
  if (a.batch <= 0 || a.total <= 0) return hipSuccess;
  if (a.rank < 1 || a.rank > PERMUTE_MAX_RANK || a.batch > 65535) return hipErrorInvalidValue;
  if ((ct_in != CT_F32 && ct_in != CT_F64) || (ct_out != CT_F32 && ct_out != CT_F64))
    return hipErrorInvalidValue;
  const long long blocks = (a.total + 255) / 256;
  const dim3 grid((unsigned)std::min<long long>(blocks, 4096), (unsigned)a.batch), blk(256);
  long long max_off = 0;
  for (int k = 0; k < a.rank; ++k) max_off += (long long)(a.dims[k] - 1) * a.in_stride[k];
  const bool small = a.total < (1LL << 31) && max_off < (1LL << 31);
  // the tiled kernel where the innermost output leg is not already read in
  // contiguous runs of 64 elements or more
  const int r = a.rank - 1;
  const bool runs = a.in_stride[r] == 1 && a.dims[r] >= 64;
  if (variant == PERMUTE_TILED || (variant == PERMUTE_AUTO && small && !runs)) {
    PermuteTileArgs t;
    int ept = 0;
    const int esize = ct_in == CT_F64 || ct_out == CT_F64 ? 16 : 8;
    if (small && plan_tiled(a, esize, &t, &ept)) {
      if (ct_in == CT_F32 && ct_out == CT_F32) return launch_tiled<CT_F32, CT_F32>(t, ept, s);
      if (ct_in == CT_F64 && ct_out == CT_F64) return launch_tiled<CT_F64, CT_F64>(t, ept, s);
      if (ct_in == CT_F32 && ct_out == CT_F64) return launch_tiled<CT_F32, CT_F64>(t, ept, s);
      return launch_tiled<CT_F64, CT_F32>(t, ept, s);
    }
    if (variant == PERMUTE_TILED) return hipErrorInvalidValue;
  }
#define DCS_PERM(I, O)                                                      \
  if (ct_in == I && ct_out == O) {                                          \
    if (small)                                                              \
      hipLaunchKernelGGL((permute32_kernel<I, O>), grid, blk, 0, s, a);     \
    else                                                                    \
      hipLaunchKernelGGL((permute_kernel<I, O>), grid, blk, 0, s, a);       \
    return hipGetLastError();                                               \
  }
  DCS_PERM(CT_F32, CT_F32)
  DCS_PERM(CT_F64, CT_F64)
  DCS_PERM(CT_F32, CT_F64)
  DCS_PERM(CT_F64, CT_F32)
#undef DCS_PERM
  return hipErrorInvalidValue;
}

}  // namespace dcs
