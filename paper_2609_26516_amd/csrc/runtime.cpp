// Host runtime behind the C ABI: state layout in device memory, chunk
// compilation into layered site operators, and the launch sequences of the
// compression step, the measurement probability and the collapse.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <array>
#include <cstdio>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "dcs.h"
#include "dcs_internal.h"
#include "runtime_shared.h"

using namespace dcs;
using cd = std::complex<double>;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// Entry points return a status and never let a C++ exception (a failed host
// allocation inside a std container, say) cross the C ABI.
template <typename F>
int guarded(F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return fail(DCS_ENOMEM, "host allocation failed");
  } catch (...) {
    return fail(DCS_EINVAL, "internal error");
  }
}

#define DCS_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(DCS_EHIP, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
  } while (0)

#define DCS_TRY(expr)          \
  do {                         \
    int r_ = (expr);           \
    if (r_ != DCS_OK) return r_; \
  } while (0)

constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

int pow2_cap(int e, int cap) {  // min(cap, 2^e) without overflow
  if (e >= 30) return cap;
  return std::min(cap, 1 << e);
}

std::vector<int> bond_dims(int n, int chi) {
  std::vector<int> d(n + 1);
  for (int b = 0; b <= n; ++b) d[b] = std::min(pow2_cap(b, chi), pow2_cap(n - b, chi));
  return d;
}

// Complex128 workspace elements of one QR item with at most `emax` matrix
// elements and at most `dmax` columns (rows <= 2 dmax).
size_t qr_ws_elems(size_t emax, size_t dmax) {
  // the blocked kernel's, or the large and spread paths' (which small
  // batches take at any size)
  return std::max(emax + (dmax / 16 + 2) * 256, qr_large_ws_elems((int)(2 * dmax), (int)dmax));
}

int ctype_of(int precision) { return precision == DCS_C128 ? CT_F64 : CT_F32; }
size_t csize_of(int ct) { return ct == CT_F32 ? 8 : 16; }

}  // namespace

namespace dcs {
int testing_fail(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace dcs

// ---------------------------------------------------------------------------
// Opaque handles

struct Split {
  int r = 0;
  std::vector<cd> left;   // [s][t][w], 2*2*r
  std::vector<cd> right;  // [w][s][t], r*2*2
};

struct TuneRec {
  int best = -1;
  double ms[GEMM_VARIANTS] = {};    // fastest trial of each tile shape
  int cnt[GEMM_VARIANTS] = {};      // trials resolved
  int issued[GEMM_VARIANTS] = {};   // trials launched
};
using TuneKey = std::array<int, 10>;

struct dcs_ctx {
  int device = 0;
  bool graphs = false;
  bool capturing = false;
  // online autotuning of GEMM tile shapes: per shape class, the first launches
  // try every tile shape (timed with events) and the fastest is kept
  bool tuning = true;
  int tune_reps = 3;
  std::map<TuneKey, TuneRec> tune;
  struct TunePending {
    TuneKey key;
    int variant;
    hipEvent_t a, b;
  };
  std::vector<TunePending> tune_pending;
  std::unordered_map<std::string, Split> split_cache;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  bool timing = false;
  // > 0 while an entry point that must allocate nothing runs: tile shapes
  // come from the decided table or the default (no timed trials), and no
  // launch is timed (both would create events)
  int no_alloc = 0;
  struct Pending {
    int cls;
    hipEvent_t a, b;
    double flops, bytes;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> free_events;
  long long launches[DCS_TIMING_CLASSES] = {};
  double ms[DCS_TIMING_CLASSES] = {};
  double flops[DCS_TIMING_CLASSES] = {};
  double bytes[DCS_TIMING_CLASSES] = {};
};

struct dcs_chunk {
  int n = 0;
  std::vector<int> w;                 // n + 1 operator bond dims
  std::vector<std::vector<cd>> site;  // W_j[wl][s][t][wr]
};

namespace {

struct Slot {
  bool live = false;
  int chi_cap = 0;
  std::vector<int> dims;  // bond dims of the current tensors
  int cur = 0;            // which of the two MPS buffers holds them
  int lc_end = 0;         // sites < lc_end are left-orthonormal
  int rc_start = 0;       // sites >= rc_start are right-orthonormal
  int ecache_bond = -1;   // left transfer matrix at this bond is cached
  int measured_q = -1;
  double n0 = 0, n1 = 0;
};

struct InitSlot {
  int chi = 0;
};

struct Layout {
  int ct = CT_F64;
  size_t cs = 16;
  int n = 0, cap = 0, chi_max = 0, wmax = 0, n_init = 0;
  std::vector<int> D;            // maximal bond dims
  std::vector<size_t> site_off;  // site offsets inside one MPS buffer
  size_t mps_bytes = 0;
  std::vector<size_t> env_off;   // bond offsets inside the environment region
  // per-slot offsets
  size_t o_mps[2] = {0, 0}, o_env = 0, o_x1 = 0, o_x2 = 0, o_f = 0, o_ws = 0, o_e = 0, o_g = 0,
         o_tx = 0, o_ty = 0, slot_stride = 0;
  // global regions
  size_t o_slots = 0, o_mpo = 0, mpo_stride = 0, o_ids = 0, o_items = 0, o_out = 0, o_init = 0,
         total = 0;
  std::vector<size_t> mpo_site_off;
};

Layout make_layout(int precision, int n, int cap, int chi_max, int wmax, int n_init) {
  Layout L;
  L.ct = ctype_of(precision);
  L.cs = csize_of(L.ct);
  L.n = n;
  L.cap = cap;
  L.chi_max = chi_max;
  L.wmax = wmax;
  L.n_init = n_init;
  L.D = bond_dims(n, chi_max);
  size_t off = 0, xmax = 0, fmax = 0;
  for (int j = 0; j < n; ++j) {
    L.site_off.push_back(off);
    const size_t e = (size_t)L.D[j] * 2 * L.D[j + 1];
    off += align_up(e * L.cs);
    fmax = std::max(fmax, e);
    xmax = std::max(xmax, e * (size_t)wmax);
  }
  L.mps_bytes = off;
  size_t eoff = 0;
  for (int b = 0; b <= n; ++b) {
    L.env_off.push_back(eoff);
    const size_t wb = (b == 0 || b == n) ? 1 : (size_t)wmax;
    eoff += align_up((size_t)L.D[b] * wb * L.D[b] * L.cs);
  }
  size_t dmax = 0;
  for (int b = 0; b <= n; ++b) dmax = std::max(dmax, (size_t)L.D[b]);
  size_t p = 0;
  L.o_mps[0] = p;
  p += L.mps_bytes;
  L.o_mps[1] = p;
  p += L.mps_bytes;
  L.o_env = p;
  p += eoff;
  L.o_x1 = p;
  p += align_up(xmax * L.cs);
  L.o_x2 = p;
  p += align_up(xmax * L.cs);
  L.o_f = p;
  p += align_up(fmax * L.cs);
  L.o_ws = p;
  p += align_up(qr_ws_elems(fmax, dmax) * 16);
  L.o_e = p;
  p += align_up(dmax * dmax * 16);
  L.o_g = p;
  p += align_up(dmax * dmax * 16);
  L.o_tx = p;
  p += align_up(2 * dmax * dmax * 16);
  L.o_ty = p;
  p += align_up(2 * dmax * dmax * 16);
  L.slot_stride = align_up(p);

  size_t g = 0;
  L.o_slots = g;
  g += L.slot_stride * (size_t)cap;
  L.o_mpo = g;
  size_t moff = 0;
  for (int j = 0; j < n; ++j) {
    L.mpo_site_off.push_back(moff);
    const size_t wl = (j == 0) ? 1 : wmax, wr = (j == n - 1) ? 1 : wmax;
    moff += align_up(wl * 4 * wr * L.cs);
  }
  L.mpo_stride = align_up(moff);
  g += L.mpo_stride * (size_t)cap;
  L.o_ids = g;
  g += align_up(sizeof(int) * (size_t)cap * 2);
  L.o_items = g;
  g += align_up(std::max(sizeof(CollapseItem), sizeof(void*)) * (size_t)(cap * (n + 2)));
  L.o_out = g;
  g += align_up(sizeof(double) * 2 * (size_t)cap);
  L.o_init = g;
  g += L.mps_bytes * (size_t)n_init;
  L.total = g;
  return L;
}

}  // namespace

struct dcs_state {
  dcs_ctx* ctx = nullptr;
  int precision = DCS_C128;
  Layout L;
  char* base = nullptr;
  size_t bytes = 0;
  std::vector<Slot> slots;
  std::vector<InitSlot> inits;
  std::vector<char> host_stage;  // pinned-equivalent staging (pageable)
  // captured launch sequences of compression steps, keyed by their signature
  // (group shapes, slot ids, buffer parity, sweeps); a signature is captured
  // the second time it is seen and replayed afterwards
  std::map<std::string, hipGraphExec_t> graphs;
  std::map<std::string, int> graph_seen;
  // starting guess of compression steps: < 0 the registered generic guess;
  // >= 0 warm start, the ket itself plus this multiple of the generic guess
  double warm_eta = -1.0;
  hipStream_t capture_stream = nullptr;   // graphs are captured here, launched on the caller's
  // pinned host staging for uploads of calls that return without
  // synchronising: a ring of buffers, each reused once its last copy is done
  static constexpr int PIN_RING = 4;
  void* pin_buf[PIN_RING] = {};
  size_t pin_bytes[PIN_RING] = {};
  hipEvent_t pin_done[PIN_RING] = {};
  int pin_next = 0;

  ~dcs_state() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    for (int k = 0; k < PIN_RING; ++k) {
      if (pin_done[k]) {
        (void)hipEventSynchronize(pin_done[k]);
        (void)hipEventDestroy(pin_done[k]);
      }
      if (pin_buf[k]) (void)hipHostFree(pin_buf[k]);
    }
  }

  char* slot_base(int id) const { return base + L.o_slots + L.slot_stride * (size_t)id; }
  int init_index(int chi) const {
    for (size_t i = 0; i < inits.size(); ++i)
      if (inits[i].chi == chi) return (int)i;
    return -1;
  }
};

// ---------------------------------------------------------------------------
// Launch timing

namespace {

struct Timed {
  dcs_ctx* c;
  hipStream_t s;
  int cls;
  double flops, bytes;
  hipEvent_t a = nullptr;
  Timed(dcs_ctx* c_, hipStream_t s_, int cls_, double f, double b)
      : c(c_), s(s_), cls(cls_), flops(f), bytes(b) {
    if (!c || !c->timing || c->no_alloc) return;
    a = take();
    (void)hipEventRecord(a, s);
  }
  hipEvent_t take() {
    if (!c->free_events.empty()) {
      hipEvent_t e = c->free_events.back();
      c->free_events.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  ~Timed() {
    if (!a) return;
    hipEvent_t b = take();
    (void)hipEventRecord(b, s);
    c->pending.push_back({cls, a, b, flops, bytes});
  }
};

void resolve_timing(dcs_ctx* c) {
  for (auto& p : c->pending) {
    (void)hipEventSynchronize(p.b);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, p.a, p.b);
    c->launches[p.cls] += 1;
    c->ms[p.cls] += ms;
    c->flops[p.cls] += p.flops;
    c->bytes[p.cls] += p.bytes;
    c->free_events.push_back(p.a);
    c->free_events.push_back(p.b);
  }
  c->pending.clear();
}

// timing classes: contraction GEMMs of the compression step by operand form
// (N N, N T, C N, J T), gate-operator application, QR, measurement, other
enum { CLS_GEMM = 0, CLS_MPO = 4, CLS_QR = 5, CLS_MEAS = 6, CLS_OTHER = 7 };

int gemm_class(int opa, int opb) {
  if (opa == OP_N && opb == OP_N) return 0;
  if (opa == OP_N && opb == OP_T) return 1;
  if (opa == OP_C && opb == OP_N) return 2;
  return 3;
}

// ---------------------------------------------------------------------------
// Batched launch builders

Operand slot_op(const dcs_state* st, size_t region_off, size_t extra) {
  Operand o;
  o.base = st->base + st->L.o_slots + region_off + extra;
  o.stride = (long long)st->L.slot_stride;
  o.by_slot = 1;
  o.pad_ = 0;
  return o;
}
Operand local_op(const void* base, long long stride) {
  Operand o;
  o.base = base;
  o.stride = stride;
  o.by_slot = 0;
  o.pad_ = 0;
  return o;
}

using GemmJob = rt::GemmJob;

int lg2_bucket(long long x) {
  int b = 0;
  while ((1LL << b) < x && b < 40) ++b;
  return b;
}

hipEvent_t take_event(dcs_ctx* c) {
  if (!c->free_events.empty()) {
    hipEvent_t e = c->free_events.back();
    c->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Tile shape for a shape class; *timed set when this launch is a tuning trial.
int tune_choose(dcs_ctx* c, const TuneKey& key, bool* timed) {
  *timed = false;
  auto it = c->tune.find(key);
  if (it != c->tune.end() && it->second.best >= 0) return it->second.best;
  const bool small = key[6] <= 5 && key[7] <= 5;   // M, N <= 32
  const int fallback = small ? GEMM_32x32 : GEMM_64x64;
  if (!c->tuning || c->capturing || c->no_alloc) return fallback;
  TuneRec& r = c->tune[key];
  const int nv = gemm_variants(key[3]);
  int v = 0;
  for (int i = 1; i < nv; ++i)
    if (r.issued[i] < r.issued[v]) v = i;
  if (r.issued[v] >= c->tune_reps) return fallback;   // all trials in flight
  r.issued[v] += 1;
  *timed = true;
  return v;
}

void tune_resolve(dcs_ctx* c) {
  for (auto& p : c->tune_pending) {
    (void)hipEventSynchronize(p.b);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, p.a, p.b);
    TuneRec& r = c->tune[p.key];
    r.ms[p.variant] = r.cnt[p.variant] ? std::min(r.ms[p.variant], (double)ms) : ms;
    r.cnt[p.variant] += 1;
    const int nv = gemm_variants(p.key[3]);
    bool done = true;
    for (int i = 0; i < nv; ++i) done = done && r.cnt[i] >= c->tune_reps;
    if (done && r.best < 0) {
      int b = 0;
      for (int i = 1; i < nv; ++i)
        if (r.ms[i] < r.ms[b]) b = i;
      r.best = b;
    }
    c->free_events.push_back(p.a);
    c->free_events.push_back(p.b);
  }
  c->tune_pending.clear();
}

int run_gemm(dcs_ctx* ctx, int ta, int tb, int tc, int tacc, int opa, int opb,
             const std::vector<GemmJob>& jobs, hipStream_t s, int cls) {
  size_t i = 0;
  while (i < jobs.size()) {
    // jobs of this launch and the shape class of the largest one
    size_t j_end = i;
    int ng = 0;
    long long big = -1;
    TuneKey key{};
    const int epi = jobs[i].epi;   // one epilogue per launch
    for (; j_end < jobs.size() && ng < GEMM_MAX_GROUPS && jobs[j_end].epi == epi; ++j_end) {
      const GemmJob& j = jobs[j_end];
      if (j.batch <= 0 || j.M <= 0 || j.N <= 0) continue;
      ++ng;
      const long long w = (long long)j.M * j.N * j.batch;
      if (w > big) {
        big = w;
        key = {ta, tb, tc, tacc, opa + 4 * epi, opb, lg2_bucket(j.M), lg2_bucket(j.N),
               lg2_bucket(j.K), lg2_bucket(j.batch)};
      }
    }
    if (ng == 0) {
      i = j_end;
      continue;
    }
    bool timed = false;
    const int variant = tune_choose(ctx, key, &timed);
    int bm = 64, bn = 64;
    gemm_tile_shape(variant, &bm, &bn);
    GemmArgs args;
    std::memset(&args, 0, sizeof(args));
    ng = 0;
    int tiles = 0;
    double flops = 0, bytes = 0;
    const double es = (ta == CT_F32 ? 8.0 : 16.0);
    for (; i < j_end; ++i) {
      const GemmJob& j = jobs[i];
      if (j.batch <= 0 || j.M <= 0 || j.N <= 0) continue;
      GemmGroup& g = args.g[ng++];
      g.a = j.a;
      g.b = j.b;
      g.c = j.c;
      g.ids = j.ids;
      g.M = j.M;
      g.N = j.N;
      g.K = j.K;
      g.lda = j.lda;
      g.ldb = j.ldb;
      g.ldc = j.ldc;
      g.batch = j.batch;
      g.w = j.w;
      g.wl = j.wl;
      g.wr = j.wr;
      // the right epilogue's tiles hold columns (0, y) and (1, y) for bn / 2 values of y
      g.tiles_n = epi == GEMM_EPI_RIGHT ? (j.N / 2 + bn / 2 - 1) / (bn / 2) : (j.N + bn - 1) / bn;
      g.tiles_per_item = ((j.M + bm - 1) / bm) * g.tiles_n;
      g.herm = j.herm && j.M == j.N && bm == bn && epi == GEMM_EPI_NONE && tacc != ACC_BF16X3;
      double part = 1.0;   // share of the product's tiles computed
      if (g.herm) {
        g.tiles_per_item = g.tiles_n * (g.tiles_n + 1) / 2;
        part = (double)g.tiles_per_item / ((double)g.tiles_n * g.tiles_n);
      }
      g.tile_begin = tiles;
      tiles += g.tiles_per_item * j.batch;
      flops += 8.0 * j.M * j.N * (double)j.K * j.batch * part;
      bytes += es * ((double)j.M * j.K + (double)j.K * j.N + (double)j.M * j.N) * j.batch;
      if (epi != GEMM_EPI_NONE)   // operator: 8 (2 wl)(2 wr) flops per (row, column) group
        flops += 8.0 * (2.0 * j.wl) * (2.0 * j.wr) * j.batch *
                 (epi == GEMM_EPI_RIGHT ? (double)(j.M / j.wl) * (j.N / 2)
                                        : (double)(j.M / 2) * (j.N / j.wr));
    }
    args.ngroups = ng;
    args.total_tiles = tiles;
    args.epi = epi;
    hipEvent_t ta_ev = nullptr, tb_ev = nullptr;
    if (timed) {
      ta_ev = take_event(ctx);
      tb_ev = take_event(ctx);
      (void)hipEventRecord(ta_ev, s);
    }
    {
      Timed t(ctx, s, cls == CLS_GEMM ? gemm_class(opa, opb) : cls, flops, bytes);
      DCS_HIP(launch_gemm(ta, tb, tc, tacc, opa, opb, variant, args, s));
    }
    if (timed) {
      (void)hipEventRecord(tb_ev, s);
      ctx->tune_pending.push_back({key, variant, ta_ev, tb_ev});
    }
  }
  return DCS_OK;
}

struct MpoJob {
  Operand in, out, w;
  const int* ids;
  int d0, d1, wl, wr, batch;
};

int run_mpo(dcs_ctx* ctx, int ct, int dir, const std::vector<MpoJob>& jobs, hipStream_t s) {
  size_t i = 0;
  while (i < jobs.size()) {
    MpoArgs args;
    std::memset(&args, 0, sizeof(args));
    int ng = 0, blocks = 0;
    double flops = 0, bytes = 0;
    const double es = (ct == CT_F32 ? 8.0 : 16.0);
    for (; i < jobs.size() && ng < MPO_MAX_GROUPS; ++i) {
      const MpoJob& j = jobs[i];
      if (j.batch <= 0) continue;
      MpoGroup& g = args.g[ng++];
      g.in = j.in;
      g.out = j.out;
      g.w = j.w;
      g.ids = j.ids;
      g.d0 = j.d0;
      g.d1 = j.d1;
      g.wl = j.wl;
      g.wr = j.wr;
      g.batch = j.batch;
      g.blk_per_item = (int)(((long long)j.d0 * j.d1 + 255) / 256);
      g.blk_begin = blocks;
      blocks += g.blk_per_item * j.batch;
      const double pairs = (double)j.d0 * j.d1 * j.batch;
      flops += pairs * 8.0 * (2.0 * j.wl) * (2.0 * j.wr);
      bytes += pairs * es * (2.0 * j.wl + 2.0 * j.wr);
    }
    if (ng == 0) continue;
    args.ngroups = ng;
    args.total_blocks = blocks;
    Timed t(ctx, s, CLS_MPO, flops, bytes);
    DCS_HIP(launch_mpo(ct, dir, args, s));
  }
  return DCS_OK;
}

using QrJob = rt::QrJob;

// Path of a QR job: 0 blocked single-workgroup kernel, left-looking form
// (m <= 512 or mode 2), 3 the spread path for the same matrices when `spread`
// (see run_qr), 1 multi-kernel large-matrix path, 2 unblocked kernel (beyond
// both).
int qr_path(const QrJob& j, bool spread) {
  if (j.mode == 2) return 0;
  if (j.m <= qr_blocked_max_rows()) return spread && j.m >= j.n ? 3 : 0;
  return j.m <= qr_large_max_rows() ? 1 : 2;
}

int run_qr(dcs_ctx* ctx, int ct_in, int ct_out, const std::vector<QrJob>& all, hipStream_t s) {
  // A call with few matrices of up to 512 rows leaves most of the chip idle
  // under one workgroup per matrix; when its largest matrix is big enough for
  // that to matter (more than 128 rows, at least 64 columns) its QRs take the
  // spread path, whose updates run over many workgroups.  Its strip updates
  // read and write the trailing matrix once per panel, so it stops paying off
  // as the batch grows (512 x 256: 0.96 against 1.78 ms for 8 matrices, 2.05
  // against 2.36 ms for 64; 192 x 96: 0.32 against 0.36 ms for 64; 128 x 64:
  // 0.155 against 0.136 ms for 16, where the blocked kernel runs four waves per
  // matrix).
  int items = 0, m_big = 0, n_big = 0;
  for (const QrJob& j : all)
    if (j.batch > 0 && j.mode != 2 && j.m <= qr_blocked_max_rows()) {
      items += j.batch;
      m_big = std::max(m_big, j.m);
      n_big = std::max(n_big, j.n);
    }
  const bool spread = items <= qr_spread_max_items() && m_big > 128 && n_big >= 64;
  for (int path : {0, 3, 1, 2}) {
    std::vector<QrJob> jobs;
    for (const QrJob& j : all)
      if (j.batch > 0 && qr_path(j, spread) == path) jobs.push_back(j);
    size_t i = 0;
    while (i < jobs.size()) {
      QrArgs args;
      std::memset(&args, 0, sizeof(args));
      int ng = 0, blocks = 0;
      size_t lds = 0;
      double flops = 0, bytes = 0;
      for (; i < jobs.size() && ng < QR_MAX_GROUPS; ++i) {
        const QrJob& j = jobs[i];
        QrGroup& g = args.g[ng++];
        g.f = j.f;
        g.q = j.q;
        g.ws = j.ws;
        g.nrm2 = j.nrm2;
        g.ids = j.ids;
        g.m = j.m;
        g.n = j.n;
        g.mode = j.mode;
        g.batch = j.batch;
        g.blk_begin = blocks;
        blocks += j.batch;
        if (j.mode != 2) lds = std::max(lds, (size_t)j.m * j.n * 16);
        const double m = j.m, n = j.n;
        // Householder factorisation + explicit thin Q (complex flops x 8)
        if (j.mode != 2) flops += 8.0 * (2.0 * m * n * n - 2.0 * n * n * n / 3.0) * j.batch;
        bytes += (m * n * (csize_of(ct_in) + csize_of(ct_out))) * j.batch;
      }
      args.ngroups = ng;
      args.total_blocks = blocks;
      int m_max = 0;
      for (int g = 0; g < ng; ++g) m_max = std::max(m_max, args.g[g].mode == 2 ? 0 : args.g[g].m);
      Timed t(ctx, s, CLS_QR, flops, bytes);
      if (path == 0) {
        args.use_lds = 1;
        // fewer matrices than about 5/8 of the CUs: factorisations and Q blocks
        // in separate launches so the Q blocks spread over the chip
        DCS_HIP(launch_qr_left(ct_in, ct_out, args, std::max(m_max, 1),
                               args.total_blocks <= qr_split_max_items(), s));
      } else if (path == 3) {
        DCS_HIP(launch_qr_spread(ct_in, ct_out, args, s));
      } else if (path == 1) {
        DCS_HIP(launch_qr_large(ct_in, ct_out, args, s));
      } else {
        args.use_lds = (lds > 0 && lds <= qr_lds_limit()) ? 1 : 0;
        DCS_HIP(launch_qr(ct_in, ct_out, args, args.use_lds ? lds : 0, s));
      }
    }
  }
  return DCS_OK;
}

struct NormJob {
  Operand a, z, out;
  const int* ids;
  int dl, dr, batch;
};

int run_norms(dcs_ctx* ctx, int ct_a, int ct_z, const std::vector<NormJob>& jobs, hipStream_t s) {
  size_t i = 0;
  while (i < jobs.size()) {
    NormArgs args;
    std::memset(&args, 0, sizeof(args));
    int ng = 0, blocks = 0;
    for (; i < jobs.size() && ng < NORM_MAX_GROUPS; ++i) {
      const NormJob& j = jobs[i];
      if (j.batch <= 0) continue;
      NormGroup& g = args.g[ng++];
      g.a = j.a;
      g.z = j.z;
      g.out = j.out;
      g.ids = j.ids;
      g.dl = j.dl;
      g.dr = j.dr;
      g.batch = j.batch;
      g.blk_begin = blocks;
      blocks += j.batch;
    }
    if (ng == 0) continue;
    args.ngroups = ng;
    args.total_blocks = blocks;
    Timed t(ctx, s, CLS_MEAS, 0, 0);
    DCS_HIP(launch_norms(ct_a, ct_z, args, s));
  }
  return DCS_OK;
}

// ---------------------------------------------------------------------------
// Argument checks

int check_ids(const dcs_state* st, int n, const int* ids, bool need_live) {
  if (n < 0 || (n > 0 && !ids)) return fail(DCS_EINVAL, "null id array");
  std::vector<char> seen(st->L.cap, 0);
  for (int i = 0; i < n; ++i) {
    const int id = ids[i];
    if (id < 0 || id >= st->L.cap)
      return fail(DCS_ECAPACITY, "branch id " + std::to_string(id) + " outside capacity");
    if (seen[id]) return fail(DCS_EINVAL, "duplicate branch id " + std::to_string(id));
    seen[id] = 1;
    if (need_live && !st->slots[id].live)
      return fail(DCS_ESTATE, "branch " + std::to_string(id) + " is not live");
  }
  return DCS_OK;
}

template <typename T>
void to_path(const cd* src, size_t count, void* dst);
template <>
void to_path<float2>(const cd* src, size_t count, void* dst) {
  float2* d = static_cast<float2*>(dst);
  for (size_t i = 0; i < count; ++i) d[i] = make_float2((float)src[i].real(), (float)src[i].imag());
}
template <>
void to_path<double2>(const cd* src, size_t count, void* dst) {
  double2* d = static_cast<double2*>(dst);
  for (size_t i = 0; i < count; ++i) d[i] = make_double2(src[i].real(), src[i].imag());
}
void to_path_ct(int ct, const cd* src, size_t count, void* dst) {
  if (ct == CT_F32)
    to_path<float2>(src, count, dst);
  else
    to_path<double2>(src, count, dst);
}

// ---------------------------------------------------------------------------
// Two-qubit gate split by a one-sided (Hestenes) Jacobi SVD of the 4 x 4
// operator-Schmidt matrix M[(s t), (s' t')] = G[(s s'), (t t')].

Split split_gate(const double* g) {
  cd M[4][4], V[4][4];
  for (int s = 0; s < 2; ++s)
    for (int sp = 0; sp < 2; ++sp)
      for (int t = 0; t < 2; ++t)
        for (int tp = 0; tp < 2; ++tp) {
          const int row = s * 2 + sp, col = t * 2 + tp;
          M[s * 2 + t][sp * 2 + tp] = cd(g[2 * (row * 4 + col)], g[2 * (row * 4 + col) + 1]);
        }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0;
    for (int p = 0; p < 3; ++p)
      for (int q = p + 1; q < 4; ++q) {
        double al = 0, be = 0;
        cd ga = 0;
        for (int i = 0; i < 4; ++i) {
          al += std::norm(M[i][p]);
          be += std::norm(M[i][q]);
          ga += std::conj(M[i][p]) * M[i][q];
        }
        const double ag = std::abs(ga);
        if (ag == 0.0 || ag <= 1e-16 * std::sqrt(al * be)) continue;
        off = std::max(off, ag / std::sqrt(al * be));
        const double zeta = (be - al) / (2.0 * ag);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        const cd ph = std::conj(ga / ag);
        for (int i = 0; i < 4; ++i) {
          const cd ap = M[i][p], aq = M[i][q] * ph;
          M[i][p] = c * ap - s * aq;
          M[i][q] = s * ap + c * aq;
          const cd vp = V[i][p], vq = V[i][q] * ph;
          V[i][p] = c * vp - s * vq;
          V[i][q] = s * vp + c * vq;
        }
      }
    if (off < 1e-15) break;
  }
  double sig[4];
  int order[4] = {0, 1, 2, 3};
  for (int k = 0; k < 4; ++k) {
    double a = 0;
    for (int i = 0; i < 4; ++i) a += std::norm(M[i][k]);
    sig[k] = std::sqrt(a);
  }
  std::stable_sort(order, order + 4, [&](int a, int b) { return sig[a] > sig[b]; });
  Split sp;
  const double smax = sig[order[0]];
  for (int k = 0; k < 4; ++k)
    if (sig[order[k]] > 1e-14 * smax) sp.r++;
  if (sp.r == 0) sp.r = 1;
  sp.left.assign(4 * sp.r, 0.0);
  sp.right.assign(4 * sp.r, 0.0);
  for (int w = 0; w < sp.r; ++w) {
    const int k = order[w];
    for (int st = 0; st < 4; ++st) sp.left[st * sp.r + w] = M[st][k];
    for (int st = 0; st < 4; ++st) sp.right[w * 4 + st] = std::conj(V[st][k]);
  }
  return sp;
}

// Product of site operators: `later` applied after `earlier`; combined bond
// index (earlier, later) with the earlier one most significant.
std::vector<cd> op_product(const std::vector<cd>& earlier, int el, int er,
                           const std::vector<cd>& later, int ll, int lr) {
  const int wl = el * ll, wr = er * lr;
  std::vector<cd> out((size_t)wl * 4 * wr, 0.0);
  for (int x = 0; x < el; ++x)
    for (int w = 0; w < ll; ++w)
      for (int s = 0; s < 2; ++s)
        for (int t = 0; t < 2; ++t)
          for (int y = 0; y < er; ++y)
            for (int v = 0; v < lr; ++v) {
              cd acc = 0;
              for (int u = 0; u < 2; ++u)
                acc += later[((w * 2 + s) * 2 + u) * lr + v] * earlier[((x * 2 + u) * 2 + t) * er + y];
              out[(((size_t)(x * ll + w) * 2 + s) * 2 + t) * wr + (y * lr + v)] = acc;
            }
  return out;
}

}  // namespace

// ---------------------------------------------------------------------------
// Fixed device scratch of dcs_overlap_noalloc: the FP64 left transfer E_j
// (at most 256 x 256 complex128) and the product TX = E_j B_j (at most
// 256 x 512) of the overlap contraction.  One copy per device, for the life
// of the process; its device address is looked up once per device (the
// array's name is only a host-side stand-in).

namespace {

constexpr size_t OVL_E_BYTES = (size_t)256 * 256 * 16;
constexpr size_t OVL_TX_BYTES = (size_t)256 * 512 * 16;
constexpr size_t OVL_SCRATCH_BYTES = OVL_E_BYTES + OVL_TX_BYTES;
static __device__ __align__(256) char scratch[OVL_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on `device` (made current by the caller).
int scratch_setup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return fail(DCS_EINVAL, "device ordinal too large");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return DCS_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(DCS_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") +
                              hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
  return DCS_OK;
}

void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (device >= 0 && device < MAX_DEVICES) ? g_scratch_ptr[device] : nullptr;
}

}  // namespace

// ===========================================================================
// C ABI

extern "C" {

const char* dcs_last_error(void) { return g_err.c_str(); }

int dcs_version(void) { return 100; }

int dcs_ctx_create(dcs_ctx** out, int device) {
  return guarded([&]() -> int {
    if (!out) return fail(DCS_EINVAL, "null output handle");
    int count = 0;
    DCS_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(DCS_EINVAL, "device ordinal out of range");
    DCS_HIP(hipSetDevice(device));
    DCS_TRY(scratch_setup(device));
    dcs_ctx* c = new dcs_ctx();
    c->device = device;
    *out = c;
    return DCS_OK;
  });
}

int dcs_ctx_destroy(dcs_ctx* ctx) {
  return guarded([&]() -> int {
    if (!ctx) return DCS_OK;
    resolve_timing(ctx);
    tune_resolve(ctx);
    for (hipEvent_t e : ctx->free_events) (void)hipEventDestroy(e);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
    return DCS_OK;
  });
}

int dcs_ctx_set_tuning(dcs_ctx* ctx, int enabled, int reps) {
  return guarded([&]() -> int {
    if (!ctx) return fail(DCS_EINVAL, "null context");
    if (reps < 1 || reps > 100) return fail(DCS_EINVAL, "reps must be in [1, 100]");
    ctx->tuning = enabled != 0;
    ctx->tune_reps = reps;
    return DCS_OK;
  });
}

int dcs_ctx_tuning_save(dcs_ctx* ctx, const char* path) {
  return guarded([&]() -> int {
    if (!ctx || !path) return fail(DCS_EINVAL, "null argument");
    tune_resolve(ctx);
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(DCS_EINVAL, std::string("cannot write ") + path);
    std::fprintf(f, "{\"format\": \"dcs-gemm-tiles-1\", \"entries\": [");
    bool first = true;
    for (auto& kv : ctx->tune) {
      if (kv.second.best < 0) continue;
      std::fprintf(f, "%s\n  {\"key\": [", first ? "" : ",");
      for (int i = 0; i < 10; ++i) std::fprintf(f, "%s%d", i ? ", " : "", kv.first[i]);
      std::fprintf(f, "], \"best\": %d, \"ms\": [", kv.second.best);
      for (int i = 0; i < GEMM_VARIANTS; ++i)
        std::fprintf(f, "%s%.6g", i ? ", " : "", kv.second.cnt[i] ? kv.second.ms[i] : -1.0);
      std::fprintf(f, "]}");
      first = false;
    }
    std::fprintf(f, "\n]}\n");
    std::fclose(f);
    return DCS_OK;
  });
}

int dcs_ctx_tuning_load(dcs_ctx* ctx, const char* path) {
  return guarded([&]() -> int {
    if (!ctx || !path) return fail(DCS_EINVAL, "null argument");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(DCS_EINVAL, std::string("cannot read ") + path);
    std::string txt;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, got);
    std::fclose(f);
    if (txt.find("dcs-gemm-tiles-1") == std::string::npos)
      return fail(DCS_EINVAL, "not a tile-shape table");
    size_t pos = 0;
    while ((pos = txt.find("\"key\": [", pos)) != std::string::npos) {
      pos += 8;
      TuneKey k{};
      int best = -1;
      const char* c = txt.c_str() + pos;
      int used = 0;
      if (std::sscanf(c, "%d, %d, %d, %d, %d, %d, %d, %d, %d, %d], \"best\": %d%n", &k[0], &k[1],
                      &k[2], &k[3], &k[4], &k[5], &k[6], &k[7], &k[8], &k[9], &best, &used) != 11)
        return fail(DCS_EINVAL, "malformed tile-shape entry");
      if (best < 0 || best >= gemm_variants(k[3])) return fail(DCS_EINVAL, "bad tile shape id");
      ctx->tune[k].best = best;
      pos += used;
    }
    return DCS_OK;
  });
}

int dcs_ctx_set_graphs(dcs_ctx* ctx, int enabled) {
  return guarded([&]() -> int {
    if (!ctx) return fail(DCS_EINVAL, "null context");
    ctx->graphs = enabled != 0;
    return DCS_OK;
  });
}

int dcs_ctx_set_timing(dcs_ctx* ctx, int enabled) {
  return guarded([&]() -> int {
    if (!ctx) return fail(DCS_EINVAL, "null context");
    ctx->timing = enabled != 0;
    return DCS_OK;
  });
}

int dcs_ctx_timing(dcs_ctx* ctx, long long* launches, double* ms, double* flops, double* bytes,
                   int reset) {
  return guarded([&]() -> int {
    if (!ctx) return fail(DCS_EINVAL, "null context");
    resolve_timing(ctx);
    for (int i = 0; i < DCS_TIMING_CLASSES; ++i) {
      if (launches) launches[i] = ctx->launches[i];
      if (ms) ms[i] = ctx->ms[i];
      if (flops) flops[i] = ctx->flops[i];
      if (bytes) bytes[i] = ctx->bytes[i];
      if (reset) {
        ctx->launches[i] = 0;
        ctx->ms[i] = ctx->flops[i] = ctx->bytes[i] = 0;
      }
    }
    return DCS_OK;
  });
}

static int check_state_args(int precision, int n, int cap, int chi_max, int wmax, int n_init) {
  if (precision != DCS_C128 && precision != DCS_C64 && precision != DCS_BF16X3)
    return fail(DCS_EINVAL, "unknown precision");
  if (n < 1 || n > 4096) return fail(DCS_EINVAL, "n_qubits out of range");
  if (cap < 1) return fail(DCS_EINVAL, "capacity must be positive");
  if (chi_max < 1 || chi_max > 1024) return fail(DCS_EINVAL, "chi_max must be in [1, 1024]");
  if (wmax < 1 || wmax > 16) return fail(DCS_EINVAL, "mpo_bond_max must be in [1, 16]");
  if (n_init < 1) return fail(DCS_EINVAL, "n_init_slots must be positive");
  return DCS_OK;
}

int dcs_state_bytes(int precision, int n_qubits, int capacity, int chi_max, int mpo_bond_max,
                    int n_init_slots, size_t* bytes_out) {
  return guarded([&]() -> int {
    DCS_TRY(check_state_args(precision, n_qubits, capacity, chi_max, mpo_bond_max, n_init_slots));
    if (!bytes_out) return fail(DCS_EINVAL, "null output");
    *bytes_out = make_layout(precision, n_qubits, capacity, chi_max, mpo_bond_max, n_init_slots).total;
    return DCS_OK;
  });
}

int dcs_state_create(dcs_ctx* ctx, dcs_state** out, int precision, int n_qubits, int capacity,
                     int chi_max, int mpo_bond_max, int n_init_slots, void* d_buffer, size_t bytes,
                     void* stream) {
  return guarded([&]() -> int {
    if (!ctx || !out) return fail(DCS_EINVAL, "null handle");
    DCS_TRY(check_state_args(precision, n_qubits, capacity, chi_max, mpo_bond_max, n_init_slots));
    Layout L = make_layout(precision, n_qubits, capacity, chi_max, mpo_bond_max, n_init_slots);
    if (!d_buffer) return fail(DCS_EINVAL, "null device buffer");
    if (reinterpret_cast<uintptr_t>(d_buffer) % ALIGN != 0)
      return fail(DCS_EINVAL, "device buffer must be 256-byte aligned");
    if (bytes < L.total)
      return fail(DCS_ENOMEM, "device buffer too small: need " + std::to_string(L.total) + " bytes");
    DCS_HIP(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    dcs_state* st = new dcs_state();
    st->ctx = ctx;
    st->precision = precision;
    st->L = L;
    st->base = static_cast<char*>(d_buffer);
    st->bytes = bytes;
    st->slots.assign(capacity, Slot());
    // boundary environments L_0 = R_n = [[1]] of every slot (never overwritten)
    std::vector<void*> ptrs;
    for (int id = 0; id < capacity; ++id) {
      char* sb = st->slot_base(id);
      ptrs.push_back(sb + L.o_env + L.env_off[0]);
      ptrs.push_back(sb + L.o_env + L.env_off[n_qubits]);
    }
    size_t done = 0;
    const size_t chunk_ptrs = (size_t)capacity * (n_qubits + 2);
    while (done < ptrs.size()) {
      const size_t cnt = std::min(chunk_ptrs, ptrs.size() - done);
      void** dptr = reinterpret_cast<void**>(st->base + L.o_items);
      hipError_t e = hipMemcpyAsync(dptr, ptrs.data() + done, cnt * sizeof(void*),
                                    hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = launch_fill_unit(L.ct, dptr, (int)cnt, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        delete st;
        return fail(DCS_EHIP, std::string("state set-up failed: ") + hipGetErrorString(e));
      }
      done += cnt;
    }
    *out = st;
    return DCS_OK;
  });
}

int dcs_state_destroy(dcs_state* st) {
  return guarded([&]() -> int {
    delete st;
    return DCS_OK;
  });
}

int dcs_state_set_init(dcs_state* st, int chi_cap, const double* gauss, void* stream) {
  return guarded([&]() -> int {
    if (!st || !gauss) return fail(DCS_EINVAL, "null argument");
    const Layout& L = st->L;
    if (chi_cap < 1 || chi_cap > L.chi_max) return fail(DCS_EINVAL, "chi_cap outside [1, chi_max]");
    int idx = st->init_index(chi_cap);
    const bool fresh = idx < 0;
    if (fresh) {
      if ((int)st->inits.size() >= L.n_init)
        return fail(DCS_ENOMEM, "all starting-guess slots are in use");
      idx = (int)st->inits.size();
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int n = L.n;
    const std::vector<int> d = bond_dims(n, chi_cap);
    std::vector<size_t> goff(n);
    size_t total = 0, emax = 0;
    for (int j = 0; j < n; ++j) {
      goff[j] = total;
      const size_t e = (size_t)d[j] * 2 * d[j + 1];
      total += e;
      emax = std::max(emax, e);
    }
    // Scratch from the state's own buffer: site j of a launch group uses the
    // per-call contraction area (x1 and x2, contiguous) of slot i = j - j0
    // for its FP64 Gaussian and that slot's QR workspace; |G|^2 goes to the
    // call output area.  None of these hold anything between calls, so live
    // branches are unaffected.  Their sizes come from chi_max >= chi_cap (the
    // QR matrices have at most 2 dmx rows and dmx columns).
    const size_t dmx = (size_t)*std::max_element(d.begin(), d.end());
    if (emax * 16 > L.o_f - L.o_x1 || qr_ws_elems(emax, dmx) * 16 > L.o_e - L.o_ws)
      return fail(DCS_ENOMEM, "internal: slot scratch too small for the starting guess");
    const int per_launch = std::min(L.cap, QR_MAX_GROUPS);
    double* nrm_dev = reinterpret_cast<double*>(st->base + L.o_out);
    char* ibase = st->base + L.o_init + L.mps_bytes * (size_t)idx;
    for (int j0 = 0; j0 < n; j0 += per_launch) {
      std::vector<QrJob> jobs;
      for (int j = j0; j < std::min(n, j0 + per_launch); ++j) {
        char* sb = st->slot_base(j - j0);
        const size_t e = (size_t)d[j] * 2 * d[j + 1];
        DCS_HIP(hipMemcpyAsync(sb + L.o_x1, gauss + 2 * goff[j], e * 16, hipMemcpyHostToDevice, s));
        QrJob q;
        q.f = local_op(sb + L.o_x1, 0);
        q.q = local_op(ibase + L.site_off[j], 0);
        q.ws = local_op(sb + L.o_ws, 0);
        q.nrm2 = local_op(nrm_dev + (j - j0), 0);
        q.ids = nullptr;
        q.batch = 1;
        if (j == 0) {
          q.m = d[0] * 2 * d[1];
          q.n = 1;
          q.mode = 2;
        } else {
          q.m = 2 * d[j + 1];
          q.n = d[j];
          q.mode = 1;
        }
        jobs.push_back(q);
      }
      DCS_TRY(run_qr(st->ctx, CT_F64, L.ct, jobs, s));
    }
    DCS_HIP(hipStreamSynchronize(s));
    // the bond cap is usable only once its guess is complete
    if (fresh) st->inits.push_back(InitSlot{chi_cap});
    return DCS_OK;
  });
}

int dcs_branch_init_zero(dcs_state* st, int n, const int* ids, const int* chi_caps, void* stream) {
  return guarded([&]() -> int {
    if (!st) return fail(DCS_EINVAL, "null state");
    DCS_TRY(check_ids(st, n, ids, false));
    if (n > 0 && !chi_caps) return fail(DCS_EINVAL, "null chi_caps");
    const Layout& L = st->L;
    for (int i = 0; i < n; ++i)
      if (chi_caps[i] < 1 || chi_caps[i] > L.chi_max)
        return fail(DCS_EINVAL, "chi cap outside [1, chi_max]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // |0...0> with unit bonds: every site tensor is the 1 x 2 x 1 vector (1, 0)
    std::vector<void*> ptrs;
    for (int i = 0; i < n; ++i) {
      char* mps = st->slot_base(ids[i]) + L.o_mps[0];
      for (int j = 0; j < L.n; ++j) ptrs.push_back(mps + L.site_off[j]);
    }
    size_t done = 0;
    const size_t room = (size_t)L.cap * (L.n + 2);
    while (done < ptrs.size()) {
      const size_t cnt = std::min(room, ptrs.size() - done);
      void** dptr = reinterpret_cast<void**>(st->base + L.o_items);
      DCS_HIP(hipMemcpyAsync(dptr, ptrs.data() + done, cnt * sizeof(void*), hipMemcpyHostToDevice, s));
      DCS_HIP(launch_fill_unit(L.ct, dptr, (int)cnt, s));
      DCS_HIP(hipStreamSynchronize(s));
      done += cnt;
    }
    for (int i = 0; i < n; ++i) {
      Slot& sl = st->slots[ids[i]];
      sl = Slot();
      sl.live = true;
      sl.chi_cap = chi_caps[i];
      sl.dims.assign(L.n + 1, 1);
      sl.cur = 0;
      sl.lc_end = L.n;
      sl.rc_start = 0;
    }
    return DCS_OK;
  });
}

int dcs_branch_set_chi(dcs_state* st, int n, const int* ids, const int* chi_caps) {
  return guarded([&]() -> int {
    if (!st) return fail(DCS_EINVAL, "null state");
    DCS_TRY(check_ids(st, n, ids, true));
    for (int i = 0; i < n; ++i)
      if (!chi_caps || chi_caps[i] < 1 || chi_caps[i] > st->L.chi_max)
        return fail(DCS_EINVAL, "chi cap outside [1, chi_max]");
    for (int i = 0; i < n; ++i) st->slots[ids[i]].chi_cap = chi_caps[i];
    return DCS_OK;
  });
}

int dcs_branch_release(dcs_state* st, int n, const int* ids) {
  return guarded([&]() -> int {
    if (!st) return fail(DCS_EINVAL, "null state");
    DCS_TRY(check_ids(st, n, ids, false));
    for (int i = 0; i < n; ++i) st->slots[ids[i]] = Slot();
    return DCS_OK;
  });
}

int dcs_branch_dims(const dcs_state* st, int id, int* dims_out) {
  return guarded([&]() -> int {
    if (!st || !dims_out) return fail(DCS_EINVAL, "null argument");
    if (id < 0 || id >= st->L.cap) return fail(DCS_ECAPACITY, "branch id outside capacity");
    const Slot& sl = st->slots[id];
    if (!sl.live) return fail(DCS_ESTATE, "branch is not live");
    for (int b = 0; b <= st->L.n; ++b) dims_out[b] = sl.dims[b];
    return DCS_OK;
  });
}

// ---------------------------------------------------------------------------
// Chunk compilation

int dcs_chunk_compile(dcs_ctx* ctx, dcs_chunk** out, int n_qubits, int n_ops, const int* q0,
                      const int* q1, const double* mats) {
  return guarded([&]() -> int {
    if (!out) return fail(DCS_EINVAL, "null handle");
    if (n_qubits < 1) return fail(DCS_EINVAL, "n_qubits must be positive");
    if (n_ops < 0 || (n_ops > 0 && (!q0 || !q1 || !mats))) return fail(DCS_EINVAL, "null op arrays");
    for (int i = 0; i < n_ops; ++i) {
      if (q0[i] < 0 || q0[i] >= n_qubits) return fail(DCS_EINVAL, "qubit out of range");
      if (q1[i] != -1) {
        if (q1[i] < 0 || q1[i] >= n_qubits) return fail(DCS_EINVAL, "qubit out of range");
        if (q1[i] == q0[i])
          return fail(DCS_EQUBITS, "two-qubit gate on (" + std::to_string(q0[i]) + ", " +
                                         std::to_string(q1[i]) + "): the qubits coincide");
      }
    }
    {
      size_t nd = 0;
      for (int i = 0; i < n_ops; ++i) nd += (q1[i] == -1) ? 8 : 32;
      for (size_t e = 0; e < nd; ++e)
        if (!std::isfinite(mats[e])) return fail(DCS_EINVAL, "non-finite gate matrix entry");
    }
    // ASAP layers: each gate goes to the first layer after the last one that
    // touches any of its qubits.  A gate on (a, b) with a > b is the gate
    // SWAP U SWAP on (b, a); a gate whose qubits are not adjacent acts as the
    // identity on the sites between them, which carry its operator bond.
    std::vector<int> last(n_qubits, -1);
    std::vector<std::vector<int>> layers;
    std::vector<size_t> mat_off(n_ops);
    std::vector<double> swapped;   // reordered matrices of the (a > b) gates
    std::vector<size_t> sw_off(n_ops, SIZE_MAX);
    size_t mo = 0;
    for (int i = 0; i < n_ops; ++i) {
      mat_off[i] = mo;
      mo += (q1[i] == -1) ? 8 : 32;
      if (q1[i] != -1 && q1[i] < q0[i]) {
        // element (s0 s1, t0 t1) of the swapped gate is element (s1 s0, t1 t0)
        const double* m = mats + mat_off[i];
        sw_off[i] = swapped.size();
        swapped.resize(swapped.size() + 32);
        double* d = swapped.data() + sw_off[i];
        for (int r = 0; r < 4; ++r)
          for (int c = 0; c < 4; ++c) {
            const int rs = ((r & 1) << 1) | (r >> 1), cs = ((c & 1) << 1) | (c >> 1);
            d[2 * (r * 4 + c)] = m[2 * (rs * 4 + cs)];
            d[2 * (r * 4 + c) + 1] = m[2 * (rs * 4 + cs) + 1];
          }
      }
      int lay = last[q0[i]];
      if (q1[i] != -1) lay = std::max(lay, last[q1[i]]);
      lay += 1;
      if ((int)layers.size() <= lay) layers.resize(lay + 1);
      layers[lay].push_back(i);
      last[q0[i]] = lay;
      if (q1[i] != -1) last[q1[i]] = lay;
    }
    dcs_chunk* ch = new dcs_chunk();
    ch->n = n_qubits;
    std::vector<int> wl(n_qubits, 1), wr(n_qubits, 1);
    ch->site.assign(n_qubits, std::vector<cd>{1.0, 0.0, 0.0, 1.0});
    for (const auto& layer : layers) {
      for (int i : layer) {
        const double* m = sw_off[i] != SIZE_MAX ? swapped.data() + sw_off[i] : mats + mat_off[i];
        const int q = q1[i] == -1 ? q0[i] : std::min(q0[i], q1[i]);
        const int qr = q1[i] == -1 ? q : std::max(q0[i], q1[i]);
        if (q1[i] == -1) {
          std::vector<cd> u(4);
          for (int k = 0; k < 4; ++k) u[k] = cd(m[2 * k], m[2 * k + 1]);
          ch->site[q] = op_product(ch->site[q], wl[q], wr[q], u, 1, 1);
        } else {
          Split local;
          const Split* spp = &local;
          if (ctx) {
            const std::string key(reinterpret_cast<const char*>(m), 32 * sizeof(double));
            auto it = ctx->split_cache.find(key);
            if (it == ctx->split_cache.end()) {
              if (ctx->split_cache.size() > 65536) ctx->split_cache.clear();
              it = ctx->split_cache.emplace(key, split_gate(m)).first;
            }
            spp = &it->second;
          } else {
            local = split_gate(m);
          }
          const Split& sp = *spp;
          ch->site[q] = op_product(ch->site[q], wl[q], wr[q], sp.left, 1, sp.r);
          wr[q] *= sp.r;
          if (qr > q + 1) {
            // identity on the physical leg, the bond index passed through
            std::vector<cd> pass((size_t)sp.r * 4 * sp.r, 0.0);
            for (int w = 0; w < sp.r; ++w)
              for (int t = 0; t < 2; ++t) pass[((size_t)(w * 2 + t) * 2 + t) * sp.r + w] = 1.0;
            for (int j = q + 1; j < qr; ++j) {
              ch->site[j] = op_product(ch->site[j], wl[j], wr[j], pass, sp.r, sp.r);
              wl[j] *= sp.r;
              wr[j] *= sp.r;
            }
          }
          ch->site[qr] = op_product(ch->site[qr], wl[qr], wr[qr], sp.right, sp.r, 1);
          wl[qr] *= sp.r;
        }
      }
    }
    ch->w.assign(n_qubits + 1, 1);
    for (int j = 0; j + 1 < n_qubits; ++j) {
      if (wr[j] != wl[j + 1]) {
        delete ch;
        return fail(DCS_EINVAL, "internal: operator bond mismatch");
      }
      ch->w[j + 1] = wr[j];
    }
    *out = ch;
    return DCS_OK;
  });
}

int dcs_gate_rank(const double* mat, int* rank_out) {
  return guarded([&]() -> int {
    if (!mat || !rank_out) return fail(DCS_EINVAL, "null argument");
    for (int e = 0; e < 32; ++e)
      if (!std::isfinite(mat[e])) return fail(DCS_EINVAL, "non-finite gate matrix entry");
    *rank_out = split_gate(mat).r;
    return DCS_OK;
  });
}

int dcs_chunk_bonds(const dcs_chunk* ch, int* w_out) {
  return guarded([&]() -> int {
    if (!ch || !w_out) return fail(DCS_EINVAL, "null argument");
    for (int b = 0; b <= ch->n; ++b) w_out[b] = ch->w[b];
    return DCS_OK;
  });
}

int dcs_chunk_export(const dcs_chunk* ch, double* out, size_t cap_doubles) {
  return guarded([&]() -> int {
    if (!ch || !out) return fail(DCS_EINVAL, "null argument");
    size_t need = 0;
    for (const auto& w : ch->site) need += 2 * w.size();
    if (need > cap_doubles) return fail(DCS_ENOMEM, "output too small for the chunk operator");
    for (const auto& w : ch->site) {
      for (const cd& z : w) {
        *out++ = z.real();
        *out++ = z.imag();
      }
    }
    return DCS_OK;
  });
}

int dcs_chunk_destroy(dcs_chunk* ch) {
  return guarded([&]() -> int {
    delete ch;
    return DCS_OK;
  });
}

// ---------------------------------------------------------------------------
// Compression step

namespace {

struct Group {
  std::vector<int> members;  // call indices
  int chi_cap = 0, cur = 0;
  std::vector<int> Db, Kb, w;
  int goff = 0;  // first call-local index of the group
  const int* ids_dev = nullptr;
  bool warm = false;   // starting guess built from the ket (every ket bond <= the bra's)
};

}  // namespace

int dcs_state_set_warm_start(dcs_state* st, int enabled, double eta) {
  return guarded([&]() -> int {
    if (!st) return fail(DCS_EINVAL, "null state");
    if (enabled && !(eta >= 0.0 && eta <= 1e6)) return fail(DCS_EINVAL, "eta must be in [0, 1e6]");
    st->warm_eta = enabled ? eta : -1.0;
    return DCS_OK;
  });
}

int dcs_compress_step(dcs_state* st, int n, const int* ids, const dcs_chunk* const* chunks,
                      int n_sweeps, double* fid_out, void* stream) {
  return guarded([&]() -> int {
    if (!st) return fail(DCS_EINVAL, "null state");
    DCS_TRY(check_ids(st, n, ids, true));
    if (n == 0) return DCS_OK;
    if (!chunks || !fid_out) return fail(DCS_EINVAL, "null chunks or fid_out");
    if (n_sweeps < 1) return fail(DCS_EINVAL, "n_sweeps must be >= 1");
    const Layout& L = st->L;
    const int nq = L.n;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int i = 0; i < n; ++i) {
      const dcs_chunk* ch = chunks[i];
      if (!ch) return fail(DCS_EINVAL, "null chunk");
      if (ch->n != nq) return fail(DCS_EINVAL, "chunk qubit count differs from the state's");
      for (int b = 1; b < nq; ++b)
        if (ch->w[b] > L.wmax)
          return fail(DCS_ENOMEM, "chunk operator bond " + std::to_string(ch->w[b]) +
                                      " exceeds the state's mpo_bond_max");
      if (st->init_index(st->slots[ids[i]].chi_cap) < 0)
        return fail(DCS_ESTATE, "no starting guess registered for bond cap " +
                                    std::to_string(st->slots[ids[i]].chi_cap));
    }
    // group branches of identical shapes
    std::map<std::vector<int>, int> key2g;
    std::vector<Group> groups;
    for (int i = 0; i < n; ++i) {
      const Slot& sl = st->slots[ids[i]];
      std::vector<int> key;
      key.push_back(sl.chi_cap);
      key.push_back(sl.cur);
      key.insert(key.end(), sl.dims.begin(), sl.dims.end());
      key.insert(key.end(), chunks[i]->w.begin(), chunks[i]->w.end());
      auto it = key2g.find(key);
      if (it == key2g.end()) {
        Group g;
        g.chi_cap = sl.chi_cap;
        g.cur = sl.cur;
        g.Db = bond_dims(nq, sl.chi_cap);
        g.Kb = sl.dims;
        g.w = chunks[i]->w;
        g.warm = st->warm_eta >= 0.0;
        for (int b = 0; b <= nq; ++b)
          if (g.Kb[b] > g.Db[b]) g.warm = false;
        groups.push_back(g);
        it = key2g.emplace(key, (int)groups.size() - 1).first;
      }
      groups[it->second].members.push_back(i);
    }
    // ids (group order) and gate operators (call-local, group order)
    std::vector<int> ids_host;
    const size_t mpo_host_bytes = L.mpo_stride * (size_t)n;
    st->host_stage.resize(std::max(st->host_stage.size(), mpo_host_bytes));
    char* mh = st->host_stage.data();
    for (auto& g : groups) {
      g.goff = (int)ids_host.size();
      for (int i : g.members) {
        const int ci = (int)ids_host.size();
        ids_host.push_back(ids[i]);
        for (int j = 0; j < nq; ++j)
          to_path_ct(L.ct, chunks[i]->site[j].data(), chunks[i]->site[j].size(),
                     mh + L.mpo_stride * ci + L.mpo_site_off[j]);
      }
    }
    int* ids_dev = reinterpret_cast<int*>(st->base + L.o_ids);
    DCS_HIP(hipMemcpyAsync(ids_dev, ids_host.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    DCS_HIP(hipMemcpyAsync(st->base + L.o_mpo, mh, mpo_host_bytes, hipMemcpyHostToDevice, s));
    for (auto& g : groups) g.ids_dev = ids_dev + g.goff;

    const int ct = L.ct;
    // contractions of the compression step: path precision, or split-BF16
    // products over the complex64 tensors
    const int acc = st->precision == DCS_BF16X3 ? ACC_BF16X3 : ct;
    const size_t cs = L.cs;
    double* nrm_dev = reinterpret_cast<double*>(st->base + L.o_out);
    auto ket_site = [&](const Group& g, int j) { return slot_op(st, L.o_mps[g.cur], L.site_off[j]); };
    auto new_site = [&](const Group& g, int j) {
      return slot_op(st, L.o_mps[1 - g.cur], L.site_off[j]);
    };
    auto env = [&](int b) { return slot_op(st, L.o_env, L.env_off[b]); };
    auto x1 = [&]() { return slot_op(st, L.o_x1, 0); };
    auto x2 = [&]() { return slot_op(st, L.o_x2, 0); };
    auto fbuf = [&]() { return slot_op(st, L.o_f, 0); };
    auto mpo = [&](const Group& g, int j) {
      return local_op(st->base + L.o_mpo + L.mpo_stride * (size_t)g.goff + L.mpo_site_off[j],
                      (long long)L.mpo_stride);
    };
    auto init_site = [&](const Group& g, int j) {
      const int ii = st->init_index(g.chi_cap);
      return local_op(st->base + L.o_init + L.mps_bytes * (size_t)ii + L.site_off[j], 0);
    };
    (void)cs;

    // moving left at site j: Y1 = K_j R_{j+1}^T, Y2 = W Y1, then (a) R_j from
    // bra_j (starting guess or LQ factor) or (b) F = L_j Y2
    // the gate operator goes into the epilogue of the contraction that
    // produces its input (complex64 / complex128 contractions, bonds <= 4)
    // (bonds of 1, 2 or 4: a tile then holds whole row and column groups)
    auto fuse = [&](int wl, int wr) {
      return acc != ACC_BF16X3 && wl <= GEMM_EPI_WMAX && wr <= GEMM_EPI_WMAX &&
             (wl & (wl - 1)) == 0 && (wr & (wr - 1)) == 0;
    };
    auto left_prologue = [&](int j) -> int {
      std::vector<GemmJob> gj;
      std::vector<MpoJob> mj;
      for (auto& g : groups) {
        const int bsz = (int)g.members.size();
        const int kl = g.Kb[j], kr = g.Kb[j + 1], dr = g.Db[j + 1], wl = g.w[j], wr = g.w[j + 1];
        if (fuse(wl, wr)) {
          GemmJob q{ket_site(g, j), env(j + 1), x2(), g.ids_dev, 2 * kl, dr * wr, kr, kr, kr, dr,
                    bsz};
          q.epi = GEMM_EPI_LEFT;
          q.w = mpo(g, j);
          q.wl = wl;
          q.wr = wr;
          gj.push_back(q);
          continue;
        }
        gj.push_back({ket_site(g, j), env(j + 1), x1(), g.ids_dev, 2 * kl, dr * wr, kr, kr, kr,
                      dr * wr, bsz});
        mj.push_back({x1(), x2(), mpo(g, j), g.ids_dev, kl, dr, wl, wr, bsz});
      }
      DCS_TRY(run_gemm(st->ctx, ct, ct, ct, acc, OP_N, OP_T, gj, s, CLS_GEMM));
      return run_mpo(st->ctx, ct, 1, mj, s);
    };
    auto right_env_from = [&](int j, bool from_init) -> int {
      std::vector<GemmJob> gj;
      for (auto& g : groups) {
        const int bsz = (int)g.members.size();
        const int kl = g.Kb[j], dl = g.Db[j], dr = g.Db[j + 1], wl = g.w[j];
        gj.push_back({from_init && !g.warm ? init_site(g, j) : new_site(g, j), x2(), env(j),
                      g.ids_dev, dl, wl * kl, 2 * dr, 2 * dr, 2 * dr, wl * kl, bsz});
      }
      return run_gemm(st->ctx, ct, ct, ct, acc, OP_J, OP_T, gj, s, CLS_GEMM);
    };
    // warm start: the ket embedded in the bra's bond dims plus eta times the
    // generic guess (seeded completion of the directions the ket lacks),
    // brought to right-canonical form from the right: M_j = L_j Q_j by LQ,
    // B_j = Q_j, M_{j-1} <- M_{j-1} L_j (L_j^T = conj(Q_j) M_j^T).  B_0 is never
    // read (the first visit forms site 0 from the environments).
    auto warm_bra = [&]() -> int {
      bool any = false;
      for (auto& g : groups) any = any || g.warm;
      if (!any) return DCS_OK;
      auto embed = [&](const Group& g, Operand dst, Operand src, Operand ini, int dl, int dr,
                       int kl, int kr, double eta) -> int {
        EmbedArgs a;
        a.dst = dst;
        a.src = src;
        a.init = ini;
        a.ids = g.ids_dev;
        a.dl = dl;
        a.dr = dr;
        a.kl = kl;
        a.kr = kr;
        a.batch = (int)g.members.size();
        a.eta = eta;
        DCS_HIP(launch_embed(ct, a, s));
        return DCS_OK;
      };
      const Operand none = local_op(nullptr, 0);
      for (auto& g : groups) {
        if (!g.warm) continue;
        for (int j = 0; j < nq; ++j)
          DCS_TRY(embed(g, new_site(g, j), ket_site(g, j), init_site(g, j), g.Db[j], g.Db[j + 1],
                        g.Kb[j], g.Kb[j + 1], st->warm_eta));
      }
      for (int j = nq - 1; j >= 1; --j) {
        std::vector<QrJob> qj;
        std::vector<GemmJob> gl, gm;
        for (auto& g : groups) {
          if (!g.warm) continue;
          const int bsz = (int)g.members.size();
          const int dl = g.Db[j], dr = g.Db[j + 1], dp = g.Db[j - 1];
          QrJob q;
          q.f = new_site(g, j);
          q.q = fbuf();
          q.ws = slot_op(st, L.o_ws, 0);
          q.nrm2 = local_op(nrm_dev + g.goff, sizeof(double));
          q.ids = g.ids_dev;
          q.m = 2 * dr;
          q.n = dl;
          q.mode = 1;
          q.batch = bsz;
          qj.push_back(q);
          gl.push_back({fbuf(), new_site(g, j), x2(), g.ids_dev, dl, dl, 2 * dr, 2 * dr, 2 * dr, dl,
                        bsz});
          gm.push_back({new_site(g, j - 1), x2(), x1(), g.ids_dev, 2 * dp, dl, dl, dl, dl, dl, bsz});
        }
        DCS_TRY(run_qr(st->ctx, ct, ct, qj, s));
        DCS_TRY(run_gemm(st->ctx, ct, ct, ct, ct, OP_J, OP_T, gl, s, CLS_GEMM));
        DCS_TRY(run_gemm(st->ctx, ct, ct, ct, ct, OP_N, OP_T, gm, s, CLS_GEMM));
        for (auto& g : groups) {
          if (!g.warm) continue;
          const int dl = g.Db[j], dr = g.Db[j + 1], dp = g.Db[j - 1];
          DCS_TRY(embed(g, new_site(g, j), fbuf(), none, dl, dr, dl, dr, 0.0));
          DCS_TRY(embed(g, new_site(g, j - 1), x1(), none, dp, dl, dp, dl, 0.0));
        }
      }
      return DCS_OK;
    };
    // moving right at site j: X1 = L_j K_j, X2 = W X1, F = X2 R_{j+1}^T
    auto right_site = [&](int j, int qr_mode) -> int {
      std::vector<GemmJob> g1, g2;
      std::vector<MpoJob> mj;
      std::vector<QrJob> qj;
      for (auto& g : groups) {
        const int bsz = (int)g.members.size();
        const int kl = g.Kb[j], kr = g.Kb[j + 1], dl = g.Db[j], dr = g.Db[j + 1];
        const int wl = g.w[j], wr = g.w[j + 1];
        if (fuse(wl, wr)) {
          GemmJob q{env(j), ket_site(g, j), x2(), g.ids_dev, dl * wl, 2 * kr, kl, kl, 2 * kr, kr,
                    bsz};
          q.epi = GEMM_EPI_RIGHT;
          q.w = mpo(g, j);
          q.wl = wl;
          q.wr = wr;
          g1.push_back(q);
        } else {
          g1.push_back({env(j), ket_site(g, j), x1(), g.ids_dev, dl * wl, 2 * kr, kl, kl, 2 * kr,
                        2 * kr, bsz});
          mj.push_back({x1(), x2(), mpo(g, j), g.ids_dev, dl, kr, wl, wr, bsz});
        }
        g2.push_back({x2(), env(j + 1), fbuf(), g.ids_dev, 2 * dl, dr, wr * kr, wr * kr, wr * kr,
                      dr, bsz});
        QrJob q;
        q.f = fbuf();
        q.q = new_site(g, j);
        q.ws = slot_op(st, L.o_ws, 0);
        q.nrm2 = local_op(nrm_dev + g.goff, sizeof(double));
        q.ids = g.ids_dev;
        q.m = (qr_mode == 2) ? 2 * dl * dr : 2 * dl;
        q.n = (qr_mode == 2) ? 1 : dr;
        q.mode = qr_mode;
        q.batch = bsz;
        qj.push_back(q);
      }
      DCS_TRY(run_gemm(st->ctx, ct, ct, ct, acc, OP_N, OP_N, g1, s, CLS_GEMM));
      DCS_TRY(run_mpo(st->ctx, ct, 0, mj, s));
      DCS_TRY(run_gemm(st->ctx, ct, ct, ct, acc, OP_N, OP_T, g2, s, CLS_GEMM));
      DCS_TRY(run_qr(st->ctx, ct, ct, qj, s));
      if (qr_mode == 2) return DCS_OK;
      std::vector<GemmJob> g3;
      for (auto& g : groups) {
        const int bsz = (int)g.members.size();
        const int kr = g.Kb[j + 1], dl = g.Db[j], dr = g.Db[j + 1], wr = g.w[j + 1];
        g3.push_back({new_site(g, j), x2(), env(j + 1), g.ids_dev, dr, wr * kr, 2 * dl, dr,
                      wr * kr, wr * kr, bsz});
      }
      return run_gemm(st->ctx, ct, ct, ct, acc, OP_C, OP_N, g3, s, CLS_GEMM);
    };
    auto left_site = [&](int j) -> int {
      DCS_TRY(left_prologue(j));
      std::vector<GemmJob> gj;
      std::vector<QrJob> qj;
      for (auto& g : groups) {
        const int bsz = (int)g.members.size();
        const int kl = g.Kb[j], dl = g.Db[j], dr = g.Db[j + 1], wl = g.w[j];
        gj.push_back({env(j), x2(), fbuf(), g.ids_dev, dl, 2 * dr, wl * kl, wl * kl, 2 * dr, 2 * dr,
                      bsz});
        QrJob q;
        q.f = fbuf();
        q.q = new_site(g, j);
        q.ws = slot_op(st, L.o_ws, 0);
        q.nrm2 = local_op(nrm_dev + g.goff, sizeof(double));
        q.ids = g.ids_dev;
        q.m = 2 * dr;
        q.n = dl;
        q.mode = 1;
        q.batch = bsz;
        qj.push_back(q);
      }
      DCS_TRY(run_gemm(st->ctx, ct, ct, ct, acc, OP_N, OP_N, gj, s, CLS_GEMM));
      DCS_TRY(run_qr(st->ctx, ct, ct, qj, s));
      return right_env_from(j, false);
    };

    std::vector<int> visits;
    for (int t = 1; t <= n_sweeps; ++t) {
      if (t % 2 == 1)
        for (int j = (t == 1 ? 0 : 1); j < nq; ++j) visits.push_back(j);
      else
        for (int j = nq - 2; j >= 0; --j) visits.push_back(j);
    }
    auto enqueue = [&]() -> int {
      DCS_TRY(warm_bra());
      // right environments of the starting guess
      for (int j = nq - 1; j >= 1; --j) {
        DCS_TRY(left_prologue(j));
        DCS_TRY(right_env_from(j, true));
      }
      for (size_t v = 0; v < visits.size(); ++v) {
        const int j = visits[v];
        if (v + 1 == visits.size()) {
          DCS_TRY(right_site(j, 2));
        } else if (visits[v + 1] == j + 1) {
          DCS_TRY(right_site(j, 0));
        } else {
          DCS_TRY(left_site(j));
        }
      }
      return DCS_OK;
    };
    if (st->ctx->graphs && !st->ctx->timing) {
      std::string sig;
      auto put = [&](int v) { sig.append(reinterpret_cast<const char*>(&v), sizeof(v)); };
      put(n_sweeps);
      for (auto& g : groups) {
        put(-1);
        put(g.warm ? 1 : 0);
        if (g.warm) sig.append(reinterpret_cast<const char*>(&st->warm_eta), sizeof(double));
        put(g.chi_cap);
        put(g.cur);
        put(g.goff);
        for (int v : g.Kb) put(v);
        for (int v : g.w) put(v);
        for (int i : g.members) put(ids[i]);
      }
      auto it = st->graphs.find(sig);
      if (it == st->graphs.end() && st->graph_seen[sig]++ >= 1) {
        if (st->graphs.size() >= 64) {
          for (auto& kv : st->graphs) (void)hipGraphExecDestroy(kv.second);
          st->graphs.clear();
        }
        // capture on the state's own stream (the caller's may be the legacy
        // default stream, which cannot capture); the kernels only read data the
        // caller's stream has produced, so the replay goes on the caller's stream
        if (!st->capture_stream)
          DCS_HIP(hipStreamCreateWithFlags(&st->capture_stream, hipStreamNonBlocking));
        const hipStream_t caller = s;
        s = st->capture_stream;
        DCS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        st->ctx->capturing = true;
        const int rc = enqueue();
        st->ctx->capturing = false;
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(s, &graph);
        s = caller;
        if (rc != DCS_OK) {
          if (graph) (void)hipGraphDestroy(graph);
          return rc;
        }
        DCS_HIP(ec);
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        DCS_HIP(ei);
        it = st->graphs.emplace(sig, exec).first;
      }
      if (it != st->graphs.end()) {
        DCS_HIP(hipGraphLaunch(it->second, s));
      } else {
        DCS_TRY(enqueue());
      }
    } else {
      DCS_TRY(enqueue());
    }
    std::vector<double> nrm(n);
    DCS_HIP(hipMemcpyAsync(nrm.data(), nrm_dev, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    DCS_HIP(hipStreamSynchronize(s));
    tune_resolve(st->ctx);
    const int centre = visits.back();
    int k = 0;
    for (auto& g : groups) {
      for (int i : g.members) {
        fid_out[i] = nrm[k++];
        Slot& sl = st->slots[ids[i]];
        sl.dims = g.Db;
        sl.cur = 1 - sl.cur;
        sl.lc_end = centre;
        sl.rc_start = centre + 1;
        sl.ecache_bond = -1;
        sl.measured_q = -1;
      }
    }
    for (int i = 0; i < n; ++i)
      if (!(fid_out[i] > 0.0) || !std::isfinite(fid_out[i]))
        return fail(DCS_ENUMERIC, "vanishing or non-finite environment tensor in branch " +
                                      std::to_string(ids[i]));
    return DCS_OK;
  });
}

// ---------------------------------------------------------------------------
// Measurement probability

namespace {

// Host -> device copy through the state's pinned ring, ordered on stream s;
// the source may be released as soon as this returns.
int stage_h2d(dcs_state* st, hipStream_t s, void* dst, const void* src, size_t bytes) {
  const int k = st->pin_next;
  st->pin_next = (k + 1) % dcs_state::PIN_RING;
  if (st->pin_done[k]) {
    DCS_HIP(hipEventSynchronize(st->pin_done[k]));
  } else {
    DCS_HIP(hipEventCreateWithFlags(&st->pin_done[k], hipEventDisableTiming));
  }
  if (st->pin_bytes[k] < bytes) {
    if (st->pin_buf[k]) DCS_HIP(hipHostFree(st->pin_buf[k]));
    st->pin_buf[k] = nullptr;
    st->pin_bytes[k] = 0;
    const size_t want = std::max<size_t>(bytes, 4096);
    DCS_HIP(hipHostMalloc(&st->pin_buf[k], want, hipHostMallocDefault));
    st->pin_bytes[k] = want;
  }
  std::memcpy(st->pin_buf[k], src, bytes);
  DCS_HIP(hipMemcpyAsync(dst, st->pin_buf[k], bytes, hipMemcpyHostToDevice, s));
  DCS_HIP(hipEventRecord(st->pin_done[k], s));
  return DCS_OK;
}

// Enqueues the outcome norms (n_0, n_1) of branch ids[i] at qubits[i] into
// the state's output area, FP64, at position pos[i] (branches grouped by
// shape).  Arguments are checked by the caller.
int enqueue_norms(dcs_state* st, int n, const int* ids, const int* qubits, hipStream_t s,
                  std::vector<int>& pos) {
  const Layout& L = st->L;
  const int ct = L.ct;

  struct MGroup {
    std::vector<int> members;
    int cur, q, e_from, e_cached, g_from;
    std::vector<int> d;
    int goff = 0;
    const int* ids_dev = nullptr;
  };
  std::map<std::vector<int>, int> key2g;
  std::vector<MGroup> groups;
  for (int i = 0; i < n; ++i) {
    const Slot& sl = st->slots[ids[i]];
    const int q = qubits[i];
    // left transfer: identity at bond min(lc_end, q); cached matrix if usable
    int e_from = std::min(sl.lc_end, q), e_cached = 0;
    if (sl.ecache_bond >= 0 && sl.ecache_bond <= q && sl.ecache_bond > e_from) {
      e_from = sl.ecache_bond;
      e_cached = 1;
    }
    const int g_from = std::max(sl.rc_start, q + 1);  // identity right transfer at this bond
    std::vector<int> key{sl.cur, q, e_from, e_cached, g_from};
    key.insert(key.end(), sl.dims.begin(), sl.dims.end());
    auto it = key2g.find(key);
    if (it == key2g.end()) {
      MGroup g;
      g.cur = sl.cur;
      g.q = q;
      g.e_from = e_from;
      g.e_cached = e_cached;
      g.g_from = g_from;
      g.d = sl.dims;
      groups.push_back(g);
      it = key2g.emplace(key, (int)groups.size() - 1).first;
    }
    groups[it->second].members.push_back(i);
  }
  std::vector<int> ids_host;
  for (auto& g : groups) {
    g.goff = (int)ids_host.size();
    for (int i : g.members) ids_host.push_back(ids[i]);
  }
  int* ids_dev = reinterpret_cast<int*>(st->base + L.o_ids);
  DCS_TRY(stage_h2d(st, s, ids_dev, ids_host.data(), sizeof(int) * n));
  for (auto& g : groups) g.ids_dev = ids_dev + g.goff;
  double* out_dev = reinterpret_cast<double*>(st->base + L.o_out);

  auto site = [&](const MGroup& g, int j) { return slot_op(st, L.o_mps[g.cur], L.site_off[j]); };
  auto ebuf = [&]() { return slot_op(st, L.o_e, 0); };
  auto gbuf = [&]() { return slot_op(st, L.o_g, 0); };
  auto tx = [&]() { return slot_op(st, L.o_tx, 0); };
  auto ty = [&]() { return slot_op(st, L.o_ty, 0); };

  // groups run one after another (their step counts differ)
  for (auto& g : groups) {
    const int bsz = (int)g.members.size();
    const int q = g.q;
    bool e_nontrivial = g.e_cached != 0;
    for (int j = g.e_from; j < q; ++j) {
      const int dl = g.d[j], dr = g.d[j + 1];
      if (!e_nontrivial) {
        // E_{j+1} = A_j^H A_j
        std::vector<GemmJob> a{{site(g, j), site(g, j), ebuf(), g.ids_dev, dr, dr, 2 * dl, dr, dr,
                                dr, bsz}};
        a[0].herm = 1;
        DCS_TRY(run_gemm(st->ctx, ct, ct, CT_F64, CT_F64, OP_C, OP_N, a, s, CLS_MEAS));
        e_nontrivial = true;
      } else {
        std::vector<GemmJob> a{{ebuf(), site(g, j), tx(), g.ids_dev, dl, 2 * dr, dl, dl, 2 * dr,
                                2 * dr, bsz}};
        DCS_TRY(run_gemm(st->ctx, CT_F64, ct, CT_F64, CT_F64, OP_N, OP_N, a, s, CLS_MEAS));
        std::vector<GemmJob> b{{site(g, j), tx(), ebuf(), g.ids_dev, dr, dr, 2 * dl, dr, dr, dr,
                                bsz}};
        b[0].herm = 1;   // A^H (E A), E Hermitian
        DCS_TRY(run_gemm(st->ctx, ct, CT_F64, CT_F64, CT_F64, OP_C, OP_N, b, s, CLS_MEAS));
      }
    }
    bool g_nontrivial = false;
    for (int j = g.g_from - 1; j > q; --j) {
      const int dl = g.d[j], dr = g.d[j + 1];
      if (!g_nontrivial) {
        // G_j = conj(A_j) A_j^T over (s, b)
        std::vector<GemmJob> a{{site(g, j), site(g, j), gbuf(), g.ids_dev, dl, dl, 2 * dr, 2 * dr,
                                2 * dr, dl, bsz}};
        a[0].herm = 1;
        DCS_TRY(run_gemm(st->ctx, ct, ct, CT_F64, CT_F64, OP_J, OP_T, a, s, CLS_MEAS));
        g_nontrivial = true;
      } else {
        std::vector<GemmJob> a{{site(g, j), gbuf(), ty(), g.ids_dev, 2 * dl, dr, dr, dr, dr, dr,
                                bsz}};
        DCS_TRY(run_gemm(st->ctx, ct, CT_F64, CT_F64, CT_F64, OP_N, OP_T, a, s, CLS_MEAS));
        std::vector<GemmJob> b{{site(g, j), ty(), gbuf(), g.ids_dev, dl, dl, 2 * dr, 2 * dr,
                                2 * dr, dl, bsz}};
        b[0].herm = 1;   // conj(A) (A G^T)^T, Hermitian as G is
        DCS_TRY(run_gemm(st->ctx, ct, CT_F64, CT_F64, CT_F64, OP_J, OP_T, b, s, CLS_MEAS));
      }
    }
    const int dl = g.d[q], dr = g.d[q + 1];
    Operand z;
    z.base = nullptr;
    z.stride = 0;
    z.by_slot = 0;
    z.pad_ = 0;
    int zct = ct;
    if (e_nontrivial) {
      std::vector<GemmJob> a{{ebuf(), site(g, q), tx(), g.ids_dev, dl, 2 * dr, dl, dl, 2 * dr,
                              2 * dr, bsz}};
      DCS_TRY(run_gemm(st->ctx, CT_F64, ct, CT_F64, CT_F64, OP_N, OP_N, a, s, CLS_MEAS));
      z = tx();
      zct = CT_F64;
    }
    if (g_nontrivial) {
      const Operand zin = e_nontrivial ? tx() : site(g, q);
      std::vector<GemmJob> a{{zin, gbuf(), ty(), g.ids_dev, 2 * dl, dr, dr, dr, dr, dr, bsz}};
      DCS_TRY(run_gemm(st->ctx, e_nontrivial ? CT_F64 : ct, CT_F64, CT_F64, CT_F64, OP_N, OP_T, a,
                       s, CLS_MEAS));
      z = ty();
      zct = CT_F64;
    }
    std::vector<NormJob> nj{
        {site(g, q), z, local_op(out_dev + 2 * g.goff, 2 * sizeof(double)), g.ids_dev, dl, dr, bsz}};
    DCS_TRY(run_norms(st->ctx, ct, zct, nj, s));
    for (int i : g.members) {
      Slot& sl = st->slots[ids[i]];
      if (e_nontrivial) sl.ecache_bond = q;
    }
  }
  pos.assign(n, 0);
  int k = 0;
  for (auto& g : groups)
    for (int i : g.members) pos[i] = k++;
  return DCS_OK;
}

int check_measure_args(dcs_state* st, int n, const int* ids, const int* qubits) {
  if (!st) return fail(DCS_EINVAL, "null state");
  DCS_TRY(check_ids(st, n, ids, true));
  if (n > 0 && !qubits) return fail(DCS_EINVAL, "null qubits");
  for (int i = 0; i < n; ++i)
    if (qubits[i] < 0 || qubits[i] >= st->L.n) return fail(DCS_EINVAL, "qubit out of range");
  return DCS_OK;
}

}  // namespace

int dcs_measure_prob(dcs_state* st, int n, const int* ids, const int* qubits, double* p0_out,
                     void* stream) {
  return guarded([&]() -> int {
    DCS_TRY(check_measure_args(st, n, ids, qubits));
    if (n == 0) return DCS_OK;
    if (!p0_out) return fail(DCS_EINVAL, "null p0_out");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int> pos;
    DCS_TRY(enqueue_norms(st, n, ids, qubits, s, pos));
    const double* out_dev = reinterpret_cast<const double*>(st->base + st->L.o_out);
    std::vector<double> nm(2 * n);
    DCS_HIP(hipMemcpyAsync(nm.data(), out_dev, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, s));
    DCS_HIP(hipStreamSynchronize(s));
    tune_resolve(st->ctx);
    for (int i = 0; i < n; ++i) {
      Slot& sl = st->slots[ids[i]];
      sl.n0 = nm[2 * pos[i]];
      sl.n1 = nm[2 * pos[i] + 1];
      sl.measured_q = qubits[i];
      const double tot = sl.n0 + sl.n1;
      if (!(tot > 0.0) || !std::isfinite(tot)) {
        sl.measured_q = -1;
        return fail(DCS_ENUMERIC, "state norm vanished or is not finite");
      }
      p0_out[i] = sl.n0 / tot;
    }
    return DCS_OK;
  });
}

int dcs_measure_sample_collapse(dcs_state* st, int n, const int* ids, const int* qubits,
                                const double* u_dev, double eps, int* outcome_dev,
                                double* pm_dev, void* stream) {
  return guarded([&]() -> int {
    DCS_TRY(check_measure_args(st, n, ids, qubits));
    if (n == 0) return DCS_OK;
    if (!u_dev || !outcome_dev || !pm_dev) return fail(DCS_EINVAL, "null device array");
    if (!(eps >= 0.0 && eps < 0.5)) return fail(DCS_EINVAL, "eps must be in [0, 0.5)");
    const Layout& L = st->L;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<int> pos;
    DCS_TRY(enqueue_norms(st, n, ids, qubits, s, pos));
    std::vector<SampleItem> items(n);
    int max_elems = 0;
    for (int i = 0; i < n; ++i) {
      const Slot& sl = st->slots[ids[i]];
      const int q = qubits[i];
      items[i].a = st->slot_base(ids[i]) + L.o_mps[sl.cur] + L.site_off[q];
      items[i].dl = sl.dims[q];
      items[i].dr = sl.dims[q + 1];
      items[i].k = pos[i];
      items[i].idx = i;
      max_elems = std::max(max_elems, sl.dims[q] * sl.dims[q + 1]);
    }
    SampleItem* items_dev = reinterpret_cast<SampleItem*>(st->base + L.o_items);
    DCS_TRY(stage_h2d(st, s, items_dev, items.data(), sizeof(SampleItem) * n));
    {
      Timed t(st->ctx, s, CLS_MEAS, 0, 0);
      DCS_HIP(launch_sample_collapse(L.ct, items_dev, n, max_elems,
                                     reinterpret_cast<const double*>(st->base + L.o_out), u_dev, eps,
                                     outcome_dev, pm_dev, s));
    }
    // the collapsed site breaks the canonical forms around it, whatever the outcome
    for (int i = 0; i < n; ++i) {
      Slot& sl = st->slots[ids[i]];
      const int q = qubits[i];
      sl.lc_end = std::min(sl.lc_end, q);
      sl.rc_start = std::max(sl.rc_start, q + 1);
      if (sl.ecache_bond > q) sl.ecache_bond = -1;
      sl.measured_q = -1;
    }
    return DCS_OK;
  });
}

// ---------------------------------------------------------------------------
// Collapse

int dcs_collapse(dcs_state* st, int n, const int* src_ids, const int* qubits, const int* outcomes,
                 const int* dst_ids, double eps, double* pm_out, void* stream) {
  return guarded([&]() -> int {
    if (!st) return fail(DCS_EINVAL, "null state");
    if (n == 0) return DCS_OK;
    if (!src_ids || !qubits || !outcomes || !dst_ids) return fail(DCS_EINVAL, "null arrays");
    const Layout& L = st->L;
    DCS_TRY(check_ids(st, n, dst_ids, false));
    std::vector<char> is_src(L.cap, 0);
    for (int i = 0; i < n; ++i) {
      const int sid = src_ids[i];
      if (sid < 0 || sid >= L.cap) return fail(DCS_ECAPACITY, "source id outside capacity");
      is_src[sid] = 1;
    }
    std::vector<double> pm(n);
    for (int i = 0; i < n; ++i) {
      const int sid = src_ids[i], did = dst_ids[i];
      const Slot& sl = st->slots[sid];
      if (!sl.live) return fail(DCS_ESTATE, "source branch is not live");
      if (sl.measured_q != qubits[i])
        return fail(DCS_ESTATE, "collapse of branch " + std::to_string(sid) + " on qubit " +
                                    std::to_string(qubits[i]) + " without a matching measurement");
      if (outcomes[i] != 0 && outcomes[i] != 1) return fail(DCS_EINVAL, "outcome must be 0 or 1");
      if (did != sid && (st->slots[did].live || is_src[did]))
        return fail(DCS_EINVAL, "destination slot " + std::to_string(did) + " is in use");
      const double nm = outcomes[i] ? sl.n1 : sl.n0;
      pm[i] = nm / (sl.n0 + sl.n1);
      if (!(pm[i] > eps))
        return fail(DCS_EZEROPROB, "outcome " + std::to_string(outcomes[i]) + " of branch " +
                                       std::to_string(sid) + " has probability " +
                                       std::to_string(pm[i]));
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    // copies first, so a source may also be collapsed in place
    std::vector<Slot> src_meta(n);
    for (int i = 0; i < n; ++i) src_meta[i] = st->slots[src_ids[i]];
    for (int i = 0; i < n; ++i) {
      const int sid = src_ids[i], did = dst_ids[i];
      if (did == sid) continue;
      const Slot& sl = src_meta[i];
      char* sb = st->slot_base(sid);
      char* db = st->slot_base(did);
      DCS_HIP(hipMemcpyAsync(db + L.o_mps[sl.cur], sb + L.o_mps[sl.cur], L.mps_bytes,
                             hipMemcpyDeviceToDevice, s));
      if (sl.ecache_bond >= 0) {
        const size_t eb = (size_t)sl.dims[sl.ecache_bond] * sl.dims[sl.ecache_bond] * 16;
        DCS_HIP(hipMemcpyAsync(db + L.o_e, sb + L.o_e, eb, hipMemcpyDeviceToDevice, s));
      }
    }
    std::vector<CollapseItem> items(n);
    int max_elems = 0;
    for (int i = 0; i < n; ++i) {
      const Slot& sl = src_meta[i];
      const int q = qubits[i];
      const double nm = outcomes[i] ? sl.n1 : sl.n0;
      items[i].a = st->slot_base(dst_ids[i]) + L.o_mps[sl.cur] + L.site_off[q];
      items[i].scale = 1.0 / std::sqrt(nm);
      items[i].dl = sl.dims[q];
      items[i].dr = sl.dims[q + 1];
      items[i].m = outcomes[i];
      items[i].pad_ = 0;
      max_elems = std::max(max_elems, sl.dims[q] * sl.dims[q + 1]);
    }
    CollapseItem* items_dev = reinterpret_cast<CollapseItem*>(st->base + L.o_items);
    DCS_HIP(hipMemcpyAsync(items_dev, items.data(), sizeof(CollapseItem) * n, hipMemcpyHostToDevice, s));
    {
      Timed t(st->ctx, s, CLS_OTHER, 0, 0);
      DCS_HIP(launch_collapse(L.ct, items_dev, n, max_elems, s));
    }
    DCS_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i) {
      Slot nsl = src_meta[i];
      const int q = qubits[i];
      nsl.live = true;
      nsl.lc_end = std::min(nsl.lc_end, q);
      nsl.rc_start = std::max(nsl.rc_start, q + 1);
      if (nsl.ecache_bond > q) nsl.ecache_bond = -1;
      nsl.measured_q = -1;
      st->slots[dst_ids[i]] = nsl;
      if (pm_out) pm_out[i] = pm[i];
    }
    return DCS_OK;
  });
}

// ---------------------------------------------------------------------------

int dcs_topk_by_weight(int n, const double* weights, int k, int* keep_idx_out, int* n_keep_out,
                       double* discarded_out) {
  return guarded([&]() -> int {
    if (n < 0 || k < 0) return fail(DCS_EINVAL, "negative size");
    if ((n > 0 && !weights) || !n_keep_out) return fail(DCS_EINVAL, "null argument");
    const int keep = std::min(n, k);
    if (keep > 0 && !keep_idx_out) return fail(DCS_EINVAL, "null keep_idx_out");
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return weights[a] > weights[b]; });
    double dropped = 0;
    for (int i = keep; i < n; ++i) dropped += weights[order[i]];
    for (int i = 0; i < keep; ++i) keep_idx_out[i] = order[i];
    *n_keep_out = keep;
    if (discarded_out) *discarded_out = dropped;
    return DCS_OK;
  });
}

int dcs_prune_adaptive(int n, const double* weights, int k_max, double mass_tol, double rel_min,
                       int* keep_idx_out, int* n_keep_out, double* discarded_out) {
  return guarded([&]() -> int {
    if (n < 0 || k_max < 1) return fail(DCS_EINVAL, "n must be >= 0 and k_max >= 1");
    if ((n > 0 && !weights) || !n_keep_out) return fail(DCS_EINVAL, "null argument");
    if (!(mass_tol >= 0.0 && mass_tol < 1.0) || !(rel_min >= 0.0 && rel_min <= 1.0))
      return fail(DCS_EINVAL, "mass_tol must be in [0, 1) and rel_min in [0, 1]");
    if (n > 0 && !keep_idx_out) return fail(DCS_EINVAL, "null keep_idx_out");
    for (int i = 0; i < n; ++i)
      if (!(weights[i] >= 0.0)) return fail(DCS_EINVAL, "weights must be non-negative");
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return weights[a] > weights[b]; });
    double total = 0;
    for (int i = 0; i < n; ++i) total += weights[i];
    const double floor_w = n > 0 ? rel_min * weights[order[0]] : 0.0;
    const double goal = (1.0 - mass_tol) * total;
    double kept = 0;
    int nk = 0;
    for (int i = 0; i < n && nk < k_max; ++i) {
      const double w = weights[order[i]];
      if (nk > 0 && (w < floor_w || (mass_tol > 0.0 && kept >= goal))) break;
      keep_idx_out[nk++] = order[i];
      kept += w;
    }
    double dropped = 0;
    for (int i = nk; i < n; ++i) dropped += weights[order[i]];
    *n_keep_out = nk;
    if (discarded_out) *discarded_out = dropped;
    return DCS_OK;
  });
}

}  // extern "C"

namespace {

// <a|b> by the FP64 left transfer E_{j+1} = A_j^H (E_j B_j), E in `E`, the
// product in `TX`; the last step writes its 1 x 1 result to `last` instead
// of E when `last` is set.
int enqueue_overlap(dcs_state* st, int id_a, int id_b, Operand E, Operand TX, void* last,
                    hipStream_t s) {
  const Layout& L = st->L;
  const int ct = L.ct;
  const Slot& A = st->slots[id_a];
  const Slot& B = st->slots[id_b];
  auto site = [&](int id, const Slot& sl, int j) {
    return local_op(st->slot_base(id) + L.o_mps[sl.cur] + L.site_off[j], 0);
  };
  for (int j = 0; j < L.n; ++j) {
    const int dla = A.dims[j], dra = A.dims[j + 1], dlb = B.dims[j], drb = B.dims[j + 1];
    const Operand out = (last && j == L.n - 1) ? local_op(last, 0) : E;
    if (j == 0) {   // E_1 = A_0^H B_0 (left bond of dimension 1)
      std::vector<GemmJob> g{{site(id_a, A, 0), site(id_b, B, 0), out, nullptr, dra, drb, 2 * dla,
                              dra, drb, drb, 1}};
      DCS_TRY(run_gemm(st->ctx, ct, ct, CT_F64, CT_F64, OP_C, OP_N, g, s, CLS_OTHER));
    } else {        // TX = E_j B_j, E_{j+1} = A_j^H TX over (a, s)
      std::vector<GemmJob> g1{{E, site(id_b, B, j), TX, nullptr, dla, 2 * drb, dlb, dlb, 2 * drb,
                               2 * drb, 1}};
      DCS_TRY(run_gemm(st->ctx, CT_F64, ct, CT_F64, CT_F64, OP_N, OP_N, g1, s, CLS_OTHER));
      std::vector<GemmJob> g2{{site(id_a, A, j), TX, out, nullptr, dra, drb, 2 * dla, dra, drb, drb,
                               1}};
      DCS_TRY(run_gemm(st->ctx, ct, CT_F64, CT_F64, CT_F64, OP_C, OP_N, g2, s, CLS_OTHER));
    }
  }
  return DCS_OK;
}

}  // namespace

extern "C" {

int dcs_overlap(dcs_state* st, int id_a, int id_b, double* out, void* stream) {
  return guarded([&]() -> int {
    if (!st || !out) return fail(DCS_EINVAL, "null argument");
    const int pair[2] = {id_a, id_b};
    DCS_TRY(check_ids(st, id_a == id_b ? 1 : 2, pair, true));
    const Layout& L = st->L;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // left transfer in slot a's measurement scratch (its cached left
    // transfer becomes invalid)
    const Operand E = local_op(st->slot_base(id_a) + L.o_e, 0);
    const Operand TX = local_op(st->slot_base(id_a) + L.o_tx, 0);
    DCS_TRY(enqueue_overlap(st, id_a, id_b, E, TX, nullptr, s));
    double v[2];
    DCS_HIP(hipMemcpyAsync(v, st->slot_base(id_a) + L.o_e, sizeof(v), hipMemcpyDeviceToHost, s));
    DCS_HIP(hipStreamSynchronize(s));
    tune_resolve(st->ctx);
    st->slots[id_a].ecache_bond = -1;
    out[0] = v[0];
    out[1] = v[1];
    return DCS_OK;
  });
}

int dcs_overlap_noalloc(dcs_state* st, int id_a, int id_b, double* out_dev, void* stream) {
  return guarded([&]() -> int {
    if (!st || !out_dev) return fail(DCS_EINVAL, "null argument");
    const int pair[2] = {id_a, id_b};
    DCS_TRY(check_ids(st, id_a == id_b ? 1 : 2, pair, true));
    const Layout& L = st->L;
    const Slot& A = st->slots[id_a];
    const Slot& B = st->slots[id_b];
    size_t e_need = 0, tx_need = 0;
    for (int j = 0; j <= L.n; ++j) e_need = std::max(e_need, (size_t)A.dims[j] * B.dims[j] * 16);
    for (int j = 0; j < L.n; ++j)
      tx_need = std::max(tx_need, (size_t)A.dims[j] * 2 * B.dims[j + 1] * 16);
    if (e_need > OVL_E_BYTES || tx_need > OVL_TX_BYTES)
      return fail(DCS_ENOMEM, "dcs_overlap_noalloc: bond dimensions above 256 need " +
                                  std::to_string(e_need + tx_need) + " bytes of scratch, the fixed "
                                  "scratch holds " + std::to_string(OVL_SCRATCH_BYTES));
    char* base = static_cast<char*>(scratch_ptr(st->ctx->device));
    if (!base) return fail(DCS_ESTATE, "no scratch address for this device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    st->ctx->no_alloc += 1;
    const int rc = enqueue_overlap(st, id_a, id_b, local_op(base, 0),
                                   local_op(base + OVL_E_BYTES, 0), out_dev, s);
    st->ctx->no_alloc -= 1;
    return rc;
  });
}

int dcs_export_mps(dcs_state* st, int id, double* host_out, size_t cap_doubles, int* dims_out,
                   void* stream) {
  return guarded([&]() -> int {
    if (!st || !host_out || !dims_out) return fail(DCS_EINVAL, "null argument");
    if (id < 0 || id >= st->L.cap) return fail(DCS_ECAPACITY, "branch id outside capacity");
    const Slot& sl = st->slots[id];
    if (!sl.live) return fail(DCS_ESTATE, "branch is not live");
    const Layout& L = st->L;
    size_t need = 0;
    for (int j = 0; j < L.n; ++j) need += 2 * (size_t)sl.dims[j] * 2 * sl.dims[j + 1];
    if (cap_doubles < need) return fail(DCS_ENOMEM, "host buffer too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<char> tmp(L.mps_bytes);
    DCS_HIP(hipMemcpyAsync(tmp.data(), st->slot_base(id) + L.o_mps[sl.cur], L.mps_bytes,
                           hipMemcpyDeviceToHost, s));
    DCS_HIP(hipStreamSynchronize(s));
    size_t o = 0;
    for (int j = 0; j < L.n; ++j) {
      const size_t e = (size_t)sl.dims[j] * 2 * sl.dims[j + 1];
      const char* src = tmp.data() + L.site_off[j];
      for (size_t k = 0; k < e; ++k) {
        if (L.ct == CT_F32) {
          const float2 v = reinterpret_cast<const float2*>(src)[k];
          host_out[o++] = v.x;
          host_out[o++] = v.y;
        } else {
          const double2 v = reinterpret_cast<const double2*>(src)[k];
          host_out[o++] = v.x;
          host_out[o++] = v.y;
        }
      }
    }
    for (int b = 0; b <= L.n; ++b) dims_out[b] = sl.dims[b];
    return DCS_OK;
  });
}

int dcs_import_mps(dcs_state* st, int id, int chi_cap, const double* host_in, const int* dims_in,
                   void* stream) {
  return guarded([&]() -> int {
    if (!st || !host_in || !dims_in) return fail(DCS_EINVAL, "null argument");
    const Layout& L = st->L;
    if (id < 0 || id >= L.cap) return fail(DCS_ECAPACITY, "branch id outside capacity");
    if (chi_cap < 1 || chi_cap > L.chi_max) return fail(DCS_EINVAL, "chi cap outside [1, chi_max]");
    if (dims_in[0] != 1 || dims_in[L.n] != 1) return fail(DCS_EINVAL, "boundary dims must be 1");
    for (int b = 0; b <= L.n; ++b)
      if (dims_in[b] < 1 || dims_in[b] > L.D[b]) return fail(DCS_EINVAL, "bond dim out of range");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<char> tmp(L.mps_bytes, 0);
    size_t o = 0;
    for (int j = 0; j < L.n; ++j) {
      const size_t e = (size_t)dims_in[j] * 2 * dims_in[j + 1];
      char* dst = tmp.data() + L.site_off[j];
      for (size_t k = 0; k < e; ++k, o += 2) {
        if (L.ct == CT_F32)
          reinterpret_cast<float2*>(dst)[k] = make_float2((float)host_in[o], (float)host_in[o + 1]);
        else
          reinterpret_cast<double2*>(dst)[k] = make_double2(host_in[o], host_in[o + 1]);
      }
    }
    DCS_HIP(hipMemcpyAsync(st->slot_base(id) + L.o_mps[0], tmp.data(), L.mps_bytes,
                           hipMemcpyHostToDevice, s));
    DCS_HIP(hipStreamSynchronize(s));
    Slot& sl = st->slots[id];
    sl = Slot();
    sl.live = true;
    sl.chi_cap = chi_cap;
    sl.dims.assign(dims_in, dims_in + L.n + 1);
    sl.cur = 0;
    sl.lc_end = 0;
    sl.rc_start = L.n;
    return DCS_OK;
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Runtime pieces shared with the tree-tensor-network entry points

namespace dcs {
namespace rt {

int fail(int code, const std::string& msg) { return ::fail(code, msg); }

int gemm(dcs_ctx* ctx, int ta, int tb, int tc, int tacc, int opa, int opb,
         const std::vector<GemmJob>& jobs, hipStream_t s, int cls) {
  return run_gemm(ctx, ta, tb, tc, tacc, opa, opb, jobs, s, cls < 0 ? CLS_GEMM : cls);
}

int qr(dcs_ctx* ctx, int ct_in, int ct_out, const std::vector<QrJob>& jobs, hipStream_t s) {
  return run_qr(ctx, ct_in, ct_out, jobs, s);
}

int permute(dcs_ctx* ctx, int ct_in, int ct_out, const PermuteArgs& a, hipStream_t s) {
  const double bytes = (double)a.total * a.batch * (csize_of(ct_in) + csize_of(ct_out));
  Timed t(ctx, s, CLS_OTHER, 0.0, bytes);
  DCS_HIP(launch_permute(ct_in, ct_out, a, s));
  return DCS_OK;
}

int ksum(dcs_ctx* ctx, const KsumArgs& a, hipStream_t s, int cls) {
  const double bytes = 16.0 * a.mn * (a.parts + 1.0) * a.batch;
  Timed t(ctx, s, cls, 2.0 * a.mn * a.parts * a.batch, bytes);
  DCS_HIP(launch_ksum(a, s));
  return DCS_OK;
}

void tune_sync(dcs_ctx* ctx) { tune_resolve(ctx); }

int ctx_device(const dcs_ctx* ctx) { return ctx->device; }

size_t qr_job_ws_elems(int m, int n, int mode) {
  if (mode == 2) return 0;
  const size_t mn = (size_t)m * n;
  if (m <= qr_large_max_rows()) return std::max(mn + ((size_t)n / 16 + 2) * 256, qr_large_ws_elems(m, n));
  return mn;
}

GateSplit split_gate(dcs_ctx* ctx, const double* m) {
  const Split* spp = nullptr;
  Split local;
  if (ctx) {
    const std::string key(reinterpret_cast<const char*>(m), 32 * sizeof(double));
    auto it = ctx->split_cache.find(key);
    if (it == ctx->split_cache.end()) {
      if (ctx->split_cache.size() > 65536) ctx->split_cache.clear();
      it = ctx->split_cache.emplace(key, ::split_gate(m)).first;
    }
    spp = &it->second;
  } else {
    local = ::split_gate(m);
    spp = &local;
  }
  GateSplit g;
  g.r = spp->r;
  g.left = spp->left;
  g.right = spp->right;
  return g;
}

}  // namespace rt
}  // namespace dcs

