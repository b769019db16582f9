// Host runtime of the tree tensor network (TTN): topology of a regular tree,
// state layout in device memory, chunks compiled into per-leaf operators whose
// two-qubit gates crossing leaves keep one named bond each, a contraction
// executor (batched transposition + batched GEMM on the shared kernels), and
// the compression step, measurement probability and collapse on trees.
//
// Every tensor carries named legs: the ket's and the bra's edge above node v,
// the bond of crossing gate g, and the input / output physical leg of qubit
// q.  A contraction sums over the legs two tensors share; the executor brings
// both operands into one of the row-major layouts the GEMM kernels take
// (transposing only when the stored order does not fit), so environments of
// any tree shape and any set of crossing gates need no operator tensor at the
// inner nodes: a gate's bond simply stays an open leg of every environment on
// the path between its two leaves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "dcs.h"
#include "dcs_internal.h"
#include "runtime_shared.h"

using namespace dcs;
using cd = std::complex<double>;
using rt::fail;
using rt::guarded;

#define TT_HIP(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(DCS_EHIP, std::string(#expr) + " failed: " + hipGetErrorString(e_));     \
  } while (0)

#define TT_TRY(expr)             \
  do {                           \
    int r_ = (expr);             \
    if (r_ != DCS_OK) return r_; \
  } while (0)

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }
int csize(int ct) { return ct == CT_F32 ? 8 : 16; }

int pow2_cap(int e, int cap) {
  if (e >= 30) return cap;
  return std::min(cap, 1 << e);
}

// ---------------------------------------------------------------------------
// Topology: levels n_0 = 1, ..., n_L = n; node ids in layer order; leaves
// (layer L-1) hold consecutive qubits.

struct Topo {
  std::vector<int> levels;
  int n = 0, L = 0, N = 0, d = 0, leaf0 = 0;
  std::vector<int> parent, qlo, qn;
  std::vector<std::vector<int>> kids;

  int build(const int* lv, int nl) {
    if (!lv || nl < 2) return fail(DCS_EINVAL, "a tree needs at least two levels");
    levels.assign(lv, lv + nl);
    if (levels[0] != 1) return fail(DCS_EINVAL, "the first level must be 1");
    for (int l = 0; l + 1 < nl; ++l)
      if (levels[l] < 1 || levels[l + 1] % levels[l] != 0 || levels[l + 1] <= levels[l])
        return fail(DCS_EINVAL, "each level must be a proper multiple of the previous one");
    n = levels.back();
    L = nl - 1;
    if (n > 62) return fail(DCS_EINVAL, "at most 62 qubits");
    N = 0;
    std::vector<int> off(L);
    for (int l = 0; l < L; ++l) {
      off[l] = N;
      N += levels[l];
    }
    leaf0 = off[L - 1];
    d = levels[L] / levels[L - 1];
    if (d > 6) return fail(DCS_EINVAL, "at most 6 qubits per leaf node");
    parent.assign(N, -1);
    kids.assign(N, {});
    qlo.assign(N, 0);
    qn.assign(N, 0);
    for (int l = 0; l < L; ++l) {
      const int per = levels[L] / levels[l];   // qubits per node of layer l
      for (int i = 0; i < levels[l]; ++i) {
        const int v = off[l] + i;
        qlo[v] = i * per;
        qn[v] = per;
        if (l > 0) parent[v] = off[l - 1] + i / (levels[l] / levels[l - 1]);
        if (l + 1 < L) {
          const int dk = levels[l + 1] / levels[l];
          for (int c = 0; c < dk; ++c) kids[v].push_back(off[l + 1] + dk * i + c);
        }
      }
    }
    for (int v = 0; v < N; ++v)
      if ((int)kids[v].size() > 6) return fail(DCS_EINVAL, "at most 6 children per node");
    return DCS_OK;
  }
  bool leaf(int v) const { return v >= leaf0; }
  int leaf_of(int q) const { return leaf0 + q / d; }
  int edge(int v, int chi) const {
    if (v == 0) return 1;
    return std::min(pow2_cap(qn[v], chi), pow2_cap(n - qn[v], chi));
  }
  std::vector<int> edges(int chi) const {
    std::vector<int> e(N);
    for (int v = 0; v < N; ++v) e[v] = edge(v, chi);
    return e;
  }
  // node dims [e_v, lower legs] for edge dims e
  std::vector<int> dims(int v, const std::vector<int>& e) const {
    std::vector<int> out{e[v]};
    if (leaf(v))
      out.insert(out.end(), d, 2);
    else
      for (int c : kids[v]) out.push_back(e[c]);
    return out;
  }
  size_t elems(int v, const std::vector<int>& e) const {
    size_t s = 1;
    for (int x : dims(v, e)) s *= (size_t)x;
    return s;
  }
  bool in_subtree(int v, int q) const { return q >= qlo[v] && q < qlo[v] + qn[v]; }
  std::vector<int> walk() const {
    std::vector<int> out{0};
    std::vector<std::pair<int, int>> st{{0, 0}};
    while (!st.empty()) {
      auto& top = st.back();
      const int v = top.first;
      if (top.second < (int)kids[v].size()) {
        const int c = kids[v][top.second++];
        out.push_back(c);
        st.push_back({c, 0});
      } else {
        st.pop_back();
        if (!st.empty()) out.push_back(st.back().first);
      }
    }
    return out;
  }
};

// Leg names.
enum { LK = 1, LB = 2, LG = 3, LT = 4, LS = 5 };
inline int legname(int kind, int idx) { return kind * (1 << 24) + idx; }

}  // namespace

// ---------------------------------------------------------------------------
// Chunk compiled for a tree

struct dcs_tchunk {
  std::vector<int> levels;
  std::vector<int> rank;                   // per crossing gate
  std::vector<std::vector<int>> cross;     // per node: gates crossing the edge above it
  std::vector<std::vector<int>> lgates;    // per leaf (index v - leaf0): its crossing gates
  std::vector<std::vector<cd>> lop;        // per leaf: [G...][S (2^d)][T (2^d)]
  std::string sig;                         // structure key (ranks and crossings)
  size_t op_elems = 0;                     // sum of the leaf operator sizes
};

namespace {

// Embedded action on the d qubits of a leaf: P[w][s][t] for the piece with
// `r` bond values acting on positions pos (1 or 2 of them), mats[w] the 2x2
// (one position) or 4x4 (two positions, first more significant) matrix.
std::vector<cd> embed_piece(int d, const std::vector<int>& pos, int r,
                            const std::vector<std::vector<cd>>& mats) {
  const int D = 1 << d;
  std::vector<cd> P((size_t)r * D * D, 0.0);
  const int k = (int)pos.size();
  for (int w = 0; w < r; ++w)
    for (int s = 0; s < D; ++s)
      for (int t = 0; t < D; ++t) {
        bool same = true;
        int ls = 0, lt = 0;
        for (int p = 0; p < d; ++p) {
          const int bs = (s >> (d - 1 - p)) & 1, bt = (t >> (d - 1 - p)) & 1;
          int which = -1;
          for (int j = 0; j < k; ++j)
            if (pos[j] == p) which = j;
          if (which < 0) {
            if (bs != bt) same = false;
          } else {
            ls |= bs << (k - 1 - which);
            lt |= bt << (k - 1 - which);
          }
        }
        if (!same) continue;
        const int m = 1 << k;
        P[((size_t)w * D + s) * D + t] = mats[w][ls * m + lt];
      }
  return P;
}

// O_new[(g_old, w)][s][t] = sum_u P[w][s][u] O_old[g_old][u][t]
std::vector<cd> leaf_compose(const std::vector<cd>& O, int gold, const std::vector<cd>& P, int r,
                             int D) {
  std::vector<cd> out((size_t)gold * r * D * D, 0.0);
  for (int go = 0; go < gold; ++go)
    for (int w = 0; w < r; ++w)
      for (int s = 0; s < D; ++s)
        for (int t = 0; t < D; ++t) {
          cd acc = 0.0;
          for (int u = 0; u < D; ++u)
            acc += P[((size_t)w * D + s) * D + u] * O[((size_t)go * D + u) * D + t];
          out[(((size_t)go * r + w) * D + s) * D + t] = acc;
        }
  return out;
}

}  // namespace

// ---------------------------------------------------------------------------
// Tree state

namespace {

struct TSlot {
  bool live = false;
  int chi_cap = 0;
  int cur = 0;
  std::vector<int> e;   // edge dims of the current tensors (e[0] = 1)
  int measured_q = -1;
  double n0 = 0, n1 = 0;
};

constexpr int NBUF = 6;   // scratch buffers of the contraction executor per slot

struct TLayout {
  int ct = CT_F64;
  size_t cs = 16;
  int cap = 0, chi_max = 0, wmax = 0, n_init = 0;
  size_t scratch = 0;                 // bytes per executor buffer
  std::vector<int> E;                 // maximal edge dims
  std::vector<size_t> node_off;       // inside one node buffer
  size_t node_bytes = 0;
  std::vector<size_t> env_off;        // per node v >= 1: U then D
  size_t env_each_max = 0;
  size_t o_nodes[2] = {0, 0}, o_env = 0, o_buf = 0, o_f = 0, o_ws = 0, o_meas = 0, slot_stride = 0;
  std::vector<size_t> meas_off;       // FP64 E_v (E_v x E_v) per node
  size_t o_slots = 0, o_ops = 0, ops_stride = 0, leaf_op_bytes = 0, o_ids = 0, o_out = 0,
         o_items = 0, items_bytes = 0, o_init = 0, o_initwork = 0, initwork_bytes = 0, total = 0;
};

TLayout make_tlayout(const Topo& T, int precision, int cap, int chi_max, int wmax,
                     size_t scratch_elems, int n_init) {
  TLayout L;
  L.ct = precision == DCS_C128 ? CT_F64 : CT_F32;
  L.cs = csize(L.ct);
  L.cap = cap;
  L.chi_max = chi_max;
  L.wmax = wmax;
  L.n_init = n_init;
  L.scratch = align_up(scratch_elems * 16);
  L.E = T.edges(chi_max);
  size_t off = 0, emax = 0;
  for (int v = 0; v < T.N; ++v) {
    L.node_off.push_back(off);
    const size_t e = T.elems(v, L.E);
    emax = std::max(emax, e);
    off += align_up(e * L.cs);
  }
  L.node_bytes = off;
  size_t eo = 0;
  L.env_off.assign(2 * T.N, 0);
  for (int v = 1; v < T.N; ++v) {
    const size_t each = align_up((size_t)L.E[v] * wmax * L.E[v] * L.cs);
    L.env_each_max = std::max(L.env_each_max, each);
    L.env_off[2 * v] = eo;
    eo += each;
    L.env_off[2 * v + 1] = eo;
    eo += each;
  }
  size_t mo = 0;
  for (int v = 0; v < T.N; ++v) {
    L.meas_off.push_back(mo);
    mo += align_up((size_t)L.E[v] * L.E[v] * 16);
  }
  // QR workspace: the largest job of any node towards any of its legs
  // (every bond cap up to chi_max: the QR path, and so its workspace, depends
  // on the shape)
  size_t ws = 0;
  for (int chi = 1; chi <= chi_max; ++chi) {
    const std::vector<int> ec = T.edges(chi);
    for (int v = 0; v < T.N; ++v) {
      const std::vector<int> dm = T.dims(v, ec);
      const size_t tot = T.elems(v, ec);
      for (size_t k = 0; k < dm.size(); ++k) {
        const int nn = dm[k], mm = (int)(tot / (size_t)dm[k]);
        ws = std::max(ws, rt::qr_job_ws_elems(mm, nn, k == 0 ? 1 : 0));
      }
    }
  }
  size_t p = 0;
  L.o_nodes[0] = p;
  p += L.node_bytes;
  L.o_nodes[1] = p;
  p += L.node_bytes;
  L.o_env = p;
  p += align_up(eo);
  L.o_buf = p;
  p += L.scratch * NBUF;
  L.o_f = p;
  p += align_up(emax * L.cs);
  L.o_ws = p;
  p += align_up(ws * 16);
  L.o_meas = p;
  p += align_up(mo);
  L.slot_stride = align_up(p);

  size_t g = 0;
  L.o_slots = g;
  g += L.slot_stride * (size_t)cap;
  // leaf operators of a call, per branch: at most wmax bond values per leaf
  const size_t D = (size_t)1 << T.d;
  L.leaf_op_bytes = align_up((size_t)wmax * D * D * L.cs);
  L.ops_stride = (size_t)(T.N - T.leaf0) * L.leaf_op_bytes;
  L.o_ops = g;
  g += L.ops_stride * (size_t)cap;
  L.o_ids = g;
  g += align_up(sizeof(int) * (size_t)cap);
  L.o_out = g;
  g += align_up(sizeof(double) * 4 * (size_t)cap);
  L.items_bytes = align_up((size_t)cap * std::max<size_t>((size_t)T.N * sizeof(void*),
                                                          sizeof(CollapseItem)));
  L.o_items = g;
  g += L.items_bytes;
  L.o_init = g;
  g += L.node_bytes * (size_t)n_init;
  // FP64 build area of a starting guess: Gaussians, isometries, R factors
  size_t iw = 0;
  for (int v = 0; v < T.N; ++v) iw += align_up(T.elems(v, L.E) * 16);
  L.initwork_bytes = 2 * iw + align_up((size_t)chi_max * chi_max * 16) + 4 * align_up(emax * 16);
  L.o_initwork = g;
  g += L.initwork_bytes;
  L.total = g;
  return L;
}

}  // namespace

struct dcs_tree {
  dcs_ctx* ctx = nullptr;
  int precision = DCS_C128;
  Topo T;
  TLayout L;
  char* base = nullptr;
  std::vector<TSlot> slots;
  std::vector<int> inits;   // bond cap of each registered guess
  char* slot_base(int id) const { return base + L.o_slots + L.slot_stride * (size_t)id; }
  int init_index(int chi) const {
    for (size_t i = 0; i < inits.size(); ++i)
      if (inits[i] == chi) return (int)i;
    return -1;
  }
};

// ---------------------------------------------------------------------------
// Contraction executor

namespace {

struct Ten {
  Operand op;
  int ct = CT_F64;
  bool conj = false;
  std::vector<int> legs, dims;
  int buf = -1;   // executor buffer holding it, or -1
  long long size() const {
    long long s = 1;
    for (int x : dims) s *= x;
    return s;
  }
};

Ten make_ten(Operand op, int ct, bool conj, const std::vector<int>& legs,
             const std::vector<int>& dims) {
  Ten t;
  t.op = op;
  t.ct = ct;
  t.conj = conj;
  for (size_t i = 0; i < legs.size(); ++i)
    if (dims[i] != 1) {   // unit legs carry no index
      t.legs.push_back(legs[i]);
      t.dims.push_back(dims[i]);
    }
  return t;
}

Operand offset_op(Operand o, size_t bytes) {
  o.base = static_cast<const char*>(o.base) + bytes;
  return o;
}

// GEMM forms the kernels provide, by storage types (A, B, C).
bool gemm_ok(int ta, int tb, int tc, int opa, int opb) {
  auto in = [&](std::initializer_list<std::pair<int, int>> l) {
    for (auto& p : l)
      if (p.first == opa && p.second == opb) return true;
    return false;
  };
  if (ta == tb && tb == tc) return in({{OP_N, OP_N}, {OP_N, OP_T}, {OP_C, OP_N}, {OP_J, OP_T}});
  if (tc != CT_F64) return false;
  if (ta == CT_F64 && tb == CT_F32) return in({{OP_N, OP_N}});
  if (ta == CT_F32 && tb == CT_F64) return in({{OP_C, OP_N}, {OP_N, OP_T}, {OP_J, OP_T}});
  if (ta == CT_F32 && tb == CT_F32) return in({{OP_C, OP_N}, {OP_J, OP_T}});
  return false;
}

struct Exec {
  dcs_tree* tr;
  hipStream_t s;
  const int* ids;   // device slot ids of the batch
  int batch;
  int tacc;         // accumulation type of compute-path contractions
  bool dry = false; // plan only: no launches, record the largest intermediate
  long long peak = 0;
  bool used[NBUF] = {};

  Operand buf_op(int b) const {
    Operand o;
    o.base = tr->base + tr->L.o_slots + tr->L.o_buf + tr->L.scratch * (size_t)b;
    o.stride = (long long)tr->L.slot_stride;
    o.by_slot = 1;
    o.pad_ = 0;
    return o;
  }
  int take(int* b) {
    if (dry) {
      *b = -1;
      return DCS_OK;
    }
    for (int i = 0; i < NBUF; ++i)
      if (!used[i]) {
        used[i] = true;
        *b = i;
        return DCS_OK;
      }
    return fail(DCS_ENOMEM, "tree contraction: executor buffers exhausted");
  }
  void give(const Ten& t) {
    if (t.buf >= 0) used[t.buf] = false;
  }
  int fits(long long elems, int ct) {
    peak = std::max(peak, elems * csize(ct) / 16);
    if (dry) return DCS_OK;
    if ((size_t)elems * csize(ct) > tr->L.scratch)
      return fail(DCS_ENOMEM, "tree contraction: an intermediate of " + std::to_string(elems) +
                                  " elements exceeds the state's scratch");
    return DCS_OK;
  }

  // Transposes `in` into leg order `order` (a permutation of its legs), with
  // its conjugation folded in and converted to `ct_out`, at `dst` (an
  // executor buffer if null).
  int permute(const Ten& in, const std::vector<int>& order, int ct_out, const Operand* dst,
              Ten* out) {
    const int r = (int)in.legs.size();
    std::vector<long long> stride(r, 1);
    for (int k = r - 2; k >= 0; --k) stride[k] = stride[k + 1] * in.dims[k + 1];
    std::vector<int> pos(order.size());
    for (size_t i = 0; i < order.size(); ++i) {
      auto it = std::find(in.legs.begin(), in.legs.end(), order[i]);
      if (it == in.legs.end()) return fail(DCS_EINVAL, "internal: permutation misses a leg");
      pos[i] = (int)(it - in.legs.begin());
    }
    // merge output neighbours that are input neighbours in the same order
    std::vector<long long> od, os;
    for (size_t i = 0; i < pos.size(); ++i) {
      const long long dd = in.dims[pos[i]], ss = stride[pos[i]];
      if (!od.empty() && os.back() == ss * dd) {
        od.back() *= dd;
        os.back() = ss;
      } else {
        od.push_back(dd);
        os.push_back(ss);
      }
    }
    if ((int)od.size() > PERMUTE_MAX_RANK) return fail(DCS_EINVAL, "internal: tensor rank too large");
    Ten t;
    t.ct = ct_out;
    t.conj = false;
    t.legs = order;
    for (int p : pos) t.dims.push_back(in.dims[p]);
    TT_TRY(fits(t.size(), ct_out));
    if (dst) {
      t.op = *dst;
    } else {
      TT_TRY(take(&t.buf));
      t.op = t.buf >= 0 ? buf_op(t.buf) : rt::local(nullptr, 0);
    }
    PermuteArgs a;
    std::memset(&a, 0, sizeof(a));
    a.in = in.op;
    a.out = t.op;
    a.ids = ids;
    a.rank = (int)od.size();
    a.conj = in.conj ? 1 : 0;
    a.batch = batch;
    a.total = t.size();
    for (int k = 0; k < a.rank; ++k) {
      a.dims[k] = (int)od[k];
      a.in_stride[k] = os[k];
    }
    if (!dry) TT_TRY(rt::permute(tr->ctx, in.ct, ct_out, a, s));
    *out = t;
    return DCS_OK;
  }

  // C = A B summed over their shared legs; C's legs are A's free legs then
  // B's free legs.  Written to `dst` when given, else to an executor buffer.
  int contract(const Ten& A0, const Ten& B0, int tc, const Operand* dst, Ten* out, int cls,
               size_t dst_bytes = 0) {
    std::vector<int> shared, fa, fb;
    for (int l : A0.legs)
      (std::find(B0.legs.begin(), B0.legs.end(), l) != B0.legs.end() ? shared : fa).push_back(l);
    for (int l : B0.legs)
      if (std::find(shared.begin(), shared.end(), l) == shared.end()) fb.push_back(l);
    auto cat = [](const std::vector<int>& x, const std::vector<int>& y) {
      std::vector<int> z = x;
      z.insert(z.end(), y.begin(), y.end());
      return z;
    };
    auto dimof = [](const Ten& t, int l) {
      return t.dims[std::find(t.legs.begin(), t.legs.end(), l) - t.legs.begin()];
    };
    // shared legs in B's order
    std::vector<int> shared_b;
    for (int l : B0.legs)
      if (std::find(shared.begin(), shared.end(), l) != shared.end()) shared_b.push_back(l);
    Ten A = A0, B = B0, tmpA, tmpB;
    bool pa = false, pb = false;
    int opa = -1, opb = -1;
    auto a_forms = [&](const Ten& a, const std::vector<int>& sh) {
      std::vector<int> f;
      if (a.legs == cat(fa, sh)) f.push_back(a.conj ? OP_J : OP_N);
      if (a.conj && a.legs == cat(sh, fa)) f.push_back(OP_C);
      return f;
    };
    auto b_forms = [&](const Ten& b, const std::vector<int>& sh) {
      std::vector<int> f;
      if (!b.conj && b.legs == cat(sh, fb)) f.push_back(OP_N);
      if (!b.conj && b.legs == cat(fb, sh)) f.push_back(OP_T);
      return f;
    };
    // 1: as stored (shared legs in A's order)
    for (int x : a_forms(A, shared))
      for (int y : b_forms(B, shared))
        if (opa < 0 && gemm_ok(A.ct, B.ct, tc, x, y)) {
          opa = x;
          opb = y;
        }
    // 2: transpose B only
    if (opa < 0) {
      for (int x : a_forms(A, shared)) {
        for (int ctb : {B.ct, (int)CT_F64}) {
          if (opa < 0 && gemm_ok(A.ct, ctb, tc, x, OP_N)) {
            TT_TRY(permute(B, cat(shared, fb), ctb, nullptr, &tmpB));
            pb = true;
            opa = x;
            opb = OP_N;
          }
        }
      }
    }
    // 3: transpose A only (shared legs in B's order)
    if (opa < 0) {
      for (int y : b_forms(B, shared_b)) {
        for (int cta : {A.ct, (int)CT_F64}) {
          if (opa < 0 && gemm_ok(cta, B.ct, tc, OP_N, y)) {
            TT_TRY(permute(A, cat(fa, shared_b), cta, nullptr, &tmpA));
            pa = true;
            shared = shared_b;
            opa = OP_N;
            opb = y;
          }
        }
      }
    }
    // 4: both into the N N form
    if (opa < 0) {
      const int cta = gemm_ok(A.ct, B.ct, tc, OP_N, OP_N) ? A.ct : tc;
      const int ctb = gemm_ok(cta, B.ct, tc, OP_N, OP_N) ? B.ct : tc;
      if (!gemm_ok(cta, ctb, tc, OP_N, OP_N)) return fail(DCS_EINVAL, "internal: no GEMM form");
      TT_TRY(permute(A, cat(fa, shared), cta, nullptr, &tmpA));
      TT_TRY(permute(B, cat(shared, fb), ctb, nullptr, &tmpB));
      pa = pb = true;
      opa = OP_N;
      opb = OP_N;
    }
    if (pa) A = tmpA;
    if (pb) B = tmpB;
    long long M = 1, N = 1, K = 1;
    for (int l : fa) M *= dimof(A, l);
    for (int l : fb) N *= dimof(B, l);
    for (int l : shared) K *= dimof(A, l);
    Ten c;
    c.ct = tc;
    c.conj = false;
    c.legs = cat(fa, fb);
    for (int l : fa) c.dims.push_back(dimof(A, l));
    for (int l : fb) c.dims.push_back(dimof(B, l));
    if (M > (1LL << 30) || N > (1LL << 30) || K > (1LL << 30))
      return fail(DCS_EINVAL, "internal: contraction too large");
    if (dst) {
      if (!dry && (size_t)c.size() * csize(tc) > dst_bytes)
        return fail(DCS_ENOMEM, "tree contraction: result larger than its destination");
      c.op = *dst;
    } else {
      TT_TRY(fits(c.size(), tc));
      TT_TRY(take(&c.buf));
      c.op = c.buf >= 0 ? buf_op(c.buf) : rt::local(nullptr, 0);
    }
    rt::GemmJob j;
    j.a = A.op;
    j.b = B.op;
    j.c = c.op;
    j.ids = ids;
    j.M = (int)M;
    j.N = (int)N;
    j.K = (int)K;
    j.lda = (opa == OP_C) ? (int)M : (int)K;
    j.ldb = (opb == OP_T) ? (int)K : (int)N;
    j.ldc = (int)N;
    j.batch = batch;
    const int acc = tc == CT_F64 ? CT_F64 : tacc;
    // Split sum: a complex128 contraction with a single output tile per item
    // and a long sum (the top-level inner products of the measurement) would
    // run as one workgroup per item; its sum is cut into chunks computed side
    // by side into an executor buffer, then added chunk by chunk in order.
    const long long item_tiles = ((M + 31) / 32) * ((N + 31) / 32) * (long long)batch;
    long long parts = 1;
    if (tc == CT_F64 && M * N <= 1024 && K >= 4096)
      parts = std::max(1LL, std::min({K / 1024, 1024 / item_tiles, (long long)GEMM_MAX_GROUPS}));
    // (without a free executor buffer the contraction runs unsplit)
    int pbuf = -1;
    if (parts > 1 && !dry) {
      for (int i = 0; i < NBUF && pbuf < 0; ++i)
        if (!used[i]) {
          used[i] = true;
          pbuf = i;
        }
      if (pbuf < 0) parts = 1;
    }
    if (parts > 1) {
      const long long kc = (K + parts - 1) / parts;
      parts = (K + kc - 1) / kc;
      TT_TRY(fits(parts * M * N, CT_F64));
      const Operand pop = pbuf >= 0 ? buf_op(pbuf) : rt::local(nullptr, 0);
      std::vector<rt::GemmJob> jobs;
      for (long long q = 0; q < parts; ++q) {
        const long long k0 = q * kc;
        rt::GemmJob jq = j;
        jq.K = (int)std::min(kc, K - k0);
        jq.a = offset_op(A.op, (size_t)(k0 * (opa == OP_C ? j.lda : 1)) * csize(A.ct));
        jq.b = offset_op(B.op, (size_t)(k0 * (opb == OP_N ? j.ldb : 1)) * csize(B.ct));
        jq.c = offset_op(pop, (size_t)(q * M * N) * csize(CT_F64));
        jq.ldc = (int)N;
        jobs.push_back(jq);
      }
      if (!dry) {
        TT_TRY(rt::gemm(tr->ctx, A.ct, B.ct, tc, acc, opa, opb, jobs, s, cls));
        KsumArgs ka;
        std::memset(&ka, 0, sizeof(ka));
        ka.part = pop;
        ka.out = c.op;
        ka.ids = ids;
        ka.parts = (int)parts;
        ka.mn = (int)(M * N);
        ka.batch = batch;
        TT_TRY(rt::ksum(tr->ctx, ka, s, cls));
      }
      Ten pt;
      pt.buf = pbuf;
      give(pt);
    } else if (!dry) {
      TT_TRY(rt::gemm(tr->ctx, A.ct, B.ct, tc, acc, opa, opb, {j}, s, cls));
    }
    if (pa) give(tmpA);
    if (pb) give(tmpB);
    *out = c;
    return DCS_OK;
  }
};

}  // namespace

// ===========================================================================
// C ABI

extern "C" {

int dcs_tree_state_bytes(int precision, int n_levels, const int* levels, int capacity, int chi_max,
                         int mpo_bond_max, size_t scratch_elems, int n_init_slots,
                         size_t* bytes_out) {
  return guarded([&]() -> int {
    if (precision != DCS_C128 && precision != DCS_C64)
      return fail(DCS_EINVAL, "trees support complex128 and complex64");
    Topo T;
    TT_TRY(T.build(levels, n_levels));
    if (capacity < 1 || chi_max < 1 || chi_max > 1024 || mpo_bond_max < 1 ||
        mpo_bond_max > 4096 || n_init_slots < 1 || !bytes_out)
      return fail(DCS_EINVAL, "bad state size argument");
    *bytes_out = make_tlayout(T, precision, capacity, chi_max, mpo_bond_max, scratch_elems,
                              n_init_slots).total;
    return DCS_OK;
  });
}

int dcs_tree_create(dcs_ctx* ctx, dcs_tree** out, int precision, int n_levels, const int* levels,
                    int capacity, int chi_max, int mpo_bond_max, size_t scratch_elems,
                    int n_init_slots, void* d_buffer, size_t bytes, void* stream) {
  return guarded([&]() -> int {
    if (!ctx || !out || !d_buffer) return fail(DCS_EINVAL, "null argument");
    size_t need = 0;
    TT_TRY(dcs_tree_state_bytes(precision, n_levels, levels, capacity, chi_max, mpo_bond_max,
                                scratch_elems, n_init_slots, &need));
    if (reinterpret_cast<uintptr_t>(d_buffer) % ALIGN != 0)
      return fail(DCS_EINVAL, "device buffer must be 256-byte aligned");
    if (bytes < need) return fail(DCS_ENOMEM, "device buffer too small: need " + std::to_string(need));
    TT_HIP(hipSetDevice(rt::ctx_device(ctx)));
    (void)stream;
    dcs_tree* t = new dcs_tree();
    t->ctx = ctx;
    t->precision = precision;
    t->T.build(levels, n_levels);
    t->L = make_tlayout(t->T, precision, capacity, chi_max, mpo_bond_max, scratch_elems,
                        n_init_slots);
    t->base = static_cast<char*>(d_buffer);
    t->slots.assign(capacity, TSlot());
    *out = t;
    return DCS_OK;
  });
}

int dcs_tree_destroy(dcs_tree* t) {
  return guarded([&]() -> int {
    delete t;
    return DCS_OK;
  });
}


int dcs_tree_set_init(dcs_tree* t, int chi_cap, const double* gauss, void* stream) {
  return guarded([&]() -> int {
    if (!t || !gauss) return fail(DCS_EINVAL, "null argument");
    const Topo& T = t->T;
    const TLayout& L = t->L;
    if (chi_cap < 1 || chi_cap > L.chi_max) return fail(DCS_EINVAL, "chi_cap outside [1, chi_max]");
    int idx = t->init_index(chi_cap);
    const bool fresh = idx < 0;
    if (fresh) {
      if ((int)t->inits.size() >= L.n_init) return fail(DCS_ENOMEM, "all starting-guess slots are in use");
      idx = (int)t->inits.size();
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const std::vector<int> e = T.edges(chi_cap);
    // FP64 build area: Gaussians G_v, then isometries Q_v, then R, then scratch
    char* w = t->base + L.o_initwork;
    std::vector<size_t> goff(T.N), qoff(T.N);
    size_t o = 0, gin = 0, emax = 0;
    for (int v = 0; v < T.N; ++v) {
      goff[v] = o;
      o += align_up(T.elems(v, L.E) * 16);
      emax = std::max(emax, T.elems(v, L.E));
    }
    for (int v = 0; v < T.N; ++v) {
      qoff[v] = o;
      o += align_up(T.elems(v, L.E) * 16);
    }
    char* R = w + o;
    char* tmp = R + align_up((size_t)L.chi_max * L.chi_max * 16);
    for (int v = 0; v < T.N; ++v) {
      const size_t ev = T.elems(v, e);
      TT_HIP(hipMemcpyAsync(w + goff[v], gauss + 2 * gin, ev * 16, hipMemcpyHostToDevice, s));
      gin += ev;
    }
    double* nrm = reinterpret_cast<double*>(t->base + L.o_out);
    const Operand ws = rt::local(t->slot_base(0) + L.o_ws, 0);
    // bottom-up: Q_v = isometry of G_v towards its upper edge (QR of G_v^T,
    // written as Q^T in node layout), R = conj(Q_v) G_v^T absorbed into the
    // parent's leg of v
    for (int v = T.N - 1; v >= 1; --v) {
      const int ev = e[v];
      const size_t tot = T.elems(v, e);
      const int rest = (int)(tot / (size_t)ev);
      rt::QrJob q;
      q.f = rt::local(w + goff[v], 0);
      q.q = rt::local(w + qoff[v], 0);
      q.ws = ws;
      q.nrm2 = rt::local(nrm, 0);
      q.ids = nullptr;
      q.m = rest;
      q.n = ev;
      q.mode = 1;
      q.batch = 1;
      TT_TRY(rt::qr(t->ctx, CT_F64, CT_F64, {q}, s));
      rt::GemmJob g;
      g.a = rt::local(w + qoff[v], 0);
      g.b = rt::local(w + goff[v], 0);
      g.c = rt::local(R, 0);
      g.ids = nullptr;
      g.M = ev;
      g.N = ev;
      g.K = rest;
      g.lda = rest;
      g.ldb = rest;
      g.ldc = ev;
      g.batch = 1;
      TT_TRY(rt::gemm(t->ctx, CT_F64, CT_F64, CT_F64, CT_F64, OP_J, OP_T, {g}, s, rt::CLS_OTHER));
      // parent p, leg k: G_p[a][i][c] <- sum_j R[i][j] G_p[a][j][c]
      const int p = T.parent[v];
      const std::vector<int> dp = T.dims(p, e);
      const int k = 1 + (int)(std::find(T.kids[p].begin(), T.kids[p].end(), v) - T.kids[p].begin());
      long long pre = 1, post = 1;
      for (int i = 0; i < k; ++i) pre *= dp[i];
      for (size_t i = k + 1; i < dp.size(); ++i) post *= dp[i];
      rt::GemmJob a;
      a.a = rt::local(R, 0);
      a.b = rt::local(w + goff[p], (long long)ev * post * 16);
      a.c = rt::local(tmp, (long long)ev * post * 16);
      a.ids = nullptr;
      a.M = ev;
      a.N = (int)post;
      a.K = ev;
      a.lda = ev;
      a.ldb = (int)post;
      a.ldc = (int)post;
      a.batch = (int)pre;
      TT_TRY(rt::gemm(t->ctx, CT_F64, CT_F64, CT_F64, CT_F64, OP_N, OP_N, {a}, s, rt::CLS_OTHER));
      TT_HIP(hipMemcpyAsync(w + goff[p], tmp, (size_t)pre * ev * post * 16, hipMemcpyDeviceToDevice, s));
    }
    {   // root: normalised
      rt::QrJob q;
      q.f = rt::local(w + goff[0], 0);
      q.q = rt::local(w + qoff[0], 0);
      q.ws = ws;
      q.nrm2 = rt::local(nrm, 0);
      q.ids = nullptr;
      q.m = (int)T.elems(0, e);
      q.n = 1;
      q.mode = 2;
      q.batch = 1;
      TT_TRY(rt::qr(t->ctx, CT_F64, CT_F64, {q}, s));
    }
    // to the path precision, into the guess slot
    char* ibase = t->base + L.o_init + L.node_bytes * (size_t)idx;
    for (int v = 0; v < T.N; ++v) {
      PermuteArgs a;
      std::memset(&a, 0, sizeof(a));
      a.in = rt::local(w + qoff[v], 0);
      a.out = rt::local(ibase + L.node_off[v], 0);
      a.ids = nullptr;
      a.rank = 1;
      a.batch = 1;
      a.total = (long long)T.elems(v, e);
      a.dims[0] = (int)a.total;
      a.in_stride[0] = 1;
      TT_TRY(rt::permute(t->ctx, CT_F64, L.ct, a, s));
    }
    TT_HIP(hipStreamSynchronize(s));
    rt::tune_sync(t->ctx);
    if (fresh) t->inits.push_back(chi_cap);
    return DCS_OK;
  });
}

int dcs_tree_branch_init_zero(dcs_tree* t, int n, const int* ids, const int* chi_caps, void* stream) {
  return guarded([&]() -> int {
    if (!t) return fail(DCS_EINVAL, "null tree");
    if (n < 0 || (n > 0 && (!ids || !chi_caps))) return fail(DCS_EINVAL, "null arrays");
    const TLayout& L = t->L;
    std::vector<char> seen(L.cap, 0);
    for (int i = 0; i < n; ++i) {
      if (ids[i] < 0 || ids[i] >= L.cap) return fail(DCS_ECAPACITY, "branch id outside capacity");
      if (seen[ids[i]]++) return fail(DCS_EINVAL, "duplicate branch id");
      if (chi_caps[i] < 1 || chi_caps[i] > L.chi_max) return fail(DCS_EINVAL, "chi cap outside [1, chi_max]");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    // |0...0> with unit edges: every node holds one nonzero entry, 1, first
    std::vector<void*> ptrs;
    for (int i = 0; i < n; ++i) {
      char* nb = t->slot_base(ids[i]) + L.o_nodes[0];
      TT_HIP(hipMemsetAsync(nb, 0, L.node_bytes, s));
      for (int v = 0; v < t->T.N; ++v) ptrs.push_back(nb + L.node_off[v]);
    }
    void** dptr = reinterpret_cast<void**>(t->base + L.o_items);
    const size_t room = L.items_bytes / sizeof(void*);
    for (size_t done = 0; done < ptrs.size();) {
      const size_t cnt = std::min(room, ptrs.size() - done);
      TT_HIP(hipMemcpyAsync(dptr, ptrs.data() + done, cnt * sizeof(void*), hipMemcpyHostToDevice, s));
      TT_HIP(launch_fill_unit(L.ct, dptr, (int)cnt, s));
      TT_HIP(hipStreamSynchronize(s));
      done += cnt;
    }
    TT_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i) {
      TSlot& sl = t->slots[ids[i]];
      sl = TSlot();
      sl.live = true;
      sl.chi_cap = chi_caps[i];
      sl.e.assign(t->T.N, 1);
    }
    return DCS_OK;
  });
}

int dcs_tree_branch_set_chi(dcs_tree* t, int n, const int* ids, const int* chi_caps) {
  return guarded([&]() -> int {
    if (!t) return fail(DCS_EINVAL, "null tree");
    for (int i = 0; i < n; ++i) {
      if (!ids || !chi_caps) return fail(DCS_EINVAL, "null arrays");
      if (ids[i] < 0 || ids[i] >= t->L.cap) return fail(DCS_ECAPACITY, "branch id outside capacity");
      if (!t->slots[ids[i]].live) return fail(DCS_ESTATE, "branch is not live");
      if (chi_caps[i] < 1 || chi_caps[i] > t->L.chi_max) return fail(DCS_EINVAL, "chi cap outside [1, chi_max]");
    }
    for (int i = 0; i < n; ++i) t->slots[ids[i]].chi_cap = chi_caps[i];
    return DCS_OK;
  });
}

int dcs_tree_branch_release(dcs_tree* t, int n, const int* ids) {
  return guarded([&]() -> int {
    if (!t) return fail(DCS_EINVAL, "null tree");
    for (int i = 0; i < n; ++i) {
      if (!ids) return fail(DCS_EINVAL, "null ids");
      if (ids[i] < 0 || ids[i] >= t->L.cap) return fail(DCS_ECAPACITY, "branch id outside capacity");
    }
    for (int i = 0; i < n; ++i) t->slots[ids[i]] = TSlot();
    return DCS_OK;
  });
}


int dcs_tree_chunk_compile(dcs_ctx* ctx, dcs_tchunk** out, int n_levels, const int* levels,
                           int n_ops, const int* q0, const int* q1, const double* mats) {
  return guarded([&]() -> int {
    if (!out) return fail(DCS_EINVAL, "null handle");
    Topo T;
    TT_TRY(T.build(levels, n_levels));
    if (n_ops < 0 || (n_ops > 0 && (!q0 || !q1 || !mats))) return fail(DCS_EINVAL, "null op arrays");
    size_t nd = 0;
    for (int i = 0; i < n_ops; ++i) {
      if (q0[i] < 0 || q0[i] >= T.n) return fail(DCS_EINVAL, "qubit out of range");
      if (q1[i] != -1 && (q1[i] < 0 || q1[i] >= T.n)) return fail(DCS_EINVAL, "qubit out of range");
      if (q1[i] == q0[i]) return fail(DCS_EQUBITS, "two-qubit gate whose qubits coincide");
      nd += q1[i] == -1 ? 8 : 32;
    }
    for (size_t e = 0; e < nd; ++e)
      if (!std::isfinite(mats[e])) return fail(DCS_EINVAL, "non-finite gate matrix entry");
    const int D = 1 << T.d, nleaf = T.N - T.leaf0;
    dcs_tchunk* ch = new dcs_tchunk();
    ch->levels = T.levels;
    ch->cross.assign(T.N, {});
    ch->lgates.assign(nleaf, {});
    ch->lop.assign(nleaf, std::vector<cd>((size_t)D * D, 0.0));
    std::vector<int> gdim(nleaf, 1);
    for (int l = 0; l < nleaf; ++l)
      for (int x = 0; x < D; ++x) ch->lop[l][(size_t)x * D + x] = 1.0;
    size_t mo = 0;
    for (int i = 0; i < n_ops; ++i) {
      const double* m = mats + mo;
      mo += q1[i] == -1 ? 8 : 32;
      const int la = T.leaf_of(q0[i]);
      const int pa = q0[i] - T.qlo[la];
      if (q1[i] == -1) {
        std::vector<cd> u(4);
        for (int k = 0; k < 4; ++k) u[k] = cd(m[2 * k], m[2 * k + 1]);
        const auto P = embed_piece(T.d, {pa}, 1, {u});
        ch->lop[la - T.leaf0] = leaf_compose(ch->lop[la - T.leaf0], gdim[la - T.leaf0], P, 1, D);
        continue;
      }
      const int lb = T.leaf_of(q1[i]);
      const int pb = q1[i] - T.qlo[lb];
      if (la == lb) {   // both qubits in one leaf: no bond
        std::vector<cd> G(16);
        for (int k = 0; k < 16; ++k) G[k] = cd(m[2 * k], m[2 * k + 1]);
        const auto P = embed_piece(T.d, {pa, pb}, 1, {G});
        ch->lop[la - T.leaf0] = leaf_compose(ch->lop[la - T.leaf0], gdim[la - T.leaf0], P, 1, D);
        continue;
      }
      const rt::GateSplit sp = rt::split_gate(ctx, m);
      const int r = sp.r, g = (int)ch->rank.size();
      ch->rank.push_back(r);
      std::vector<std::vector<cd>> lm(r, std::vector<cd>(4)), rm(r, std::vector<cd>(4));
      for (int w = 0; w < r; ++w)
        for (int st = 0; st < 4; ++st) {
          lm[w][st] = sp.left[(size_t)st * r + w];
          rm[w][st] = sp.right[(size_t)w * 4 + st];
        }
      const int ia = la - T.leaf0, ib = lb - T.leaf0;
      ch->lop[ia] = leaf_compose(ch->lop[ia], gdim[ia], embed_piece(T.d, {pa}, r, lm), r, D);
      gdim[ia] *= r;
      ch->lgates[ia].push_back(g);
      ch->lop[ib] = leaf_compose(ch->lop[ib], gdim[ib], embed_piece(T.d, {pb}, r, rm), r, D);
      gdim[ib] *= r;
      ch->lgates[ib].push_back(g);
      // the bond crosses every edge on the path between the two leaves
      int a = la, b = lb;
      while (a != b) {
        ch->cross[a].push_back(g);
        ch->cross[b].push_back(g);
        a = T.parent[a];
        b = T.parent[b];
      }
    }
    std::string sig;
    auto put = [&](int v) { sig.append(reinterpret_cast<const char*>(&v), sizeof(v)); };
    for (int r : ch->rank) put(r);
    put(-1);
    for (int v = 0; v < T.N; ++v) {
      for (int gg : ch->cross[v]) put(gg);
      put(-2);
    }
    ch->sig = sig;
    for (auto& o : ch->lop) ch->op_elems += o.size();
    *out = ch;
    return DCS_OK;
  });
}

int dcs_tchunk_destroy(dcs_tchunk* ch) {
  return guarded([&]() -> int {
    delete ch;
    return DCS_OK;
  });
}

int dcs_tchunk_bonds(const dcs_tchunk* ch, int* w_out, int cap) {
  return guarded([&]() -> int {
    if (!ch || !w_out) return fail(DCS_EINVAL, "null argument");
    if (cap < (int)ch->cross.size()) return fail(DCS_ENOMEM, "output too small");
    for (size_t v = 0; v < ch->cross.size(); ++v) {
      long long w = 1;
      for (int g : ch->cross[v]) w *= ch->rank[g];
      w_out[v] = (int)std::min<long long>(w, 1 << 30);
    }
    return DCS_OK;
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Compression step, measurement and collapse on trees

namespace {

struct TGroup {
  std::vector<int> members;   // call indices
  int chi_cap = 0, cur = 0, goff = 0, init_idx = 0, q = -1;
  std::vector<int> Kb, Db;
  const dcs_tchunk* ch = nullptr;
  const int* ids_dev = nullptr;
};

std::vector<int> node_legs(const Topo& T, int v, int edge_kind, int phys_kind) {
  std::vector<int> l{legname(edge_kind, v)};
  if (T.leaf(v))
    for (int q = T.qlo[v]; q < T.qlo[v] + T.qn[v]; ++q) l.push_back(legname(phys_kind, q));
  else
    for (int c : T.kids[v]) l.push_back(legname(edge_kind, c));
  return l;
}

Operand slot_operand(const dcs_tree* t, size_t off) {
  Operand o;
  o.base = t->base + t->L.o_slots + off;
  o.stride = (long long)t->L.slot_stride;
  o.by_slot = 1;
  o.pad_ = 0;
  return o;
}

// Compression step of one group of branches (equal shapes and chunk
// structure): right... upward environments of the starting guess, then the
// walk of every sweep; each visited node is set to F / |F| and the centre
// moves on by a QR towards the next node; the last visit (the root) keeps T
// and leaves |F|^2 in the output area.
int compress_group(dcs_tree* t, Exec& ex, const TGroup& g, int n_sweeps) {
  const Topo& T = t->T;
  const TLayout& L = t->L;
  const dcs_tchunk& ch = *g.ch;
  const int ct = L.ct, bsz = (int)g.members.size();
  std::vector<std::vector<int>> Ul(T.N), Ud(T.N), Dl(T.N), Dd(T.N);
  auto ket = [&](int v) {
    return make_ten(slot_operand(t, L.o_nodes[g.cur] + L.node_off[v]), ct, false,
                    node_legs(T, v, LK, LT), T.dims(v, g.Kb));
  };
  auto bra_guess = [&](int v) {
    return make_ten(rt::local(t->base + L.o_init + L.node_bytes * (size_t)g.init_idx + L.node_off[v], 0),
                    ct, true, node_legs(T, v, LB, LS), T.dims(v, g.Db));
  };
  auto bra_new = [&](int v) {
    return make_ten(slot_operand(t, L.o_nodes[1 - g.cur] + L.node_off[v]), ct, true,
                    node_legs(T, v, LB, LS), T.dims(v, g.Db));
  };
  auto oper = [&](int l) {
    std::vector<int> legs, dims;
    for (int gg : ch.lgates[l - T.leaf0]) {
      legs.push_back(legname(LG, gg));
      dims.push_back(ch.rank[gg]);
    }
    for (int q = T.qlo[l]; q < T.qlo[l] + T.qn[l]; ++q) {
      legs.push_back(legname(LS, q));
      dims.push_back(2);
    }
    for (int q = T.qlo[l]; q < T.qlo[l] + T.qn[l]; ++q) {
      legs.push_back(legname(LT, q));
      dims.push_back(2);
    }
    return make_ten(rt::local(t->base + L.o_ops + L.ops_stride * (size_t)g.goff +
                                  L.leaf_op_bytes * (size_t)(l - T.leaf0),
                              (long long)L.ops_stride),
                    ct, false, legs, dims);
  };
  auto envU = [&](int v) {
    Ten x;
    x.op = slot_operand(t, L.o_env + L.env_off[2 * v]);
    x.ct = ct;
    x.legs = Ul[v];
    x.dims = Ud[v];
    return x;
  };
  auto envD = [&](int v) {
    Ten x;
    x.op = slot_operand(t, L.o_env + L.env_off[2 * v + 1]);
    x.ct = ct;
    x.legs = Dl[v];
    x.dims = Dd[v];
    return x;
  };
  // X <- X . Y (X given back to the executor)
  auto absorb = [&](Ten& X, const Ten& Y) -> int {
    Ten Z;
    TT_TRY(ex.contract(X, Y, ct, nullptr, &Z, rt::CLS_BY_FORM));
    ex.give(X);
    X = Z;
    return DCS_OK;
  };
  // everything below v (ket, operator, children's environments)
  auto below = [&](int v, int skip, Ten* X) -> int {
    *X = ket(v);
    if (T.leaf(v)) TT_TRY(absorb(*X, oper(v)));
    for (int c : T.kids[v])
      if (c != skip) TT_TRY(absorb(*X, envU(c)));
    return DCS_OK;
  };
  auto write_env = [&](Ten& X, const Ten& bra, size_t off, std::vector<int>& legs,
                       std::vector<int>& dims) -> int {
    const Operand dst = slot_operand(t, L.o_env + off);
    Ten E;
    TT_TRY(ex.contract(X, bra, ct, &dst, &E, rt::CLS_BY_FORM, L.env_each_max));
    ex.give(X);
    legs = E.legs;
    dims = E.dims;
    return DCS_OK;
  };
  double* out = reinterpret_cast<double*>(t->base + L.o_out);
  auto qr = [&](Operand f, Operand q, int m, int n, int mode) -> int {
    if (m < n || n < 1) return fail(DCS_EINVAL, "internal: QR of a wide matrix");
    if (ex.dry) return DCS_OK;
    rt::QrJob j;
    j.f = f;
    j.q = q;
    j.ws = slot_operand(t, L.o_ws);
    j.nrm2 = rt::local(out + g.goff, sizeof(double));
    j.ids = g.ids_dev;
    j.m = m;
    j.n = n;
    j.mode = mode;
    j.batch = bsz;
    return rt::qr(t->ctx, ct, ct, {j}, ex.s);
  };

  // upward environments of the starting guess, bottom-up
  for (int v = T.N - 1; v >= 1; --v) {
    Ten X;
    TT_TRY(below(v, -1, &X));
    TT_TRY(write_env(X, bra_guess(v), L.env_off[2 * v], Ul[v], Ud[v]));
  }
  std::vector<int> visits;
  const std::vector<int> w = T.walk();
  for (int sw = 0; sw < n_sweeps; ++sw) visits.insert(visits.end(), w.begin() + (sw ? 1 : 0), w.end());
  for (size_t i = 0; i < visits.size(); ++i) {
    const int v = visits[i];
    Ten X = ket(v);
    if (T.leaf(v)) TT_TRY(absorb(X, oper(v)));
    if (v != 0) TT_TRY(absorb(X, envD(v)));
    for (int c : T.kids[v]) TT_TRY(absorb(X, envU(c)));
    const Ten B = bra_new(v);   // node order of the bra legs (unit legs dropped)
    Ten F;
    if (X.legs == B.legs) {
      F = X;
    } else {
      const Operand fdst = slot_operand(t, L.o_f);
      TT_TRY(ex.permute(X, B.legs, ct, &fdst, &F));
      ex.give(X);
    }
    const long long tot = F.size();
    if (i + 1 == visits.size()) {
      TT_TRY(qr(F.op, B.op, (int)tot, 1, 2));
      ex.give(F);
      break;
    }
    const int u = visits[i + 1];
    if (u == T.parent[v]) {
      const int n = g.Db[v];
      TT_TRY(qr(F.op, B.op, (int)(tot / n), n, 1));
      ex.give(F);
      Ten Y;
      TT_TRY(below(v, -1, &Y));
      TT_TRY(write_env(Y, bra_new(v), L.env_off[2 * v], Ul[v], Ud[v]));
    } else {
      const int lc = legname(LB, u);
      std::vector<int> order;
      for (int l : B.legs)
        if (l != lc) order.push_back(l);
      const bool has = std::find(B.legs.begin(), B.legs.end(), lc) != B.legs.end();
      if (has) order.push_back(lc);
      Ten Fp;
      TT_TRY(ex.permute(F, order, ct, nullptr, &Fp));
      ex.give(F);
      const int n = g.Db[u];
      Ten Q = Fp;
      int qb = -1;
      TT_TRY(ex.take(&qb));
      Q.buf = qb;
      Q.op = qb >= 0 ? ex.buf_op(qb) : rt::local(nullptr, 0);
      TT_TRY(qr(Fp.op, Q.op, (int)(tot / n), n, 0));
      ex.give(Fp);
      Ten Bw;
      const Operand bdst = B.op;
      TT_TRY(ex.permute(Q, B.legs, ct, &bdst, &Bw));
      ex.give(Q);
      Ten Y = ket(v);
      if (v != 0) TT_TRY(absorb(Y, envD(v)));
      for (int c : T.kids[v])
        if (c != u) TT_TRY(absorb(Y, envU(c)));
      TT_TRY(write_env(Y, bra_new(v), L.env_off[2 * u + 1], Dl[u], Dd[u]));
    }
  }
  return DCS_OK;
}

// n_m = <psi|P_m|psi> (m = 0, 1) of qubit g.q for every branch of the group,
// by FP64 contraction from the leaves up: E_v[b][k] = the subtree of v
// contracted with its conjugate; the projector acts in the measured leaf.
// Results: (re, im) of n_m at out[4 (goff + b) + 2 m].
int measure_group(dcs_tree* t, Exec& ex, const TGroup& g) {
  const Topo& T = t->T;
  const TLayout& L = t->L;
  const int ct = L.ct;
  const int lq = T.leaf_of(g.q), lt = legname(LT, g.q);
  std::vector<std::vector<int>> El(T.N), Ed(T.N);
  double* out = reinterpret_cast<double*>(t->base + L.o_out);
  auto ket = [&](int v) {
    return make_ten(slot_operand(t, L.o_nodes[g.cur] + L.node_off[v]), ct, false,
                    node_legs(T, v, LK, LT), T.dims(v, g.Kb));
  };
  auto as_bra = [&](Ten x) {
    for (int& l : x.legs)
      if (l / (1 << 24) == LK) l = legname(LB, l % (1 << 24));
    x.conj = true;
    return x;
  };
  for (int m = 0; m < 2; ++m) {
    for (int v = T.N - 1; v >= 0; --v) {
      const Operand dst = v == 0 ? rt::local(out + 4 * g.goff + 2 * m, 4 * sizeof(double))
                                 : slot_operand(t, L.o_meas + L.meas_off[v]);
      const size_t dst_bytes = v == 0 ? 16 : (size_t)L.E[v] * L.E[v] * 16;
      Ten E;
      if (T.leaf(v)) {
        const Ten K = ket(v);
        if (v == lq) {
          std::vector<int> order{lt};
          for (int l : K.legs)
            if (l != lt) order.push_back(l);
          Ten Kp;
          TT_TRY(ex.permute(K, order, ct, nullptr, &Kp));
          Ten S = Kp;
          S.buf = -1;
          S.legs.erase(S.legs.begin());
          S.dims.erase(S.dims.begin());
          S.op = offset_op(Kp.op, (size_t)m * (size_t)S.size() * csize(ct));
          TT_TRY(ex.contract(as_bra(S), S, CT_F64, &dst, &E, rt::CLS_MEAS, dst_bytes));
          ex.give(Kp);
        } else {
          TT_TRY(ex.contract(as_bra(K), K, CT_F64, &dst, &E, rt::CLS_MEAS, dst_bytes));
        }
      } else {
        Ten X = ket(v);
        for (int c : T.kids[v]) {
          Ten Ec;
          Ec.op = slot_operand(t, L.o_meas + L.meas_off[c]);
          Ec.ct = CT_F64;
          Ec.legs = El[c];
          Ec.dims = Ed[c];
          Ten Z;
          TT_TRY(ex.contract(X, Ec, CT_F64, nullptr, &Z, rt::CLS_MEAS));
          ex.give(X);
          X = Z;
        }
        TT_TRY(ex.contract(as_bra(ket(v)), X, CT_F64, &dst, &E, rt::CLS_MEAS, dst_bytes));
        ex.give(X);
      }
      El[v] = E.legs;
      Ed[v] = E.dims;
    }
  }
  return DCS_OK;
}

int check_tree_ids(const dcs_tree* t, int n, const int* ids) {
  if (n < 0 || (n > 0 && !ids)) return fail(DCS_EINVAL, "null id array");
  std::vector<char> seen(t->L.cap, 0);
  for (int i = 0; i < n; ++i) {
    if (ids[i] < 0 || ids[i] >= t->L.cap) return fail(DCS_ECAPACITY, "branch id outside capacity");
    if (seen[ids[i]]++) return fail(DCS_EINVAL, "duplicate branch id");
    if (!t->slots[ids[i]].live) return fail(DCS_ESTATE, "branch is not live");
  }
  return DCS_OK;
}

void to_path(int ct, const std::vector<cd>& src, char* dst) {
  for (size_t i = 0; i < src.size(); ++i) {
    if (ct == CT_F32) {
      float* f = reinterpret_cast<float*>(dst) + 2 * i;
      f[0] = (float)src[i].real();
      f[1] = (float)src[i].imag();
    } else {
      double* f = reinterpret_cast<double*>(dst) + 2 * i;
      f[0] = src[i].real();
      f[1] = src[i].imag();
    }
  }
}

}  // namespace

extern "C" {

int dcs_tree_chunk_scratch(const dcs_tchunk* ch, int chi_bra, int chi_ket, size_t* elems_out) {
  return guarded([&]() -> int {
    if (!ch || !elems_out) return fail(DCS_EINVAL, "null argument");
    if (chi_bra < 1 || chi_ket < 1) return fail(DCS_EINVAL, "bond caps must be positive");
    dcs_tree t;
    TT_TRY(t.T.build(ch->levels.data(), (int)ch->levels.size()));
    t.L = make_tlayout(t.T, DCS_C128, 1, std::max(chi_bra, chi_ket), 4096, 0, 1);
    Exec ex{&t, nullptr, nullptr, 1, CT_F64};
    ex.dry = true;
    TGroup g;
    g.members = {0};
    g.chi_cap = chi_bra;
    g.Kb = t.T.edges(chi_ket);
    g.Db = t.T.edges(chi_bra);
    g.ch = ch;
    TT_TRY(compress_group(&t, ex, g, 2));
    for (int q = 0; q < t.T.n; q += t.T.d) {
      g.q = q;
      g.Kb = t.T.edges(chi_bra);
      TT_TRY(measure_group(&t, ex, g));
    }
    *elems_out = (size_t)ex.peak;
    return DCS_OK;
  });
}

int dcs_tree_compress_step(dcs_tree* t, int n, const int* ids, const dcs_tchunk* const* chunks,
                           int n_sweeps, double* fid_out, void* stream) {
  return guarded([&]() -> int {
    if (!t) return fail(DCS_EINVAL, "null tree");
    TT_TRY(check_tree_ids(t, n, ids));
    if (n == 0) return DCS_OK;
    if (!chunks || !fid_out) return fail(DCS_EINVAL, "null chunks or fid_out");
    if (n_sweeps < 1) return fail(DCS_EINVAL, "n_sweeps must be >= 1");
    const Topo& T = t->T;
    const TLayout& L = t->L;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int i = 0; i < n; ++i) {
      const dcs_tchunk* ch = chunks[i];
      if (!ch) return fail(DCS_EINVAL, "null chunk");
      if (ch->levels != T.levels) return fail(DCS_EINVAL, "chunk compiled for another tree");
      for (int v = 1; v < T.N; ++v) {
        long long w = 1;
        for (int g : ch->cross[v]) w *= ch->rank[g];
        if (w > L.wmax)
          return fail(DCS_ENOMEM, "chunk operator bond " + std::to_string(w) +
                                      " exceeds the state's mpo_bond_max");
      }
      if (t->init_index(t->slots[ids[i]].chi_cap) < 0)
        return fail(DCS_ESTATE, "no starting guess registered for bond cap " +
                                    std::to_string(t->slots[ids[i]].chi_cap));
    }
    std::map<std::string, int> key2g;
    std::vector<TGroup> groups;
    for (int i = 0; i < n; ++i) {
      const TSlot& sl = t->slots[ids[i]];
      std::string key = chunks[i]->sig;
      auto put = [&](int v) { key.append(reinterpret_cast<const char*>(&v), sizeof(v)); };
      put(sl.chi_cap);
      put(sl.cur);
      for (int x : sl.e) put(x);
      auto it = key2g.find(key);
      if (it == key2g.end()) {
        TGroup g;
        g.chi_cap = sl.chi_cap;
        g.cur = sl.cur;
        g.Kb = sl.e;
        g.Db = T.edges(sl.chi_cap);
        g.ch = chunks[i];
        g.init_idx = t->init_index(sl.chi_cap);
        groups.push_back(g);
        it = key2g.emplace(key, (int)groups.size() - 1).first;
      }
      groups[it->second].members.push_back(i);
    }
    // slot ids and leaf operators (call-local, group order)
    std::vector<int> ids_host;
    std::vector<char> ops((size_t)L.ops_stride * n, 0);
    for (auto& g : groups) {
      g.goff = (int)ids_host.size();
      for (int i : g.members) {
        const int ci = (int)ids_host.size();
        ids_host.push_back(ids[i]);
        for (size_t l = 0; l < chunks[i]->lop.size(); ++l)
          to_path(L.ct, chunks[i]->lop[l], ops.data() + L.ops_stride * ci + L.leaf_op_bytes * l);
      }
    }
    int* ids_dev = reinterpret_cast<int*>(t->base + L.o_ids);
    TT_HIP(hipMemcpyAsync(ids_dev, ids_host.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    TT_HIP(hipMemcpyAsync(t->base + L.o_ops, ops.data(), ops.size(), hipMemcpyHostToDevice, s));
    for (auto& g : groups) {
      g.ids_dev = ids_dev + g.goff;
      Exec ex{t, s, g.ids_dev, (int)g.members.size(), L.ct};
      TT_TRY(compress_group(t, ex, g, n_sweeps));
    }
    std::vector<double> nrm(n);
    TT_HIP(hipMemcpyAsync(nrm.data(), t->base + L.o_out, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    TT_HIP(hipStreamSynchronize(s));
    rt::tune_sync(t->ctx);
    int k = 0;
    for (auto& g : groups)
      for (int i : g.members) {
        fid_out[i] = nrm[k++];
        TSlot& sl = t->slots[ids[i]];
        sl.e = g.Db;
        sl.cur = 1 - sl.cur;
        sl.measured_q = -1;
      }
    for (int i = 0; i < n; ++i)
      if (!(fid_out[i] > 0.0) || !std::isfinite(fid_out[i]))
        return fail(DCS_ENUMERIC, "vanishing or non-finite environment tensor in branch " +
                                      std::to_string(ids[i]));
    return DCS_OK;
  });
}

int dcs_tree_measure_prob(dcs_tree* t, int n, const int* ids, const int* qubits, double* p0_out,
                          void* stream) {
  return guarded([&]() -> int {
    if (!t) return fail(DCS_EINVAL, "null tree");
    TT_TRY(check_tree_ids(t, n, ids));
    if (n == 0) return DCS_OK;
    if (!qubits || !p0_out) return fail(DCS_EINVAL, "null arrays");
    const Topo& T = t->T;
    const TLayout& L = t->L;
    for (int i = 0; i < n; ++i)
      if (qubits[i] < 0 || qubits[i] >= T.n) return fail(DCS_EINVAL, "qubit out of range");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::map<std::vector<int>, int> key2g;
    std::vector<TGroup> groups;
    for (int i = 0; i < n; ++i) {
      const TSlot& sl = t->slots[ids[i]];
      std::vector<int> key{sl.cur, qubits[i]};
      key.insert(key.end(), sl.e.begin(), sl.e.end());
      auto it = key2g.find(key);
      if (it == key2g.end()) {
        TGroup g;
        g.cur = sl.cur;
        g.q = qubits[i];
        g.Kb = sl.e;
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
    int* ids_dev = reinterpret_cast<int*>(t->base + L.o_ids);
    TT_HIP(hipMemcpyAsync(ids_dev, ids_host.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    for (auto& g : groups) {
      g.ids_dev = ids_dev + g.goff;
      Exec ex{t, s, g.ids_dev, (int)g.members.size(), CT_F64};
      TT_TRY(measure_group(t, ex, g));
    }
    std::vector<double> nm(4 * (size_t)n);
    TT_HIP(hipMemcpyAsync(nm.data(), t->base + L.o_out, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, s));
    TT_HIP(hipStreamSynchronize(s));
    rt::tune_sync(t->ctx);
    int k = 0;
    for (auto& g : groups)
      for (int i : g.members) {
        TSlot& sl = t->slots[ids[i]];
        sl.n0 = nm[4 * k];
        sl.n1 = nm[4 * k + 2];
        ++k;
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

int dcs_tree_collapse(dcs_tree* t, int n, const int* src_ids, const int* qubits,
                      const int* outcomes, const int* dst_ids, double eps, double* pm_out,
                      void* stream) {
  return guarded([&]() -> int {
    if (!t) return fail(DCS_EINVAL, "null tree");
    if (n == 0) return DCS_OK;
    if (!src_ids || !qubits || !outcomes || !dst_ids) return fail(DCS_EINVAL, "null arrays");
    const Topo& T = t->T;
    const TLayout& L = t->L;
    std::vector<char> is_src(L.cap, 0), seen(L.cap, 0);
    for (int i = 0; i < n; ++i) {
      if (src_ids[i] < 0 || src_ids[i] >= L.cap || dst_ids[i] < 0 || dst_ids[i] >= L.cap)
        return fail(DCS_ECAPACITY, "branch id outside capacity");
      if (seen[dst_ids[i]]++) return fail(DCS_EINVAL, "duplicate destination id");
      is_src[src_ids[i]] = 1;
    }
    std::vector<double> pm(n);
    for (int i = 0; i < n; ++i) {
      const TSlot& sl = t->slots[src_ids[i]];
      if (!sl.live) return fail(DCS_ESTATE, "source branch is not live");
      if (sl.measured_q != qubits[i]) return fail(DCS_ESTATE, "collapse without a matching measurement");
      if (outcomes[i] != 0 && outcomes[i] != 1) return fail(DCS_EINVAL, "outcome must be 0 or 1");
      if (dst_ids[i] != src_ids[i] && (t->slots[dst_ids[i]].live || is_src[dst_ids[i]]))
        return fail(DCS_EINVAL, "destination slot is in use");
      const double nmv = outcomes[i] ? sl.n1 : sl.n0;
      pm[i] = nmv / (sl.n0 + sl.n1);
      if (!(pm[i] > eps)) return fail(DCS_EZEROPROB, "outcome of vanishing probability");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<TSlot> meta(n);
    for (int i = 0; i < n; ++i) meta[i] = t->slots[src_ids[i]];
    for (int i = 0; i < n; ++i) {
      if (dst_ids[i] == src_ids[i]) continue;
      const size_t o = L.o_nodes[meta[i].cur];
      TT_HIP(hipMemcpyAsync(t->slot_base(dst_ids[i]) + o, t->slot_base(src_ids[i]) + o,
                            L.node_bytes, hipMemcpyDeviceToDevice, s));
    }
    std::vector<CollapseItem> items(n);
    int max_elems = 0;
    for (int i = 0; i < n; ++i) {
      const int q = qubits[i], l = T.leaf_of(q), p = q - T.qlo[l];
      const double nmv = outcomes[i] ? meta[i].n1 : meta[i].n0;
      items[i].a = t->slot_base(dst_ids[i]) + L.o_nodes[meta[i].cur] + L.node_off[l];
      items[i].scale = 1.0 / std::sqrt(nmv);
      items[i].dl = meta[i].e[l] << p;
      items[i].dr = 1 << (T.d - 1 - p);
      items[i].m = outcomes[i];
      items[i].pad_ = 0;
      max_elems = std::max(max_elems, items[i].dl * items[i].dr);
    }
    CollapseItem* dev = reinterpret_cast<CollapseItem*>(t->base + L.o_items);
    TT_HIP(hipMemcpyAsync(dev, items.data(), sizeof(CollapseItem) * n, hipMemcpyHostToDevice, s));
    TT_HIP(launch_collapse(L.ct, dev, n, max_elems, s));
    TT_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i) {
      TSlot ns = meta[i];
      ns.live = true;
      ns.measured_q = -1;
      t->slots[dst_ids[i]] = ns;
      if (pm_out) pm_out[i] = pm[i];
    }
    return DCS_OK;
  });
}

int dcs_tree_export(dcs_tree* t, int id, double* host_out, size_t cap_doubles, int* dims_out,
                    void* stream) {
  return guarded([&]() -> int {
    if (!t || !host_out || !dims_out) return fail(DCS_EINVAL, "null argument");
    if (id < 0 || id >= t->L.cap) return fail(DCS_ECAPACITY, "branch id outside capacity");
    const TSlot& sl = t->slots[id];
    if (!sl.live) return fail(DCS_ESTATE, "branch is not live");
    const Topo& T = t->T;
    const TLayout& L = t->L;
    size_t need = 0;
    for (int v = 0; v < T.N; ++v) need += 2 * T.elems(v, sl.e);
    if (cap_doubles < need) return fail(DCS_ENOMEM, "host buffer too small");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<char> tmp(L.node_bytes);
    TT_HIP(hipMemcpyAsync(tmp.data(), t->slot_base(id) + L.o_nodes[sl.cur], L.node_bytes,
                          hipMemcpyDeviceToHost, s));
    TT_HIP(hipStreamSynchronize(s));
    size_t o = 0;
    for (int v = 0; v < T.N; ++v) {
      const size_t e = T.elems(v, sl.e);
      const char* src = tmp.data() + L.node_off[v];
      for (size_t k = 0; k < e; ++k) {
        if (L.ct == CT_F32) {
          const float* f = reinterpret_cast<const float*>(src) + 2 * k;
          host_out[o++] = f[0];
          host_out[o++] = f[1];
        } else {
          const double* f = reinterpret_cast<const double*>(src) + 2 * k;
          host_out[o++] = f[0];
          host_out[o++] = f[1];
        }
      }
    }
    for (int v = 0; v < T.N; ++v) dims_out[v] = sl.e[v];
    return DCS_OK;
  });
}

int dcs_tree_n_nodes(const int* levels, int n_levels, int* n_nodes_out) {
  return guarded([&]() -> int {
    if (!n_nodes_out) return fail(DCS_EINVAL, "null argument");
    Topo T;
    TT_TRY(T.build(levels, n_levels));
    *n_nodes_out = T.N;
    return DCS_OK;
  });
}

}  // extern "C"
