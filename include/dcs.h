/*
 * dcs.h -- C ABI of the MI355X (gfx950) library for tensor-network simulation
 * of dynamic circuits: the MPS compression step of a unitary chunk, the
 * measurement probability, the collapse on an outcome and top-M branch
 * retention.
 *
 * Method (Fulginiti, Poggiali, Mendl, "Tensor Network Simulation of Dynamic
 * Circuits"):
 *   Sec. III-B    MPS state: site tensors A_j[chi_j][2][chi_{j+1}]
 *   Sec. III-C    compression step of a unitary chunk (Defs. "Unitary chunk",
 *                 "Compression step"), optimum T = F / sqrt(<F|F>), partial
 *                 fidelity f, global fidelity = product of the f
 *   Sec. IV-A     branch = (p, classical register, TN state)
 *   Sec. IV-B1    p_m = <psi|P_m|psi> by contraction; collapse = projector on
 *                 the local leg and renormalisation by 1/sqrt(p_m)
 *   Sec. IV-C     chunk construction (done by the caller)
 *   Alg. 1 / 2    single-path sampling and multi-path branching with top-M
 *                 retention (control flow done by the caller)
 *
 * Conventions
 *   - Every function returns an int status: DCS_OK (0) or a negative code;
 *     no function aborts or throws.  dcs_last_error() gives a thread-local
 *     message for the last failure on the calling thread.
 *   - Complex numbers on the host are interleaved (re, im) doubles.
 *   - Device memory of a state is owned by the caller (one buffer of
 *     dcs_state_bytes() bytes, at least 256-byte aligned) and must outlive the
 *     state; the library never frees it and makes no device allocation of its
 *     own: every device scratch area a call uses lies inside that buffer.
 *     (Pinned host staging buffers are allocated on first use and held by the
 *     state until dcs_state_destroy.)  Host arrays are only read during a
 *     call.  Opaque handles are owned by the caller and released with the
 *     matching *_destroy.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All device work
 *     of a call is enqueued on it; calls that return host values synchronise
 *     that stream before returning.
 *   - Qubit q of the chain is the paper's Q_{q+1}.  A two-qubit gate may act
 *     on any two distinct qubits, in either order (dcs_chunk_compile carries
 *     the operator bond of a gate on non-adjacent qubits across the sites
 *     between them).
 *   - Bond dimensions are fixed and zero padded: for bond cap chi the bond b
 *     (between sites b-1 and b) has chi_b = min(chi, 2^b, 2^(n-b)).
 *   - A state holds `capacity` branch slots; a branch is named by its slot
 *     id in [0, capacity).  Calls that take arrays of ids run all listed
 *     branches together (batched launches); ids in one call must be distinct.
 *   - Calls on one state are not thread-safe; use one host thread per state.
 */
#ifndef DCS_H
#define DCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum dcs_status {
  DCS_OK = 0,
  DCS_EINVAL = -1,      /* bad argument (range, null pointer, duplicate id) */
  DCS_EQUBITS = -2,     /* two-qubit gate whose two qubits coincide         */
  DCS_ENONLOCAL = DCS_EQUBITS,   /* former name of DCS_EQUBITS (from when gates
                                    had to act on adjacent qubits)          */
  DCS_EZEROPROB = -3,   /* collapse on an outcome with p_m <= eps           */
  DCS_ECAPACITY = -4,   /* branch id outside the state's capacity           */
  DCS_ENOMEM = -5,      /* buffer too small / chunk operator wider than the
                           state's maximum operator bond                     */
  DCS_EHIP = -6,        /* a HIP runtime call failed                        */
  DCS_ESTATE = -7,      /* call not valid in the branch's current state
                           (branch not live, collapse without a measurement,
                           no starting guess registered for its bond cap)   */
  DCS_ENUMERIC = -8     /* vanishing environment tensor (<F|F> = 0)         */
};

enum dcs_precision {
  DCS_C128 = 0,         /* complex128 storage and contractions (FP64 MFMA)  */
  DCS_C64 = 1,          /* complex64 storage, contractions on FP32 MFMA with
                           FP32 accumulation; QR, norms, probabilities and
                           renormalisation stay in FP64                      */
  DCS_BF16X3 = 2        /* complex64 storage; the compression-step
                           contractions run as split-BF16 products (each FP32
                           component = bf16 hi + bf16 lo, three BF16 MFMA
                           products per real product, FP32 accumulation);
                           gate operators in FP32; QR, norms, probabilities
                           and renormalisation in FP64                       */
};

typedef struct dcs_ctx dcs_ctx;
typedef struct dcs_state dcs_state;
typedef struct dcs_chunk dcs_chunk;

/* Thread-local message of the last failed call ("" if none). */
const char *dcs_last_error(void);

/* Library ABI version (major * 100 + minor). */
int dcs_version(void);

/* Context bound to one HIP device: holds host-side caches (gate splits,
 * pinned staging) and optional launch timing.  `device` is a HIP ordinal. */
int dcs_ctx_create(dcs_ctx **out, int device);
int dcs_ctx_destroy(dcs_ctx *ctx);

/* Autotuning of the contraction tile shapes (64x64, 32x32, 128x64, 64x128
 * output tiles per workgroup), on by default: for every shape class (operand
 * types and forms, power-of-two buckets of M, N, K and batch) the first
 * launches try each tile shape `reps` times, timed with HIP events, and the
 * fastest is used from then on.  All shapes give bit-identical results.
 * dcs_ctx_tuning_save / _load write and read the decided table as JSON. */
int dcs_ctx_set_tuning(dcs_ctx *ctx, int enabled, int reps);
int dcs_ctx_tuning_save(dcs_ctx *ctx, const char *path);
int dcs_ctx_tuning_load(dcs_ctx *ctx, const char *path);

/* Capture the launch sequence of dcs_compress_step into a HIP graph and
 * replay it when the same signature recurs (same branch slots, shapes,
 * operator bonds, sweeps and buffer parity), off by default.  A signature is
 * run eagerly the first time, captured the second time, replayed afterwards;
 * the per-call uploads (slot ids, gate operators) stay outside the graph.
 * Ignored while launch timing is on.  Graphs are owned by the state. */
int dcs_ctx_set_graphs(dcs_ctx *ctx, int enabled);

/* Per-kernel-class launch timing with HIP events on the caller's stream
 * (off by default).  Classes (DCS_TIMING_CLASSES of them): 0-3 the
 * contraction GEMMs of the compression step by operand form (0 A B, 1 A B^T,
 * 2 A^H B, 3 conj(A) B^T), 4 gate-operator application, 5 QR/LQ gauge shift,
 * 6 measurement contractions, 7 other.  dcs_ctx_timing returns, per class,
 * the number of launches, their summed duration in ms, and the algorithmic
 * flops and operand bytes (unpadded shapes) of those launches. */
#define DCS_TIMING_CLASSES 8
int dcs_ctx_set_timing(dcs_ctx *ctx, int enabled);
int dcs_ctx_timing(dcs_ctx *ctx, long long *launches, double *ms, double *flops,
                   double *bytes, int reset);

/* Bytes of device memory a state needs: `precision` a dcs_precision; n_qubits
 * >= 1; capacity branch slots; chi_max the largest bond cap any branch uses;
 * mpo_bond_max the largest operator bond dimension of any chunk that will be
 * compressed (1-2 layers of 2-qubit gates: 4; 3 layers: 16); n_init_slots the
 * number of distinct bond caps with a registered starting guess. */
int dcs_state_bytes(int precision, int n_qubits, int capacity, int chi_max,
                    int mpo_bond_max, int n_init_slots, size_t *bytes_out);

/* Create a state over the caller's device buffer `d_buffer` of `bytes` bytes
 * (from dcs_state_bytes with the same arguments).  All slots start released. */
int dcs_state_create(dcs_ctx *ctx, dcs_state **out, int precision, int n_qubits,
                     int capacity, int chi_max, int mpo_bond_max, int n_init_slots,
                     void *d_buffer, size_t bytes, void *stream);
int dcs_state_destroy(dcs_state *st);

/* Register the starting guess of every compression step into bond cap
 * `chi_cap` (Sec. III-C leaves it open; here a fixed generic right-canonical
 * MPS).  `gauss` holds the random Gaussian site tensors G_j (host, complex128
 * interleaved, sites j = 0..n-1 concatenated, each row-major
 * [chi_j][2][chi_{j+1}] for the padded dims of chi_cap).  Site j >= 1 becomes
 * the orthonormal-row factor of LQ(G_j as chi_j x 2chi_{j+1}) (FP64 on the
 * GPU); site 0 becomes G_0 / |G_0|.  The Gaussians are staged through the
 * per-call scratch of the state's slots (live branches keep their contents);
 * the bond cap is registered only once its guess is complete, so after a
 * failure no compression step can use a partial guess.  Re-registering a cap
 * replaces its guess.  Synchronises `stream`. */
int dcs_state_set_init(dcs_state *st, int chi_cap, const double *gauss, void *stream);

/* Make the listed slots live branches in |0...0> (A_j[0][0][0] = 1) with bond
 * caps chi_caps[i] (1 <= cap <= chi_max). */
int dcs_branch_init_zero(dcs_state *st, int n, const int *ids, const int *chi_caps,
                         void *stream);
/* Change the bond cap the next compression step of each branch compresses
 * into (the current tensors keep their dims until then). */
int dcs_branch_set_chi(dcs_state *st, int n, const int *ids, const int *chi_caps);
/* Release slots (their contents become undefined). */
int dcs_branch_release(dcs_state *st, int n, const int *ids);
/* Bond dims chi_0..chi_n (n_qubits+1 ints) of a live branch's tensors. */
int dcs_branch_dims(const dcs_state *st, int id, int *dims_out);

/* Compile one chunk (Def. "Unitary chunk", Sec. IV-C) of n_ops unitaries in
 * time order into one layered operator per site: q0[i] the first qubit, q1[i]
 * the second qubit of a two-qubit gate (any other qubit) or -1 for a
 * one-qubit gate; `mats` holds the matrices back to back (complex128
 * interleaved, row-major, 2x2 or 4x4 in basis |q0 q1> with q0 the more
 * significant bit).  Gates are placed in ASAP layers; a two-qubit gate is
 * split across its qubits by an SVD of its operator-Schmidt matrix (singular
 * values above 1e-14 of the largest kept, r of them); per site the layer
 * operators are multiplied in time order.  A gate on non-adjacent qubits a <
 * b is exact: the sites strictly between them get the identity with the
 * gate's bond of dimension r passed through, so every bond a..b-1 is
 * multiplied by r (the chunk's bond j is the product of the ranks of the
 * gates spanning it).  A gate with q0 > q1 is applied as its qubit-swapped
 * matrix on (q1, q0).  Errors: DCS_EQUBITS for q0 == q1, DCS_EINVAL for a
 * qubit out of range or a non-finite matrix entry.  Host-only; the handle is independent of any state.
 * `ctx` may be NULL (no caching of gate splits across calls). */
int dcs_chunk_compile(dcs_ctx *ctx, dcs_chunk **out, int n_qubits, int n_ops,
                      const int *q0, const int *q1, const double *mats);
/* Operator-Schmidt rank r (1, 2 or 4) of one two-qubit gate (16 complex128
 * interleaved, row-major, as in dcs_chunk_compile): the bond dimension the
 * gate adds to every bond it spans.  Lets a caller close a chunk before its
 * operator bond would exceed the state's mpo_bond_max.  DCS_EINVAL for a
 * non-finite entry.  Host-only, pure. */
int dcs_gate_rank(const double *mat, int *rank_out);
/* Operator bond dims w_0..w_n (n_qubits+1 ints; w_0 = w_n = 1). */
int dcs_chunk_bonds(const dcs_chunk *ch, int *w_out);
/* Host copy of the compiled operator: the sites W_0..W_{n-1} back to back,
 * each row-major [w_j][2 (out)][2 (in)][w_{j+1}] complex128 interleaved
 * (2 * sum w_j*4*w_{j+1} doubles, at most cap_doubles, else DCS_ENOMEM). */
int dcs_chunk_export(const dcs_chunk *ch, double *out, size_t cap_doubles);
int dcs_chunk_destroy(dcs_chunk *ch);

/* Compression step (Sec. III-C) of branch ids[i] with chunk chunks[i], all
 * branches swept together: starting guess of the branch's bond cap, right
 * environments, then n_sweeps alternating sweeps (first left-to-right over
 * sites 0..n-1, then right-to-left over n-2..0, ...).  At each visited site
 * F = environment contraction, T = F/|F|; QR (moving right) or LQ (moving
 * left) of T in FP64 gives the site tensor and the next environment; the last
 * update keeps T and gives the partial fidelity f = <F|F>, written to
 * fid_out[i] (host).  Afterwards the orthogonality centre is site 0 (even
 * n_sweeps) or n-1 (odd).  Synchronises `stream`. */
int dcs_compress_step(dcs_state *st, int n, const int *ids,
                      const dcs_chunk *const *chunks, int n_sweeps, double *fid_out,
                      void *stream);

/* Starting guess of the compression steps of this state (the paper leaves
 * the initial state of the variational compression open, Sec. III-C).
 * enabled = 0 (default): the generic guess registered for the branch's bond
 * cap.  enabled != 0: warm start from the ket, B = right-canonical form of
 * (ket embedded in the bra's bond dims) + eta * (generic guess), the second
 * term filling the directions the ket lacks with seeded ones; built on the
 * GPU by an LQ chain from the right (B_j = Q_j of M_j = L_j Q_j, L_j absorbed
 * into site j-1).  Branches whose ket has a bond wider than the bra's keep
 * the generic guess.  eta in [0, 1e6], else DCS_EINVAL.  Host-only. */
int dcs_state_set_warm_start(dcs_state *st, int enabled, double eta);

/* Measurement probability (Sec. IV-B1) of qubit qubits[i] of branch ids[i]:
 * n_m = <psi|P_m|psi> (m = 0, 1) contracted in FP64 from the network,
 * p0_out[i] = n_0 / (n_0 + n_1) (host).  The norms are kept for the next
 * dcs_collapse of that branch.  Synchronises `stream`. */
int dcs_measure_prob(dcs_state *st, int n, const int *ids, const int *qubits,
                     double *p0_out, void *stream);

/* Collapse (Sec. IV-B1, Alg. 2 "Collapse"): for each i, the branch src_ids[i]
 * measured on qubits[i] by the last dcs_measure_prob becomes, in slot
 * dst_ids[i], P_m psi / sqrt(n_m) with m = outcomes[i]: the slice 1-m of the
 * site tensor is zeroed and slice m scaled by 1/sqrt(n_m) (FP64 factor).
 * dst == src collapses in place; otherwise the branch is first copied to the
 * (released) slot dst, which becomes live with the source's bond cap.  All
 * copies happen before any in-place update, so one source may feed two
 * children (one in place, one copied).  pm_out[i] = n_m / (n_0 + n_1) (host,
 * may be NULL).  DCS_EZEROPROB if p_m <= eps (nothing is changed). */
int dcs_collapse(dcs_state *st, int n, const int *src_ids, const int *qubits,
                 const int *outcomes, const int *dst_ids, double eps, double *pm_out,
                 void *stream);

/* Measurement, sampling and collapse without a host round trip (Alg. 1 with
 * the outcome drawn on the device; Sec. IV-B1 probabilities and projection).
 * For each i: p_0 of branch ids[i] at qubits[i] as in dcs_measure_prob, then
 * outcome m = 0 if u_dev[i] < p_0 else 1; if p_m <= eps the other outcome
 * is taken (an event of probability at most eps); the branch is collapsed in
 * place (slice 1-m zeroed, slice m scaled by 1/sqrt(n_m) in FP64).
 * u_dev (double[n]), outcome_dev (int[n]) and pm_dev (double[n], p_m) are
 * device memory.  Enqueued on the stream without host synchronisation; the
 * caller reads the outcomes when it needs them (e.g. for classical control).
 * A branch whose norm vanished gets outcome -1, p_m NaN and is left as is.
 * Errors (checked on the host, before any work): EINVAL, ECAPACITY, ESTATE. */
int dcs_measure_sample_collapse(dcs_state *st, int n, const int *ids, const int *qubits,
                                const double *u_dev, double eps, int *outcome_dev,
                                double *pm_dev, void *stream);

/* Top-M retention (Alg. 2, after a measurement): indices of the k largest of
 * weights[0..n) in descending order, ties in index order (stable), into
 * keep_idx_out (capacity >= min(n, k)); *n_keep_out = min(n, k);
 * *discarded_out = sum of the weights not kept.  Host-only, pure. */
int dcs_topk_by_weight(int n, const double *weights, int k, int *keep_idx_out,
                       int *n_keep_out, double *discarded_out);

/* Adaptive pruning of the branch set, beyond the fixed top-M (the paper's
 * closing remarks name it as an open direction; this rule is ours).  The
 * branches are visited in descending weight (stable, as in
 * dcs_topk_by_weight) and kept while all of: fewer than k_max are kept; the
 * weight is at least rel_min times the largest weight; and, if mass_tol > 0,
 * the mass kept so far is below (1 - mass_tol) times the total (total summed
 * in index order, kept mass in visiting order).  The heaviest branch is
 * always kept (n > 0).  mass_tol = rel_min = 0 is dcs_topk_by_weight with
 * k = k_max.  keep_idx_out: capacity >= min(n, k_max), indices in visiting
 * order; *discarded_out = sum of the weights not kept.  Errors: EINVAL for n
 * < 0, k_max < 1, mass_tol outside [0, 1), rel_min outside [0, 1], a
 * negative or NaN weight, or a null pointer.  Host-only, pure. */
int dcs_prune_adaptive(int n, const double *weights, int k_max, double mass_tol,
                       double rel_min, int *keep_idx_out, int *n_keep_out,
                       double *discarded_out);

/* <a|b> = sum over all indices of conj(A) B for branches id_a (bra) and id_b
 * (ket) of one state, by the FP64 left-transfer contraction E_{j+1} =
 * A_j^H (E_j B_j) on the contraction kernels (Sec. III-B state overlap; the
 * fidelity |<a|b>|^2 / (<a|a><b|b>) compares two states).  The branches may
 * have different bond caps.  out: host, 2 doubles (re, im).  Uses the
 * measurement scratch of id_a.  Synchronises the stream.  Errors: EINVAL,
 * ECAPACITY, ESTATE (branch not live), EHIP. */
int dcs_overlap(dcs_state *st, int id_a, int id_b, double *out, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): dcs_overlap without any
 * allocation and without host synchronisation.  The transfer matrices live
 * in a fixed device array of the library (3 MiB per device, held until the
 * process ends): branches whose bond dimensions exceed 256 are rejected with
 * DCS_ENOMEM.  No tile-shape trials and no launch timing run in this call;
 * slot a's cached measurement transfer is left intact.  out_dev: device
 * memory, 2 doubles (re, im), written by the last contraction on `stream`.
 * All calls on one device share that array and nothing in it needs to start
 * at zero, but calls that overlap in time on one device (other streams, other
 * host threads) race on it: order them on one stream.  Errors: EINVAL,
 * ECAPACITY, ESTATE, ENOMEM, EHIP. */
int dcs_overlap_noalloc(dcs_state *st, int id_a, int id_b, double *out_dev, void *stream);

/* FP64 host copy of branch `id`'s MPS: sites concatenated, each row-major
 * [chi_j][2][chi_{j+1}] complex128 interleaved (2 * sum chi_j*2*chi_{j+1}
 * doubles, at most cap_doubles); dims_out gets chi_0..chi_n. */
int dcs_export_mps(dcs_state *st, int id, double *host_out, size_t cap_doubles,
                   int *dims_out, void *stream);
/* Load an MPS into branch `id` (becomes live, bond cap chi_cap) from the same
 * layout; dims_in[b] <= min(chi_max, 2^b, 2^(n-b)), dims_in[0] = dims_in[n]
 * = 1.  No canonical form is assumed. */
int dcs_import_mps(dcs_state *st, int id, int chi_cap, const double *host_in,
                   const int *dims_in, void *stream);

/* ------------------------------------------------------------------------
 * Tree tensor network (Sec. III-B, TTN paragraph: the paper's second ansatz,
 * whose compression step it takes from the work it builds on).  Readings:
 *   - structure (n_0 = 1, n_1, ..., n_L = n qubits), each level a proper
 *     multiple of the previous one; nodes numbered in layer order (root 0);
 *     the qubits are the leaves in order: leaf node i of layer L-1 holds
 *     qubits i d .. i d + d - 1, d = n_L / n_{L-1};
 *   - a node tensor's legs are [edge to the parent (dimension 1 at the root),
 *     then its children's edges in order, or its qubits' physical legs in
 *     order], row-major, complex interleaved; the edge above a node whose
 *     subtree holds s qubits has the fixed, zero-padded dimension
 *     min(chi, 2^s, 2^(n-s)) for bond cap chi;
 *   - compression step: the starting guess is canonical towards the root;
 *     a sweep walks from the root through every subtree and back (each edge
 *     twice, children in order); every visited node becomes T = F/sqrt(<F|F>)
 *     and the centre moves to the next node of the walk by a QR of T with the
 *     edge towards that node as its column index (FP64); the last visit (the
 *     root) keeps T and gives f = <F|F>;
 *   - measurement: n_m = <psi|P_m|psi> contracted in FP64 from the leaves up;
 *     collapse projects the qubit's leg in its leaf node and rescales by
 *     1/sqrt(n_m).
 * Two-qubit gates act on any two distinct qubits: a gate inside one leaf is
 * part of that leaf's operator; a gate across leaves is split by an SVD of
 * its operator-Schmidt matrix and its bond (rank r) is carried by every edge
 * on the tree path between the two leaves (the edge's operator bond is the
 * product of the ranks of the gates crossing it).  Precisions: DCS_C128 and
 * DCS_C64 (contractions on FP32 MFMA, QR and measurement in FP64).  Memory,
 * streams, errors and branch slots follow the MPS calls above. */
typedef struct dcs_tree dcs_tree;
typedef struct dcs_tchunk dcs_tchunk;

/* Number of nodes of the tree with the given levels. */
int dcs_tree_n_nodes(const int *levels, int n_levels, int *n_nodes_out);

/* Bytes of device memory of a tree state: capacity branch slots, bond caps up
 * to chi_max, operator bonds (per edge) up to mpo_bond_max, contraction
 * intermediates of up to scratch_elems complex128-sized elements (from
 * dcs_tree_chunk_scratch), n_init_slots registered starting guesses. */
int dcs_tree_state_bytes(int precision, int n_levels, const int *levels, int capacity,
                         int chi_max, int mpo_bond_max, size_t scratch_elems,
                         int n_init_slots, size_t *bytes_out);
int dcs_tree_create(dcs_ctx *ctx, dcs_tree **out, int precision, int n_levels,
                    const int *levels, int capacity, int chi_max, int mpo_bond_max,
                    size_t scratch_elems, int n_init_slots, void *d_buffer, size_t bytes,
                    void *stream);
int dcs_tree_destroy(dcs_tree *t);

/* Starting guess for bond cap chi_cap: `gauss` holds a Gaussian tensor per
 * node (node order, node layout for the padded dims of chi_cap, complex128
 * interleaved).  From the deepest layer up, node v becomes the isometry of
 * its QR with the upper edge as the column index and the R factor is
 * absorbed into the parent's leg of v; the root is normalised.  Built in FP64
 * in the state's buffer, stored in the path precision.  Synchronises. */
int dcs_tree_set_init(dcs_tree *t, int chi_cap, const double *gauss, void *stream);

/* Branch slots: |0...0> (every edge of dimension 1), bond caps, release. */
int dcs_tree_branch_init_zero(dcs_tree *t, int n, const int *ids, const int *chi_caps,
                              void *stream);
int dcs_tree_branch_set_chi(dcs_tree *t, int n, const int *ids, const int *chi_caps);
int dcs_tree_branch_release(dcs_tree *t, int n, const int *ids);

/* Chunk (Sec. IV-C) compiled for the tree with the given levels: gates in time
 * order as in dcs_chunk_compile.  Host-only. */
int dcs_tree_chunk_compile(dcs_ctx *ctx, dcs_tchunk **out, int n_levels, const int *levels,
                           int n_ops, const int *q0, const int *q1, const double *mats);
int dcs_tchunk_destroy(dcs_tchunk *ch);
/* Operator bond of the edge above each node (n_nodes ints, 1 at the root). */
int dcs_tchunk_bonds(const dcs_tchunk *ch, int *w_out, int cap);
/* Largest contraction intermediate (complex128-sized elements) of a
 * compression step of this chunk from a ket of bond cap chi_ket into a bra
 * of cap chi_bra, and of the measurements that follow.  Host-only. */
int dcs_tree_chunk_scratch(const dcs_tchunk *ch, int chi_bra, int chi_ket, size_t *elems_out);

/* Compression step (as dcs_compress_step) of the listed tree branches;
 * fid_out[i] = f.  Synchronises. */
int dcs_tree_compress_step(dcs_tree *t, int n, const int *ids, const dcs_tchunk *const *chunks,
                           int n_sweeps, double *fid_out, void *stream);
/* p0_out[i] = n_0 / (n_0 + n_1) of qubit qubits[i]; norms kept for the
 * collapse.  Synchronises. */
int dcs_tree_measure_prob(dcs_tree *t, int n, const int *ids, const int *qubits, double *p0_out,
                          void *stream);
/* As dcs_collapse. */
int dcs_tree_collapse(dcs_tree *t, int n, const int *src_ids, const int *qubits,
                      const int *outcomes, const int *dst_ids, double eps, double *pm_out,
                      void *stream);
/* FP64 host copy of a branch: node tensors in node order, node layout for the
 * current edge dims (dims_out: the edge above each node, n_nodes ints). */
int dcs_tree_export(dcs_tree *t, int id, double *host_out, size_t cap_doubles, int *dims_out,
                    void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DCS_H */
