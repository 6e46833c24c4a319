/*
 * ttn.h -- C ABI of the MI355X (gfx950) tree-tensor-network trajectory engine.
 *
 * The engine simulates Monte Carlo quantum trajectories (Sec. III.C of
 * Barone, Jaschke, Siloi, Montangero, "Color code thresholds under
 * circuit-level noise beyond the Pauli framework") of a batch of B
 * independent pure states, each stored as a binary tree tensor network
 * (Sec. III.B, App. B / Fig. 7): a complete binary tree over L = 2^D leaves,
 * one qubit per leaf (unused leaves allowed), 3-leg node tensors
 * T[a][b][u] (left child, right child, parent), kept in canonical form around
 * an isometry centre.  Gates act along the tree path between the two leaves;
 * bonds are truncated to chi_max by dropping the smallest Schmidt values
 * (Sec. IV.A).  Noise channels are the systematic X rotation (SRX, Eq. 1) and
 * amplitude damping unravelled by its Kraus operators (Eq. 2-3), plus their
 * Pauli twirls (Eq. 9).
 *
 * Conventions common to every entry point
 *  - Every function returns ttn_status: TTN_OK (0) or a negative error code.
 *    No C++ exception crosses the ABI.  ttn_last_error(ctx) returns the last
 *    message for that context (valid until the next call on it).
 *  - Device pointers are plain HIP device addresses (e.g. torch tensor
 *    data_ptr()); host pointers are marked "host".  The caller owns every
 *    input/output buffer; the context owns its tensor pool and workspaces.
 *  - Work is enqueued on the context's HIP stream and is asynchronous unless
 *    marked [sync].  One context = one stream; a context is not thread-safe.
 *  - Trajectory row r of a batch uses the random stream keyed by
 *    (seed, traj_offset + r): Philox4x64-10, draw k = 64-bit word k mod 4 of
 *    the block at counter (k/4 + 1, 0, 0, 0), u = (w >> 11) * 2^-53.  Results
 *    therefore do not depend on B or on how rows are split into batches.
 *  - Precision: dtype TTN_C64 stores tensors in complex64 and contracts on
 *    FP32 MFMA with FP32 accumulation; Gram matrices, eigen-decompositions,
 *    norms and Born/Kraus probabilities are FP64.  TTN_C128 is FP64
 *    throughout.
 *
 * Error codes
 *  TTN_EINVAL     bad argument (qubit out of range, q0 == q1, non-finite or
 *                 unsupported matrix, chi_max < 1, unknown dtype/basis,
 *                 bad sizes); nothing was enqueued.
 *  TTN_ENOMEM     device allocation failed (reduce the batch).
 *  TTN_EDEVICE    a HIP runtime call failed.
 *  TTN_ENONFINITE a trajectory's norm became zero or non-finite; the row is
 *                 flagged (ttn_stats.flagged_rows) and the others continue.
 *  TTN_EPROB      a forced outcome had probability < 1e-300; log P = -inf is
 *                 written for that row.
 */
#ifndef TTN_H_
#define TTN_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ttn_status;
enum {
  TTN_OK = 0,
  TTN_EINVAL = -1,
  TTN_ENOMEM = -2,
  TTN_EDEVICE = -3,
  TTN_ENONFINITE = -4,
  TTN_EPROB = -5
};

enum { TTN_C64 = 0, TTN_C128 = 1 };

/* Amplitude-damping unravelling (Sec. III.C, Eq. 2-3 and the Trotterised
 * effective Hamiltonian).  Both jump with probability p1 = gamma <n1> to
 * K1 psi / sqrt(p1).  TTN_AD_KRAUS (default): no jump evolves by
 * K0 = diag(1, sqrt(1 - gamma)), which makes the trajectory average equal the
 * channel of Eq. 2 exactly.  TTN_AD_TROTTER: no jump evolves by the paper's
 * Trotterised gate exp(-(dt/2) L1^dag L1) = diag(1, e^{-gamma/2}) with
 * L1 = K1 / sqrt(dt), renormalised; it equals K0 to first order in gamma. */
enum { TTN_AD_KRAUS = 0, TTN_AD_TROTTER = 1 };

/* op-list record: 9 int32 per op (see ttn_oplist_upload) */
enum { TTN_OP_INIT = 0, TTN_OP_CNOT = 1, TTN_OP_SRX = 2, TTN_OP_AD = 3, TTN_OP_PAULI = 4, TTN_OP_MEAS = 5 };

typedef struct ttn_ctx ttn_ctx;
typedef struct ttn_oplist ttn_oplist;

typedef struct {
  int32_t n_qubits;              /* N >= 1 */
  const int32_t* leaf_of_qubit;  /* host [n_qubits], injective into [0, L), L = smallest power of 2 >= N (>= 2) */
  int32_t chi_max;               /* bond-dimension cap (1 .. 128: bonds double to 2 chi_max while a controlled gate rides on them) */
  double cutoff;                 /* keep Schmidt values with s^2 / sum s^2 > cutoff (>= 0) */
  int32_t dtype;                 /* TTN_C64 or TTN_C128 */
  int32_t ad_mode;               /* TTN_AD_KRAUS or TTN_AD_TROTTER */
  int32_t batch;                 /* B trajectories held by the context (>= 1) */
  uint64_t seed;                 /* random stream key, first word */
  void* stream;                  /* hipStream_t, NULL = default stream */
} ttn_config;

typedef struct {
  int32_t max_rank;          /* largest bond dimension over rows and bonds at the end */
  double discarded_weight;   /* sum over rows and truncations of the discarded fraction */
  int64_t degenerate_cuts;   /* cuts that fell inside a near-degenerate cluster */
  int32_t flagged_rows;      /* rows with a non-finite/zero norm or an impossible forced outcome */
  int64_t hops;              /* isometry-centre moves per row */
  int64_t launches;          /* kernel launches enqueued */
  double gemm_flops;         /* real flops of the contraction GEMMs, padded shapes, whole batch */
  double gram_flops;         /* real flops of the FP64 Gram GEMMs, padded shapes, whole batch */
  int64_t block_hops;        /* centre moves solved as two diagonal blocks (controlled-gate zip) */
} ttn_stats;

/* [sync] Validates the configuration and allocates the tensor pool and
 * workspaces for `batch` rows.  The state is the product |0...0>. */
ttn_status ttn_create(const ttn_config* cfg, ttn_ctx** out);

/* [sync] Frees everything the context owns (waits for its stream). */
ttn_status ttn_destroy(ttn_ctx* ctx);

const char* ttn_last_error(const ttn_ctx* ctx);

/* Product state (Sec. III: data start in |0>): qubit q in |0> (basis[q] = 0)
 * or |+> (basis[q] = 1), all bonds of dimension 1, centre at the root.
 * basis: host [n_qubits] or NULL (all |0>). */
ttn_status ttn_init_product(ttn_ctx* ctx, const uint8_t* basis);

/* Single-qubit gate or error on qubit q of every row: the one-qubit
 * operations of the circuit model (Sec. II.A, Fig. 1b-e: an error location
 * after a gate acts on one qubit, e.g. the SRX rotation of Eq. 1), applied to
 * the qubit's physical leg of its bottom tree node (Sec. III.B).
 * u: device float64 [rows][2][2][2] = (row-major matrix, re/im); row stride
 * 8 doubles, or 0 to broadcast one matrix.  A unitary on a physical leg keeps
 * the canonical form, so no centre move is made; a non-unitary matrix must
 * be followed by a measurement or explicit renormalisation by the caller.
 * Errors: TTN_EINVAL for a bad qubit, a null matrix or a negative stride. */
ttn_status ttn_apply_1q(ttn_ctx* ctx, int32_t q, const double* u, int64_t row_stride);

/* Two-qubit gate of the syndrome-extraction circuit (the CNOTs of Sec. II.A,
 * Fig. 1a) on a TTN: applied along the tree path between the two leaves, at a
 * cost that grows with their distance in the tree, O(log N) (Sec. III.B),
 * with the bonds it widens truncated by dropping the smallest Schmidt values
 * (Sec. IV.A).  g: host float64 [4][4][2], row-major, q0 the high bit (a host
 * matrix: its block structure decides on the host which qubit the zip starts
 * from; the 16 entries are copied to a context-owned device buffer for the
 * sibling case), qubits q0 != q1.  Sibling leaves: applied on their shared
 * node.  Otherwise the gate must be controlled on one of the two qubits
 * (block diagonal in its index, e.g. CNOT, CZ): it is split as
 * sum_k |k><k| (x) B_k, the index k is carried along the tree path from one
 * leaf to the other while the centre moves (exact, only numerically zero
 * Schmidt values dropped), and a sweep back truncates every bond of the path
 * to chi_max / cutoff.  Errors: TTN_EINVAL for bad qubits, a non-finite
 * matrix, or a non-controlled gate between non-siblings. */
ttn_status ttn_apply_2q(ttn_ctx* ctx, int32_t q0, int32_t q1, const double* g);

/* Born-rule measurement of qubit q in basis 0 (Z) or 1 (X): the ancilla
 * readout of every syndrome round and the final data readout of the memory
 * experiment (Sec. III, Fig. 1a), sampled per trajectory (Sec. III.C); outcome
 * 0 = the +1 eigenvector.  Moves the isometry centre to q's node, computes
 * p0 = |Pi_0 psi|^2 / |psi|^2 in FP64, takes outcome 0 iff u < p0 with
 * u = draw `draw` of the row's stream (or the forced outcome), projects and
 * rescales to unit norm, and adds log p(outcome) to logp.
 * forced: device uint8 [rows] or NULL; bits: device uint8 [rows] (out);
 * logp: device float64 [rows] (accumulated). */
ttn_status ttn_measure_project(ttn_ctx* ctx, int32_t q, int32_t basis, const uint8_t* forced,
                               uint8_t* bits, double* logp, uint64_t traj_offset, int32_t draw);

/* Quantum jump of a two-outcome Kraus channel {K0, K1} on qubit q (Eq. 2-3
 * for amplitude damping): p1 = |K1 psi|^2 / |psi|^2 (FP64, centre at q),
 * branch 1 iff u < p1 (or forced), psi -> K_branch psi / sqrt(p_branch),
 * logp += log p_branch.  k: device float64 [rows][2][2][2][2] =
 * (K0, K1; row-major; re/im), row stride 16 doubles or 0 to broadcast.
 * forced: device int8 [rows] or NULL; branch: device int8 [rows] (out). */
ttn_status ttn_kraus_jump(ttn_ctx* ctx, int32_t q, const double* k, int64_t row_stride,
                          const int8_t* forced, int8_t* branch, double* logp,
                          uint64_t traj_offset, int32_t draw);

/* [sync] Upload an op list: host int32 [n_ops][9] with columns
 *   op, q0, q1, arg, loc, draw, rec, prev, tick
 * op: TTN_OP_INIT (q0 prepared in basis arg = 0 |0> / 1 |+> from its known
 *     previous state: never measured (prev = -1) or measured in basis prev
 *     with the outcome in record column rec -- the reset),
 *     TTN_OP_CNOT (control q0, target q1), TTN_OP_SRX (exp(-i theta X/2),
 *     theta = theta[row][loc]), TTN_OP_AD (amplitude damping, gamma[row][loc],
 *     draw), TTN_OP_PAULI (twirled channel: arg 0 = SRX twirl, 1 = AD twirl,
 *     draw), TTN_OP_MEAS (basis arg, record column rec, draw).
 * n_loc / n_rec / n_draws: parameter columns, record bits, draws per row. */
ttn_status ttn_oplist_upload(ttn_ctx* ctx, const int32_t* ops, int32_t n_ops, int32_t n_loc,
                             int32_t n_rec, int32_t n_draws, ttn_oplist** out);
ttn_status ttn_oplist_free(ttn_oplist* ol);

/* One Monte Carlo shot per row of the memory experiment of Sec. III (Fig. 1):
 * the data start in |0>, C rounds of syndrome extraction with an error
 * location after every gate, idle step and (re)initialisation (Fig. 1b-e),
 * then the final data readout; each row is one quantum trajectory (Sec. III.C)
 * of the TTN state, so averages over rows estimate the noisy circuit's
 * output distribution.  Runs the whole op list on every row, starting from
 * the product state (ttn_init_product is called internally with every qubit
 * in |0>).
 * theta, gamma: device float64 [rows][n_loc] with row stride params_stride
 * (0 = broadcast one row); may be NULL when the op list has no such op.
 * records: device uint8 [rows][n_rec]; branches: device int8 [rows][n_ad]
 * (n_ad = number of AD ops; may be NULL if none); logp: device float64
 * [rows] (overwritten with sum log p).  st: host, may be NULL; filling it
 * synchronises the stream. */
ttn_status ttn_batch_run_circuit(ttn_ctx* ctx, const ttn_oplist* ol, const double* theta,
                                 const double* gamma, int64_t params_stride, uint64_t traj_offset,
                                 uint8_t* records, int8_t* branches, double* logp, ttn_stats* st);

/* Launch mode of ttn_batch_run_circuit (no passage of the paper: how the
 * library issues the work of Sec. III.C's trajectories).
 *  TTN_RUN_DYNAMIC (default): after each centre move the host reads the
 *    batch's largest kept count and pads the new bond to it (one small
 *    device-to-host read per move; shapes follow the batch's ranks).
 *  TTN_RUN_STATIC: no host read; every bond keeps its static padded bound
 *    (chi_max or the bond's physical bound, doubled while a controlled gate
 *    rides on it); each row's kept values are a prefix and the rest is zero,
 *    so results agree with the dynamic mode up to floating-point summation
 *    order (tile shapes follow the padded dimensions).  Launch shapes depend
 *    only on the op list.
 *  TTN_RUN_GRAPH: static shapes, and the whole op list is captured once into
 *    a HIP graph per (op list, argument buffers, probability trace) on a
 *    stream the context owns and replayed on later calls, ordered after the
 *    context's stream by events; the first call with new buffers runs eagerly
 *    and captures, later calls write the trajectory offset to device memory
 *    and launch the graph (bit-identical to TTN_RUN_STATIC).  Profiling is
 *    unavailable in this mode (TTN_EINVAL).
 * Changing the mode waits for the stream and drops a captured graph.
 * captures / replays (may be null) receive the graph counts so far.
 * Errors: TTN_EINVAL for an unknown mode. */
enum { TTN_RUN_DYNAMIC = 0, TTN_RUN_STATIC = 1, TTN_RUN_GRAPH = 2 };
ttn_status ttn_set_run_mode(ttn_ctx* ctx, int32_t mode, int64_t* captures, int64_t* replays);

/* log P(record) of given records and Kraus branches: the probability of one
 * trajectory of Sec. III.C, i.e. the product of the Born probabilities of its
 * measurement outcomes and the jump / no-jump probabilities of its Kraus
 * branches (Eq. 2-3), computed by one pass with every sampled event forced
 * instead of drawn.  Same op list and parameters as above; records
 * device uint8 [rows][n_rec], branches device int8 [rows][n_ad] (NULL if
 * no AD op); logp device float64 [rows] (out). */
ttn_status ttn_log_prob(ttn_ctx* ctx, const ttn_oplist* ol, const uint8_t* records,
                        const int8_t* branches, const double* theta, const double* gamma,
                        int64_t params_stride, double* logp, ttn_stats* st);

/* [sync] log P(record) as ttn_log_prob and its derivatives by every
 * location's parameters: dtheta[row][l] = d log P / d theta_l (the SRX angle
 * of Eq. 1 at location l), dgamma[row][l] = d log P / d gamma_l (the damping
 * of Eq. 2-3; the recorded Kraus branch is held fixed: a jump contributes
 * 1/gamma, no jump the derivative of K0).  Reverse mode: the adjoint state
 * A_>^dagger psi_N is carried backwards through the adjoint of every op
 * (SRX(-theta), CNOT, the recorded projector, K^dagger, the inverse reset)
 * in a second context of the same configuration (allocated on first use),
 * and every layer of noise ops between two other ops is differentiated
 * through the leaf environments of the contraction <lambda| N |psi>; the
 * state before each layer is recomputed from at most 16 snapshots taken on
 * the forward pass (device memory: the second context, the snapshots and one
 * environment per bond are allocated for the call).  Exact for untruncated
 * runs; with truncation it is the derivative of the same approximation
 * applied to both states.  The op list must not hold twirled (PAULI) ops.
 * theta, gamma: as for ttn_batch_run_circuit (both required; pass zeros for
 * an absent channel); logp device float64 [rows] (out); dtheta, dgamma
 * device float64 [rows][n_loc] (out, overwritten).  Returns TTN_EPROB when a
 * forced outcome had probability < 1e-300 or an overlap vanished (those rows
 * are flagged). */
ttn_status ttn_log_prob_grad(ttn_ctx* ctx, const ttn_oplist* ol, const uint8_t* records,
                             const int8_t* branches, const double* theta, const double* gamma,
                             int64_t params_stride, double* logp, double* dtheta, double* dgamma,
                             ttn_stats* st);

/* Per-draw probability trace (test and statistics export of the same runs):
 * with probs set (device float64 [rows][stride], stride >= the op list's
 * n_draws), every later ttn_batch_run_circuit / ttn_log_prob /
 * ttn_measure_project / ttn_kraus_jump writes, for each sampled event, the
 * probability of the outcome taken (the Born probability of a measurement
 * outcome, the jump or no-jump probability of an AD op, the probability of
 * the Pauli chosen by a twirled op; Sec. III.C) to probs[row][draw]; columns of
 * draws that did not happen are left untouched.  probs = NULL stops the
 * trace.  The buffer must stay allocated while the trace is on.  Errors:
 * TTN_EINVAL for stride < 1 with a non-null buffer. */
ttn_status ttn_trace_probs(ttn_ctx* ctx, double* probs, int64_t stride);

/* Logical readout (final-data lookup decoder): fail[row] = parity of the
 * data bits XOR parity of the minimum-weight correction of their Z-check
 * syndrome.  data_rec: host int32 [n_data] record columns of the final data
 * bits (n_data <= 64); checks: host uint8 [n_checks][n_data] incidence
 * (n_checks <= 24).  records: device uint8 [rows][n_rec]; fail: device uint8
 * [rows].  Builds the leader table on the host (breadth-first search over
 * single flips, qubits in ascending order) and decodes on the device. */
ttn_status ttn_decode(ttn_ctx* ctx, const uint8_t* records, int32_t n_rec, const int32_t* data_rec,
                      int32_t n_data, const uint8_t* checks, int32_t n_checks, uint8_t* fail);

/* Logical readout as ttn_decode, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the leader-parity table (2^n_checks bytes), the data
 * record columns and the check masks are staged in a fixed library-owned
 * device array of TTN_DECODE_STATIC_SCRATCH_BYTES per GPU, held until the
 * process ends (its address on a device is resolved when the first context
 * is created there), instead of buffers the context allocates on first use.
 * Limit: n_checks <= TTN_DECODE_STATIC_MAX_CHECKS (16; d <= 7 colour codes
 * have at most 18 plaquettes, so d = 7 needs ttn_decode), n_data <= 64;
 * larger sizes return TTN_EINVAL.  Every call on a GPU shares that GPU's
 * array and overwrites every byte the kernel reads: calls that overlap on one
 * GPU (other streams, other threads) race.  [sync]: returns after the decode
 * has run (the table is built on the host and copied with the call).  Same
 * arguments and outputs as ttn_decode. */
#define TTN_DECODE_STATIC_MAX_CHECKS 16
#define TTN_DECODE_STATIC_SCRATCH_BYTES (65536 + 512)
ttn_status ttn_decode_static(ttn_ctx* ctx, const uint8_t* records, int32_t n_rec, const int32_t* data_rec,
                             int32_t n_data, const uint8_t* checks, int32_t n_checks, uint8_t* fail);

/* Move the isometry centre through every node (depth-first) so each bond is
 * re-decomposed and truncated with the context's rule; afterwards the bond
 * dimensions are the Schmidt ranks above the cutoff. */
ttn_status ttn_compress(ttn_ctx* ctx);

/* [sync] Test exports.  ttn_to_statevector contracts row `row` into all
 * 2^N amplitudes (qubit 0 the most significant bit), amp: device float64
 * [2^N][2], N <= 26.  ttn_bond_dims writes the current dimension of the
 * bond above every node 1..L-1 of row `row` (node 1 = root, children 2i,
 * 2i+1) to dims: host int32 [L] (dims[0] unused). */
ttn_status ttn_to_statevector(ttn_ctx* ctx, int32_t row, double* amp);
ttn_status ttn_bond_dims(ttn_ctx* ctx, int32_t row, int32_t* dims);

/* [sync] Uniforms of the rows' streams: out device float64 [rows][n_draws]
 * for rows traj_offset .. traj_offset + rows - 1. */
ttn_status ttn_uniforms(ttn_ctx* ctx, uint64_t traj_offset, int32_t rows, int32_t n_draws, double* out);

/* Host-side evaluation of the same counter-based generator (no GPU needed). */
double ttn_philox_uniform_host(uint64_t seed, uint64_t traj, uint64_t draw);

/* Host-side sweep plan of the coset-ordered eigensolver for N = 2^k,
 * k = 2 .. 8 (no GPU needed): a cyclic Jacobi sweep visits every pair of
 * the N indices once (Sec. III.B's truncations solve G = V diag(s^2) V^H by
 * such sweeps); this one is the matchings {(i, i ^ d)}, d = 1 .. N - 1,
 * in groups.  groups[g] = a | b << 8 | m << 16: the group applies the m
 * matchings a, b, a ^ b (first m of them), all inside the cosets of
 * {0, a, b, a ^ b}.  Writes at most cap entries; returns the number of
 * groups, or -1 for k outside 2 .. 8 or cap too small. */
int32_t ttn_test_sweep_plan(int32_t k, uint32_t* groups, int32_t cap);

/* [sync] Kernel-level test exports (not part of the simulation path; the
 * same kernels the engine launches).  Buffers are device memory of the
 * context's dtype (complex64 = 2 floats, complex128 = 2 doubles per
 * element); *_elems give their sizes in complex elements and the call fails
 * with TTN_EINVAL if the operation would reach past them.
 *  ttn_test_leg_apply: out[t][..a..] = sum_i W[t][a][i] T[t][..i..] on leg
 *    `leg` (0, 1, 2) of T [rows][d0][d1][d2]; W [rows][newd][n], n = d[leg].
 *  Both GEMM exports run in the fixed rule's tile shape, or in the one that
 *  ttn_autotune(ctx, 2 + c, ...) forces.
 *  ttn_test_gram: G[t][i][j] = sum over the other legs of
 *    conj(T[..i..]) T[..j..], G float64 [ksplit][rows][n][n][2] (FP64
 *    accumulation): with ksplit > 1 the sum runs in ksplit parts, one per
 *    slice, and G is the sum of the slices.  G is Hermitian and, as in the
 *    engine, output tiles wholly below the diagonal are not written: every
 *    i <= j is (the upper triangle the solvers read).
 *  ttn_test_eigh, ttn_test_move: read only the upper triangle (i <= j) of
 *    each row's G.
 *  ttn_test_eigh: the factors of a centre move computed from G (as in
 *    ttn_ctx's hops): W_iso[t][a][i] = V[i][a] / s_a, W_abs[t][a][i] =
 *    conj(V[i][a]) s_a / |s_kept|, a < rank[t] in descending s, zero beyond;
 *    rows <= batch, n <= 2 * min(chi_max, ...) of the context; sweeps
 *    (device int32 [rows] or NULL) receives the Jacobi sweep count.
 *    blocks = 2: G is block diagonal with two n/2 blocks, solved apart; the
 *    cutoff refers to the whole trace, block b fills rows [b new_pad/2,
 *    (b+1) new_pad/2) and columns [b n/2, (b+1) n/2) of the factors (zeros
 *    in the other block's columns), at most cap values per block; rank and
 *    sweeps are not written. */
ttn_status ttn_test_leg_apply(ttn_ctx* ctx, int32_t rows, const int32_t* dims3, int32_t leg, const void* T,
                              int64_t t_elems, const void* W, int64_t w_elems, int32_t newd, void* out,
                              int64_t out_elems);
ttn_status ttn_test_gram(ttn_ctx* ctx, int32_t rows, const int32_t* dims3, int32_t leg, const void* T,
                         int64_t t_elems, double* G, int64_t g_elems, int32_t ksplit);
ttn_status ttn_test_eigh(ttn_ctx* ctx, int32_t rows, int32_t n, int32_t new_pad, int32_t cap, double cutoff,
                         const double* G, int64_t g_elems, void* W_iso, void* W_abs, int64_t w_elems,
                         int32_t* rank, int32_t* sweeps, int32_t blocks);
/* ttn_test_move: the factors of an exact centre move by pivoted Cholesky
 * (the QR route of complex64 contexts): same arguments and outputs as
 * ttn_test_eigh (without sweeps), n <= 64 per diagonal block, or n <= 128
 * without blocks; the rank is the number of pivots above cutoff x trace, at
 * most cap.  For n > 64 the call behaves as the batch driver's try before a
 * truncating eigen-decomposition: a row whose weight above the cutoff needs
 * more than cap pivots gets rank -1 and its W rows are left untouched. */
ttn_status ttn_test_move(ttn_ctx* ctx, int32_t rows, int32_t n, int32_t new_pad, int32_t cap, double cutoff,
                         const double* G, int64_t g_elems, void* W_iso, void* W_abs, int64_t w_elems,
                         int32_t* rank, int32_t blocks);

/* Profiling.  While enabled, every kernel launch of the context is
 * bracketed by HIP events on its stream, grouped by kernel class, and the
 * algorithmic work of the launches is added to per-row ledgers from the
 * actual (unpadded) dimensions of each row:
 *   eigensolver   36 n^3 real flops for an n x n complex Hermitian
 *                 eigen-decomposition with vectors, n = the number of
 *                 non-zero eigenvalues;
 *   Gram          8 n^2 r real flops (n as above, r = product of the other
 *                 two actual leg dimensions), per diagonal block when the
 *                 move is block diagonal;
 *   contraction   8 k n r real flops for each of the two factor products
 *                 (k = kept values);
 *   exact move    8 (r^2 (3n - 2r) / 3 + r^3 / 3) real flops for a pivoted
 *                 Cholesky factorisation of rank r and the inverse of its
 *                 r x r triangle (n = the problem size after dropping zero
 *                 rows).
 * The Gram and contraction classes also ledger algorithmic HBM bytes: every
 * operand read once and every result written once at the actual dimensions
 * (complex64 / complex128 tensor elements, FP64 complex Gram entries), i.e.
 * Gram  es (n0 + n1) r + 16 (n0^2 + n1^2),  contraction  es ((n + k) r + 2 k n)
 * per side of the move and per diagonal block.
 * The Gram and contraction ledgers track the actual leg dimensions from the
 * last state reset (ttn_init_product, or the start of a run) on: enable
 * profiling before it.  Enabling resets the counters (the first enable
 * creates the library's pool of timing events, so that none is created
 * while a profiled run is timed).  ttn_profile_read
 * [sync] returns, for one class, the summed elapsed milliseconds, the number
 * of launches, the ledgered flops and (alg_bytes may be null) the ledgered
 * bytes (0 for classes without a ledger). */
enum {
  TTN_CLASS_CONTRACT = 0,     /* c64/c128 leg contractions (MFMA)           */
  TTN_CLASS_GRAM = 1,         /* FP64 Gram matrices (MFMA)                  */
  TTN_CLASS_EIGH_SMALL = 2,   /* Jacobi eigensolver, n <= 64, vectors in LDS */
  TTN_CLASS_EIGH_LARGE = 3,   /* Jacobi eigensolver, n > 64 (circle- and coset-ordered solvers and the vector replay) */
  TTN_CLASS_LEAF = 4,         /* bottom-node gates, measurements, jumps     */
  TTN_CLASS_EXTEND = 5,       /* controlled-gate index extensions           */
  TTN_CLASS_OTHER = 6,
  TTN_CLASS_MOVE = 7,         /* pivoted-Cholesky exact centre moves        */
  TTN_NCLASS = 8
};
ttn_status ttn_profile_enable(ttn_ctx* ctx, int32_t on);
ttn_status ttn_profile_read(ttn_ctx* ctx, int32_t cls, double* ms, int64_t* launches, double* alg_flops,
                            double* alg_bytes);

/* Tile-shape tuner for the batched contractions and Gram matrices (no
 * passage of the paper: launch tuning of this library).  Every such launch
 * runs in one of six output-tile shapes (64x64, 128x32, 32x128, 16x128, and
 * 32x32 and 16x16 with the K range split over the wavefronts); by default a
 * fixed rule on the output dimensions picks it.  With on = 1, a launch whose
 * shape (kind, M, N, K, inner/outer K split, batch sizes, split-K, operand
 * layouts) has not been measured yet first runs once in every tile shape
 * that fits it (the 16-row shapes for at most 16 rows) on its own
 * operands, timed with events on the context's stream (the stream is
 * synchronised: tuning stalls the host), and the fastest is kept for that
 * shape; results do not depend on the choice beyond floating-point
 * summation order.  on = 0 stops measuring new shapes but keeps using the
 * measured ones; on = -1 forgets them and returns to the fixed rule.
 * on = 2 + c (c = 0..5: 64x64, 128x32, 32x128, 32x32, 16x16, 16x128) runs
 * every launch in tile shape c, whatever it fits, until the next call
 * (testing each shape on any problem); 0, 1 and -1 end it.
 * shapes / changed (may be null) receive the number of shapes measured and
 * how many of them differ from the fixed rule.  Errors: TTN_EINVAL for
 * other values of on. */
ttn_status ttn_autotune(ttn_ctx* ctx, int32_t on, int64_t* shapes, int64_t* changed);

/* Library build identification (no GPU needed). */
const char* ttn_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TTN_H_ */
