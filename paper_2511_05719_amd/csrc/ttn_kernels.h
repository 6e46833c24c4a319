// Internal launch interface of the TTN engine's HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ttn {

// ---------------------------------------------------------------- GEMM ----
enum GemmKind { GEMM_C64 = 0, GEMM_C128 = 1, GEMM_GRAM_C64 = 2, GEMM_GRAM_C128 = 3 };

struct GemmDesc {
  const void* A;
  const void* B;
  void* C;
  int M, N, K, Kin;   // K index l = (l / Kin, l % Kin) with strides (l1, l2)
  // N index j = (j / Nin, j % Nin) with strides (sBj1, sBj) on B and (sCj1,
  // sCj) on C when 0 < Nin < N (N a multiple of Nin); otherwise one stride
  int Nin;
  long long sBj1, sCj1;
  int H;              // inner batch size (>= 1)
  int G2;             // block batch size (0 or 1: none; 2: the two diagonal
                      // blocks of a block-diagonal operand, strides s?g)
  long long sAt, sAh, sAi, sAl1, sAl2, sAg;
  long long sBt, sBh, sBl1, sBl2, sBj, sBg;
  long long sCt, sCh, sCi, sCj, sCg;
  int ksplit;               // 0 or 1: one K range; k > 1: k partial products
  long long sCz;            // element stride between the partial products of C
  int conjA, conjB;
  int a_m_fast, b_n_fast;   // operand dimension that is unit-stride on load
  int same_ab;              // A and B are one operand with one layout (a Gram matrix): a
                            // diagonal tile of a square tile shape stages it once
  int herm;                 // C is Hermitian: output tiles wholly below the diagonal are
                            // neither computed nor written (readers use the upper triangle)
  int tilesN;               // filled by the launcher
  // Per-trajectory extents (all optional).  A node tensor is stored padded
  // to the batch's largest bond dimensions, and trajectory t's entries are
  // zero beyond its own extent on each bond (a prefix).  With ext set, a
  // field e > 0 names the bond whose extent ext[t * ext_stride + e] bounds
  // that dimension, e < 0 the new bond of the move in progress, whose extent
  // is knew[t * 4], and e = 0 leaves it padded.  Output tiles beyond the
  // extent are written as zeros without K work; the K loop stops at
  // extent(eKo) * extent(eKi) with l = (l / Kin_t, l % Kin_t), Kin_t =
  // min(Kin, extent(eKi)).
  const int* ext;
  const int* knew;
  long long ext_stride;
  int eM, eN, eH;           // M <= extent(eM) * mM, N <= extent(eN) * mN, H <= extent(eH)
  int mM, mN;               // (with Nin: eN, mN bound j % Nin, eNo bounds j / Nin)
  int eNo;
  int eKo, eKi;             // outer (l / Kin) and inner (l % Kin) parts of K
  // Bands (optional, band = 1): only rows [bM0, bM1), columns [bN0, bN1) and
  // inner batches [bH0, bH1) can be non-zero; output tiles wholly outside
  // are written as zeros without K work (a block-structured leg of the node).
  // With Nin, [bN0, bN1) bounds j % Nin (element by element) and [bNo0,
  // bNo1) bounds j / Nin.
  int band;
  int bM0, bM1, bN0, bN1, bH0, bH1, bNo0, bNo1;
};

// cfg: one of the kZgemmCfgs tile shapes (64x64, 128x32, 32x128, 32x32 and
// 16x16 with the K chunk split over the waves, 16x128), or -1 for the fixed
// rule
constexpr int kZgemmCfgs = 6;
hipError_t launch_zgemm(const GemmDesc& d, int batch, int kind, hipStream_t st, int cfg = -1);
// the fixed rule's tile shape for d, and its output tiles per (t, g, h)
int zgemm_rule_cfg(const GemmDesc& d);
// whether the tuner should measure tile shape cfg for d
bool zgemm_cfg_useful(const GemmDesc& d, int cfg);
long long zgemm_tiles(const GemmDesc& d);

// ---------------------------------------------------------------- EIGH ----
// Hermitian eigen-decomposition of the per-trajectory Gram matrix of one
// bond (FP64 Jacobi), truncation, and the two factor matrices of the centre
// move:  W_iso[a][i] = V[i][a] / s_a  and  W_abs[a][i] = conj(V[i][a]) s_a / |s_kept|
// for the kept a (descending eigenvalue order), zero rows beyond.
struct EighDesc {
  const double2* G;     // [batch][n][n]
  int n;                // matrix size (bond dimension before the move)
  int new_pad;          // rows of the W outputs (padded bond dimension after)
  int cap;              // at most this many kept values (chi cap)
  double cutoff;        // keep lambda_a > cutoff * sum(lambda)
  void* W_iso;          // [batch][new_pad][n]  (float2 or double2)
  void* W_abs;          // [batch][new_pad][n]
  int out_c128;         // 1: W in double2, 0: float2
  int blocks;           // 1, or 2: G is block diagonal, solve the halves apart
  int* rank_out;        // [batch] stride rank_stride (may be null)
  int* rank_max;        // [batch] stride rank_stride: running maximum (may be null)
  long long rank_stride;
  double* flops_acc;    // [batch] += algorithmic flops (may be null)
  int* sweeps_out;      // [batch] Jacobi sweeps used (may be null)
  double* disc_acc;     // [batch] += discarded weight fraction
  int* flags;           // [batch] |= 1 on non-finite / zero norm
  int* degen_acc;       // [batch] += 1 on a cut inside a near-degenerate cluster
  // workspace for n > 64 (per problem: a row, or a diagonal block of a row)
  double* rot_log;      // [problems][log_stride]: per step, (c, s) of each pair
  int max_steps;
  double* lam_sorted;   // [batch][n]
  int* order;           // [batch][n]
  int* kept;            // [batch]
  double* scale_abs;    // [batch]
  int* nsteps;          // [batch]
  int* nk_out;          // [batch][4]: (non-zero eigenvalues, kept) of block 0, block 1 (may be null)
  // [problems] (may be null): the pivoted Cholesky of 65..128 columns writes
  // 1 where it has written the factors, 0 where the weight above the cutoff
  // needs more than cap pivots; the large eigensolver skips the 1s
  int* done;
  double tol;           // rotate a pair while |g_pq| > tol sqrt(g_pp g_qq) (0: 1e-15)
  int early_stop;       // 1: also stop once every off-diagonal ratio is below sqrt(tol) / 4
  int gsplit;           // G is the sum of gsplit partial products (0 or 1: one)
  long long gslice;     // element stride between them
  long long log_stride; // doubles of rot_log per problem (problem = row, or (row, block))
  double2* gpk;         // problems of size > 128: packed G in device memory, [batch][256 * 257 / 2]
  // problems above 64: the circle-ordered solver runs on aux_stream beside
  // the coset-ordered one (fork after ev_fork on the caller's stream, joined
  // through ev_join before the vector replay); all null: one stream
  hipStream_t aux_stream;
  hipEvent_t ev_fork, ev_join;
};
hipError_t launch_eigh(const EighDesc& d, int batch, hipStream_t st);
// one-time set-up of the eigensolver kernels on the current device (idempotent)
hipError_t eigh_prepare();
// Exact (non-truncating) centre-move factors by pivoted Cholesky of G, same
// outputs as launch_eigh (rank = pivots above cutoff x trace, at most cap);
// problems of size <= 64 per block, or <= 128 without blocks (with done)
hipError_t launch_pchol(const EighDesc& d, int batch, hipStream_t st);
int eigh_max_sweeps();
// size that the solver pads a problem above 64 to (a power of two, >= 4):
// its rotation log holds eigh_max_sweeps() * (N - 1) matchings of N / 2 pairs
int eigh_padded_size(int n);
// the coset-ordered solver's sweep plan for N = 2^k (a | b << 8 | m << 16
// per group): the number of groups, or -1 (k outside 2 .. 8, cap too small)
int eigh_sweep_plan(int k, unsigned* groups, int cap);

// ----------------------------------------------------------- LEAF OPS ----
// One op on one or both physical legs of a bottom node, for every trajectory.
enum LeafOpKind {
  LOP_MATRIX = 0,     // explicit 2x2 per trajectory or broadcast (mat)
  LOP_SRX = 1,        // exp(-i theta X / 2), theta = params[row][loc]
  LOP_PAULI_SRX = 2,  // twirled SRX: X with p = sin^2(theta/2), draw
  LOP_PAULI_AD = 3,   // twirled AD: I/X/Y/Z, draw
  LOP_INIT = 4,       // prepare basis state from the known previous state
  LOP_CNOT = 5,       // both legs: control leg `leg`, target the other
  LOP_GATE4 = 6,      // both legs: explicit 4x4 (leg 0 = high bit)
  LOP_MEAS = 7,       // Born measurement (centre here), draw or forced
  LOP_KRAUS_AD = 8,   // amplitude-damping jump (centre here), draw or forced
  LOP_KRAUS_MAT = 9,  // two explicit Kraus matrices (centre here)
};

struct LeafOp {
  int kind;
  int leg;           // physical leg (0 = a, 1 = b) of the qubit
  int arg;           // INIT: target basis; MEAS: basis; PAULI: unused
  int prev;          // INIT: previous measurement basis (-1 none)
  int rec;           // MEAS: record index; INIT: previous record index
  int loc;           // parameter column
  int draw;          // RNG draw index
  int branch;        // KRAUS: branch column
};

constexpr int kMaxLeafOps = 40;
struct LeafBatch {
  LeafOp ops[kMaxLeafOps];      // executed in order by every row
  void* node_ptr[kMaxLeafOps];  // per op: base pointer of its bottom node tensor
  int node_u[kMaxLeafOps];      // per op: padded up-leg dimension of that node
  int n_ops;
  int n_rows;          // trajectories in this batch
  int c128;
  const double* theta; long long theta_row_stride;   // [rows][n_loc] (row stride 0 = broadcast)
  const double* gamma; long long gamma_row_stride;
  const double* mat;   long long mat_row_stride;     // LOP_MATRIX / GATE4 / KRAUS_MAT data
  uint8_t* records; long long rec_stride;
  const uint8_t* forced_rec; long long forced_rec_stride;
  int8_t* branches; long long br_stride;
  const int8_t* forced_br; long long forced_br_stride;
  double* logp;
  double* probs; long long probs_stride;             // [rows][stride]: probability of each sampled event (may be null)
  int ad_trotter;      // 1: LOP_KRAUS_AD without a jump applies diag(1, e^{-gamma/2}), renormalised
  int* flags;
  uint64_t seed;
  uint64_t traj_offset;
  const uint64_t* traj_offset_dev;   // if set, the offset is read from device memory (graph replays)
  int adjoint;         // 1: apply each op's adjoint (SRX, INIT, CNOT, forced MEAS and
                       //    KRAUS_AD), rescaled to unit norm; no log P, records or branches
};
hipError_t launch_leaf_ops(const LeafBatch& b, hipStream_t st);

// ------------------------------------------------------ DATA MOVEMENT ----
// Copy a node into a larger zeroed buffer with one or two legs doubled
// (the operator-Schmidt index k of a controlled gate rides on those legs).
struct ExtendDesc {
  const void* src; void* dst;
  int d0, d1, d2;          // source dims
  int leg_in, leg_out;     // legs doubled (leg_out = -1: none)
  int mode;                // 0: delta-thread (block k on both legs)
                           // 1: leg_in doubled, block k = bmat[k] applied on the
                           //    physical leg ctrl_leg (start or end of the gate)
  int ctrl_leg;            // mode 1: physical leg the 2x2 blocks act on
  double bmat[2][2][2][2]; // mode 1: (k, row, col, re/im)
  long long src_stride, dst_stride;   // per trajectory
  int c128;
};
hipError_t launch_extend(const ExtendDesc& d, int batch, hipStream_t st);

hipError_t launch_fill_zero(void* p, long long bytes, hipStream_t st);

// product state of one node for every row: a bottom node holds |s0>|s1>
// (s = 0 -> |0>, 1 -> |+>) with up dimension 1; an internal node is the 1x1x1
// tensor 1.
struct InitDesc {
  void* ptr;
  int bottom;
  int basis0, basis1;
  int c128;
};
hipError_t launch_init_product(const InitDesc& d, int batch, hipStream_t st);
hipError_t launch_fill_i32(int* p, int value, long long n, hipStream_t st);
hipError_t launch_fill_f64(double* p, double value, long long n, hipStream_t st);
hipError_t launch_fill_u64(uint64_t* p, uint64_t value, long long n, hipStream_t st);
// n complex ones (complex64 or complex128)
hipError_t launch_fill_cone(void* p, int c128, long long n, hipStream_t st);

// logical readout: fail[t] = parity(data) ^ parity(leader(syndrome(data)))
hipError_t launch_decode(const uint8_t* records, long long rec_stride, const int* data_rec, int n_data,
                         const uint32_t* check_masks /*[P] bitmask over data index*/, int n_checks,
                         const uint8_t* leader_parity /*[2^P]*/, uint8_t* fail, int batch, hipStream_t st);

// Work ledger of the profiler: per-row actual leg dimensions adim[B][L][3]
// (the padded shapes of the launches are upper bounds of these), updated
// after every centre move and leg doubling, and the algorithmic flops of the
// Gram and contraction launches computed from them.
struct LedgerHop {
  int* adim;
  const int* nk;        // [B][4] written by the eigensolver (EighDesc::nk_out)
  int L;
  int x, lx, y, ly;     // centre moved from x (leg lx) to y (leg ly)
  double* gram_acc;     // [B]
  double* contract_acc; // [B]
  // algorithmic HBM bytes of the same launches (each operand read once, each
  // result written once, at the actual dimensions): es bytes per tensor
  // element, 16 per FP64 complex Gram entry
  double* gram_bytes;   // [B]
  double* contract_bytes; // [B]
  int es;
};
hipError_t launch_ledger_hop(const LedgerHop& d, int batch, hipStream_t st);
hipError_t launch_ledger_double(int* adim, int L, int node, int l0, int l1, int batch, hipStream_t st);
hipError_t launch_ledger_reset(int* adim, int L, int batch, hipStream_t st);

// out[c] = max over rows t of nk[t][c], c = 0..3 (one workgroup)
hipError_t launch_nk_max(const int* nk, int batch, int* out, hipStream_t st);
// per-row copy of one column: dst[t * dst_stride] = src[t * src_stride]
// (a bond's per-row extents from the kept counts of its move)
hipError_t launch_set_ext(int* dst, long long dst_stride, const int* src, long long src_stride, int batch,
                          hipStream_t st);

// ------------------------------------------------------------ ADJOINT ----
// Noise ops of one leaf inside one layer of the adjoint gradient (applied in
// list order), and the bottom-node environment kernels (ttn_adjoint.hip).
enum NoiseKind { NOISE_SRX = 0, NOISE_AD = 1 };
constexpr int kMaxLeafNoise = 8;
struct LeafNoise {
  int n;
  int kind[kMaxLeafNoise];
  int loc[kMaxLeafNoise];      // parameter column
  int branch[kMaxLeafNoise];   // NOISE_AD: branch column of the record
};
struct EnvParams {
  const double* theta;
  const double* gamma;
  long long pstride;           // row stride of theta / gamma (0: shared)
  const int8_t* branches;      // [rows][br_stride] recorded Kraus branches
  long long br_stride;
};
struct EnvBottom {
  const void* lam;             // adjoint tree's bottom node [rows][2][2][ul]
  const void* psi;             // state tree's bottom node [rows][2][2][up]
  int ul, up;                  // up-bond dimensions (<= 4)
  void* out;                   // up environment [rows][ul][up] (k_env_bottom_up)
  const void* down;            // down environment [rows][ul][up] (k_env_leaf_grad)
  LeafNoise nz[2];             // noise ops on leaf 0 (leg a) and leaf 1 (leg b)
  EnvParams par;
  double* dtheta;              // [rows][gstride] += d log P / d theta
  double* dgamma;              // [rows][gstride] += d log P / d gamma
  long long gstride;
  int* flags;                  // [rows] |= 8 on a vanishing overlap
  int c128;
};
hipError_t launch_env_bottom_up(const EnvBottom& d, int batch, hipStream_t st);
hipError_t launch_env_leaf_grad(const EnvBottom& d, int batch, hipStream_t st);

// uniform draws for tests
hipError_t launch_philox_uniforms(uint64_t seed, uint64_t traj_offset, int n_draws, double* out, int batch,
                                  hipStream_t st);

}  // namespace ttn
