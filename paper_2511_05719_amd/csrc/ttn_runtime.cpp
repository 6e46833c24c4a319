// Host runtime of the TTN trajectory engine: tree metadata, tensor pool,
// isometry-centre moves, the controlled-gate zip, the op-list runner and the
// C ABI declared in include/ttn.h.
//
// Layout.  The tree is heap-numbered: node 1 is the root, node i has
// children 2i (leg a) and 2i+1 (leg b) and parent i/2 (leg u); nodes
// L/2 .. L-1 are bottom nodes whose legs a, b are the physical legs of leaves
// 2(i - L/2) and 2(i - L/2) + 1.  The root keeps an up leg of dimension 1
// (instead of being absorbed into a child, Fig. 7), so every node is 3-leg.
// All B rows of a node live in one buffer, row-major [B][a][b][u]; the leg
// dimensions are padded to values the host knows (the per-row Schmidt ranks
// are <= the padding and the padding is zero).  After each centre move's
// eigen-decomposition the host reads one small record, the largest kept
// count over the rows, and pads the new bond to exactly that: the shapes of
// all launches follow the batch's actual ranks, which fall again after
// measurements, instead of staying at their static bounds.
//
// Pool.  A node's buffer must hold its largest shape: two legs doubled while
// a controlled gate's index rides on them.  Nodes with equal capacity share
// a size class with two spare buffers; a contraction writes into a spare of
// the node's class and the old buffer becomes the spare.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ttn.h"
#include "ttn_device.h"
#include "ttn_kernels.h"

using namespace ttn;

// Device scratch of ttn_decode_static: the decoder's leader-parity table
// (2^n_checks bytes, n_checks <= 16), then the data-record columns (64 int32)
// and the check masks (24 x 2 uint32).  One copy per GPU, held until the
// process ends; its device address is looked up once per device when the
// first context on that device is created (the host-side name is only a
// stand-in and is never passed to a kernel or a copy).
constexpr size_t kScratchTable = (size_t)1 << 16;
constexpr size_t kScratchDataRec = kScratchTable;              // 64 int32
constexpr size_t kScratchMasks = kScratchDataRec + 64 * sizeof(int);   // 48 uint32
constexpr size_t kScratchBytes = kScratchMasks + 256;
static_assert(((size_t)1 << TTN_DECODE_STATIC_MAX_CHECKS) == kScratchTable, "table size");
static_assert(kScratchBytes == TTN_DECODE_STATIC_SCRATCH_BYTES, "scratch size");
static __device__ __align__(256) uint8_t scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {nullptr};

// the current device's copy of `scratch` (looked up on first use there)
static hipError_t scratch_for_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

enum {
  CLS_GEMM = TTN_CLASS_CONTRACT, CLS_GRAM = TTN_CLASS_GRAM, CLS_EIGH_SMALL = TTN_CLASS_EIGH_SMALL,
  CLS_EIGH_LARGE = TTN_CLASS_EIGH_LARGE, CLS_LEAF = TTN_CLASS_LEAF, CLS_EXTEND = TTN_CLASS_EXTEND,
  CLS_OTHER = TTN_CLASS_OTHER, CLS_MOVE = TTN_CLASS_MOVE
};

namespace {

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  int cls = -1;
  bool used = false;
};

inline int ilog2(int x) { int r = 0; while ((1 << r) < x) ++r; return r; }

}  // namespace

struct ttn_oplist {
  ttn_ctx* ctx = nullptr;
  std::vector<int32_t> ops;
  std::vector<int> ad_col;     // per op: branch column of an AD op (-1 otherwise)
  int n_ops = 0, n_loc = 0, n_rec = 0, n_draws = 0, n_ad = 0;
};

struct ttn_ctx {
  // configuration
  int N = 0, L = 0, B = 0, c128 = 0, chi = 1;
  int ad_trotter = 0;          // AD without a jump: Trotterised gate instead of K0
  double cutoff = 0.0;
  uint64_t seed = 0;
  hipStream_t st = nullptr;
  size_t es = 8;
  std::vector<int> leaf_of_qubit, qubit_at_leaf, nq_below;
  // state
  std::vector<std::array<int, 3>> dims;
  std::vector<int> node_buf, node_cls;
  std::vector<size_t> cls_elems;
  std::vector<Buf> bufs;
  int centre = 1;
  int nmax = 2;        // largest bond dimension a Gram can have
  int gslices = 1;     // partial-product slices of the Gram workspace
  // workspaces
  double2* G = nullptr;
  void* Wi = nullptr;
  void* Wa = nullptr;
  double* rot_log = nullptr;
  int max_steps = 0;
  long long log_stride = 0;    // doubles of rot_log per eigen-problem
  double2* gpk = nullptr;      // packed Gram matrices of problems above 128 (device memory)
  double* lam_sorted = nullptr;
  int* order = nullptr;
  int* kept = nullptr;
  double* scale_abs = nullptr;
  int* nsteps = nullptr;
  int* rank_table = nullptr;   // [B][L] bond above node e
  // [B][L] per-row prefix extent of the bond above node e: the row's entries
  // beyond it are zero on both nodes of the bond; trusted only where
  // ext_ok[e] (a bond doubled by a controlled gate is not, until a plain
  // move re-factors it)
  int* ext = nullptr;
  std::vector<char> ext_ok;
  int* rank_max = nullptr;     // [B][L] running maximum of rank_table
  double* disc_acc = nullptr;  // [B]
  int* flags = nullptr;        // [B]
  int* degen_acc = nullptr;    // [B]
  double* gate4 = nullptr;     // [4][4][2] device copy of a sibling two-qubit gate
  uint8_t* scratch_dev = nullptr;  // device address of `scratch` on the context's GPU
  double* trace = nullptr;     // per-draw probability trace (caller's buffer) or null
  long long trace_stride = 0;
  uint8_t* leader = nullptr;   // decoder table (device)
  size_t leader_bytes = 0;
  int* dec_datarec = nullptr;
  uint32_t* dec_masks = nullptr;
  // pending bottom-node ops
  std::vector<LeafOp> pend_ops;
  std::vector<int> pend_node;
  LeafBatch run{};             // run-level pointers of the pending ops
  // profiling: HIP events around every launch of each kernel class
  bool prof = false;
  // profiling: a ring of event pairs created once and recycled (a slot's
  // elapsed time is added to its class's total before the slot is reused)
  struct ProfSlot { hipEvent_t a, b; int cls; bool pending; };
  std::vector<ProfSlot> prof_ring;
  size_t prof_pos = 0;
  double prof_ms[TTN_NCLASS] = {0.0};
  int64_t prof_n[TTN_NCLASS] = {0};
  double* ledger[TTN_NCLASS] = {nullptr};   // device [B] algorithmic flops per class (or null)
  double* ledger_bytes[TTN_NCLASS] = {nullptr};   // device [B] algorithmic HBM bytes (Gram, contraction)
  double* ledger_mem = nullptr;             // [7][B]: flops of eigh small, eigh large, Gram, contraction,
                                            // move; bytes of Gram, contraction
  int* adim = nullptr;                      // [B][L][3] actual leg dimensions (profiling)
  int* nk = nullptr;                        // [B][4] eigensolver counts of the last move
  int* qr_done = nullptr;                   // [B] rows of a move factored by the pivoted Cholesky
  int* nk_max = nullptr;                    // [4] their maxima over rows (device)
  int* nk_host = nullptr;                   // [4] pinned host copy
  // stats
  int64_t hops = 0, launches = 0, block_hops = 0;
  int last_kb[2] = {0, 0};     // batch-max kept counts of the two blocks of the last block move
  // GEMM tile-shape tuner: per launch shape, the measured fastest tile shape
  int tune_on = 0;
  int force_cfg = -1;           // >= 0: every GEMM launch in this tile shape (testing)
  std::map<std::array<long long, 14>, int> tune;
  int64_t tuned_shapes = 0, tuned_changed = 0;
  hipEvent_t tune_ev[2] = {nullptr, nullptr};
  // the eigensolver's auxiliary stream (default priority) and its fork/join
  // events, created with the eigensolver workspace for bonds above 64
  hipStream_t st_aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  ttn_ctx* adj = nullptr;      // twin context holding the adjoint state (created on first use)
  // run modes (ttn_set_run_mode): dynamic shapes with one host read per move,
  // or static shapes (bonds padded to their static bounds, no host read),
  // eager or captured once into a HIP graph and replayed
  int run_mode = TTN_RUN_DYNAMIC;
  bool capturing = false;
  uint64_t* d_traj = nullptr;  // device copy of the trajectory offset of static-shape runs
  hipStream_t st_graph = nullptr;               // capture / replay stream (created on first use)
  hipEvent_t ev_gin = nullptr, ev_gout = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::array<uintptr_t, 8> graph_key{};
  int64_t graph_captures = 0, graph_replays = 0;
  double gemm_flops = 0.0, gram_flops = 0.0;
  std::string err;
};

#define TTN_CHECK_HIP(expr)                                                        \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                \
      return TTN_EDEVICE;                                                          \
    }                                                                              \
  } while (0)

#define TTN_TRY(expr)                 \
  do {                                \
    ttn_status s_ = (expr);           \
    if (s_ != TTN_OK) return s_;      \
  } while (0)

static ttn_status fail(ttn_ctx* ctx, ttn_status code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

// ------------------------------------------------------------- tree info ----
static inline bool is_bottom(const ttn_ctx* c, int node) { return node >= c->L / 2; }
static inline int bottom_of(const ttn_ctx* c, int q, int* leg) {
  const int l = c->leaf_of_qubit[q];
  *leg = l & 1;
  return c->L / 2 + l / 2;
}
static inline int leg_toward(int x, int y) {
  if (y == x / 2) return 2;
  if (y == 2 * x) return 0;
  return 1;   // y == 2x + 1
}
static inline int bond_node(int x, int y) { return (y == x / 2) ? x : y; }
// Schmidt-rank bound of the bond above node e (qubits on either side)
static inline long long phys_bound(const ttn_ctx* c, int e) {
  const int a = c->nq_below[e], b = c->N - a;
  const int m = std::min(a, b);
  return m >= 40 ? (1ll << 40) : (1ll << m);
}
static inline int bond_cap(const ttn_ctx* c, int e) {
  return (int)std::min<long long>((long long)c->chi, phys_bound(c, e));
}
static inline long long elems(const std::array<int, 3>& d) { return (long long)d[0] * d[1] * d[2]; }

static std::vector<int> tree_path(int a, int b) {
  std::vector<int> pa{a}, pb{b};
  while (pa.back() != pb.back()) {
    if (pa.back() > pb.back()) pa.push_back(pa.back() / 2);
    else pb.push_back(pb.back() / 2);
  }
  for (int i = (int)pb.size() - 2; i >= 0; --i) pa.push_back(pb[i]);
  return pa;
}

// ---------------------------------------------------------------- pool ----
static int acquire(ttn_ctx* c, int cls) {
  for (size_t i = 0; i < c->bufs.size(); ++i)
    if (c->bufs[i].cls == cls && !c->bufs[i].used) {
      c->bufs[i].used = true;
      return (int)i;
    }
  return -1;
}
static void adopt(ttn_ctx* c, int node, int buf) {
  c->bufs[c->node_buf[node]].used = false;
  c->node_buf[node] = buf;
}
static inline void* node_ptr(ttn_ctx* c, int node) { return c->bufs[c->node_buf[node]].p; }

// ----------------------------------------------------------- profiling ----
// Event pairs live in a ring of kProfRing slots created when profiling is
// first enabled, so that no event is created while a profiled run is timed.
// Reusing a slot first adds its elapsed time to its class (the host waits
// on every hop, so the slot's events have long completed by then).
static constexpr size_t kProfRing = 8192;
static hipError_t prof_harvest(ttn_ctx* ctx, ttn_ctx::ProfSlot& s) {
  if (!s.pending) return hipSuccess;
  s.pending = false;
  hipError_t e = hipEventSynchronize(s.b);
  if (e != hipSuccess) return e;
  float ms = 0.0f;
  e = hipEventElapsedTime(&ms, s.a, s.b);
  if (e != hipSuccess) return e;
  ctx->prof_ms[s.cls] += ms;
  return hipSuccess;
}
static void prof_begin(ttn_ctx* ctx, int cls, hipEvent_t* stop) {
  *stop = nullptr;
  if (!ctx->prof || ctx->prof_ring.empty()) return;
  auto& s = ctx->prof_ring[ctx->prof_pos];
  if (prof_harvest(ctx, s) != hipSuccess) return;
  ctx->prof_pos = (ctx->prof_pos + 1) % ctx->prof_ring.size();
  s.cls = cls;
  s.pending = true;
  ++ctx->prof_n[cls];
  hipEventRecord(s.a, ctx->st);
  *stop = s.b;
}
static void prof_end(ttn_ctx* ctx, hipEvent_t stop) {
  if (stop) hipEventRecord(stop, ctx->st);
}
struct ProfScope {
  ttn_ctx* c;
  hipEvent_t e;
  ProfScope(ttn_ctx* ctx, int cls) : c(ctx) { prof_begin(ctx, cls, &e); }
  ~ProfScope() { prof_end(c, e); }
};

// -------------------------------------------------------- contractions ----
// Largest element offset a GEMM operand can touch (host-side bounds check:
// no launch is made whose indexing could leave its buffer).
static long long extent(long long batch, long long sT, int G2, long long sG, int H, long long sH, int M,
                        long long sM, int K, int Kin, long long s1, long long s2) {
  const long long kq = (K - 1) / Kin, kr = (K >= Kin) ? Kin - 1 : K - 1;
  return (batch - 1) * sT + (long long)(G2 - 1) * sG + (long long)(H - 1) * sH + (long long)(M - 1) * sM +
         kq * s1 + kr * s2 + 1;
}
static bool gemm_fits(const GemmDesc& g, int batch, long long capA, long long capB, long long capC) {
  if (g.M < 1 || g.N < 1 || g.K < 1 || g.H < 1 || g.Kin < 1) return false;
  const int G2 = std::max(g.G2, 1);
  const bool nsplit = g.Nin > 0 && g.Nin < g.N;
  if (nsplit && g.N % g.Nin != 0) return false;
  // the largest column offset on B and C (a split index: both parts at their last value)
  const long long jB = nsplit ? (long long)(g.N / g.Nin - 1) * g.sBj1 + (long long)(g.Nin - 1) * g.sBj
                              : (long long)(g.N - 1) * g.sBj;
  const long long jC = nsplit ? (long long)(g.N / g.Nin - 1) * g.sCj1 + (long long)(g.Nin - 1) * g.sCj
                              : (long long)(g.N - 1) * g.sCj;
  const long long eA = extent(batch, g.sAt, G2, g.sAg, g.H, g.sAh, g.M, g.sAi, g.K, g.Kin, g.sAl1, g.sAl2);
  const long long eB = extent(batch, g.sBt, G2, g.sBg, g.H, g.sBh, 1, 0, g.K, g.Kin, g.sBl1, g.sBl2) + jB;
  const long long eC = (long long)(batch - 1) * g.sCt + (long long)(G2 - 1) * g.sCg + (long long)(g.H - 1) * g.sCh +
                       (long long)(g.M - 1) * g.sCi + jC + (long long)(std::max(g.ksplit, 1) - 1) * g.sCz + 1;
  return eA <= capA && eB <= capB && eC <= capC;
}

// T'[.., a, ..] = sum_i W[a][i] T[.., i, ..] on leg `leg`, W: [rows][wrows][n]
// (rows a < newd <= wrows are used)
static GemmDesc leg_desc(const void* T, std::array<int, 3> d, int leg, const void* W, int wrows, int newd,
                         void* out) {
  const int n = d[leg];
  GemmDesc g{};
  g.H = 1;
  const long long sT = elems(d);
  std::array<int, 3> e = d;
  e[leg] = newd;
  const long long sO = elems(e);
  if (leg == 0) {
    const long long R = (long long)d[1] * d[2];
    g.A = W; g.sAt = (long long)wrows * n; g.sAi = n; g.sAl2 = 1; g.a_m_fast = 0;
    g.B = T; g.sBt = sT; g.sBl2 = R; g.sBj = 1; g.b_n_fast = 1;
    g.C = out; g.sCt = sO; g.sCi = R; g.sCj = 1;
    g.M = newd; g.N = (int)R; g.K = n;
  } else if (leg == 2) {
    const long long R = (long long)d[0] * d[1];
    g.A = T; g.sAt = sT; g.sAi = n; g.sAl2 = 1; g.a_m_fast = 0;
    g.B = W; g.sBt = (long long)wrows * n; g.sBl2 = 1; g.sBj = n; g.b_n_fast = 0;
    g.C = out; g.sCt = sO; g.sCi = newd; g.sCj = 1;
    g.M = (int)R; g.N = newd; g.K = n;
  } else {
    // the middle leg: one GEMM per row over the split column index (a, u)
    // of T[a][i][u] (strides (n d2, 1)) and of the output (newd d2, 1)
    g.A = W; g.sAt = (long long)wrows * n; g.sAi = n; g.sAl2 = 1; g.a_m_fast = 0;
    g.B = T; g.sBt = sT; g.sBl2 = d[2]; g.sBj = 1; g.sBj1 = (long long)n * d[2]; g.b_n_fast = d[2] >= 4;
    g.C = out; g.sCt = sO; g.sCi = d[2]; g.sCj = 1; g.sCj1 = (long long)newd * d[2];
    g.M = newd; g.N = d[0] * d[2]; g.Nin = d[2]; g.K = n;
  }
  g.Kin = g.K;
  return g;
}

// G[t][i][j] = sum_rest conj(T[..i..]) T[..j..] on leg `leg` (FP64 result)
static GemmDesc gram_desc(const void* T, std::array<int, 3> d, int leg, double2* G) {
  const int n = d[leg];
  GemmDesc g{};
  g.H = 1;
  const long long sT = elems(d);
  g.conjA = 1;
  g.same_ab = 1;
  g.herm = 1;
  g.A = T; g.B = T; g.sAt = sT; g.sBt = sT;
  g.C = G; g.sCt = (long long)n * n; g.sCi = n; g.sCj = 1;
  g.M = n; g.N = n;
  if (leg == 0) {
    const long long R = (long long)d[1] * d[2];
    g.sAi = R; g.sAl1 = d[2]; g.sAl2 = 1; g.a_m_fast = 0;
    g.sBl1 = d[2]; g.sBl2 = 1; g.sBj = R; g.b_n_fast = 0;
    g.K = (int)R; g.Kin = d[2];
  } else if (leg == 2) {
    const long long R = (long long)d[0] * d[1];
    g.sAi = 1; g.sAl1 = (long long)d[1] * n; g.sAl2 = n; g.a_m_fast = 1;
    g.sBl1 = (long long)d[1] * n; g.sBl2 = n; g.sBj = 1; g.b_n_fast = 1;
    g.K = (int)R; g.Kin = d[1];
  } else {
    g.sAi = d[2]; g.sAl1 = (long long)n * d[2]; g.sAl2 = 1; g.a_m_fast = 0;
    g.sBl1 = (long long)n * d[2]; g.sBl2 = 1; g.sBj = d[2]; g.b_n_fast = 0;
    g.K = d[0] * d[2]; g.Kin = d[2];
  }
  return g;
}

// Block-diagonal moves (two independent halves of the bond, Sec. III.B
// zip): the Gram matrix is needed only on its two diagonal blocks and both
// factor matrices are block diagonal, so every product splits into two
// half-size products (here on the block index g).
static void gram_split(GemmDesc& g) {
  const int h = g.M / 2;
  g.G2 = 2;
  g.sAg = h * g.sAi;
  g.sBg = h * g.sBj;
  g.sCg = h * (g.sCi + g.sCj);
  g.M = h;
  g.N = h;
}
// Bond id of leg `leg` of `node` whose per-row extents can be trusted, else
// 0 (physical legs of bottom nodes, the root's dimension-1 leg, and bonds
// doubled by a controlled gate).
static int ext_bond(const ttn_ctx* ctx, int node, int leg) {
  int e;
  if (leg == 2) e = node;
  else if (is_bottom(ctx, node)) return 0;
  else e = 2 * node + leg;
  return (e > 1 && e < ctx->L && ctx->ext_ok[e]) ? e : 0;
}
// Per-row extents of a contraction on `leg` of `node` whose new bond (the
// output rows of W) has the per-row kept counts of the move in progress
// (newb = true) or is padded.  The contracted leg's extent bounds K.
static void ext_leg(const ttn_ctx* ctx, GemmDesc& g, int node, std::array<int, 3> d, int leg, bool newb,
                    bool kb) {
  g.ext = ctx->ext; g.knew = ctx->nk + 1; g.ext_stride = ctx->L;
  const int bn = newb ? -1 : 0;
  const int bk = kb ? ext_bond(ctx, node, leg) : 0;
  if (leg == 0) {
    g.eM = bn; g.mM = 1; g.eN = ext_bond(ctx, node, 1); g.mN = d[2];
  } else if (leg == 2) {
    g.eM = ext_bond(ctx, node, 0); g.mM = d[1]; g.eN = bn; g.mN = 1;
  } else {
    g.eNo = ext_bond(ctx, node, 0); g.eM = bn; g.mM = 1; g.eN = ext_bond(ctx, node, 2); g.mN = 1;
  }
  g.eKi = bk;
}
// Per-row extents of the Gram matrix of `leg` of `node`: its rows and
// columns run over that leg (unless split in blocks), K over the other two.
static void ext_gram(const ttn_ctx* ctx, GemmDesc& g, int node, int leg, bool blocks) {
  g.ext = ctx->ext; g.knew = nullptr; g.ext_stride = ctx->L;
  const int bl = blocks ? 0 : ext_bond(ctx, node, leg);
  g.eM = bl; g.mM = 1; g.eN = bl; g.mN = 1;
  const int o = leg == 0 ? 1 : 0, i = leg == 2 ? 1 : 2;
  g.eKo = ext_bond(ctx, node, o);
  g.eKi = ext_bond(ctx, node, i);
}
static long long buf_elems(const ttn_ctx* ctx, int b) { return (long long)(ctx->bufs[b].bytes / ctx->es); }
static long long ws_elems(const ttn_ctx* ctx) { return (long long)ctx->B * ctx->nmax * ctx->nmax; }
static long long gslice_elems(const ttn_ctx* ctx) { return ws_elems(ctx); }
// a Gram launch with fewer workgroups than this splits its K range
constexpr long long kGramTargetWgs = 1024;

static inline void* offset_ptr(const void* p, long long elems, size_t es) {
  return (void*)((const char*)p + elems * (long long)es);
}

// One batched GEMM launch of the hot path with its tile shape: the tuned
// one for this launch shape if the tuner has measured it; with tuning on, a
// shape not seen before is first run once in each of its tile shapes on
// its own operands (every shape computes the same product, overwriting C),
// timed with events on the context's stream, and the fastest is kept.
static ttn_status run_gemm(ttn_ctx* ctx, const GemmDesc& g, int kind) {
  const std::array<long long, 14> key = {kind, g.M, g.N, g.K, g.Kin, g.H, std::max(g.G2, 1), std::max(g.ksplit, 1),
                                         g.a_m_fast, g.b_n_fast, g.conjA, g.conjB, g.ext != nullptr, ctx->B};
  auto it = ctx->tune.find(key);
  int cfg = ctx->force_cfg >= 0 ? ctx->force_cfg : (it != ctx->tune.end() ? it->second : -1);
  if (cfg < 0 && ctx->tune_on && !ctx->capturing) {
    if (!ctx->tune_ev[0]) {
      TTN_CHECK_HIP(hipEventCreate(&ctx->tune_ev[0]));
      TTN_CHECK_HIP(hipEventCreate(&ctx->tune_ev[1]));
    }
    float best_ms = 0.0f;
    for (int c = 0; c < kZgemmCfgs; ++c) {
      if (!zgemm_cfg_useful(g, c)) continue;
      TTN_CHECK_HIP(launch_zgemm(g, ctx->B, kind, ctx->st, c));          // warm
      TTN_CHECK_HIP(hipEventRecord(ctx->tune_ev[0], ctx->st));
      TTN_CHECK_HIP(launch_zgemm(g, ctx->B, kind, ctx->st, c));
      TTN_CHECK_HIP(hipEventRecord(ctx->tune_ev[1], ctx->st));
      TTN_CHECK_HIP(hipEventSynchronize(ctx->tune_ev[1]));
      float ms = 0.0f;
      TTN_CHECK_HIP(hipEventElapsedTime(&ms, ctx->tune_ev[0], ctx->tune_ev[1]));
      if (cfg < 0 || ms < best_ms) {
        best_ms = ms;
        cfg = c;
      }
    }
    ctx->tune[key] = cfg;
    ++ctx->tuned_shapes;
    if (cfg != zgemm_rule_cfg(g)) ++ctx->tuned_changed;
  }
  TTN_CHECK_HIP(launch_zgemm(g, ctx->B, kind, ctx->st, cfg));
  return TTN_OK;
}

// T' = W applied on leg `leg` of the node in src_buf, written to dst_buf with
// that leg of dimension newd.  W is [rows][wrows][n].  blocks = 2: W is block
// diagonal with diagonal blocks [wrows/2][n/2]; block b contributes kb[b]
// rows, placed at new indices [kb[0] * b, kb[0] * b + kb[b]) (newd = kb[0] + kb[1]).
// A leg of a node that carries a controlled gate's block index alongside
// the contracted leg: the node is zero unless both are in the same block,
// and block b of that leg spans [lo[b], hi[b]).
struct Partner {
  int leg = -1;
  int lo[2] = {0, 0};
  int hi[2] = {0, 0};
};

// The band of the GEMM's flattened rest dimension that block b of a partner
// leg maps to (nothing when the partner leg is the inner, faster part of a
// flattened dimension: its band would be strided).
static void set_band(GemmDesc& g, std::array<int, 3> d, int leg, const Partner& pt, int b) {
  const int lo = pt.lo[b], hi = pt.hi[b];
  g.bM0 = 0; g.bM1 = 1 << 30; g.bN0 = 0; g.bN1 = 1 << 30; g.bH0 = 0; g.bH1 = 1 << 30;
  g.bNo0 = 0; g.bNo1 = 1 << 30;
  g.band = 1;
  if (leg == 0 && pt.leg == 1) { g.bN0 = lo * d[2]; g.bN1 = hi * d[2]; }
  else if (leg == 2 && pt.leg == 0) { g.bM0 = lo * d[1]; g.bM1 = hi * d[1]; }
  else if (leg == 1 && pt.leg == 0) { g.bNo0 = lo; g.bNo1 = hi; }    // the outer part (a) of the split index
  else if (leg == 1 && pt.leg == 2) { g.bN0 = lo; g.bN1 = hi; }      // its inner part (u)
  else g.band = 0;
}

static ttn_status leg_apply(ttn_ctx* ctx, int node, int src_buf, std::array<int, 3> d, int leg, const void* W,
                            int wrows, int newd, int dst_buf, int blocks = 1, const int* kb = nullptr,
                            const Partner* pt = nullptr) {
  const int n = d[leg];
  const bool wA = (leg != 2);
  const long long capT = buf_elems(ctx, src_buf), capW = ws_elems(ctx), capC = buf_elems(ctx, dst_buf);
  const int nb = blocks > 1 ? 2 : 1;
  int off = 0;
  for (int b = 0; b < nb; ++b) {
    GemmDesc g = leg_desc(ctx->bufs[src_buf].p, d, leg, W, wrows, newd, ctx->bufs[dst_buf].p);
    // rows of W beyond a row's kept count are zero: the new bond's extent is
    // that count (for the two halves of a block move the padded bound)
    ext_leg(ctx, g, node, d, leg, nb == 1, nb == 1);
    long long oT = 0, oW = 0, oC = 0;
    if (nb == 2) {
      const int rows_b = kb[b];
      if (rows_b == 0) continue;
      oW = (long long)b * (wrows / 2) * n + (long long)b * (n / 2);
      if (leg == 2) {
        oT = (long long)b * (n / 2) * g.sAl2;
        oC = (long long)off * g.sCj;
        g.N = rows_b;
      } else {
        oT = (long long)b * (n / 2) * g.sBl2;
        oC = (long long)off * g.sCi;
        g.M = rows_b;
      }
      g.K = n / 2;
      g.Kin = g.K;
      off += rows_b;
      if (wA) { g.A = offset_ptr(g.A, oW, ctx->es); g.B = offset_ptr(g.B, oT, ctx->es); }
      else { g.A = offset_ptr(g.A, oT, ctx->es); g.B = offset_ptr(g.B, oW, ctx->es); }
      g.C = offset_ptr(g.C, oC, ctx->es);
      if (pt && pt->leg >= 0 && pt->leg != leg) set_band(g, d, leg, *pt, b);
    }
    if (!gemm_fits(g, ctx->B, wA ? capW - oW : capT - oT, wA ? capT - oT : capW - oW, capC - oC))
      return fail(ctx, TTN_EINVAL, "internal: contraction exceeds its buffers");
    ctx->gemm_flops += 8.0 * (double)g.M * g.N * g.K * g.H * ctx->B;
    ++ctx->launches;
    ProfScope ps(ctx, CLS_GEMM);
    TTN_TRY(run_gemm(ctx, g, ctx->c128 ? GEMM_C128 : GEMM_C64));
  }
  return TTN_OK;
}

// The Gram matrix of leg `leg` of the node in src_buf into ctx->G.  When the
// output has too few tiles to occupy the chip, K is split over up to
// ctx->gslices workgroups per tile, each writing its partial product to its
// own slice of G (the eigensolver sums the slices); *nsplit returns the count.
// With a controlled gate's index on two legs of the node (the outgoing leg
// `leg`, split in halves, and the incoming leg in_leg, whose block b spans
// rows [b kin0, b kin0 + kin[b]) after the previous block move), the node is
// zero unless both legs are in the same block, so block b of the Gram
// matrix needs only the incoming rows of block b: K runs over
// kh = max(kin) incoming rows, from 0 for block 0 and from d[in_leg] - kh
// for block 1 (both ranges cover their block and stay inside the leg).
static ttn_status gram(ttn_ctx* ctx, int node, int src_buf, std::array<int, 3> d, int leg, int blocks,
                       int* nsplit, int in_leg = -1, const int* kin = nullptr) {
  GemmDesc g = gram_desc(ctx->bufs[src_buf].p, d, leg, ctx->G);
  ext_gram(ctx, g, node, leg, blocks > 1);
  if (blocks > 1) gram_split(g);
  // (skipped when the split does not describe the leg, e.g. after a move in
  // which every row lost its norm)
  if (blocks > 1 && in_leg >= 0 && in_leg != leg && kin && kin[0] >= 0 && kin[1] >= 0 &&
      kin[0] + kin[1] == d[in_leg] && std::max(kin[0], kin[1]) >= 1) {
    const int din = d[in_leg];
    const int kh = std::max(kin[0], kin[1]);
    const bool outer = in_leg < 3 - leg - in_leg;      // K = (lower leg, higher leg) of the other two
    const long long s_in = outer ? g.sAl1 : g.sAl2;   // A and B share the node's strides
    const long long shift = (long long)(din - kh) * s_in;
    g.sAg += shift;
    g.sBg += shift;
    if (outer) {
      g.K = kh * g.Kin;
      g.eKo = 0;
    } else {
      g.K = (g.K / g.Kin) * kh;
      g.Kin = kh;
      g.eKi = 0;
    }
  }
  const long long wgs = (long long)ctx->B * std::max(g.G2, 1) * zgemm_tiles(g);
  int ks = (int)std::min<long long>((kGramTargetWgs + wgs - 1) / wgs, ctx->gslices);
  ks = std::max(1, std::min(ks, g.K / 256));
  g.ksplit = ks;
  g.sCz = gslice_elems(ctx);
  *nsplit = ks;
  if (!gemm_fits(g, ctx->B, buf_elems(ctx, src_buf), buf_elems(ctx, src_buf), ws_elems(ctx) * ctx->gslices))
    return fail(ctx, TTN_EINVAL, "internal: Gram exceeds its buffers");
  ctx->gram_flops += 8.0 * (double)g.M * g.N * g.K * std::max(g.G2, 1) * ctx->B;
  ++ctx->launches;
  ProfScope ps(ctx, CLS_GRAM);
  TTN_TRY(run_gemm(ctx, g, ctx->c128 ? GEMM_GRAM_C128 : GEMM_GRAM_C64));
  return TTN_OK;
}

// eigensolver workspaces of the context
static void eigh_ws(const ttn_ctx* ctx, EighDesc& ed) {
  ed.rot_log = ctx->rot_log; ed.max_steps = ctx->max_steps; ed.log_stride = ctx->log_stride;
  ed.lam_sorted = ctx->lam_sorted; ed.order = ctx->order; ed.kept = ctx->kept;
  ed.scale_abs = ctx->scale_abs; ed.nsteps = ctx->nsteps; ed.gpk = ctx->gpk;
  ed.aux_stream = ctx->st_aux; ed.ev_fork = ctx->ev_fork; ed.ev_join = ctx->ev_join;
  if (ctx->capturing) {        // one stream inside a captured graph
    ed.aux_stream = nullptr; ed.ev_fork = nullptr; ed.ev_join = nullptr;
  }
}

// Move the isometry centre from x to its neighbour y (Sec. III.B: the
// canonical form that makes local Schmidt values and Born probabilities
// local): factor x = (x V S^-1)(S V^H) across the bond, keep the first factor
// in x, absorb the second into y, truncating to `cap` values above `cutoff`.
// The batch's kept counts of the last eigen-decomposition: kb[b] = the
// largest number of values any row kept in block b.  The only device-to-host
// read of a centre move: the new bond is padded to what some row uses, not to
// its static bound, so padding never accumulates on bonds whose rank fell.
static ttn_status read_kept(ttn_ctx* ctx, int kb[2]) {
  TTN_CHECK_HIP(launch_nk_max(ctx->nk, ctx->B, ctx->nk_max, ctx->st));
  TTN_CHECK_HIP(hipMemcpyAsync(ctx->nk_host, ctx->nk_max, 4 * sizeof(int), hipMemcpyDeviceToHost, ctx->st));
  TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
  kb[0] = ctx->nk_host[1];
  kb[1] = ctx->nk_host[3];
  return TTN_OK;
}

// exact: the move keeps every value above the cutoff (the cap cannot bind).
// Complex64 contexts factor such moves, and truncating moves whose bond is
// no wider than the cap (only the cutoff can drop values), by pivoted
// Cholesky (QR) instead of the eigensolver when the problem fits it (n <= 64
// per block): the bond then keeps a basis of the same kept space rather than
// the Schmidt basis, which nothing downstream needs.
static ttn_status hop(ttn_ctx* ctx, int x, int y, double cutoff, int cap, int new_pad, int blocks = 1,
                      int in_leg = -1, const int* kin = nullptr, const Partner* px = nullptr,
                      const Partner* py = nullptr, bool exact = false) {
  const int lx = leg_toward(x, y), ly = leg_toward(y, x);
  const int e = bond_node(x, y);
  std::array<int, 3> dx = ctx->dims[x], dy = ctx->dims[y];
  const int n = dx[lx];
  if (n != dy[ly]) return fail(ctx, TTN_EINVAL, "internal: bond dimension mismatch");
  if (n > ctx->nmax || new_pad > ctx->nmax)
    return fail(ctx, TTN_EINVAL, "internal: bond dimension exceeds workspace");
  if (blocks > 1 && ((n & 1) || (new_pad & 1))) return fail(ctx, TTN_EINVAL, "internal: odd block size");
  int gsplit = 1;
  TTN_TRY(gram(ctx, x, ctx->node_buf[x], dx, lx, blocks, &gsplit, in_leg, kin));
  EighDesc ed{};
  ed.G = ctx->G; ed.n = n; ed.new_pad = new_pad; ed.cap = cap; ed.cutoff = cutoff;
  ed.gsplit = gsplit; ed.gslice = gslice_elems(ctx);
  ed.W_iso = ctx->Wi; ed.W_abs = ctx->Wa; ed.out_c128 = ctx->c128;
  ed.blocks = blocks;
  ed.rank_out = blocks > 1 ? nullptr : ctx->rank_table + e;
  ed.rank_max = blocks > 1 ? nullptr : ctx->rank_max + e;
  ed.rank_stride = ctx->L;
  const bool large = (n / blocks + ((n / blocks) & 1)) > 64;
  const bool qr = !ctx->c128 && !large && (blocks > 1 ? exact : n <= cap);
  ed.flops_acc = ctx->ledger[qr ? CLS_MOVE : large ? CLS_EIGH_LARGE : CLS_EIGH_SMALL];
  ed.disc_acc = ctx->disc_acc; ed.flags = ctx->flags; ed.degen_acc = ctx->degen_acc;
  eigh_ws(ctx, ed);
  ed.nk_out = ctx->nk;
  // complex64 factors carry ~1e-7 relative error, so off-diagonal Gram
  // entries below 1e-12 of the diagonal change nothing they hold
  ed.tol = ctx->c128 ? 1e-15 : 1e-10;
  ed.early_stop = ctx->c128 ? 0 : 1;
  // complex64 rows without blocks of 65..128 columns: the pivoted Cholesky
  // first, which factors every row whose weight above the cutoff fits the
  // cap (the move then drops nothing but that cutoff); the eigensolver
  // takes the rest
  const bool try_qr = !ctx->c128 && large && blocks == 1 && n <= 128;
  if (qr) {
    ++ctx->launches;
    ProfScope ps(ctx, CLS_MOVE);
    TTN_CHECK_HIP(launch_pchol(ed, ctx->B, ctx->st));
  } else if (try_qr) {
    {
      EighDesc eq = ed;
      eq.flops_acc = ctx->ledger[CLS_MOVE];
      eq.done = ctx->qr_done;
      ++ctx->launches;
      ProfScope ps(ctx, CLS_MOVE);
      TTN_CHECK_HIP(launch_pchol(eq, ctx->B, ctx->st));
    }
    ed.done = ctx->qr_done;
    ctx->launches += 2;
    ProfScope ps(ctx, CLS_EIGH_LARGE);
    TTN_CHECK_HIP(launch_eigh(ed, ctx->B, ctx->st));
  } else {
    ctx->launches += large ? 2 : 1;
    ProfScope ps(ctx, large ? CLS_EIGH_LARGE : CLS_EIGH_SMALL);
    TTN_CHECK_HIP(launch_eigh(ed, ctx->B, ctx->st));
  }
  int kb[2];
  if (ctx->run_mode == TTN_RUN_DYNAMIC) {
    TTN_TRY(read_kept(ctx, kb));
  } else {
    // static shapes: the new bond keeps its padded bound (each row's kept
    // values are a prefix, the rest of the factor rows are zero)
    kb[0] = blocks > 1 ? new_pad / 2 : new_pad;
    kb[1] = blocks > 1 ? new_pad / 2 : 0;
  }
  if (kb[0] < 0 || kb[1] < 0 || kb[0] + kb[1] > new_pad || (blocks > 1 && std::max(kb[0], kb[1]) > new_pad / 2))
    return fail(ctx, TTN_EDEVICE, "internal: kept count out of range");
  int newd = blocks > 1 ? kb[0] + kb[1] : kb[0];
  ctx->last_kb[0] = kb[0];
  ctx->last_kb[1] = blocks > 1 ? kb[1] : 0;
  if (newd == 0) {             // every row lost its norm (flagged): keep one zero column
    newd = 1;
    kb[0] = 1;
  }
  const int bx = acquire(ctx, ctx->node_cls[x]);
  if (bx < 0) return fail(ctx, TTN_EINVAL, "internal: pool exhausted");
  TTN_TRY(leg_apply(ctx, x, ctx->node_buf[x], dx, lx, ctx->Wi, new_pad, newd, bx, blocks, kb, px));
  adopt(ctx, x, bx);
  const int by = acquire(ctx, ctx->node_cls[y]);
  if (by < 0) return fail(ctx, TTN_EINVAL, "internal: pool exhausted");
  TTN_TRY(leg_apply(ctx, y, ctx->node_buf[y], dy, ly, ctx->Wa, new_pad, newd, by, blocks, kb, py));
  adopt(ctx, y, by);
  // the bond's new per-row extents: the kept counts (a block move leaves
  // them untrusted until the truncating sweep re-factors the bond)
  if (blocks > 1) {
    ctx->ext_ok[e] = 0;
  } else {
    ++ctx->launches;
    TTN_CHECK_HIP(launch_set_ext(ctx->ext + e, ctx->L, ctx->nk + 1, 4, ctx->B, ctx->st));
    ctx->ext_ok[e] = 1;
  }
  ctx->dims[x][lx] = newd;
  ctx->dims[y][ly] = newd;
  ctx->centre = y;
  ++ctx->hops;
  if (blocks > 1) ++ctx->block_hops;
  if (ctx->prof) {
    LedgerHop lh{};
    lh.adim = ctx->adim; lh.nk = ctx->nk; lh.L = ctx->L;
    lh.x = x; lh.lx = lx; lh.y = y; lh.ly = ly;
    lh.gram_acc = ctx->ledger[CLS_GRAM];
    lh.contract_acc = ctx->ledger[CLS_GEMM];
    lh.gram_bytes = ctx->ledger_bytes[CLS_GRAM];
    lh.contract_bytes = ctx->ledger_bytes[CLS_GEMM];
    lh.es = (int)ctx->es;
    TTN_CHECK_HIP(launch_ledger_hop(lh, ctx->B, ctx->st));
  }
  return TTN_OK;
}

// plain moves of the centre (exact: no gate has widened the bond) and the
// truncating sweep after a controlled gate
static ttn_status hop_truncating(ttn_ctx* ctx, int x, int y, bool exact = false) {
  const int e = bond_node(x, y);
  const int n = ctx->dims[x][leg_toward(x, y)];
  const int cap = bond_cap(ctx, e);
  return hop(ctx, x, y, ctx->cutoff, cap, std::min(n, cap), 1, -1, nullptr, nullptr, nullptr, exact);
}

static ttn_status flush_leaf(ttn_ctx* ctx);

static ttn_status move_centre(ttn_ctx* ctx, int target) {
  if (ctx->centre == target) return TTN_OK;
  TTN_TRY(flush_leaf(ctx));
  std::vector<int> p = tree_path(ctx->centre, target);
  for (size_t i = 0; i + 1 < p.size(); ++i) TTN_TRY(hop_truncating(ctx, p[i], p[i + 1], true));
  return TTN_OK;
}

// --------------------------------------------------------- bottom ops ----
static ttn_status flush_leaf(ttn_ctx* ctx) {
  size_t i = 0;
  while (i < ctx->pend_ops.size()) {
    LeafBatch b = ctx->run;
    b.n_ops = 0;
    for (; i < ctx->pend_ops.size() && b.n_ops < kMaxLeafOps; ++i) {
      const int node = ctx->pend_node[i];
      if (!is_bottom(ctx, node) || ctx->dims[node][0] != 2 || ctx->dims[node][1] != 2 ||
          4ll * ctx->dims[node][2] * ctx->B > buf_elems(ctx, ctx->node_buf[node]))
        return fail(ctx, TTN_EINVAL, "internal: bottom-node op on a malformed node");
      b.ops[b.n_ops] = ctx->pend_ops[i];
      b.node_ptr[b.n_ops] = node_ptr(ctx, node);
      b.node_u[b.n_ops] = ctx->dims[node][2];
      ++b.n_ops;
    }
    b.n_rows = ctx->B;
    b.c128 = ctx->c128;
    b.flags = ctx->flags;
    b.seed = ctx->seed;
    b.ad_trotter = ctx->ad_trotter;
    b.probs = b.adjoint ? nullptr : ctx->trace;
    b.probs_stride = ctx->trace_stride;
    ++ctx->launches;
    ProfScope ps(ctx, CLS_LEAF);
    TTN_CHECK_HIP(launch_leaf_ops(b, ctx->st));
  }
  ctx->pend_ops.clear();
  ctx->pend_node.clear();
  return TTN_OK;
}

static void push_leaf(ttn_ctx* ctx, int node, const LeafOp& op) {
  ctx->pend_ops.push_back(op);
  ctx->pend_node.push_back(node);
}

static LeafOp leaf_op(int kind, int leg) {
  LeafOp o{};
  o.kind = kind; o.leg = leg; o.prev = -1; o.rec = -1; o.loc = 0; o.draw = 0; o.branch = 0; o.arg = 0;
  return o;
}

// ----------------------------------------------------- controlled gate ----
// Zip moves across bonds of at least this (doubled) dimension are solved as
// two diagonal blocks; below it one dense solve costs less than the extra
// launches.
constexpr int kBlockMin = 16;

// g = sum_k P_k (x) B_k with P_k = |v_k><v_k| orthogonal projectors on the
// `start` qubit.  The start node gets its up bond doubled into (k, u) with
// block k = P_k applied; the index k then rides along the tree path
// (delta-copied on both path legs of every node it passes) while the centre
// moves one node at a time toward the other end, where block k receives B_k.
// Because the P_k project onto orthogonal subspaces of a qubit on the near
// side, every Gram matrix on the way is that of the exact state, so only
// numerically zero values are dropped.  A sweep back to the start then
// truncates every path bond with the context's rule (Sec. IV.A).
static ttn_status controlled_gate(ttn_ctx* ctx, int qs, const double P[2][2][2][2], int qe,
                                  const double Bm[2][2][2][2]) {
  int ls, le;
  const int ns = bottom_of(ctx, qs, &ls), ne = bottom_of(ctx, qe, &le);
  TTN_TRY(move_centre(ctx, ns));
  TTN_TRY(flush_leaf(ctx));
  const std::vector<int> path = tree_path(ns, ne);
  const int m = (int)path.size() - 1;
  // split at the start
  {
    ExtendDesc x{};
    const std::array<int, 3> d = ctx->dims[ns];
    x.src = node_ptr(ctx, ns);
    x.d0 = d[0]; x.d1 = d[1]; x.d2 = d[2];
    x.leg_in = 2; x.leg_out = -1; x.mode = 1; x.ctrl_leg = ls;
    std::memcpy(x.bmat, P, sizeof(x.bmat));
    x.src_stride = elems(d);
    x.dst_stride = elems(d) * 2;
    x.c128 = ctx->c128;
    const int b = acquire(ctx, ctx->node_cls[ns]);
    if (b < 0) return fail(ctx, TTN_EINVAL, "internal: pool exhausted");
    if (elems(d) * 2 * ctx->B > buf_elems(ctx, b)) return fail(ctx, TTN_EINVAL, "internal: split exceeds buffer");
    x.dst = ctx->bufs[b].p;
    ++ctx->launches;
    ProfScope ps(ctx, CLS_EXTEND);
    TTN_CHECK_HIP(launch_extend(x, ctx->B, ctx->st));
    adopt(ctx, ns, b);
    ctx->dims[ns][2] *= 2;
    ctx->ext_ok[ns] = 0;
    if (ctx->prof) TTN_CHECK_HIP(launch_ledger_double(ctx->adim, ctx->L, ns, 2, -1, ctx->B, ctx->st));
  }
  bool prev_block = false;      // the last forward move was a block move (kin: its kept counts)
  int kin[2] = {0, 0};
  for (int i = 0; i < m; ++i) {
    const int x = path[i], y = path[i + 1];
    const int ly = leg_toward(y, x);
    ExtendDesc ex{};
    const std::array<int, 3> d = ctx->dims[y];
    ex.src = node_ptr(ctx, y);
    ex.d0 = d[0]; ex.d1 = d[1]; ex.d2 = d[2];
    ex.c128 = ctx->c128;
    ex.src_stride = elems(d);
    std::array<int, 3> e = d;
    if (y == ne) {
      ex.mode = 1; ex.leg_in = 2; ex.leg_out = -1; ex.ctrl_leg = le;
      std::memcpy(ex.bmat, Bm, sizeof(ex.bmat));
      e[2] *= 2;
    } else {
      const int lo = leg_toward(y, path[i + 2]);
      ex.mode = 0; ex.leg_in = ly; ex.leg_out = lo;
      e[ly] *= 2;
      e[lo] *= 2;
    }
    ex.dst_stride = elems(e);
    const int b = acquire(ctx, ctx->node_cls[y]);
    if (b < 0) return fail(ctx, TTN_EINVAL, "internal: pool exhausted");
    if (elems(e) * ctx->B > buf_elems(ctx, b)) return fail(ctx, TTN_EINVAL, "internal: extension exceeds buffer");
    ex.dst = ctx->bufs[b].p;
    ++ctx->launches;
    {
      ProfScope ps(ctx, CLS_EXTEND);
      TTN_CHECK_HIP(launch_extend(ex, ctx->B, ctx->st));
    }
    adopt(ctx, y, b);
    ctx->dims[y] = e;
    ctx->ext_ok[bond_node(x, y)] = 0;
    if (y != ne) ctx->ext_ok[bond_node(y, path[i + 2])] = 0;
    if (ctx->prof)
      TTN_CHECK_HIP(launch_ledger_double(ctx->adim, ctx->L, y, ex.leg_in, ex.leg_out, ctx->B, ctx->st));
    // exact move across (x, y): the bond can hold the near side's full space
    const int n = ctx->dims[x][leg_toward(x, y)];
    const int qnear = (y == x / 2) ? ctx->nq_below[x] : ctx->N - ctx->nq_below[y];
    const long long near_dim = qnear >= 30 ? (1ll << 30) : (1ll << qnear);
    if (n >= kBlockMin) {
      // the Gram matrix is block diagonal in k: two independent halves;
      // after a block move into x, x's incoming leg is block structured too
      const int in_leg = prev_block ? leg_toward(x, path[i - 1]) : -1;
      // the legs that carry the index next to the moving bond: x's incoming
      // leg (blocks of the previous move) and y's outgoing leg (halves)
      Partner px, py;
      if (in_leg >= 0 && kin[0] + kin[1] == ctx->dims[x][in_leg]) {
        px.leg = in_leg;
        px.lo[0] = 0; px.hi[0] = kin[0];
        px.lo[1] = kin[0]; px.hi[1] = kin[0] + kin[1];
      }
      if (y != ne) {
        py.leg = leg_toward(y, path[i + 2]);
        const int half = ctx->dims[y][py.leg] / 2;
        py.lo[0] = 0; py.hi[0] = half;
        py.lo[1] = half; py.hi[1] = 2 * half;
      }
      TTN_TRY(hop(ctx, x, y, ctx->cutoff, n / 2, n, 2, in_leg, kin, &px, &py, true));
      prev_block = true;
      kin[0] = ctx->last_kb[0];
      kin[1] = ctx->last_kb[1];
    } else {
      const int pad = (int)std::min<long long>(n, near_dim);
      TTN_TRY(hop(ctx, x, y, ctx->cutoff, pad, pad, 1, -1, nullptr, nullptr, nullptr, true));
      prev_block = false;
    }
  }
  for (int i = m; i > 0; --i) TTN_TRY(hop_truncating(ctx, path[i], path[i - 1]));
  return TTN_OK;
}

static void proj(double P[2][2][2][2], int basis) {
  std::memset(P, 0, sizeof(double) * 16);
  if (basis == 0) {            // |0><0|, |1><1|
    P[0][0][0][0] = 1.0;
    P[1][1][1][0] = 1.0;
  } else {                     // |+><+|, |-><-|
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        P[0][i][j][0] = 0.5;
        P[1][i][j][0] = (i == j) ? 0.5 : -0.5;
      }
  }
}

static ttn_status cnot(ttn_ctx* ctx, int c, int t) {
  int lc, lt;
  const int nc = bottom_of(ctx, c, &lc), nt = bottom_of(ctx, t, &lt);
  if (nc == nt) {
    push_leaf(ctx, nc, leaf_op(LOP_CNOT, lc));
    return TTN_OK;
  }
  // CNOT = |0><0| (x) I + |1><1| (x) X  =  I (x) |+><+| + Z (x) |-><-|:
  // start the zip at whichever end is nearer the current centre
  const int dc = (int)tree_path(ctx->centre, nc).size();
  const int dt = (int)tree_path(ctx->centre, nt).size();
  double P[2][2][2][2], Bm[2][2][2][2];
  std::memset(Bm, 0, sizeof(Bm));
  if (dc <= dt) {
    proj(P, 0);
    Bm[0][0][0][0] = 1; Bm[0][1][1][0] = 1;        // I
    Bm[1][0][1][0] = 1; Bm[1][1][0][0] = 1;        // X
    return controlled_gate(ctx, c, P, t, Bm);
  }
  proj(P, 1);
  Bm[0][0][0][0] = 1; Bm[0][1][1][0] = 1;          // I
  Bm[1][0][0][0] = 1; Bm[1][1][1][0] = -1;         // Z
  return controlled_gate(ctx, t, P, c, Bm);
}

// ----------------------------------------------------------- run setup ----
static ttn_status reset_state(ttn_ctx* ctx, const uint8_t* basis) {
  TTN_TRY(flush_leaf(ctx));
  for (int node = 1; node < ctx->L; ++node) {
    ctx->dims[node] = is_bottom(ctx, node) ? std::array<int, 3>{2, 2, 1} : std::array<int, 3>{1, 1, 1};
    InitDesc d{};
    d.ptr = node_ptr(ctx, node);
    d.bottom = is_bottom(ctx, node);
    d.c128 = ctx->c128;
    if (d.bottom) {
      const int l0 = 2 * (node - ctx->L / 2);
      const int q0 = ctx->qubit_at_leaf[l0], q1 = ctx->qubit_at_leaf[l0 + 1];
      d.basis0 = (basis && q0 >= 0) ? basis[q0] : 0;
      d.basis1 = (basis && q1 >= 0) ? basis[q1] : 0;
    }
    ++ctx->launches;
    TTN_CHECK_HIP(launch_init_product(d, ctx->B, ctx->st));
  }
  ctx->centre = 1;
  TTN_CHECK_HIP(launch_fill_i32(ctx->rank_table, 1, (long long)ctx->B * ctx->L, ctx->st));
  TTN_CHECK_HIP(launch_fill_i32(ctx->ext, 1, (long long)ctx->B * ctx->L, ctx->st));
  ctx->ext_ok.assign(ctx->L, 1);
  TTN_CHECK_HIP(launch_fill_i32(ctx->rank_max, 1, (long long)ctx->B * ctx->L, ctx->st));
  TTN_CHECK_HIP(launch_ledger_reset(ctx->adim, ctx->L, ctx->B, ctx->st));
  TTN_CHECK_HIP(launch_fill_i32(ctx->flags, 0, ctx->B, ctx->st));
  TTN_CHECK_HIP(launch_fill_i32(ctx->degen_acc, 0, ctx->B, ctx->st));
  TTN_CHECK_HIP(launch_fill_f64(ctx->disc_acc, 0.0, ctx->B, ctx->st));
  ctx->launches += 6;
  return TTN_OK;
}

static ttn_status fill_stats(ttn_ctx* ctx, ttn_stats* st) {
  if (!st) return TTN_OK;
  TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
  std::vector<int> ranks((size_t)ctx->B * ctx->L), flags(ctx->B), degen(ctx->B);
  std::vector<double> disc(ctx->B);
  TTN_CHECK_HIP(hipMemcpy(ranks.data(), ctx->rank_max, ranks.size() * 4, hipMemcpyDeviceToHost));
  TTN_CHECK_HIP(hipMemcpy(flags.data(), ctx->flags, flags.size() * 4, hipMemcpyDeviceToHost));
  TTN_CHECK_HIP(hipMemcpy(degen.data(), ctx->degen_acc, degen.size() * 4, hipMemcpyDeviceToHost));
  TTN_CHECK_HIP(hipMemcpy(disc.data(), ctx->disc_acc, disc.size() * 8, hipMemcpyDeviceToHost));
  st->max_rank = 1;
  for (int t = 0; t < ctx->B; ++t)
    for (int e = 2; e < ctx->L; ++e) st->max_rank = std::max(st->max_rank, ranks[(size_t)t * ctx->L + e]);
  st->discarded_weight = 0.0;
  st->degenerate_cuts = 0;
  st->flagged_rows = 0;
  for (int t = 0; t < ctx->B; ++t) {
    st->discarded_weight += disc[t];
    st->degenerate_cuts += degen[t];
    st->flagged_rows += flags[t] != 0;
  }
  st->hops = ctx->hops;
  st->launches = ctx->launches;
  st->gemm_flops = ctx->gemm_flops;
  st->gram_flops = ctx->gram_flops;
  st->block_hops = ctx->block_hops;
  return TTN_OK;
}

// Run-level pointers of an op-list execution (see LeafBatch).
static void setup_run(ttn_ctx* ctx, const ttn_oplist* ol, const double* theta, const double* gamma, int64_t pstride,
                      uint64_t traj_offset, uint8_t* records, int8_t* branches, double* logp,
                      const uint8_t* forced_rec, const int8_t* forced_br, int adjoint) {
  LeafBatch& r = ctx->run;
  r = LeafBatch{};
  r.theta = theta; r.theta_row_stride = pstride;
  r.gamma = gamma; r.gamma_row_stride = pstride;
  r.records = records; r.rec_stride = ol->n_rec;
  r.forced_rec = forced_rec; r.forced_rec_stride = ol->n_rec;
  r.branches = branches; r.br_stride = ol->n_ad;
  r.forced_br = forced_br; r.forced_br_stride = ol->n_ad;
  r.logp = logp;
  r.traj_offset = traj_offset;
  r.traj_offset_dev = ctx->run_mode != TTN_RUN_DYNAMIC ? ctx->d_traj : nullptr;
  r.adjoint = adjoint;
}

// Op k of the list on the context's state (its adjoint when the run is an
// adjoint run: the caller walks the list backwards).
static ttn_status exec_op(ttn_ctx* ctx, const ttn_oplist* ol, int k) {
  const int32_t* o = &ol->ops[(size_t)k * 9];
  const int op = o[0], q0 = o[1], q1 = o[2], arg = o[3], loc = o[4], draw = o[5], rec = o[6], prev = o[7];
  int leg;
  const int node = bottom_of(ctx, q0, &leg);
  switch (op) {
    case TTN_OP_INIT: {
      LeafOp l = leaf_op(LOP_INIT, leg);
      l.arg = arg; l.prev = prev; l.rec = rec;
      push_leaf(ctx, node, l);
      break;
    }
    case TTN_OP_CNOT:
      TTN_TRY(cnot(ctx, q0, q1));
      break;
    case TTN_OP_SRX: {
      LeafOp l = leaf_op(LOP_SRX, leg);
      l.loc = loc;
      push_leaf(ctx, node, l);
      break;
    }
    case TTN_OP_PAULI: {
      if (ctx->run.adjoint) return fail(ctx, TTN_EINVAL, "twirled ops have no adjoint run");
      LeafOp l = leaf_op(arg == 0 ? LOP_PAULI_SRX : LOP_PAULI_AD, leg);
      l.loc = loc; l.draw = draw;
      push_leaf(ctx, node, l);
      break;
    }
    case TTN_OP_AD: {
      TTN_TRY(move_centre(ctx, node));
      LeafOp l = leaf_op(LOP_KRAUS_AD, leg);
      l.loc = loc; l.draw = draw; l.branch = ol->ad_col[k];
      push_leaf(ctx, node, l);
      break;
    }
    case TTN_OP_MEAS: {
      TTN_TRY(move_centre(ctx, node));
      LeafOp l = leaf_op(LOP_MEAS, leg);
      l.arg = arg; l.rec = rec; l.draw = draw;
      push_leaf(ctx, node, l);
      break;
    }
    default:
      return fail(ctx, TTN_EINVAL, "unknown op code");
  }
  return TTN_OK;
}

static ttn_status run_oplist(ttn_ctx* ctx, const ttn_oplist* ol, const double* theta, const double* gamma,
                             int64_t pstride, uint64_t traj_offset, uint8_t* records, int8_t* branches,
                             double* logp, const uint8_t* forced_rec, const int8_t* forced_br, ttn_stats* st) {
  if (!ol || ol->ctx != ctx) return fail(ctx, TTN_EINVAL, "op list belongs to another context");
  if (!records || !logp) return fail(ctx, TTN_EINVAL, "records and logp are required");
  if (ol->n_ad > 0 && !branches && !forced_br) return fail(ctx, TTN_EINVAL, "branches required (AD ops)");
  if (ctx->trace && ctx->trace_stride < ol->n_draws)
    return fail(ctx, TTN_EINVAL, "probability trace narrower than the op list's draws");
  ctx->hops = 0; ctx->launches = 0; ctx->block_hops = 0; ctx->gemm_flops = 0.0; ctx->gram_flops = 0.0;
  TTN_TRY(reset_state(ctx, nullptr));
  TTN_CHECK_HIP(launch_fill_f64(logp, 0.0, ctx->B, ctx->st));
  if (ctx->run_mode != TTN_RUN_DYNAMIC && !ctx->capturing)
    TTN_CHECK_HIP(launch_fill_u64(ctx->d_traj, traj_offset, 1, ctx->st));
  setup_run(ctx, ol, theta, gamma, pstride, traj_offset, records, branches, logp, forced_rec, forced_br, 0);
  for (int k = 0; k < ol->n_ops; ++k) TTN_TRY(exec_op(ctx, ol, k));
  TTN_TRY(flush_leaf(ctx));
  ctx->run = LeafBatch{};
  if (st) TTN_TRY(fill_stats(ctx, st));
  return TTN_OK;
}

// ================================================================ C ABI ====
extern "C" {

const char* ttn_version(void) { return "ttn-mi355x 0.1 (gfx950)"; }

double ttn_philox_uniform_host(uint64_t seed, uint64_t traj, uint64_t draw) {
  return philox_uniform(seed, traj, draw);
}

int32_t ttn_test_sweep_plan(int32_t k, uint32_t* groups, int32_t cap) {
  return eigh_sweep_plan(k, groups, cap);
}

const char* ttn_last_error(const ttn_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

ttn_status ttn_create(const ttn_config* cfg, ttn_ctx** out) {
  if (!cfg || !out) return TTN_EINVAL;
  *out = nullptr;
  if (cfg->n_qubits < 1 || !cfg->leaf_of_qubit || cfg->chi_max < 1 || cfg->batch < 1 ||
      !(cfg->cutoff >= 0.0) || (cfg->dtype != TTN_C64 && cfg->dtype != TTN_C128) ||
      (cfg->ad_mode != TTN_AD_KRAUS && cfg->ad_mode != TTN_AD_TROTTER))
    return TTN_EINVAL;
  ttn_ctx* ctx = new ttn_ctx();
  ctx->N = cfg->n_qubits;
  int L = 2;
  while (L < ctx->N) L *= 2;
  ctx->L = L;
  ctx->B = cfg->batch;
  ctx->c128 = cfg->dtype == TTN_C128;
  ctx->ad_trotter = cfg->ad_mode == TTN_AD_TROTTER;
  ctx->es = ctx->c128 ? 16 : 8;
  ctx->chi = cfg->chi_max;
  ctx->cutoff = cfg->cutoff;
  ctx->seed = cfg->seed;
  ctx->st = (hipStream_t)cfg->stream;
  ctx->leaf_of_qubit.assign(cfg->leaf_of_qubit, cfg->leaf_of_qubit + ctx->N);
  ctx->qubit_at_leaf.assign(L, -1);
  for (int q = 0; q < ctx->N; ++q) {
    const int l = ctx->leaf_of_qubit[q];
    if (l < 0 || l >= L || ctx->qubit_at_leaf[l] >= 0) {
      delete ctx;
      return TTN_EINVAL;
    }
    ctx->qubit_at_leaf[l] = q;
  }
  ctx->nq_below.assign(L, 0);
  for (int node = L - 1; node >= 1; --node) {
    if (node >= L / 2) {
      const int l0 = 2 * (node - L / 2);
      ctx->nq_below[node] = (ctx->qubit_at_leaf[l0] >= 0) + (ctx->qubit_at_leaf[l0 + 1] >= 0);
    } else {
      ctx->nq_below[node] = ctx->nq_below[2 * node] + ctx->nq_below[2 * node + 1];
    }
  }
  // largest Gram: a doubled bond during a controlled gate
  int nmax = 2;
  for (int e = 2; e < L; ++e) nmax = std::max(nmax, 2 * bond_cap(ctx, e));
  ctx->nmax = nmax;
  if (nmax > 256) {
    delete ctx;
    return TTN_EINVAL;   // the FP64 Jacobi solver takes bonds up to 256 (chi_max <= 128)
  }
  // node capacities and size classes
  std::vector<size_t> cap_el(L, 0);
  for (int node = 1; node < L; ++node) {
    const long long cu = node == 1 ? 1 : bond_cap(ctx, node);
    if (node >= L / 2) cap_el[node] = (size_t)(2 * 2 * 2 * cu);
    else cap_el[node] = (size_t)(4ll * bond_cap(ctx, 2 * node) * bond_cap(ctx, 2 * node + 1) * cu);
  }
  ctx->node_cls.assign(L, -1);
  ctx->node_buf.assign(L, -1);
  ctx->dims.assign(L, {1, 1, 1});
  for (int node = 1; node < L; ++node) {
    int cls = -1;
    for (size_t c = 0; c < ctx->cls_elems.size(); ++c)
      if (ctx->cls_elems[c] == cap_el[node]) cls = (int)c;
    if (cls < 0) {
      cls = (int)ctx->cls_elems.size();
      ctx->cls_elems.push_back(cap_el[node]);
    }
    ctx->node_cls[node] = cls;
  }
  auto bail = [&](ttn_status s) {
    ttn_destroy(ctx);
    return s;
  };
  for (size_t c = 0; c < ctx->cls_elems.size(); ++c) {
    int count = 2;
    for (int node = 1; node < L; ++node) count += ctx->node_cls[node] == (int)c;
    for (int i = 0; i < count; ++i) {
      Buf b;
      b.cls = (int)c;
      b.bytes = ctx->cls_elems[c] * ctx->es * (size_t)ctx->B;
      b.bytes = (b.bytes + 255) & ~(size_t)255;
      if (hipMalloc(&b.p, b.bytes) != hipSuccess) return bail(TTN_ENOMEM);
      ctx->bufs.push_back(b);
    }
  }
  for (int node = 1; node < L; ++node) {
    const int b = acquire(ctx, ctx->node_cls[node]);
    ctx->node_buf[node] = b;
  }
  const size_t Bz = (size_t)ctx->B;
  const int n2 = nmax;
  const int nlog = eigh_padded_size(n2);      // the solver's padded size for problems above 64
  ctx->max_steps = eigh_max_sweeps() * (nlog - 1);
  bool ok = true;
  ctx->gslices = (int)std::max<long long>(1, std::min<long long>(8, 2048 / ctx->B));
  ok &= hipMalloc((void**)&ctx->G, ctx->gslices * Bz * n2 * n2 * sizeof(double2)) == hipSuccess;
  ok &= hipMalloc(&ctx->Wi, Bz * n2 * n2 * ctx->es) == hipSuccess;
  ok &= hipMalloc(&ctx->Wa, Bz * n2 * n2 * ctx->es) == hipSuccess;
  // eigen-problems above 64 keep a rotation log: one per row, or one per
  // diagonal block when the blocks themselves exceed 64 (bonds above 128)
  ctx->log_stride = (long long)ctx->max_steps * (nlog / 2) * 3;
  const size_t log_problems = n2 > 128 ? 2 * Bz : Bz;
  if (n2 > 64) {
    ok &= hipMalloc((void**)&ctx->rot_log, log_problems * ctx->log_stride * sizeof(double)) == hipSuccess;
    ok &= hipStreamCreateWithFlags(&ctx->st_aux, hipStreamNonBlocking) == hipSuccess;
    ok &= hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) == hipSuccess;
    ok &= hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) == hipSuccess;
  }
  // (the solver strides the packed matrices by the size of a 256-wide one)
  if (n2 > 128) ok &= hipMalloc((void**)&ctx->gpk, Bz * (size_t)(256 * 257 / 2) * sizeof(double2)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->lam_sorted, Bz * n2 * sizeof(double)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->order, Bz * n2 * sizeof(int)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->kept, 2 * Bz * sizeof(int)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->scale_abs, 2 * Bz * sizeof(double)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->nsteps, 2 * Bz * sizeof(int)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->rank_table, Bz * L * sizeof(int)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->ext, Bz * L * sizeof(int)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->rank_max, Bz * L * sizeof(int)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->ledger_mem, 7 * Bz * sizeof(double)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->adim, Bz * L * 3 * sizeof(int)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->nk, Bz * 4 * sizeof(int)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->qr_done, Bz * sizeof(int)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->nk_max, 4 * sizeof(int)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->gate4, 32 * sizeof(double)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->d_traj, sizeof(uint64_t)) == hipSuccess;
  ok &= hipHostMalloc((void**)&ctx->nk_host, 4 * sizeof(int), hipHostMallocDefault) == hipSuccess;
  if (ok) {
    ctx->ledger[CLS_EIGH_SMALL] = ctx->ledger_mem;
    ctx->ledger[CLS_EIGH_LARGE] = ctx->ledger_mem + Bz;
    ctx->ledger[CLS_GRAM] = ctx->ledger_mem + 2 * Bz;
    ctx->ledger[CLS_GEMM] = ctx->ledger_mem + 3 * Bz;
    ctx->ledger[CLS_MOVE] = ctx->ledger_mem + 4 * Bz;
    ctx->ledger_bytes[CLS_GRAM] = ctx->ledger_mem + 5 * Bz;
    ctx->ledger_bytes[CLS_GEMM] = ctx->ledger_mem + 6 * Bz;
    ok &= launch_fill_f64(ctx->ledger_mem, 0.0, 7ll * ctx->B, ctx->st) == hipSuccess;
  }
  ok &= hipMalloc((void**)&ctx->disc_acc, Bz * sizeof(double)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->flags, Bz * sizeof(int)) == hipSuccess;
  ok &= hipMalloc((void**)&ctx->degen_acc, Bz * sizeof(int)) == hipSuccess;
  if (!ok) return bail(TTN_ENOMEM);
  {
    void* sp = nullptr;
    if (scratch_for_current_device(&sp) != hipSuccess) return bail(TTN_EDEVICE);
    ctx->scratch_dev = (uint8_t*)sp;
  }
  if (eigh_prepare() != hipSuccess) return bail(TTN_EDEVICE);
  if (reset_state(ctx, nullptr) != TTN_OK) return bail(TTN_EDEVICE);
  if (hipStreamSynchronize(ctx->st) != hipSuccess) return bail(TTN_EDEVICE);
  *out = ctx;
  return TTN_OK;
}

ttn_status ttn_destroy(ttn_ctx* ctx) {
  if (!ctx) return TTN_EINVAL;
  hipStreamSynchronize(ctx->st);
  if (ctx->adj) ttn_destroy(ctx->adj);
  for (auto& b : ctx->bufs) hipFree(b.p);
  for (hipEvent_t e : ctx->tune_ev)
    if (e) hipEventDestroy(e);
  if (ctx->st_aux) {
    hipStreamSynchronize(ctx->st_aux);
    hipStreamDestroy(ctx->st_aux);
  }
  if (ctx->ev_fork) hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) hipEventDestroy(ctx->ev_join);
  if (ctx->graph_exec) hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) hipGraphDestroy(ctx->graph);
  if (ctx->st_graph) {
    hipStreamSynchronize(ctx->st_graph);
    hipStreamDestroy(ctx->st_graph);
  }
  if (ctx->ev_gin) hipEventDestroy(ctx->ev_gin);
  if (ctx->ev_gout) hipEventDestroy(ctx->ev_gout);
  for (auto& e : ctx->prof_ring) {
    hipEventDestroy(e.a);
    hipEventDestroy(e.b);
  }
  void* ws[] = {ctx->G, ctx->Wi, ctx->Wa, ctx->rot_log, ctx->gpk, ctx->lam_sorted, ctx->order, ctx->kept,
                ctx->scale_abs, ctx->nsteps, ctx->rank_table, ctx->ext, ctx->rank_max, ctx->ledger_mem,
                ctx->adim, ctx->nk, ctx->qr_done, ctx->nk_max, ctx->gate4, ctx->d_traj,
                ctx->disc_acc, ctx->flags,
                ctx->degen_acc, ctx->leader, ctx->dec_datarec, ctx->dec_masks};
  for (void* p : ws)
    if (p) hipFree(p);
  if (ctx->nk_host) hipHostFree(ctx->nk_host);
  delete ctx;
  return TTN_OK;
}

ttn_status ttn_init_product(ttn_ctx* ctx, const uint8_t* basis) {
  if (!ctx) return TTN_EINVAL;
  if (basis)
    for (int q = 0; q < ctx->N; ++q)
      if (basis[q] > 1) return fail(ctx, TTN_EINVAL, "basis must be 0 or 1");
  return reset_state(ctx, basis);
}

ttn_status ttn_apply_1q(ttn_ctx* ctx, int32_t q, const double* u, int64_t row_stride) {
  if (!ctx) return TTN_EINVAL;
  if (q < 0 || q >= ctx->N || !u || row_stride < 0) return fail(ctx, TTN_EINVAL, "bad qubit or matrix");
  int leg;
  const int node = bottom_of(ctx, q, &leg);
  TTN_TRY(flush_leaf(ctx));
  ctx->run = LeafBatch{};
  ctx->run.mat = u;
  ctx->run.mat_row_stride = row_stride;
  LeafOp l = leaf_op(LOP_MATRIX, leg);
  push_leaf(ctx, node, l);
  ttn_status s = flush_leaf(ctx);
  ctx->run = LeafBatch{};
  return s;
}

ttn_status ttn_apply_2q(ttn_ctx* ctx, int32_t q0, int32_t q1, const double* g) {
  if (!ctx) return TTN_EINVAL;
  if (q0 < 0 || q1 < 0 || q0 >= ctx->N || q1 >= ctx->N || q0 == q1 || !g)
    return fail(ctx, TTN_EINVAL, "bad qubits or gate");
  for (int i = 0; i < 32; ++i)
    if (!std::isfinite(g[i])) return fail(ctx, TTN_EINVAL, "non-finite gate");
  int l0, l1;
  const int n0 = bottom_of(ctx, q0, &l0), n1 = bottom_of(ctx, q1, &l1);
  auto G = [&](int r, int c, int ri) { return g[(r * 4 + c) * 2 + ri]; };
  if (n0 == n1) {
    // reorder to (leg a, leg b) bit order
    static thread_local double m[32];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) {
        int rr = r, cc = c;
        if (l0 == 1) {   // q0 on leg b: swap bits
          rr = ((r & 1) << 1) | (r >> 1);
          cc = ((c & 1) << 1) | (c >> 1);
        }
        m[(rr * 4 + cc) * 2] = G(r, c, 0);
        m[(rr * 4 + cc) * 2 + 1] = G(r, c, 1);
      }
    TTN_TRY(flush_leaf(ctx));
    // stream-ordered copy into the context's gate buffer: an earlier gate's
    // kernel has read its matrix before this copy runs
    TTN_CHECK_HIP(hipMemcpyAsync(ctx->gate4, m, sizeof(m), hipMemcpyHostToDevice, ctx->st));
    ctx->run = LeafBatch{};
    ctx->run.mat = ctx->gate4;
    ctx->run.mat_row_stride = 0;
    push_leaf(ctx, n0, leaf_op(LOP_GATE4, 0));
    ttn_status s = flush_leaf(ctx);
    ctx->run = LeafBatch{};
    // the host copy is thread-local and may be overwritten by the next call
    TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
    return s;
  }
  // controlled on q0 (block diagonal in q0's index) or on q1
  auto off0 = [&]() {
    double s = 0;
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c)
        if ((r >> 1) != (c >> 1)) s += std::fabs(G(r, c, 0)) + std::fabs(G(r, c, 1));
    return s;
  };
  auto off1 = [&]() {
    double s = 0;
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c)
        if ((r & 1) != (c & 1)) s += std::fabs(G(r, c, 0)) + std::fabs(G(r, c, 1));
    return s;
  };
  double P[2][2][2][2], Bm[2][2][2][2];
  proj(P, 0);
  if (off0() == 0.0) {
    for (int k = 0; k < 2; ++k)
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          for (int z = 0; z < 2; ++z) Bm[k][i][j][z] = G(k * 2 + i, k * 2 + j, z);
    return controlled_gate(ctx, q0, P, q1, Bm);
  }
  if (off1() == 0.0) {
    for (int k = 0; k < 2; ++k)
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          for (int z = 0; z < 2; ++z) Bm[k][i][j][z] = G(i * 2 + k, j * 2 + k, z);
    return controlled_gate(ctx, q1, P, q0, Bm);
  }
  return fail(ctx, TTN_EINVAL, "non-sibling gate must be controlled on one of its qubits");
}

ttn_status ttn_measure_project(ttn_ctx* ctx, int32_t q, int32_t basis, const uint8_t* forced, uint8_t* bits,
                               double* logp, uint64_t traj_offset, int32_t draw) {
  if (!ctx) return TTN_EINVAL;
  if (q < 0 || q >= ctx->N || (basis != 0 && basis != 1) || !bits || !logp || draw < 0)
    return fail(ctx, TTN_EINVAL, "bad measurement arguments");
  if (ctx->trace && draw >= ctx->trace_stride) return fail(ctx, TTN_EINVAL, "draw beyond the probability trace");
  int leg;
  const int node = bottom_of(ctx, q, &leg);
  TTN_TRY(move_centre(ctx, node));
  TTN_TRY(flush_leaf(ctx));
  ctx->run = LeafBatch{};
  ctx->run.records = bits; ctx->run.rec_stride = 1;
  ctx->run.forced_rec = forced; ctx->run.forced_rec_stride = 1;
  ctx->run.logp = logp;
  ctx->run.traj_offset = traj_offset;
  LeafOp l = leaf_op(LOP_MEAS, leg);
  l.arg = basis; l.rec = 0; l.draw = draw;
  push_leaf(ctx, node, l);
  ttn_status s = flush_leaf(ctx);
  ctx->run = LeafBatch{};
  return s;
}

ttn_status ttn_kraus_jump(ttn_ctx* ctx, int32_t q, const double* k, int64_t row_stride, const int8_t* forced,
                          int8_t* branch, double* logp, uint64_t traj_offset, int32_t draw) {
  if (!ctx) return TTN_EINVAL;
  if (q < 0 || q >= ctx->N || !k || !branch || !logp || row_stride < 0 || draw < 0)
    return fail(ctx, TTN_EINVAL, "bad Kraus arguments");
  if (ctx->trace && draw >= ctx->trace_stride) return fail(ctx, TTN_EINVAL, "draw beyond the probability trace");
  int leg;
  const int node = bottom_of(ctx, q, &leg);
  TTN_TRY(move_centre(ctx, node));
  TTN_TRY(flush_leaf(ctx));
  ctx->run = LeafBatch{};
  ctx->run.mat = k; ctx->run.mat_row_stride = row_stride;
  ctx->run.branches = branch; ctx->run.br_stride = 1;
  ctx->run.forced_br = forced; ctx->run.forced_br_stride = 1;
  ctx->run.logp = logp;
  ctx->run.traj_offset = traj_offset;
  LeafOp l = leaf_op(LOP_KRAUS_MAT, leg);
  l.loc = 0; l.draw = draw; l.branch = 0;
  push_leaf(ctx, node, l);
  ttn_status s = flush_leaf(ctx);
  ctx->run = LeafBatch{};
  return s;
}

ttn_status ttn_oplist_upload(ttn_ctx* ctx, const int32_t* ops, int32_t n_ops, int32_t n_loc, int32_t n_rec,
                             int32_t n_draws, ttn_oplist** out) {
  if (!ctx) return TTN_EINVAL;
  if (!ops || n_ops < 0 || n_loc < 0 || n_rec < 0 || n_draws < 0 || !out)
    return fail(ctx, TTN_EINVAL, "bad op list");
  ttn_oplist* ol = new ttn_oplist();
  ol->ctx = ctx;
  ol->ops.assign(ops, ops + (size_t)n_ops * 9);
  ol->n_ops = n_ops; ol->n_loc = n_loc; ol->n_rec = n_rec; ol->n_draws = n_draws;
  for (int k = 0; k < n_ops; ++k) {
    const int32_t* o = &ops[(size_t)k * 9];
    const int op = o[0], q0 = o[1], q1 = o[2];
    bool bad = q0 < 0 || q0 >= ctx->N || op < 0 || op > 5;
    if (op == TTN_OP_CNOT) bad |= q1 < 0 || q1 >= ctx->N || q1 == q0;
    if (op == TTN_OP_SRX || op == TTN_OP_AD || op == TTN_OP_PAULI) bad |= o[4] < 0 || o[4] >= n_loc;
    if (op == TTN_OP_AD || op == TTN_OP_PAULI || op == TTN_OP_MEAS) bad |= o[5] < 0 || o[5] >= n_draws;
    if (op == TTN_OP_MEAS) bad |= o[6] < 0 || o[6] >= n_rec || (o[3] != 0 && o[3] != 1);
    if (op == TTN_OP_INIT) bad |= (o[3] != 0 && o[3] != 1) || o[7] < -1 || o[7] > 1 || (o[7] >= 0 && (o[6] < 0 || o[6] >= n_rec));
    if (op == TTN_OP_PAULI) bad |= (o[3] != 0 && o[3] != 1);
    if (bad) {
      delete ol;
      return fail(ctx, TTN_EINVAL, "op " + std::to_string(k) + " is malformed");
    }
    ol->ad_col.push_back(op == TTN_OP_AD ? ol->n_ad : -1);
    ol->n_ad += op == TTN_OP_AD;
  }
  *out = ol;
  return TTN_OK;
}

ttn_status ttn_oplist_free(ttn_oplist* ol) {
  delete ol;
  return TTN_OK;
}

// Graph mode: the op list is captured once per (op list, argument buffers)
// on the context's own capture stream (a graph cannot be captured on the
// default stream) and launched there, ordered after the caller's stream by
// events; the trajectory offset is the only argument that changes between
// launches, and it lives in device memory (ctx->d_traj), written before
// each launch.  Capturing executes nothing, so the host's record of the
// node buffers after the capture is that of the graph's end state, which
// every launch reproduces.  (The eigensolver's one-time set-up, which may
// not be captured, runs at context creation.)
static ttn_status graph_run(ttn_ctx* ctx, const ttn_oplist* ol, const double* theta, const double* gamma,
                            int64_t pstride, uint64_t traj_offset, uint8_t* records, int8_t* branches,
                            double* logp, ttn_stats* st) {
  if (ctx->prof) return fail(ctx, TTN_EINVAL, "profiling is not available in graph mode");
  if (!ol || ol->ctx != ctx) return fail(ctx, TTN_EINVAL, "op list belongs to another context");
  if (!ctx->st_graph) {
    TTN_CHECK_HIP(hipStreamCreateWithFlags(&ctx->st_graph, hipStreamNonBlocking));
    TTN_CHECK_HIP(hipEventCreateWithFlags(&ctx->ev_gin, hipEventDisableTiming));
    TTN_CHECK_HIP(hipEventCreateWithFlags(&ctx->ev_gout, hipEventDisableTiming));
  }
  const std::array<uintptr_t, 8> key = {(uintptr_t)ol, (uintptr_t)theta, (uintptr_t)gamma, (uintptr_t)pstride,
                                        (uintptr_t)records, (uintptr_t)branches, (uintptr_t)logp,
                                        (uintptr_t)ctx->trace};
  TTN_TRY(flush_leaf(ctx));   // pending single-qubit ops, on the caller's stream
  hipStream_t caller = ctx->st;
  TTN_CHECK_HIP(hipEventRecord(ctx->ev_gin, caller));
  TTN_CHECK_HIP(hipStreamWaitEvent(ctx->st_graph, ctx->ev_gin, 0));
  ttn_status s = TTN_OK;
  ctx->st = ctx->st_graph;
  if (!ctx->graph_exec || key != ctx->graph_key) {
    if (ctx->graph_exec) hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    {
      hipError_t e = hipStreamBeginCapture(ctx->st, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) {
        s = fail(ctx, TTN_EDEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
      } else {
        ctx->capturing = true;
        const ttn_status sc = run_oplist(ctx, ol, theta, gamma, pstride, traj_offset, records, branches, logp,
                                         nullptr, nullptr, nullptr);
        ctx->capturing = false;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(ctx->st, &g);
        if (sc != TTN_OK) {
          s = sc;
        } else if (e != hipSuccess || !g) {
          s = fail(ctx, TTN_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        } else {
          ctx->graph = g;
          e = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
          if (e != hipSuccess) {
            ctx->graph_exec = nullptr;
            s = fail(ctx, TTN_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
          } else {
            ctx->graph_key = key;
            ++ctx->graph_captures;
          }
        }
        if (s != TTN_OK && g && !ctx->graph) hipGraphDestroy(g);
      }
    }
  }
  if (s == TTN_OK) {
    hipError_t e = launch_fill_u64(ctx->d_traj, traj_offset, 1, ctx->st);
    if (e == hipSuccess) e = hipGraphLaunch(ctx->graph_exec, ctx->st);
    if (e != hipSuccess) s = fail(ctx, TTN_EDEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    else ++ctx->graph_replays;
  }
  ctx->st = caller;
  TTN_CHECK_HIP(hipEventRecord(ctx->ev_gout, ctx->st_graph));
  TTN_CHECK_HIP(hipStreamWaitEvent(caller, ctx->ev_gout, 0));
  if (s == TTN_OK && st) TTN_TRY(fill_stats(ctx, st));
  return s;
}

ttn_status ttn_batch_run_circuit(ttn_ctx* ctx, const ttn_oplist* ol, const double* theta, const double* gamma,
                                 int64_t params_stride, uint64_t traj_offset, uint8_t* records, int8_t* branches,
                                 double* logp, ttn_stats* st) {
  if (!ctx) return TTN_EINVAL;
  if (params_stride < 0) return fail(ctx, TTN_EINVAL, "negative parameter stride");
  ttn_status s;
  if (ctx->run_mode == TTN_RUN_GRAPH)
    s = graph_run(ctx, ol, theta, gamma, params_stride, traj_offset, records, branches, logp, st);
  else
    s = run_oplist(ctx, ol, theta, gamma, params_stride, traj_offset, records, branches, logp, nullptr, nullptr, st);
  if (s == TTN_OK && st && st->flagged_rows > 0) return TTN_ENONFINITE;
  return s;
}

ttn_status ttn_set_run_mode(ttn_ctx* ctx, int32_t mode, int64_t* captures, int64_t* replays) {
  if (!ctx) return TTN_EINVAL;
  if (mode < TTN_RUN_DYNAMIC || mode > TTN_RUN_GRAPH) return fail(ctx, TTN_EINVAL, "unknown run mode");
  TTN_TRY(flush_leaf(ctx));
  if (ctx->run_mode != mode) {
    TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
    if (ctx->graph_exec) hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    ctx->run_mode = mode;
  }
  if (captures) *captures = ctx->graph_captures;
  if (replays) *replays = ctx->graph_replays;
  return TTN_OK;
}

ttn_status ttn_log_prob(ttn_ctx* ctx, const ttn_oplist* ol, const uint8_t* records, const int8_t* branches,
                        const double* theta, const double* gamma, int64_t params_stride, double* logp,
                        ttn_stats* st) {
  if (!ctx) return TTN_EINVAL;
  if (!records || params_stride < 0) return fail(ctx, TTN_EINVAL, "records required");
  if (ol && ol->n_ad > 0 && !branches) return fail(ctx, TTN_EINVAL, "branches required (AD ops)");
  // forced run: the record buffer is read (and rewritten with identical bits)
  ttn_status s = run_oplist(ctx, ol, theta, gamma, params_stride, 0, const_cast<uint8_t*>(records),
                            nullptr, logp, records, branches, st);
  if (s == TTN_OK && st && st->flagged_rows > 0) return TTN_EPROB;
  return s;
}

// ------------------------------------------------------- log P gradient ----
// Reverse-mode derivative of log P of a forced record by every location's
// theta and gamma (see ttn_adjoint.hip for the formula).  The forward pass
// keeps snapshots of the state at the start of some noise layers; the
// backward pass carries the adjoint state lambda in a twin context from the
// final state to the first op, applying each op's adjoint, and at every
// noise layer restores the nearest earlier snapshot, re-runs the state to
// the layer's start and contracts the two trees into the layer's leaf
// environments.

namespace {
struct Snapshot {
  std::vector<std::array<int, 3>> dims;
  std::vector<char> ext_ok;
  int centre = 1;
  void* mem = nullptr;
  std::vector<size_t> off;
};
struct NoiseLayer { int k0, k1; };
constexpr int kMaxSnapshots = 16;
}  // namespace

static void snap_free(Snapshot& s) {
  if (s.mem) hipFree(s.mem);
  s.mem = nullptr;
}

static ttn_status snap_take(ttn_ctx* c, Snapshot& s) {
  ttn_ctx* ctx = c;
  TTN_TRY(flush_leaf(c));
  snap_free(s);
  s.dims = c->dims;
  s.ext_ok = c->ext_ok;
  s.centre = c->centre;
  s.off.assign(c->L + 1, 0);
  size_t tot = 0;
  for (int node = 1; node < c->L; ++node) {
    s.off[node] = tot;
    tot += ((size_t)c->B * elems(c->dims[node]) * c->es + 255) & ~(size_t)255;
  }
  s.off[c->L] = tot;                      // the per-row bond extents
  tot += (size_t)c->B * c->L * sizeof(int);
  if (hipMalloc(&s.mem, tot) != hipSuccess) {
    s.mem = nullptr;
    return fail(c, TTN_ENOMEM, "snapshot allocation failed (reduce the batch)");
  }
  for (int node = 1; node < c->L; ++node)
    TTN_CHECK_HIP(hipMemcpyAsync((char*)s.mem + s.off[node], node_ptr(c, node),
                                 (size_t)c->B * elems(c->dims[node]) * c->es, hipMemcpyDeviceToDevice, c->st));
  TTN_CHECK_HIP(hipMemcpyAsync((char*)s.mem + s.off[c->L], c->ext, (size_t)c->B * c->L * sizeof(int),
                               hipMemcpyDeviceToDevice, c->st));
  return TTN_OK;
}

// into c (the snapshot's own context or its twin: same tree and pool)
static ttn_status snap_restore(ttn_ctx* c, const Snapshot& s) {
  ttn_ctx* ctx = c;
  TTN_TRY(flush_leaf(c));
  if ((int)s.dims.size() != c->L) return fail(c, TTN_EINVAL, "internal: snapshot of another tree");
  for (int node = 1; node < c->L; ++node) {
    const long long n = (long long)c->B * elems(s.dims[node]);
    if (n > buf_elems(c, c->node_buf[node])) return fail(c, TTN_EINVAL, "internal: snapshot exceeds the pool");
    TTN_CHECK_HIP(hipMemcpyAsync(node_ptr(c, node), (const char*)s.mem + s.off[node], (size_t)n * c->es,
                                 hipMemcpyDeviceToDevice, c->st));
  }
  TTN_CHECK_HIP(hipMemcpyAsync(c->ext, (const char*)s.mem + s.off[c->L], (size_t)c->B * c->L * sizeof(int),
                               hipMemcpyDeviceToDevice, c->st));
  c->dims = s.dims;
  c->ext_ok = s.ext_ok;
  c->centre = s.centre;
  return TTN_OK;
}

// C[t][i][j] = sum over the two other legs of conj(A[..i..]) Bt[..j..]; A and
// Bt agree on those legs' dimensions
static GemmDesc cross_desc(const void* A, std::array<int, 3> dA, const void* Bt, std::array<int, 3> dB, int leg,
                           void* C) {
  GemmDesc g{};
  g.H = 1;
  g.conjA = 1;
  g.A = A; g.B = Bt; g.C = C;
  g.sAt = elems(dA); g.sBt = elems(dB);
  g.M = dA[leg]; g.N = dB[leg];
  g.sCt = (long long)g.M * g.N; g.sCi = g.N; g.sCj = 1;
  if (leg == 0) {
    const long long R = (long long)dA[1] * dA[2];
    g.sAi = R; g.sAl2 = 1; g.a_m_fast = 0;
    g.sBj = R; g.sBl2 = 1; g.b_n_fast = 0;
    g.K = (int)R; g.Kin = g.K;
  } else if (leg == 2) {
    g.sAi = 1; g.sAl2 = dA[2]; g.a_m_fast = 1;
    g.sBj = 1; g.sBl2 = dB[2]; g.b_n_fast = 1;
    g.K = dA[0] * dA[1]; g.Kin = g.K;
  } else {
    g.sAi = dA[2]; g.sAl1 = (long long)dA[1] * dA[2]; g.sAl2 = 1; g.a_m_fast = 0;
    g.sBj = dB[2]; g.sBl1 = (long long)dB[1] * dB[2]; g.sBl2 = 1; g.b_n_fast = 0;
    g.K = dA[0] * dA[2]; g.Kin = dA[2];
  }
  return g;
}

static ttn_status env_gemm(ttn_ctx* c, const GemmDesc& g, long long capA, long long capB, long long capC) {
  ttn_ctx* ctx = c;
  if (!gemm_fits(g, c->B, capA, capB, capC)) return fail(c, TTN_EINVAL, "internal: environment exceeds its buffers");
  ++c->launches;
  TTN_CHECK_HIP(launch_zgemm(g, c->B, c->c128 ? GEMM_C128 : GEMM_C64, c->st, c->force_cfg));
  return TTN_OK;
}

// out = W applied on leg `leg` of T (W: [rows][newd][d[leg]])
static ttn_status env_apply(ttn_ctx* c, const void* T, std::array<int, 3> d, long long capT, int leg, const void* W,
                            long long capW, int newd, void* out, long long capOut) {
  GemmDesc g = leg_desc(T, d, leg, W, newd, newd, out);
  const bool wA = (leg != 2);
  return env_gemm(c, g, wA ? capW : capT, wA ? capT : capW, capOut);
}

struct EnvWork {
  std::vector<void*> up, down;       // per node [B][cap^2]
  std::vector<long long> cap_el;     // elements per env buffer
  void* t1 = nullptr;
  void* t2 = nullptr;
  long long t_el = 0;
  ~EnvWork() {
    for (void* p : up) if (p) hipFree(p);
    for (void* p : down) if (p) hipFree(p);
    if (t1) hipFree(t1);
    if (t2) hipFree(t2);
  }
};

static ttn_status env_alloc(ttn_ctx* c, EnvWork& w) {
  w.up.assign(c->L, nullptr);
  w.down.assign(c->L, nullptr);
  w.cap_el.assign(c->L, 0);
  long long tmax = 1;
  for (int node = 1; node < c->L; ++node) {
    const long long cu = node == 1 ? 1 : bond_cap(c, node);
    w.cap_el[node] = (long long)c->B * cu * cu;
    if (hipMalloc(&w.up[node], w.cap_el[node] * c->es) != hipSuccess ||
        hipMalloc(&w.down[node], w.cap_el[node] * c->es) != hipSuccess)
      return fail(c, TTN_ENOMEM, "environment allocation failed");
    if (!is_bottom(c, node)) tmax = std::max(tmax, (long long)bond_cap(c, 2 * node) * bond_cap(c, 2 * node + 1) * cu);
  }
  w.t_el = (long long)c->B * tmax;
  if (hipMalloc(&w.t1, w.t_el * c->es) != hipSuccess || hipMalloc(&w.t2, w.t_el * c->es) != hipSuccess)
    return fail(c, TTN_ENOMEM, "environment allocation failed");
  return TTN_OK;
}

// leaf environments of the layer ops [k0, k1) between state ps (before the
// layer) and adjoint state lm (after it), accumulated into dtheta / dgamma
static ttn_status env_layer(ttn_ctx* ps, ttn_ctx* lm, const ttn_oplist* ol, int k0, int k1, EnvWork& w,
                            const EnvParams& par, double* dtheta, double* dgamma) {
  ttn_ctx* ctx = ps;
  TTN_TRY(flush_leaf(ps));
  TTN_TRY(flush_leaf(lm));
  const int L = ps->L, B = ps->B;
  std::vector<LeafNoise> nz(L);
  for (auto& z : nz) z.n = 0;
  std::vector<char> noisy(L, 0);
  for (int k = k0; k < k1; ++k) {
    const int32_t* o = &ol->ops[(size_t)k * 9];
    const int leaf = ps->leaf_of_qubit[o[1]];
    LeafNoise& z = nz[leaf];
    if (z.n >= kMaxLeafNoise) return fail(ps, TTN_EINVAL, "internal: noise layer too deep");
    z.kind[z.n] = o[0] == TTN_OP_SRX ? NOISE_SRX : NOISE_AD;
    z.loc[z.n] = o[4];
    z.branch[z.n] = ol->ad_col[k];
    ++z.n;
    for (int node = L / 2 + leaf / 2; node >= 1; node /= 2) noisy[node] = 1;
  }
  auto bottom_desc = [&](int node) {
    EnvBottom d{};
    d.lam = node_ptr(lm, node);
    d.psi = node_ptr(ps, node);
    d.ul = lm->dims[node][2];
    d.up = ps->dims[node][2];
    const int l0 = 2 * (node - L / 2);
    d.nz[0] = nz[l0];
    d.nz[1] = nz[l0 + 1];
    d.par = par;
    d.dtheta = dtheta;
    d.dgamma = dgamma;
    d.gstride = ol->n_loc;
    d.flags = ps->flags;
    d.c128 = ps->c128;
    return d;
  };
  // up environments, leaves to root
  for (int x = L - 1; x >= 1; --x) {
    const std::array<int, 3> dl = lm->dims[x], dp = ps->dims[x];
    if ((long long)B * dl[2] * dp[2] > w.cap_el[x]) return fail(ps, TTN_EINVAL, "internal: environment too large");
    if (is_bottom(ps, x)) {
      if (dl[0] != 2 || dl[1] != 2 || dp[0] != 2 || dp[1] != 2) return fail(ps, TTN_EINVAL, "internal: bottom dims");
      EnvBottom d = bottom_desc(x);
      d.out = w.up[x];
      ++ps->launches;
      TTN_CHECK_HIP(launch_env_bottom_up(d, B, ps->st));
      continue;
    }
    const int a = 2 * x, b = 2 * x + 1;
    const std::array<int, 3> t1 = {dl[0], dp[1], dp[2]};
    const std::array<int, 3> t2 = {dl[0], dl[1], dp[2]};
    TTN_TRY(env_apply(ps, node_ptr(ps, x), dp, buf_elems(ps, ps->node_buf[x]), 0, w.up[a], w.cap_el[a], dl[0],
                      w.t1, w.t_el));
    TTN_TRY(env_apply(ps, w.t1, t1, w.t_el, 1, w.up[b], w.cap_el[b], dl[1], w.t2, w.t_el));
    TTN_TRY(env_gemm(ps, cross_desc(node_ptr(lm, x), dl, w.t2, t2, 2, w.up[x]), buf_elems(lm, lm->node_buf[x]),
                     w.t_el, w.cap_el[x]));
  }
  // down environments, root to the bottom nodes that carry noise
  if (ps->dims[1][2] != 1 || lm->dims[1][2] != 1) return fail(ps, TTN_EINVAL, "internal: root up dimension");
  TTN_CHECK_HIP(launch_fill_cone(w.down[1], ps->c128, B, ps->st));
  for (int x = 1; x < L / 2; ++x) {
    if (!noisy[x]) continue;
    const std::array<int, 3> dl = lm->dims[x], dp = ps->dims[x];
    const int a = 2 * x, b = 2 * x + 1;
    const long long capX = buf_elems(ps, ps->node_buf[x]), capL = buf_elems(lm, lm->node_buf[x]);
    if (noisy[a]) {
      const std::array<int, 3> t1 = {dp[0], dl[1], dp[2]};
      const std::array<int, 3> t2 = {dp[0], dl[1], dl[2]};
      TTN_TRY(env_apply(ps, node_ptr(ps, x), dp, capX, 1, w.up[b], w.cap_el[b], dl[1], w.t1, w.t_el));
      TTN_TRY(env_apply(ps, w.t1, t1, w.t_el, 2, w.down[x], w.cap_el[x], dl[2], w.t2, w.t_el));
      TTN_TRY(env_gemm(ps, cross_desc(node_ptr(lm, x), dl, w.t2, t2, 0, w.down[a]), capL, w.t_el, w.cap_el[a]));
    }
    if (noisy[b]) {
      const std::array<int, 3> t1 = {dl[0], dp[1], dp[2]};
      const std::array<int, 3> t2 = {dl[0], dp[1], dl[2]};
      TTN_TRY(env_apply(ps, node_ptr(ps, x), dp, capX, 0, w.up[a], w.cap_el[a], dl[0], w.t1, w.t_el));
      TTN_TRY(env_apply(ps, w.t1, t1, w.t_el, 2, w.down[x], w.cap_el[x], dl[2], w.t2, w.t_el));
      TTN_TRY(env_gemm(ps, cross_desc(node_ptr(lm, x), dl, w.t2, t2, 1, w.down[b]), capL, w.t_el, w.cap_el[b]));
    }
  }
  for (int x = L / 2; x < L; ++x) {
    if (!noisy[x]) continue;
    EnvBottom d = bottom_desc(x);
    d.down = w.down[x];
    ++ps->launches;
    TTN_CHECK_HIP(launch_env_leaf_grad(d, B, ps->st));
  }
  return TTN_OK;
}

static ttn_status ensure_twin(ttn_ctx* ctx) {
  if (ctx->adj) return TTN_OK;
  ttn_config cfg{};
  cfg.n_qubits = ctx->N;
  cfg.leaf_of_qubit = ctx->leaf_of_qubit.data();
  cfg.chi_max = ctx->chi;
  cfg.cutoff = ctx->cutoff;
  cfg.dtype = ctx->c128 ? TTN_C128 : TTN_C64;
  cfg.ad_mode = ctx->ad_trotter ? TTN_AD_TROTTER : TTN_AD_KRAUS;
  cfg.batch = ctx->B;
  cfg.seed = ctx->seed;
  cfg.stream = ctx->st;
  ttn_ctx* t = nullptr;
  const ttn_status s = ttn_create(&cfg, &t);
  if (s != TTN_OK) return fail(ctx, s, "adjoint context: allocation failed");
  ctx->adj = t;
  return TTN_OK;
}

static ttn_status log_prob_grad(ttn_ctx* ctx, const ttn_oplist* ol, const uint8_t* records, const int8_t* branches,
                                const double* theta, const double* gamma, int64_t pstride, double* logp,
                                double* dtheta, double* dgamma, uint8_t* rec_copy, double* logp_scr,
                                ttn_stats* st) {
  // noise layers
  std::vector<NoiseLayer> layers;
  {
    std::vector<int> depth(ctx->L, 0);
    int k = 0;
    while (k < ol->n_ops) {
      const int op = ol->ops[(size_t)k * 9];
      if (op != TTN_OP_SRX && op != TTN_OP_AD) { ++k; continue; }
      NoiseLayer ly{k, k};
      std::fill(depth.begin(), depth.end(), 0);
      while (k < ol->n_ops) {
        const int32_t* o = &ol->ops[(size_t)k * 9];
        if (o[0] != TTN_OP_SRX && o[0] != TTN_OP_AD) break;
        int& dq = depth[ctx->leaf_of_qubit[o[1]]];
        if (dq == kMaxLeafNoise) break;
        ++dq;
        ++k;
      }
      ly.k1 = k;
      layers.push_back(ly);
    }
  }
  const int nl = (int)layers.size();
  const int every = std::max(1, (nl + kMaxSnapshots - 1) / kMaxSnapshots);
  std::vector<Snapshot> snaps(nl);
  struct Cleanup {
    std::vector<Snapshot>* s;
    ~Cleanup() { for (auto& x : *s) snap_free(x); }
  } cleanup{&snaps};
  ttn_ctx* lm = ctx->adj;

  // forward pass, snapshots at the start of every `every`-th layer
  ctx->hops = 0; ctx->launches = 0; ctx->block_hops = 0; ctx->gemm_flops = 0.0; ctx->gram_flops = 0.0;
  TTN_TRY(reset_state(ctx, nullptr));
  TTN_CHECK_HIP(launch_fill_f64(logp, 0.0, ctx->B, ctx->st));
  setup_run(ctx, ol, theta, gamma, pstride, 0, rec_copy, nullptr, logp, records, branches, 0);
  int pos = 0;
  for (int r = 0; r < nl; r += every) {
    for (; pos < layers[r].k0; ++pos) TTN_TRY(exec_op(ctx, ol, pos));
    TTN_TRY(snap_take(ctx, snaps[r]));
  }
  for (; pos < ol->n_ops; ++pos) TTN_TRY(exec_op(ctx, ol, pos));
  TTN_TRY(flush_leaf(ctx));
  ctx->run.logp = logp_scr;     // re-runs below must not add to log P again

  // adjoint state = final state
  {
    Snapshot fin;
    TTN_TRY(snap_take(ctx, fin));
    TTN_TRY(reset_state(lm, nullptr));
    setup_run(lm, ol, theta, gamma, pstride, 0, rec_copy, nullptr, logp_scr, records, branches, 1);
    const ttn_status s = snap_restore(lm, fin);
    TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
    snap_free(fin);
    TTN_TRY(s);
  }
  EnvWork w;
  TTN_TRY(env_alloc(ctx, w));
  EnvParams par{};
  par.theta = theta; par.gamma = gamma; par.pstride = pstride;
  par.branches = branches; par.br_stride = ol->n_ad;
  TTN_CHECK_HIP(launch_fill_f64(dtheta, 0.0, (long long)ctx->B * ol->n_loc, ctx->st));
  TTN_CHECK_HIP(launch_fill_f64(dgamma, 0.0, (long long)ctx->B * ol->n_loc, ctx->st));

  int k = ol->n_ops - 1;
  int r = nl - 1;
  while (k >= 0) {
    if (r >= 0 && k == layers[r].k1 - 1) {
      const int c = (r / every) * every;
      TTN_TRY(snap_restore(ctx, snaps[c]));
      for (int q = layers[c].k0; q < layers[r].k0; ++q) TTN_TRY(exec_op(ctx, ol, q));
      TTN_TRY(env_layer(ctx, lm, ol, layers[r].k0, layers[r].k1, w, par, dtheta, dgamma));
      for (int q = layers[r].k1 - 1; q >= layers[r].k0; --q) TTN_TRY(exec_op(lm, ol, q));
      k = layers[r].k0 - 1;
      --r;
    } else {
      TTN_TRY(exec_op(lm, ol, k));
      --k;
    }
  }
  TTN_TRY(flush_leaf(lm));
  TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
  ctx->run = LeafBatch{};
  lm->run = LeafBatch{};
  if (st) {
    TTN_TRY(fill_stats(ctx, st));
    std::vector<int> fl(ctx->B);
    TTN_CHECK_HIP(hipMemcpy(fl.data(), lm->flags, fl.size() * 4, hipMemcpyDeviceToHost));
    std::vector<int> fp(ctx->B);
    TTN_CHECK_HIP(hipMemcpy(fp.data(), ctx->flags, fp.size() * 4, hipMemcpyDeviceToHost));
    st->flagged_rows = 0;
    for (int t = 0; t < ctx->B; ++t) st->flagged_rows += (fl[t] != 0) || (fp[t] != 0);
    st->hops += lm->hops;
    st->launches += lm->launches;
  }
  return TTN_OK;
}

ttn_status ttn_log_prob_grad(ttn_ctx* ctx, const ttn_oplist* ol, const uint8_t* records, const int8_t* branches,
                             const double* theta, const double* gamma, int64_t params_stride, double* logp,
                             double* dtheta, double* dgamma, ttn_stats* st) {
  if (!ctx) return TTN_EINVAL;
  if (!ol || ol->ctx != ctx) return fail(ctx, TTN_EINVAL, "op list belongs to another context");
  if (!records || !theta || !gamma || !logp || !dtheta || !dgamma || params_stride < 0)
    return fail(ctx, TTN_EINVAL, "records, parameters and outputs are required");
  if (ol->n_ad > 0 && !branches) return fail(ctx, TTN_EINVAL, "branches required (AD ops)");
  if (ctx->ad_trotter && ol->n_ad > 0)
    return fail(ctx, TTN_EINVAL, "the gradient is defined for the exact Kraus unravelling (ad_mode TTN_AD_KRAUS)");
  for (int k = 0; k < ol->n_ops; ++k)
    if (ol->ops[(size_t)k * 9] == TTN_OP_PAULI)
      return fail(ctx, TTN_EINVAL, "the gradient needs the non-twirled channels (op list has twirled ops)");
  ctx->err.clear();
  TTN_TRY(ensure_twin(ctx));
  ctx->adj->err.clear();
  uint8_t* rec_copy = nullptr;
  double* logp_scr = nullptr;
  const size_t rec_bytes = (size_t)ctx->B * std::max(ol->n_rec, 1);
  if (hipMalloc((void**)&rec_copy, rec_bytes) != hipSuccess ||
      hipMalloc((void**)&logp_scr, (size_t)ctx->B * sizeof(double)) != hipSuccess) {
    if (rec_copy) hipFree(rec_copy);
    return fail(ctx, TTN_ENOMEM, "scratch allocation failed");
  }
  ttn_status s = TTN_OK;
  if (ol->n_rec > 0 &&
      hipMemcpyAsync(rec_copy, records, (size_t)ctx->B * ol->n_rec, hipMemcpyDeviceToDevice, ctx->st) != hipSuccess)
    s = fail(ctx, TTN_EDEVICE, "record copy failed");
  if (s == TTN_OK)
    s = log_prob_grad(ctx, ol, records, branches, theta, gamma, params_stride, logp, dtheta, dgamma, rec_copy,
                      logp_scr, st);
  if (s != TTN_OK && ctx->adj && ctx->err.empty()) ctx->err = ctx->adj->err;
  hipStreamSynchronize(ctx->st);
  hipFree(rec_copy);
  hipFree(logp_scr);
  ctx->run = LeafBatch{};
  if (s == TTN_OK && st && st->flagged_rows > 0) return TTN_EPROB;
  return s;
}

ttn_status ttn_trace_probs(ttn_ctx* ctx, double* probs, int64_t stride) {
  if (!ctx) return TTN_EINVAL;
  if (probs && stride < 1) return fail(ctx, TTN_EINVAL, "trace stride must be >= 1");
  ctx->trace = probs;
  ctx->trace_stride = probs ? stride : 0;
  return TTN_OK;
}

// Leader-parity table of the final-data decoder: par[s] = parity of the
// first minimum-weight flip pattern that breadth-first search over single
// flips (qubits in ascending order) reaches with syndrome s; masks: the check
// rows as two 32-bit words over the data index.
static void decoder_table(const uint8_t* checks, int n_checks, int n_data, std::vector<uint8_t>& par,
                          std::vector<uint32_t>& masks) {
  std::vector<uint32_t> col(n_data, 0);
  masks.assign(2 * (size_t)std::max(n_checks, 1), 0);
  for (int p = 0; p < n_checks; ++p)
    for (int k = 0; k < n_data; ++k)
      if (checks[(size_t)p * n_data + k]) {
        col[k] |= 1u << p;
        if (k < 32) masks[2 * p] |= 1u << k;
        else masks[2 * p + 1] |= 1u << (k - 32);
      }
  const size_t S = (size_t)1 << n_checks;
  par.assign(S, 0);
  std::vector<uint8_t> seen(S, 0);
  std::deque<uint32_t> dq;
  seen[0] = 1;
  dq.push_back(0);
  std::vector<std::vector<uint8_t>> pattern(1, std::vector<uint8_t>(n_data, 0));
  std::vector<int> pat_of(S, -1);
  pat_of[0] = 0;
  while (!dq.empty()) {
    const uint32_t s = dq.front();
    dq.pop_front();
    const std::vector<uint8_t> cur = pattern[pat_of[s]];
    for (int k = 0; k < n_data; ++k) {
      if (cur[k]) continue;
      const uint32_t s2 = s ^ col[k];
      if (seen[s2]) continue;
      seen[s2] = 1;
      std::vector<uint8_t> nxt = cur;
      nxt[k] = 1;
      par[s2] = par[s] ^ 1;
      pat_of[s2] = (int)pattern.size();
      pattern.push_back(nxt);
      dq.push_back(s2);
    }
  }
}

static ttn_status decode_args(ttn_ctx* ctx, const uint8_t* records, int32_t n_rec, const int32_t* data_rec,
                              int32_t n_data, const uint8_t* checks, int32_t n_checks, uint8_t* fail_out,
                              int max_checks) {
  if (!records || !data_rec || !checks || !fail_out || n_data < 1 || n_data > 64 || n_checks < 0 ||
      n_checks > max_checks || n_rec < 1)
    return fail(ctx, TTN_EINVAL, "bad decoder arguments (n_data 1..64, n_checks 0.." +
                                     std::to_string(max_checks) + ")");
  for (int k = 0; k < n_data; ++k)
    if (data_rec[k] < 0 || data_rec[k] >= n_rec) return fail(ctx, TTN_EINVAL, "bad data record index");
  return TTN_OK;
}

ttn_status ttn_decode(ttn_ctx* ctx, const uint8_t* records, int32_t n_rec, const int32_t* data_rec, int32_t n_data,
                      const uint8_t* checks, int32_t n_checks, uint8_t* fail_out) {
  if (!ctx) return TTN_EINVAL;
  TTN_TRY(decode_args(ctx, records, n_rec, data_rec, n_data, checks, n_checks, fail_out, 24));
  std::vector<uint8_t> par;
  std::vector<uint32_t> masks;
  decoder_table(checks, n_checks, n_data, par, masks);
  const size_t S = par.size();
  if (ctx->leader_bytes < S) {
    if (ctx->leader) hipFree(ctx->leader);
    ctx->leader = nullptr;
    TTN_CHECK_HIP(hipMalloc((void**)&ctx->leader, S));
    ctx->leader_bytes = S;
  }
  if (!ctx->dec_datarec) TTN_CHECK_HIP(hipMalloc((void**)&ctx->dec_datarec, 64 * sizeof(int)));
  if (!ctx->dec_masks) TTN_CHECK_HIP(hipMalloc((void**)&ctx->dec_masks, 2 * 24 * sizeof(uint32_t)));
  TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
  TTN_CHECK_HIP(hipMemcpy(ctx->leader, par.data(), S, hipMemcpyHostToDevice));
  TTN_CHECK_HIP(hipMemcpy(ctx->dec_datarec, data_rec, n_data * sizeof(int), hipMemcpyHostToDevice));
  TTN_CHECK_HIP(hipMemcpy(ctx->dec_masks, masks.data(), masks.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  TTN_CHECK_HIP(launch_decode(records, n_rec, ctx->dec_datarec, n_data, ctx->dec_masks, n_checks, ctx->leader,
                              fail_out, ctx->B, ctx->st));
  return TTN_OK;
}

ttn_status ttn_decode_static(ttn_ctx* ctx, const uint8_t* records, int32_t n_rec, const int32_t* data_rec,
                             int32_t n_data, const uint8_t* checks, int32_t n_checks, uint8_t* fail_out) {
  if (!ctx) return TTN_EINVAL;
  TTN_TRY(decode_args(ctx, records, n_rec, data_rec, n_data, checks, n_checks, fail_out, TTN_DECODE_STATIC_MAX_CHECKS));
  if (!ctx->scratch_dev) return fail(ctx, TTN_EDEVICE, "static scratch not resolved for this device");
  std::vector<uint8_t> par;
  std::vector<uint32_t> masks;
  decoder_table(checks, n_checks, n_data, par, masks);
  // every byte the kernel reads is rewritten here: the table's 2^n_checks
  // entries, the n_data record columns and the n_checks mask pairs
  uint8_t* base = ctx->scratch_dev;
  int* d_datarec = (int*)(base + kScratchDataRec);
  uint32_t* d_masks = (uint32_t*)(base + kScratchMasks);
  TTN_CHECK_HIP(hipMemcpyAsync(base, par.data(), par.size(), hipMemcpyHostToDevice, ctx->st));
  TTN_CHECK_HIP(hipMemcpyAsync(d_datarec, data_rec, n_data * sizeof(int), hipMemcpyHostToDevice, ctx->st));
  TTN_CHECK_HIP(hipMemcpyAsync(d_masks, masks.data(), masks.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                               ctx->st));
  TTN_CHECK_HIP(launch_decode(records, n_rec, d_datarec, n_data, d_masks, n_checks, base, fail_out, ctx->B,
                              ctx->st));
  // the host-side table must outlive the copies
  TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
  return TTN_OK;
}

ttn_status ttn_compress(ttn_ctx* ctx) {
  if (!ctx) return TTN_EINVAL;
  TTN_TRY(flush_leaf(ctx));
  // depth-first tour: every bond is crossed in both directions
  std::vector<int> tour;
  std::vector<std::pair<int, int>> stack{{1, 0}};
  tour.push_back(1);
  while (!stack.empty()) {
    auto& top = stack.back();
    const int node = top.first;
    if (!is_bottom(ctx, node) && top.second < 2) {
      const int child = 2 * node + top.second;
      ++top.second;
      stack.push_back({child, 0});
      tour.push_back(child);
    } else {
      stack.pop_back();
      if (!stack.empty()) tour.push_back(stack.back().first);
    }
  }
  TTN_TRY(move_centre(ctx, 1));
  for (size_t i = 0; i + 1 < tour.size(); ++i) TTN_TRY(hop_truncating(ctx, tour[i], tour[i + 1]));
  return TTN_OK;
}

ttn_status ttn_to_statevector(ttn_ctx* ctx, int32_t row, double* amp) {
  if (!ctx) return TTN_EINVAL;
  if (row < 0 || row >= ctx->B || !amp || ctx->N > 26) return fail(ctx, TTN_EINVAL, "bad row or N > 26");
  TTN_TRY(flush_leaf(ctx));
  TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
  typedef std::complex<double> cd;
  const int L = ctx->L;
  std::vector<std::vector<cd>> T(L);
  for (int node = 1; node < L; ++node) {
    const long long ne = elems(ctx->dims[node]);
    std::vector<cd> h(ne);
    if (ctx->c128) {
      TTN_CHECK_HIP(hipMemcpy(h.data(), (char*)node_ptr(ctx, node) + (size_t)row * ne * 16, ne * 16,
                              hipMemcpyDeviceToHost));
    } else {
      std::vector<std::complex<float>> f(ne);
      TTN_CHECK_HIP(hipMemcpy(f.data(), (char*)node_ptr(ctx, node) + (size_t)row * ne * 8, ne * 8,
                              hipMemcpyDeviceToHost));
      for (long long i = 0; i < ne; ++i) h[i] = cd(f[i].real(), f[i].imag());
    }
    T[node] = std::move(h);
  }
  // bottom-up: v[node] = [2^(qubits below)][u], qubits in leaf order
  std::vector<std::vector<cd>> v(L);
  std::vector<std::vector<int>> qs(L);
  for (int node = L - 1; node >= 1; --node) {
    const auto d = ctx->dims[node];
    if (node >= L / 2) {
      const int l0 = 2 * (node - L / 2);
      const int q0 = ctx->qubit_at_leaf[l0], q1 = ctx->qubit_at_leaf[l0 + 1];
      const int na = q0 >= 0 ? 2 : 1, nb = q1 >= 0 ? 2 : 1;
      std::vector<cd> out((size_t)na * nb * d[2]);
      for (int a = 0; a < na; ++a)
        for (int b = 0; b < nb; ++b)
          for (int u = 0; u < d[2]; ++u) out[((size_t)a * nb + b) * d[2] + u] = T[node][((size_t)a * 2 + b) * d[2] + u];
      v[node] = std::move(out);
      if (q0 >= 0) qs[node].push_back(q0);
      if (q1 >= 0) qs[node].push_back(q1);
    } else {
      const auto& va = v[2 * node];
      const auto& vb = v[2 * node + 1];
      const size_t ra = va.size() / d[0], rb = vb.size() / d[1];
      std::vector<cd> tmp(ra * d[1] * d[2], cd(0, 0));   // sum_i va[x][i] T[i][j][u]
      for (size_t x = 0; x < ra; ++x)
        for (int i = 0; i < d[0]; ++i) {
          const cd a = va[x * d[0] + i];
          if (a == cd(0, 0)) continue;
          for (int j = 0; j < d[1]; ++j)
            for (int u = 0; u < d[2]; ++u) tmp[(x * d[1] + j) * d[2] + u] += a * T[node][((size_t)i * d[1] + j) * d[2] + u];
        }
      std::vector<cd> out(ra * rb * d[2], cd(0, 0));
      for (size_t x = 0; x < ra; ++x)
        for (size_t y = 0; y < rb; ++y)
          for (int j = 0; j < d[1]; ++j) {
            const cd b = vb[y * d[1] + j];
            if (b == cd(0, 0)) continue;
            for (int u = 0; u < d[2]; ++u) out[(x * rb + y) * d[2] + u] += b * tmp[(x * d[1] + j) * d[2] + u];
          }
      v[node] = std::move(out);
      qs[node] = qs[2 * node];
      qs[node].insert(qs[node].end(), qs[2 * node + 1].begin(), qs[2 * node + 1].end());
      v[2 * node].clear();
      v[2 * node + 1].clear();
    }
  }
  const auto& root = v[1];
  const std::vector<int>& order = qs[1];   // qubits in leaf order, first = most significant
  const int N = ctx->N;
  std::vector<double> outh((size_t)2 << N, 0.0);
  for (size_t idx = 0; idx < ((size_t)1 << N); ++idx) {
    // idx in leaf order -> qubit-order index
    size_t qi = 0;
    for (int p = 0; p < N; ++p) {
      const int bit = (idx >> (N - 1 - p)) & 1;
      qi |= (size_t)bit << (N - 1 - order[p]);
    }
    outh[2 * qi] = root[idx].real();
    outh[2 * qi + 1] = root[idx].imag();
  }
  TTN_CHECK_HIP(hipMemcpy(amp, outh.data(), outh.size() * sizeof(double), hipMemcpyHostToDevice));
  return TTN_OK;
}

ttn_status ttn_bond_dims(ttn_ctx* ctx, int32_t row, int32_t* dims) {
  if (!ctx) return TTN_EINVAL;
  if (row < 0 || row >= ctx->B || !dims) return fail(ctx, TTN_EINVAL, "bad row");
  TTN_TRY(flush_leaf(ctx));
  TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
  std::vector<int> r(ctx->L);
  TTN_CHECK_HIP(hipMemcpy(r.data(), ctx->rank_table + (size_t)row * ctx->L, ctx->L * sizeof(int),
                          hipMemcpyDeviceToHost));
  dims[0] = 0;
  dims[1] = 1;
  for (int e = 2; e < ctx->L; ++e) dims[e] = r[e];
  return TTN_OK;
}

ttn_status ttn_autotune(ttn_ctx* ctx, int32_t on, int64_t* shapes, int64_t* changed) {
  if (!ctx) return TTN_EINVAL;
  if (on < -1 || on >= 2 + kZgemmCfgs) return fail(ctx, TTN_EINVAL, "on must be -1, 0, 1 or 2 + a tile shape");
  ctx->force_cfg = on >= 2 ? on - 2 : -1;
  if (on >= 2) {
    ctx->tune_on = 0;
  } else if (on == -1) {
    ctx->tune.clear();
    ctx->tuned_shapes = 0;
    ctx->tuned_changed = 0;
    ctx->tune_on = 0;
  } else {
    ctx->tune_on = on;
  }
  if (shapes) *shapes = ctx->tuned_shapes;
  if (changed) *changed = ctx->tuned_changed;
  return TTN_OK;
}

ttn_status ttn_profile_enable(ttn_ctx* ctx, int32_t on) {
  if (!ctx) return TTN_EINVAL;
  TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
  ctx->prof = on != 0;
  for (auto& e : ctx->prof_ring) e.pending = false;
  for (int c = 0; c < TTN_NCLASS; ++c) {
    ctx->prof_ms[c] = 0.0;
    ctx->prof_n[c] = 0;
  }
  while (ctx->prof && ctx->prof_ring.size() < kProfRing) {
    // timing-only events: no system-scope fence (cache writeback and
    // invalidation) at each record, which would also slow the work it brackets
    ttn_ctx::ProfSlot e{nullptr, nullptr, 0, false};
    TTN_CHECK_HIP(hipEventCreateWithFlags(&e.a, hipEventDisableSystemFence));
    if (hipEventCreateWithFlags(&e.b, hipEventDisableSystemFence) != hipSuccess) {
      hipEventDestroy(e.a);
      return fail(ctx, TTN_EDEVICE, "hipEventCreate failed");
    }
    ctx->prof_ring.push_back(e);
  }
  TTN_CHECK_HIP(launch_fill_f64(ctx->ledger_mem, 0.0, 7ll * ctx->B, ctx->st));
  return TTN_OK;
}

ttn_status ttn_profile_read(ttn_ctx* ctx, int32_t cls, double* ms, int64_t* launches, double* alg_flops,
                            double* alg_bytes) {
  if (!ctx) return TTN_EINVAL;
  if (cls < 0 || cls >= TTN_NCLASS || !ms || !launches || !alg_flops) return fail(ctx, TTN_EINVAL, "bad class");
  TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
  for (auto& e : ctx->prof_ring) TTN_CHECK_HIP(prof_harvest(ctx, e));
  *ms = ctx->prof_ms[cls];
  *launches = ctx->prof_n[cls];
  *alg_flops = 0.0;
  if (ctx->ledger[cls]) {
    std::vector<double> f(ctx->B);
    TTN_CHECK_HIP(hipMemcpy(f.data(), ctx->ledger[cls], ctx->B * sizeof(double), hipMemcpyDeviceToHost));
    for (double v : f) *alg_flops += v;
  }
  if (alg_bytes) {
    *alg_bytes = 0.0;
    if (ctx->ledger_bytes[cls]) {
      std::vector<double> f(ctx->B);
      TTN_CHECK_HIP(hipMemcpy(f.data(), ctx->ledger_bytes[cls], ctx->B * sizeof(double), hipMemcpyDeviceToHost));
      for (double v : f) *alg_bytes += v;
    }
  }
  return TTN_OK;
}

ttn_status ttn_uniforms(ttn_ctx* ctx, uint64_t traj_offset, int32_t rows, int32_t n_draws, double* out) {
  if (!ctx) return TTN_EINVAL;
  if (rows < 0 || n_draws < 0 || !out) return fail(ctx, TTN_EINVAL, "bad arguments");
  TTN_CHECK_HIP(launch_philox_uniforms(ctx->seed, traj_offset, n_draws, out, rows, ctx->st));
  TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
  return TTN_OK;
}

ttn_status ttn_test_leg_apply(ttn_ctx* ctx, int32_t rows, const int32_t* dims3, int32_t leg, const void* T,
                              int64_t t_elems, const void* W, int64_t w_elems, int32_t newd, void* out,
                              int64_t out_elems) {
  if (!ctx) return TTN_EINVAL;
  if (rows < 1 || !dims3 || leg < 0 || leg > 2 || !T || !W || !out || newd < 1)
    return fail(ctx, TTN_EINVAL, "bad arguments");
  std::array<int, 3> d{dims3[0], dims3[1], dims3[2]};
  if (d[0] < 1 || d[1] < 1 || d[2] < 1) return fail(ctx, TTN_EINVAL, "bad dims");
  GemmDesc g = leg_desc(T, d, leg, W, newd, newd, out);
  const bool wA = (leg != 2);
  if (!gemm_fits(g, rows, wA ? w_elems : t_elems, wA ? t_elems : w_elems, out_elems))
    return fail(ctx, TTN_EINVAL, "buffers too small for the contraction");
  TTN_CHECK_HIP(launch_zgemm(g, rows, ctx->c128 ? GEMM_C128 : GEMM_C64, ctx->st, ctx->force_cfg));
  TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
  return TTN_OK;
}

ttn_status ttn_test_move(ttn_ctx* ctx, int32_t rows, int32_t n, int32_t new_pad, int32_t cap, double cutoff,
                         const double* G, int64_t g_elems, void* W_iso, void* W_abs, int64_t w_elems,
                         int32_t* rank, int32_t blocks) {
  if (!ctx) return TTN_EINVAL;
  if (rows < 1 || rows > ctx->B || n < 1 || n / blocks > (blocks == 1 ? 128 : 64) || new_pad < 1 ||
      new_pad > ctx->nmax || cap < 1 || !G || !W_iso || !W_abs || (blocks != 1 && blocks != 2) ||
      (blocks == 1 && !rank) || (blocks == 2 && ((n & 1) || (new_pad & 1))))
    return fail(ctx, TTN_EINVAL,
                "bad arguments (rows <= batch, n <= 128, or <= 64 per block, new_pad <= workspace)");
  if (g_elems < (int64_t)rows * n * n || w_elems < (int64_t)rows * new_pad * n)
    return fail(ctx, TTN_EINVAL, "buffers too small for the factorisation");
  EighDesc ed{};
  ed.G = (const double2*)G; ed.n = n; ed.new_pad = new_pad; ed.cap = cap; ed.cutoff = cutoff;
  ed.W_iso = W_iso; ed.W_abs = W_abs; ed.out_c128 = ctx->c128;
  ed.blocks = blocks;
  ed.rank_out = blocks == 1 ? rank : nullptr; ed.rank_stride = 1;
  const bool tried = blocks == 1 && n > 64;
  if (tried) ed.done = ctx->qr_done;
  TTN_CHECK_HIP(launch_pchol(ed, rows, ctx->st));
  TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
  if (tried) {
    std::vector<int> dn(rows), rk(rows);
    TTN_CHECK_HIP(hipMemcpy(dn.data(), ctx->qr_done, rows * sizeof(int), hipMemcpyDeviceToHost));
    TTN_CHECK_HIP(hipMemcpy(rk.data(), rank, rows * sizeof(int), hipMemcpyDeviceToHost));
    for (int t = 0; t < rows; ++t)
      if (!dn[t]) rk[t] = -1;
    TTN_CHECK_HIP(hipMemcpy(rank, rk.data(), rows * sizeof(int), hipMemcpyHostToDevice));
  }
  return TTN_OK;
}

ttn_status ttn_test_gram(ttn_ctx* ctx, int32_t rows, const int32_t* dims3, int32_t leg, const void* T,
                         int64_t t_elems, double* G, int64_t g_elems, int32_t ksplit) {
  if (!ctx) return TTN_EINVAL;
  if (rows < 1 || !dims3 || leg < 0 || leg > 2 || !T || !G || ksplit < 1 || ksplit > 64)
    return fail(ctx, TTN_EINVAL, "bad arguments");
  std::array<int, 3> d{dims3[0], dims3[1], dims3[2]};
  if (d[0] < 1 || d[1] < 1 || d[2] < 1) return fail(ctx, TTN_EINVAL, "bad dims");
  GemmDesc g = gram_desc(T, d, leg, (double2*)G);
  g.ksplit = ksplit;
  g.sCz = (long long)rows * d[leg] * d[leg];
  if (!gemm_fits(g, rows, t_elems, t_elems, g_elems)) return fail(ctx, TTN_EINVAL, "buffers too small for the Gram");
  TTN_CHECK_HIP(launch_zgemm(g, rows, ctx->c128 ? GEMM_GRAM_C128 : GEMM_GRAM_C64, ctx->st, ctx->force_cfg));
  TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
  return TTN_OK;
}

ttn_status ttn_test_eigh(ttn_ctx* ctx, int32_t rows, int32_t n, int32_t new_pad, int32_t cap, double cutoff,
                         const double* G, int64_t g_elems, void* W_iso, void* W_abs, int64_t w_elems,
                         int32_t* rank, int32_t* sweeps, int32_t blocks) {
  if (!ctx) return TTN_EINVAL;
  if (rows < 1 || rows > ctx->B || n < 1 || n > ctx->nmax || new_pad < 1 || new_pad > ctx->nmax || cap < 1 || !G ||
      !W_iso || !W_abs || (blocks != 1 && blocks != 2) || (blocks == 1 && !rank) ||
      (blocks == 2 && ((n & 1) || (new_pad & 1))))
    return fail(ctx, TTN_EINVAL, "bad arguments (rows <= batch, n and new_pad <= workspace)");
  if (g_elems < (int64_t)rows * n * n || w_elems < (int64_t)rows * new_pad * n)
    return fail(ctx, TTN_EINVAL, "buffers too small for the eigen-decomposition");
  EighDesc ed{};
  ed.G = (const double2*)G; ed.n = n; ed.new_pad = new_pad; ed.cap = cap; ed.cutoff = cutoff;
  ed.W_iso = W_iso; ed.W_abs = W_abs; ed.out_c128 = ctx->c128;
  ed.blocks = blocks;
  ed.sweeps_out = blocks == 1 ? sweeps : nullptr;
  ed.rank_out = blocks == 1 ? rank : nullptr; ed.rank_stride = 1;
  eigh_ws(ctx, ed);
  ed.nk_out = ctx->prof ? ctx->nk : nullptr;
  // the convergence settings of the batch driver's moves
  ed.tol = ctx->c128 ? 1e-15 : 1e-10;
  ed.early_stop = ctx->c128 ? 0 : 1;
  TTN_CHECK_HIP(launch_eigh(ed, rows, ctx->st));
  TTN_CHECK_HIP(hipStreamSynchronize(ctx->st));
  return TTN_OK;
}

}  // extern "C"
