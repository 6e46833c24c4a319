// FP64 Hermitian eigen-decomposition of the per-trajectory bond Gram matrix
// by cyclic two-sided Jacobi, and the factors of the isometry-centre move.
//
// The Gram matrix G = M^H M of the node reshaped with the bond as its column
// index has eigenvalues s_a^2 (the squared singular values of M, i.e. the
// squared Schmidt values when the rest of the network is an isometry) and
// eigenvectors V (the right singular vectors).  The centre moves across the
// bond by M = (M V S^-1) (S V^H): the first factor stays behind as the new
// isometry, the second is absorbed by the neighbour.  Truncation keeps the
// largest s_a with s_a^2 / sum s^2 > cutoff, at most `cap` of them, and
// renormalises the kept part (the paper truncates the smallest Schmidt
// coefficients, Sec. IV.A).
//
// One workgroup per problem.  G lives in LDS as its packed upper triangle
// (<= 132 KB at n = 128).  Each Jacobi step rotates n/2 disjoint index pairs
// chosen by the round-robin (circle) schedule, so every pair is visited once
// per sweep; a step updates every 2 x 2 block (P, Q) of G by J_P^H G_PQ J_Q.
// For n <= 64 the eigenvectors are accumulated in LDS next to G; for larger n
// each step's rotations go to a log that a second kernel replays onto row
// blocks of V.  Problems above 64 whose size is near a power of two use
// another cyclic order instead, the XOR matchings grouped by cosets (below),
// which applies three steps per pass over G.
//
// Block-diagonal mode (blocks = 2): while a controlled gate's index rides on
// a bond, the Gram matrix is block diagonal (the two halves carry orthogonal
// projections of the start qubit), so each diagonal half is solved by its
// own workgroup; cutoff and normalisation refer to the trace of the whole
// matrix, and each workgroup writes its own diagonal block of the factors
// (and zeros in its rows of the other block).
#include <vector>

#include "ttn_device.h"
#include "ttn_kernels.h"

namespace ttn {

constexpr int kMaxSweeps = 24;
constexpr int kVLdsMax = 64;
constexpr int kThreadsSmall = 512;    // n <= 64: G and V in LDS
constexpr int kThreadsLarge = 1024;   // n > 64: G alone fills the LDS, one workgroup per CU
int eigh_max_sweeps() { return kMaxSweeps; }

__device__ inline int pidx(int i, int j, int n) {   // packed upper triangle, i <= j
  // (both factors are below 2^24: the full-rate 24-bit multiply)
  return (int)((unsigned)__umul24((unsigned)i, (unsigned)(2 * n - i + 1)) >> 1) + (j - i);
}
// Problems above 64 whose compacted even size n2 is at least 15/16 of the
// next power of two are solved by coset-grouped sweeps on the padded matrix;
// the others by circle-ordered sweeps on n2 (padding would cost more than the
// grouping saves: at N = 128 the circle order is the faster one up to
// n2 = 116, the coset order from 120).
__device__ inline int padded_pow2(int n) {
  int N = 4;
  while (N < n) N <<= 1;
  return N;
}
__device__ inline bool coset_order(int n) {
  const int n2 = n + (n & 1);
  return n2 > 64 && 16 * n2 >= 15 * padded_pow2(n2);
}

// circle-method pairing for step s of an even size n (no integer division)
__device__ inline void pair_of(int n, int s, int j, int* p, int* q) {
  int a, b;
  if (j == 0) { a = n - 1; b = s; }
  else {
    a = s + j; if (a >= n - 1) a -= n - 1;
    b = s - j; if (b < 0) b += n - 1;
  }
  *p = a < b ? a : b;
  *q = a < b ? b : a;
}

struct Rot { double c; double2 s; double delta; };
// a rotation in tangent form, J = c [[1, t], [-conj(t), 1]] (s = c t), so
// that the two-sided block update needs two fused multiply-adds per real
// component and one scaling by c_P c_Q at the end
struct RotT { double2 t; double c; double delta; };

__device__ inline double2 c_sub_mul_conj(double2 a, double2 b, double2 t) {   // a - b conj(t)
  return make_double2(fma(-b.x, t.x, fma(-b.y, t.y, a.x)), fma(-b.y, t.x, fma(b.x, t.y, a.y)));
}
__device__ inline double2 c_add_mul(double2 a, double2 b, double2 t) {        // a + b t
  return make_double2(fma(b.x, t.x, fma(-b.y, t.y, a.x)), fma(b.x, t.y, fma(b.y, t.x, a.y)));
}
__device__ inline double2 c_sub_mul(double2 a, double2 b, double2 t) {        // a - b t
  return make_double2(fma(-b.x, t.x, fma(b.y, t.y, a.x)), fma(-b.x, t.y, fma(-b.y, t.x, a.y)));
}
__device__ inline double2 c_add_mul_conj(double2 a, double2 b, double2 t) {   // a + b conj(t)
  return make_double2(fma(b.x, t.x, fma(b.y, t.y, a.x)), fma(b.y, t.x, fma(-b.x, t.y, a.y)));
}
// the imaginary part with its sign bit flipped by m (0 or the sign bit)
__device__ inline double2 conj_if(double2 v, unsigned long long m) {
  v.y = __longlong_as_double(__double_as_longlong(v.y) ^ (long long)m);
  return v;
}

// entry o of one row's Gram matrix: the sum of its partial products when the
// Gram launch split its K range
__device__ inline double2 gram_at(const EighDesc& d, const double2* G, long long o) {
  double2 v = G[o];
  for (int z = 1; z < d.gsplit; ++z) v = cadd(v, G[o + z * d.gslice]);
  return v;
}

// entry (r, c) of a row's Hermitian Gram matrix from its upper triangle
// (the Gram launch skips the output tiles wholly below the diagonal)
__device__ inline double2 gram_herm(const EighDesc& d, const double2* G, int r, int c) {
  return r <= c ? gram_at(d, G, (long long)r * d.n + c) : cconj(gram_at(d, G, (long long)c * d.n + r));
}

struct Problem {       // one diagonal block of one trajectory's matrix
  long long t;
  int k;               // block index
  int n;               // block size
  int off;             // row/column offset of the block in G and in W
  int pad;             // rows of W owned by this block
  int pad_off;         // first such row
};

__device__ inline Problem problem_of(const EighDesc& d, long long bid) {
  Problem p;
  const int nb = d.blocks > 1 ? 2 : 1;
  p.t = bid / nb;
  p.k = (int)(bid % nb);
  p.n = d.n / nb;
  p.off = p.k * p.n;
  p.pad = d.new_pad / nb;
  p.pad_off = p.k * p.pad;
  return p;
}

// Rows of a problem's block of G with a non-zero diagonal, in order.  A
// Gram matrix with g_ii = 0 has row and column i exactly zero (padding of a
// bond beyond this trajectory's dimension, or the unused rows of a block),
// so the eigenproblem is solved on the compacted matrix of the m rows kept:
// cidx[c] = original row of compacted index c (c < m), inv[i] = c or -1.
// One original row per thread (pb.n <= blockDim.x); every thread returns m.
template <int NW>
__device__ int compact_rows(const EighDesc& d, const double2* G, const Problem& pb, int* cidx, int* inv,
                            int* wcount) {
  const int i = threadIdx.x, lane = i & 63, wave = i >> 6;
  bool nz = false;
  if (i < pb.n) nz = gram_at(d, G, (long long)(pb.off + i) * d.n + pb.off + i).x > 0.0;
  const unsigned long long mask = __ballot(nz);
  if (lane == 0) wcount[wave] = __popcll(mask);
  __syncthreads();
  int base = 0, m = 0;
  for (int w = 0; w < NW; ++w) {
    if (w < wave) base += wcount[w];
    m += wcount[w];
  }
  if (i < pb.n) {
    const int c = base + __popcll(mask & ((1ull << lane) - 1ull));
    inv[i] = nz ? c : -1;
    if (nz) cidx[c] = i;
  }
  __syncthreads();
  return m;
}

template <typename S, typename VT>
__device__ void write_factors(const EighDesc& d, const Problem& pb, const VT* V /* compacted n2 x n2 */,
                              int n2, const int* inv, const int* order, const double* lam_sorted, int k,
                              double scale_abs) {
  S* Wi = (S*)d.W_iso + pb.t * (long long)d.new_pad * d.n;
  S* Wa = (S*)d.W_abs + pb.t * (long long)d.new_pad * d.n;
  const int nrows = pb.n;
  // own block: rows pad_off .. pad_off + pad, columns off + [0, n); rows of
  // the block outside the compacted problem get zeros
  for (int idx = threadIdx.x; idx < pb.pad * nrows; idx += blockDim.x) {
    const int a = idx / nrows;
    const int i = idx % nrows;
    double2 wi = make_double2(0.0, 0.0), wa = make_double2(0.0, 0.0);
    if (a < k && inv[i] >= 0) {
      const double2 v = to_d2(V[(long long)inv[i] * n2 + order[a]]);
      const double s = sqrt(lam_sorted[a]);
      wi = cscale(v, 1.0 / s);
      wa = cscale(cconj(v), s * scale_abs);
    }
    const long long o = (long long)(pb.pad_off + a) * d.n + pb.off + i;
    Wi[o] = from_d2<S>(wi);
    Wa[o] = from_d2<S>(wa);
  }
  if (d.blocks > 1) {
    // zeros of my rows in the other block's columns
    const int other = (1 - pb.k) * pb.n;
    for (int idx = threadIdx.x; idx < pb.pad * nrows; idx += blockDim.x) {
      const int a = idx / nrows;
      const int i = idx % nrows;
      const long long o = (long long)(pb.pad_off + a) * d.n + other + i;
      Wi[o] = from_d2<S>(make_double2(0.0, 0.0));
      Wa[o] = from_d2<S>(make_double2(0.0, 0.0));
    }
  }
}

// Convergence.  A pair is rotated while |g_pq| > tol sqrt(g_pp g_qq) (and
// above 0.1 tol of the trace).  After each sweep the whole matrix is
// checked: the solver stops when no off-diagonal entry passes that test (the
// next sweep would rotate nothing), or, with early_stop, when none reaches
// sqrt(tol) / 4 of sqrt(g_pp g_qq) (cyclic Jacobi converges quadratically,
// so the next sweep would typically leave nothing above tol; complex64 runs
// only).  The check reads the matrix, not the ratios met at the rotations:
// a rotation between nearly equal diagonal entries turns by up to 45 degrees
// however small its own entry, and can carry large entries past the pairs
// the sweep has already visited.
// VT: element type of the eigenvector matrix kept in LDS (kVinLds).  Runs
// whose factors are complex64 accumulate it in complex64, which halves its
// LDS footprint so that two problems share a CU.
// NMAX: largest problem size; above 128 the packed G (526 KB at 256) lives in
// device memory (d.gpk) instead of LDS.
template <bool kVinLds, int NT, typename VT, int NMAX>
__global__ void __launch_bounds__(NT) k_jacobi(EighDesc d) {
  extern __shared__ double2 smem[];
  const long long pid = blockIdx.x;                    // problem: a row, or (row, block)
  if (!kVinLds && d.done && d.done[pid]) return;       // factored by the pivoted Cholesky
  const Problem pb = problem_of(d, pid);
  const long long t = pb.t;
  const double2* G = d.G + t * (long long)d.n * d.n;
  __shared__ int cidx[NMAX];
  __shared__ int inv[NMAX];
  __shared__ int wcount[NT / 64];
  const int n = compact_rows<NT / 64>(d, G, pb, cidx, inv, wcount);   // compacted size
  if (!kVinLds && coset_order(n)) return;        // solved by k_jacobi_coset
  const int n2 = n + (n & 1);          // even size, a zero dummy index if odd
  const int h = n2 / 2;
  const int npk = n2 * (n2 + 1) / 2;
  const int nblk = h * (h - 1) / 2;
  constexpr bool kGlobalG = NMAX > 128;
  double2* Gp = kGlobalG ? d.gpk + pid * (long long)(NMAX * (NMAX + 1) / 2) : smem;   // packed G
  VT* V = reinterpret_cast<VT*>(smem + npk);           // [n2][n2] if kVinLds
  __shared__ RotT rot[NMAX / 2];
  __shared__ int pq_s[NMAX / 2];                                    // this step's pairs, p | q << 16
  // this step's pairs in bytes: {16 p, 16 q, 16 rowbase(p), 16 rowbase(q)};
  // entry (i, j), i <= j, of the packed triangle is element rowbase(i) + j
  __shared__ int4 pinfo[NMAX / 2];
  __shared__ unsigned short blk[(NMAX / 2) * (NMAX / 2 - 1) / 2];   // (P, Q), P < Q: off-diagonal 2x2 blocks
  __shared__ double lam[NMAX];
  __shared__ int order_s[NMAX];
  __shared__ double red[NT];
  __shared__ double trace_s;

  for (int idx = threadIdx.x; idx < npk; idx += blockDim.x) {
    int i = 0, rem = idx;
    while (rem >= n2 - i) { rem -= n2 - i; ++i; }
    const int j = i + rem;
    Gp[idx] = (i < n && j < n) ? gram_at(d, G, (long long)(pb.off + cidx[i]) * d.n + pb.off + cidx[j])
                               : make_double2(0.0, 0.0);
  }
  for (int idx = threadIdx.x; idx < nblk; idx += blockDim.x) {
    int P = 0, rem = idx;
    while (rem >= h - 1 - P) { rem -= h - 1 - P; ++P; }
    blk[idx] = (unsigned short)(P | ((P + 1 + rem) << 8));
  }
  if (kVinLds)
    for (int idx = threadIdx.x; idx < n2 * n2; idx += blockDim.x)
      V[idx] = from_d2<VT>(make_double2((idx / n2 == idx % n2) ? 1.0 : 0.0, 0.0));
  // trace of the whole matrix (both blocks in block-diagonal mode)
  double part = 0.0;
  for (int i = threadIdx.x; i < d.n; i += blockDim.x) part += gram_at(d, G, (long long)i * d.n + i).x;
  red[threadIdx.x] = part;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) trace_s = red[0];
  __syncthreads();
  const double tr = trace_s;
  const bool finite = isfinite(tr) && tr > 0.0;

  int step_count = 0, sweeps_done = 0;
  double* log = d.rot_log ? d.rot_log + pid * d.log_stride : nullptr;
  const double tol = d.tol > 0.0 ? d.tol : 1e-15;
  const double stop_ratio = d.early_stop ? 0.25 * sqrt(tol) : 0.0;
  const double stop_ratio2 = stop_ratio * stop_ratio;
  const double floor2 = (0.1 * tol * tr) * (0.1 * tol * tr);
  if (n2 >= 2 && finite) {
    const int vgroups = NT / h;                 // V update: row groups of h threads
    const int vP = threadIdx.x % h, vr0 = threadIdx.x / h;
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
      for (int s = 0; s < n2 - 1; ++s) {
        // -- rotation parameters of the n2/2 pairs (the tests on squares,
        //    one reciprocal square root for |b| and one for c: the serial
        //    part of every step) --
        if (threadIdx.x < h) {
          int p, q;
          pair_of(n2, s, threadIdx.x, &p, &q);
          pq_s[threadIdx.x] = p | (q << 16);
          const int rbp = pidx(p, p, n2) - p, rbq = pidx(q, q, n2) - q;
          pinfo[threadIdx.x] = make_int4(16 * p, 16 * q, 16 * rbp, 16 * rbq);
          const double a = Gp[rbp + p].x, dd = Gp[rbq + q].x;
          const double2 b = Gp[rbp + q];
          const double ab2 = cabs2(b);
          const double ad = fabs(a * dd);
          RotT r;
          r.c = 1.0; r.t = make_double2(0.0, 0.0); r.delta = 0.0;
          if (ab2 > tol * tol * ad && ab2 > floor2 && ab2 > 0.0) {
            const double inv_ab = rsqrt(ab2);
            const double th = 0.5 * (dd - a) * inv_ab;
            const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            const double tn = tt * inv_ab;
            r.c = rsqrt(1.0 + tt * tt);
            r.t = make_double2(tn * b.x, tn * b.y);
            r.delta = tt * (ab2 * inv_ab);
            // the pair's own 2x2 diagonal block (no other block of this
            // step touches these three entries)
            Gp[rbp + p] = make_double2(a - r.delta, 0.0);
            Gp[rbq + q] = make_double2(dd + r.delta, 0.0);
            Gp[rbp + q] = make_double2(0.0, 0.0);
          }
          rot[threadIdx.x] = r;
          if (!kVinLds && log) {
            double* e = log + ((long long)step_count * h + threadIdx.x) * 3;
            e[0] = r.c; e[1] = r.c * r.t.x; e[2] = r.c * r.t.y;
          }
        }
        __syncthreads();
        // -- G <- J^H G J on the off-diagonal blocks --
        const char* Gb = reinterpret_cast<const char*>(Gp);
        for (int idx = threadIdx.x; idx < nblk; idx += blockDim.x) {
          const unsigned short pq = blk[idx];
          const int P = pq & 0xff, Q = pq >> 8;
          const RotT rP = rot[P], rQ = rot[Q];
          if (rP.delta == 0.0 && rQ.delta == 0.0) continue;
          const int4 eP = pinfo[P], eQ = pinfo[Q];
          // entry (i, j) of the block: byte offset of its upper-triangle
          // slot, and the sign mask that conjugates a lower-triangle entry
          const bool u00 = eP.x <= eQ.x, u01 = eP.x <= eQ.y, u10 = eP.y <= eQ.x, u11 = eP.y <= eQ.y;
          const int o00 = u00 ? eP.z + eQ.x : eQ.z + eP.x;
          const int o01 = u01 ? eP.z + eQ.y : eQ.w + eP.x;
          const int o10 = u10 ? eP.w + eQ.x : eQ.z + eP.y;
          const int o11 = u11 ? eP.w + eQ.y : eQ.w + eP.y;
          constexpr unsigned long long kSign = 0x8000000000000000ull;
          const unsigned long long m00 = u00 ? 0ull : kSign, m01 = u01 ? 0ull : kSign;
          const unsigned long long m10 = u10 ? 0ull : kSign, m11 = u11 ? 0ull : kSign;
          const double2 g00 = conj_if(*reinterpret_cast<const double2*>(Gb + o00), m00);
          const double2 g01 = conj_if(*reinterpret_cast<const double2*>(Gb + o01), m01);
          const double2 g10 = conj_if(*reinterpret_cast<const double2*>(Gb + o10), m10);
          const double2 g11 = conj_if(*reinterpret_cast<const double2*>(Gb + o11), m11);
          // X = G_PQ J_Q, J = [[c, s], [-conj(s), c]], s = c t; then
          // Y = J_P^H X (the products with c and s as written: the
          // tangent form with one c_P c_Q scaling at the end changes the
          // rounding enough to move stabilizer-state records off their
          // exact values in complex64 runs)
          const double2 sQ = cscale(rQ.t, rQ.c), sP = cscale(rP.t, rP.c);
          const double2 sQc = cconj(sQ), sPc = cconj(sP);
          const double2 x00 = csub(cscale(g00, rQ.c), cmul(g01, sQc));
          const double2 x01 = cadd(cmul(g00, sQ), cscale(g01, rQ.c));
          const double2 x10 = csub(cscale(g10, rQ.c), cmul(g11, sQc));
          const double2 x11 = cadd(cmul(g10, sQ), cscale(g11, rQ.c));
          const double2 y00 = csub(cscale(x00, rP.c), cmul(sP, x10));
          const double2 y01 = csub(cscale(x01, rP.c), cmul(sP, x11));
          const double2 y10 = cadd(cmul(sPc, x00), cscale(x10, rP.c));
          const double2 y11 = cadd(cmul(sPc, x01), cscale(x11, rP.c));
          char* Gw = reinterpret_cast<char*>(Gp);
          *reinterpret_cast<double2*>(Gw + o00) = conj_if(y00, m00);
          *reinterpret_cast<double2*>(Gw + o01) = conj_if(y01, m01);
          *reinterpret_cast<double2*>(Gw + o10) = conj_if(y10, m10);
          *reinterpret_cast<double2*>(Gw + o11) = conj_if(y11, m11);
        }
        if (kVinLds) {
          // V <- V J (columns p, q of every row): thread owns pair vP on
          // the rows vr0, vr0 + vgroups, ...
          if (threadIdx.x < vgroups * h) {
            const RotT rP = rot[vP];
            if (rP.delta != 0.0) {
              const int eP = pq_s[vP];
              const int p = eP & 0xffff, q = eP >> 16;
              for (int r = vr0; r < n2; r += vgroups) {
                const double2 vp = to_d2(V[r * n2 + p]), vq = to_d2(V[r * n2 + q]);
                V[r * n2 + p] = from_d2<VT>(cscale(c_sub_mul_conj(vp, vq, rP.t), rP.c));
                V[r * n2 + q] = from_d2<VT>(cscale(c_add_mul(vq, vp, rP.t), rP.c));
              }
            }
          }
        }
        ++step_count;
        __syncthreads();
      }
      ++sweeps_done;
      // converged: no off-diagonal entry left that passes the rotation test
      // and reaches the stop ratio
      int big = 0;
      for (int e = threadIdx.x; e < n2 * n2; e += blockDim.x) {
        const int i = e / n2, j = e - (e / n2) * n2;
        if (j <= i) continue;
        const int rbi = pidx(i, i, n2) - i;
        const double ad = fabs(Gp[rbi + i].x * Gp[pidx(j, j, n2)].x);
        const double ab2 = cabs2(Gp[rbi + j]);
        if (ab2 > tol * tol * ad && ab2 > floor2 && ab2 > 0.0 && ab2 >= stop_ratio2 * ad) big = 1;
      }
      if (!__syncthreads_or(big)) break;
    }
  }
  // -- eigenvalues, descending order, truncation --
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double l = Gp[pidx(i, i, n2)].x;
    lam[i] = (isfinite(l) && l > 0.0) ? l : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    int rk = 0;
    const double li = lam[i];
    for (int j = 0; j < n; ++j) rk += (lam[j] > li) || (lam[j] == li && j < i);
    order_s[rk] = i;
  }
  __syncthreads();
  __shared__ int k_s;
  __shared__ double scale_s;
  if (threadIdx.x == 0) {
    double mine = 0.0;
    for (int i = 0; i < n; ++i) mine += lam[i];
    const double tot = d.blocks > 1 ? tr : mine;
    int k = 0;
    double kept = 0.0;
    const int lim = min(min(d.cap, pb.pad), n);
    if (finite && tot > 0.0) {
      while (k < lim && lam[order_s[k]] > d.cutoff * tot) { kept += lam[order_s[k]]; ++k; }
    }
    if (d.blocks > 1) {
      // the joint state is normalised by the whole trace (the tiny dropped
      // parts are renormalised by the truncating sweep that follows)
      scale_s = finite ? 1.0 / sqrt(tr) : 0.0;
      if (!finite && d.flags) atomicOr(d.flags + t, 1);
      if (d.disc_acc && tot > 0.0) atomicAdd(d.disc_acc + t, (mine - kept) / tot);
    } else {
      if (!(kept > 0.0) || !isfinite(kept)) {
        k = 0;
        if (d.flags) d.flags[t] |= 1;
        scale_s = 0.0;
      } else {
        scale_s = 1.0 / sqrt(kept);
      }
      if (d.disc_acc && tot > 0.0) d.disc_acc[t] += (tot - kept) / tot;
      if (d.degen_acc && k > 0 && k < n) {
        const double lk1 = lam[order_s[k - 1]], lk = lam[order_s[k]];
        if (lk > d.cutoff * tot && lk1 - lk <= 1e-6 * lk1) d.degen_acc[t] += 1;
      }
      if (d.rank_out) d.rank_out[t * d.rank_stride] = k;
      if (d.rank_max) d.rank_max[t * d.rank_stride] = max(d.rank_max[t * d.rank_stride], k);
    }
    if (d.flops_acc || d.nk_out) {
      // algorithmic work of an n x n complex Hermitian eigen-decomposition
      // with vectors: 36 n^3 real flops (9 n^3 for the real symmetric case,
      // Golub & Van Loan, times 4 for complex arithmetic), n = the number of
      // non-zero eigenvalues (the actual bond dimension)
      int na = 0;
      for (int i = 0; i < n; ++i) na += lam[i] > 1e-15 * tot;
      const double f = 36.0 * (double)na * na * na;
      if (d.flops_acc) {
        if (d.blocks > 1) atomicAdd(d.flops_acc + t, f);
        else d.flops_acc[t] += f;
      }
      if (d.nk_out) {
        d.nk_out[t * 4 + 2 * pb.k] = na;
        d.nk_out[t * 4 + 2 * pb.k + 1] = k;
        if (d.blocks <= 1) { d.nk_out[t * 4 + 2] = 0; d.nk_out[t * 4 + 3] = 0; }
      }
    }
    k_s = k;
    if (d.sweeps_out) d.sweeps_out[t] = sweeps_done;
    if (!kVinLds) {
      d.kept[pid] = k;
      d.scale_abs[pid] = scale_s;
      d.nsteps[pid] = step_count;
    }
  }
  __syncthreads();
  if (kVinLds) {
    __shared__ double lam_sorted[NMAX];
    for (int a = threadIdx.x; a < n; a += blockDim.x) lam_sorted[a] = lam[order_s[a]];
    __syncthreads();
    if (d.out_c128)
      write_factors<double2>(d, pb, V, n2, inv, order_s, lam_sorted, k_s, scale_s);
    else
      write_factors<float2>(d, pb, V, n2, inv, order_s, lam_sorted, k_s, scale_s);
  } else {
    // (per problem pb.n slots; the compacted problem uses the first n)
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
      d.order[pid * pb.n + a] = order_s[a];
      d.lam_sorted[pid * pb.n + a] = lam[order_s[a]];
    }
  }
}

// ---------------------------------------------------------------------------
// Problems above 64 whose compacted size is near a power of two (see
// coset_order): coset-grouped sweeps.
//
// The compacted matrix is padded with zero rows to N = 2^k (zero rows never
// rotate).  A sweep is the N - 1 matchings M_d = {(i, i ^ d) : i < i ^ d},
// d = 1 .. N - 1, which together visit every pair once, taken in groups of
// up to three from one subgroup H = {0, a, b, a ^ b} of (Z_2)^k: {a, b,
// a ^ b}, {a, b} or {a}.  Every matching of a group maps each coset {r, r ^ a,
// r ^ b, r ^ a ^ b} of H onto itself, so the group's rotations act inside
// 4 x 4 blocks: two lanes per coset compute them on its diagonal block in
// registers (one matching after another, as cyclic Jacobi does; each lane
// one of the matching's two disjoint rotations), and then every off-diagonal
// block (Q, R) gets U_Q^H G_QR U_R with one read and one write of G per group
// instead of one per matching.
// ---------------------------------------------------------------------------
constexpr int kPlanMaxK = 8;                  // N <= 256
struct SweepPlan {
  int ngroups[kPlanMaxK + 1];
  unsigned grp[kPlanMaxK + 1][256];           // a | b << 8 | m << 16 (m matchings: a, b, a ^ b)
  unsigned char dseq[kPlanMaxK + 1][256];     // the matchings of one sweep in order
};
__constant__ SweepPlan c_plan;

__device__ inline int hibit(int x) { return 31 - __clz(x); }
// x with a zero bit inserted at position b
__device__ inline int insert_zero(int x, int b) { return ((x >> b) << (b + 1)) | (x & ((1 << b) - 1)); }
// pair index of (i, i ^ d), i < i ^ d, within matching d: i without bit hibit(d)
__device__ inline int pair_index(int i, int hb) { return ((i >> (hb + 1)) << hb) | (i & ((1 << hb) - 1)); }

// rotation of the pair (p, q), p < q, with g_pp = a, g_qq = dd, g_pq = b
// (the tests of the circle-ordered solver).  With w = dd - a and
// D = |w| + sqrt(w^2 + 4 |b|^2): t = 2 sign(w) b / D (the smaller-angle
// root), delta = 2 sign(w) |b|^2 / D, and c = (1 + |t|^2)^-1/2;
// one square root, one reciprocal (refined twice by Newton's iteration, D
// >= |w| > 0) and one reciprocal square root.  ic = 1 / c.
__device__ __forceinline__ RotT jacobi_rot(double a, double dd, double2 b, double tol, double floor2,
                                  double stop_ratio2, bool* rotated, bool* big, double* ic) {
  RotT r;
  r.c = 1.0; r.t = make_double2(0.0, 0.0); r.delta = 0.0;
  *ic = 1.0;
  const double ab2 = cabs2(b);
  const double ad = fabs(a * dd);
  *rotated = false; *big = false;
  if (ab2 > tol * tol * ad && ab2 > floor2 && ab2 > 0.0) {
    *big = ab2 >= stop_ratio2 * ad;
    const double w = dd - a;
    const double D = fabs(w) + sqrt(fma(w, w, 4.0 * ab2));
    double y = __builtin_amdgcn_rcp(D);
    y = fma(y, fma(-D, y, 1.0), y);
    y = fma(y, fma(-D, y, 1.0), y);
    const double g = (w >= 0.0 ? 2.0 : -2.0) * y;
    r.t = make_double2(g * b.x, g * b.y);
    r.delta = g * ab2;
    const double x = fma(4.0 * ab2, y * y, 1.0);     // 1 + |t|^2
    r.c = rsqrt(x);
    *ic = x * r.c;
    *rotated = true;
  }
  return r;
}

// slots of the two pairs of matching J of a coset (r, r ^ a, r ^ b, r ^ a ^ b):
// a: (0, 1), (2, 3); b: (0, 2), (1, 3); a ^ b: (0, 3), (1, 2)
template <int J> struct CosetPairs {
  static constexpr int s00 = 0, s01 = J == 0 ? 1 : (J == 1 ? 2 : 3);
  static constexpr int s10 = J == 0 ? 2 : 1, s11 = J == 2 ? 2 : 3;
};
template <int S> __device__ inline int comp(const int4& v) {
  return S == 0 ? v.x : (S == 1 ? v.y : (S == 2 ? v.z : v.w));
}

struct RotCtl { double tol, floor2, stop_ratio2; };

// The rotation of one pair of a coset's diagonal block (entries a = B_00,
// dd = B_11, b = B_01 in slot order, slot indices i0, i1), computed in slot
// order: the same rotation as in index order, relabelled (t -> -conj(t),
// delta -> -delta when the first slot holds the larger index).  Its log entry
// is written in index order.
__device__ __forceinline__ RotT coset_rot(double a, double dd, double2 b, int i0, int i1, int hb,
                                          const RotCtl& rc, double* e, bool* rotated, bool* big, double* ic) {
  bool bg;
  const RotT r = jacobi_rot(a, dd, b, rc.tol, rc.floor2, rc.stop_ratio2, rotated, &bg, ic);
  *big |= bg;
  e += (long long)pair_index(min(i0, i1), hb) * 3;
  const double tx = i0 < i1 ? r.t.x : -r.t.x;
  e[0] = r.c; e[1] = r.c * tx; e[2] = r.c * r.t.y;
  return r;
}

// Coefficients of one rotation for the off-diagonal blocks.  Rows (and
// columns) of a coset carry pending scales sigma (products of the c's of the
// group's earlier rotations), so a rotation of slots (S0, S1) becomes
// X0 <- X0 - alpha X1, X1 <- X1 + beta X0 with alpha = t sigma1 / sigma0,
// beta = conj(t) sigma0 / sigma1 (and the conjugate coefficients on the
// column side), and the scales multiply by c; every entry is scaled once,
// after the group.
struct RotAB { double2 alpha, beta; };

// Matching J of a group on a coset's diagonal block B (members v), worked by
// two lanes that both hold B: lane ln computes the rotation of pair ln (its
// log entry and off-diagonal coefficients), the lanes swap them, and both
// rotate the cross block between the pairs from both sides, set each pair's
// own 2 x 2 block to its exact diagonal form and advance the pending scales
// sig (and their inverses isig).  Returns whether a pair rotated.
template <int J>
__device__ __forceinline__ bool coset_matching(double2 (&B)[4][4], double (&sig)[4], double (&isig)[4],
                                               const int4& v, int dm, int ln, const RotCtl& rc, double* log_step,
                                               RotAB (&rec)[2], bool* big) {
  using S = CosetPairs<J>;
  constexpr int a0 = S::s00, a1 = S::s01, b0 = S::s10, b1 = S::s11;
  const bool hi = ln != 0;
  bool rot;
  double ic;
  const RotT r = coset_rot(hi ? B[b0][b0].x : B[a0][a0].x, hi ? B[b1][b1].x : B[a1][a1].x,
                           hi ? B[b0][b1] : B[a0][a1], hi ? comp<b0>(v) : comp<a0>(v),
                           hi ? comp<b1>(v) : comp<a1>(v), hibit(dm), rc, log_step, &rot, big, &ic);
  {
    const double s0 = hi ? sig[b0] : sig[a0], s1 = hi ? sig[b1] : sig[a1];
    const double is0 = hi ? isig[b0] : isig[a0], is1 = hi ? isig[b1] : isig[a1];
    RotAB ab;
    ab.alpha = cscale(r.t, s1 * is0);
    ab.beta = cscale(cconj(r.t), s0 * is1);
    rec[ln] = ab;
  }
  RotT ro;
  ro.t = make_double2(__shfl_xor(r.t.x, 1), __shfl_xor(r.t.y, 1));
  ro.c = __shfl_xor(r.c, 1);
  ro.delta = __shfl_xor(r.delta, 1);
  const double ico = __shfl_xor(ic, 1);
  const bool roto = __shfl_xor((int)rot, 1) != 0;
  const RotT r0 = hi ? ro : r, r1 = hi ? r : ro;
  const bool rot0 = hi ? roto : rot, rot1 = hi ? rot : roto;
  const double ic0 = hi ? ico : ic, ic1 = hi ? ic : ico;
  sig[a0] *= r0.c; sig[a1] *= r0.c; sig[b0] *= r1.c; sig[b1] *= r1.c;
  isig[a0] *= ic0; isig[a1] *= ic0; isig[b0] *= ic1; isig[b1] *= ic1;
  if (!rot0 && !rot1) return false;
  // cross block C = B[{a0, a1}][{b0, b1}] <- J0^H C J1
  double2 c00 = B[a0][b0], c01 = B[a0][b1], c10 = B[a1][b0], c11 = B[a1][b1];
  {
    const double2 x00 = c_sub_mul(c00, c10, r0.t), x10 = c_add_mul_conj(c10, c00, r0.t);
    const double2 x01 = c_sub_mul(c01, c11, r0.t), x11 = c_add_mul_conj(c11, c01, r0.t);
    const double cc = r0.c * r1.c;
    c00 = cscale(c_sub_mul_conj(x00, x01, r1.t), cc);
    c01 = cscale(c_add_mul(x01, x00, r1.t), cc);
    c10 = cscale(c_sub_mul_conj(x10, x11, r1.t), cc);
    c11 = cscale(c_add_mul(x11, x10, r1.t), cc);
  }
  B[a0][b0] = c00; B[a0][b1] = c01; B[a1][b0] = c10; B[a1][b1] = c11;
  B[b0][a0] = cconj(c00); B[b1][a0] = cconj(c01); B[b0][a1] = cconj(c10); B[b1][a1] = cconj(c11);
  if (rot0) {
    B[a0][a0].x -= r0.delta; B[a1][a1].x += r0.delta;
    B[a0][a1] = make_double2(0.0, 0.0); B[a1][a0] = make_double2(0.0, 0.0);
  }
  if (rot1) {
    B[b0][b0].x -= r1.delta; B[b1][b1].x += r1.delta;
    B[b0][b1] = make_double2(0.0, 0.0); B[b1][b0] = make_double2(0.0, 0.0);
  }
  return true;
}

// matching J on an off-diagonal block: rows by coset Q's coefficients (from
// the left), columns by coset R's (from the right, conjugated)
template <int S0, int S1>
__device__ __forceinline__ void ab_rows(double2 (&X)[4][4], const RotAB& r) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const double2 x0 = X[S0][u], x1 = X[S1][u];
    X[S0][u] = c_sub_mul(x0, x1, r.alpha);
    X[S1][u] = c_add_mul(x1, x0, r.beta);
  }
}
template <int S0, int S1>
__device__ __forceinline__ void ab_cols(double2 (&X)[4][4], const RotAB& r) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double2 x0 = X[s][S0], x1 = X[s][S1];
    X[s][S0] = c_sub_mul_conj(x0, x1, r.alpha);
    X[s][S1] = c_add_mul_conj(x1, x0, r.beta);
  }
}
template <int J>
__device__ __forceinline__ void coset_block(double2 (&X)[4][4], const RotAB (&a)[2], const RotAB (&b)[2]) {
  using S = CosetPairs<J>;
  ab_rows<S::s00, S::s01>(X, a[0]);
  ab_rows<S::s10, S::s11>(X, a[1]);
  ab_cols<S::s00, S::s01>(X, b[0]);
  ab_cols<S::s10, S::s11>(X, b[1]);
}

// byte offset of entry (i, j) (byte indices 16 i, 16 j; packed row bases
// rbi, rbj in bytes) and the mask that conjugates a lower-triangle entry
__device__ inline int coset_off(int i16, int rbi, int j16, int rbj) { return i16 < j16 ? rbi + j16 : rbj + i16; }
__device__ inline unsigned long long coset_msk(int i16, int j16) {
  return i16 < j16 ? 0ull : 0x8000000000000000ull;
}

constexpr int kThreadsCoset = 512;
template <int NMAX>
__global__ void __launch_bounds__(kThreadsCoset) k_jacobi_coset(EighDesc d) {
  constexpr int NT = kThreadsCoset;
  constexpr int NQ = NMAX / 4;
  extern __shared__ double2 smem[];
  const long long pid = blockIdx.x;
  if (d.done && d.done[pid]) return;                   // factored by the pivoted Cholesky
  const Problem pb = problem_of(d, pid);
  const long long t = pb.t;
  const double2* G = d.G + t * (long long)d.n * d.n;
  __shared__ int cidx[NMAX];
  __shared__ int inv[NMAX];
  __shared__ int wcount[NT / 64];
  const int n = compact_rows<NT / 64>(d, G, pb, cidx, inv, wcount);
  if (!coset_order(n)) return;              // solved by the circle-ordered k_jacobi
  int kk = 2;
  while ((1 << kk) < n) ++kk;
  const int N = 1 << kk;
  const int npk = N * (N + 1) / 2;
  const int nq = N / 4;
  const int nblk = nq * (nq - 1) / 2;
  constexpr bool kGlobalG = NMAX > 128;
  double2* Gp = kGlobalG ? d.gpk + pid * (long long)(NMAX * (NMAX + 1) / 2) : smem;
  __shared__ RotAB rq[NQ][3][2];            // this group's off-diagonal coefficients: coset, matching, pair
  __shared__ double4 qsig[NQ];              // the cosets' scales after the group
  __shared__ int4 qm[NQ];                   // coset members r, r ^ a, r ^ b, r ^ a ^ b, in bytes (16 i)
  __shared__ int4 qrb[NQ];                  // their packed row bases, in bytes
  __shared__ int qact[NQ];                  // the coset rotated in this group
  __shared__ unsigned short blk[NQ * (NQ - 1) / 2];
  __shared__ double lam[NMAX];
  __shared__ int order_s[NMAX];
  __shared__ double wsum[NT / 64];
  __shared__ double trace_s;

  for (int idx = threadIdx.x; idx < npk; idx += NT) {
    int i = 0, rem = idx;
    while (rem >= N - i) { rem -= N - i; ++i; }
    const int j = i + rem;
    Gp[idx] = (i < n && j < n) ? gram_at(d, G, (long long)(pb.off + cidx[i]) * d.n + pb.off + cidx[j])
                               : make_double2(0.0, 0.0);
  }
  for (int idx = threadIdx.x; idx < nblk; idx += NT) {
    int Q = 0, rem = idx;
    while (rem >= nq - 1 - Q) { rem -= nq - 1 - Q; ++Q; }
    blk[idx] = (unsigned short)(Q | ((Q + 1 + rem) << 8));
  }
  // trace of the whole matrix (both blocks in block-diagonal mode)
  {
    double part = 0.0;
    for (int i = threadIdx.x; i < d.n; i += NT) part += gram_at(d, G, (long long)i * d.n + i).x;
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += wsum[w];
      trace_s = s;
    }
    __syncthreads();
  }
  const double tr = trace_s;
  const bool finite = isfinite(tr) && tr > 0.0;

  int step_count = 0, sweeps_done = 0;
  double* log = d.rot_log + pid * d.log_stride;
  const int hN = N / 2;
  const double tol = d.tol > 0.0 ? d.tol : 1e-15;
  const double stop_ratio = d.early_stop ? 0.25 * sqrt(tol) : 0.0;
  const double stop_ratio2 = stop_ratio * stop_ratio;
  const double floor2 = (0.1 * tol * tr) * (0.1 * tol * tr);
  const int ngroups = c_plan.ngroups[kk];
  const char* Gb = reinterpret_cast<const char*>(Gp);
  char* Gw = reinterpret_cast<char*>(Gp);
  constexpr unsigned long long kSign = 0x8000000000000000ull;
  if (n >= 2 && finite) {
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
      bool my_big = false;       // (the rotations' own stop-ratio flags; convergence is checked below)
      for (int g = 0; g < ngroups; ++g) {
        const unsigned gi = c_plan.grp[kk][g];
        const int ga = gi & 0xff, gbv = (gi >> 8) & 0xff, m = (int)(gi >> 16);
        // -- each coset's diagonal block: the group's rotations one matching
        //    after another, in registers --
        //    (two lanes per coset, lane ln working pair ln of each matching)
        if (threadIdx.x < 2 * nq) {
          const int Q = threadIdx.x >> 1, ln = threadIdx.x & 1;
          int e1 = ga, e2 = gbv;
          if (hibit(e2) == hibit(e1)) e2 ^= e1;
          const int h1 = hibit(e1), h2 = hibit(e2);
          const int lo = min(h1, h2), hi = max(h1, h2);
          const int r0 = insert_zero(insert_zero(Q, lo), hi);
          const int4 v = make_int4(r0, r0 ^ ga, r0 ^ gbv, r0 ^ ga ^ gbv);
          const int4 v16 = make_int4(16 * v.x, 16 * v.y, 16 * v.z, 16 * v.w);
          const int4 rb16 = make_int4(16 * (pidx(v.x, v.x, N) - v.x), 16 * (pidx(v.y, v.y, N) - v.y),
                                      16 * (pidx(v.z, v.z, N) - v.z), 16 * (pidx(v.w, v.w, N) - v.w));
          double2 B[4][4];
#define COSET_LD(S, U, CS, CU)                                                                       \
  B[S][U] = conj_if(*reinterpret_cast<const double2*>(Gb + coset_off(v16.CS, rb16.CS, v16.CU, rb16.CU)), \
                    coset_msk(v16.CS, v16.CU));                                                        \
  B[U][S] = cconj(B[S][U]);
          B[0][0] = make_double2(reinterpret_cast<const double2*>(Gb + rb16.x + v16.x)->x, 0.0);
          B[1][1] = make_double2(reinterpret_cast<const double2*>(Gb + rb16.y + v16.y)->x, 0.0);
          B[2][2] = make_double2(reinterpret_cast<const double2*>(Gb + rb16.z + v16.z)->x, 0.0);
          B[3][3] = make_double2(reinterpret_cast<const double2*>(Gb + rb16.w + v16.w)->x, 0.0);
          COSET_LD(0, 1, x, y) COSET_LD(0, 2, x, z) COSET_LD(0, 3, x, w)
          COSET_LD(1, 2, y, z) COSET_LD(1, 3, y, w) COSET_LD(2, 3, z, w)
#undef COSET_LD
          const RotCtl rc{tol, floor2, stop_ratio2};
          double* lg = log + (long long)step_count * hN * 3;
          double sig[4] = {1.0, 1.0, 1.0, 1.0}, isig[4] = {1.0, 1.0, 1.0, 1.0};
          bool act = coset_matching<0>(B, sig, isig, v, ga, ln, rc, lg, rq[Q][0], &my_big);
          if (m > 1) act |= coset_matching<1>(B, sig, isig, v, gbv, ln, rc, lg + hN * 3, rq[Q][1], &my_big);
          if (m > 2)
            act |= coset_matching<2>(B, sig, isig, v, ga ^ gbv, ln, rc, lg + 2 * hN * 3, rq[Q][2], &my_big);
          if (act) {
            // (both lanes hold the same block; each stores half of it)
#define COSET_ST(S, U, CS, CU)                                                                       \
  *reinterpret_cast<double2*>(Gw + coset_off(v16.CS, rb16.CS, v16.CU, rb16.CU)) =                       \
      conj_if(B[S][U], coset_msk(v16.CS, v16.CU));
            if (ln == 0) {
              *reinterpret_cast<double2*>(Gw + rb16.x + v16.x) = B[0][0];
              *reinterpret_cast<double2*>(Gw + rb16.y + v16.y) = B[1][1];
              COSET_ST(0, 1, x, y) COSET_ST(0, 2, x, z) COSET_ST(0, 3, x, w)
            } else {
              *reinterpret_cast<double2*>(Gw + rb16.z + v16.z) = B[2][2];
              *reinterpret_cast<double2*>(Gw + rb16.w + v16.w) = B[3][3];
              COSET_ST(1, 2, y, z) COSET_ST(1, 3, y, w) COSET_ST(2, 3, z, w)
            }
#undef COSET_ST
          }
          if (ln == 0) {
            qsig[Q] = make_double4(sig[0], sig[1], sig[2], sig[3]);
            qact[Q] = act;
            qm[Q] = v16;
            qrb[Q] = rb16;
          }
        }
        __syncthreads();
        // -- off-diagonal blocks: G_QR <- U_Q^H G_QR U_R --
        for (int idx = threadIdx.x; idx < nblk; idx += NT) {
          const unsigned short qr = blk[idx];
          const int Q = qr & 0xff, R = qr >> 8;
          if (!qact[Q] && !qact[R]) continue;
          const int4 mq = qm[Q], bq = qrb[Q], mr = qm[R], br = qrb[R];
          double2 X[4][4];
#define COSET_LD(S, U, CS, CU)                                                                       \
  X[S][U] = conj_if(*reinterpret_cast<const double2*>(Gb + coset_off(mq.CS, bq.CS, mr.CU, br.CU)),     \
                    coset_msk(mq.CS, mr.CU));
#define COSET_ROW(S, CS) COSET_LD(S, 0, CS, x) COSET_LD(S, 1, CS, y) COSET_LD(S, 2, CS, z) COSET_LD(S, 3, CS, w)
          COSET_ROW(0, x) COSET_ROW(1, y) COSET_ROW(2, z) COSET_ROW(3, w)
#undef COSET_ROW
#undef COSET_LD
          coset_block<0>(X, rq[Q][0], rq[R][0]);
          if (m > 1) coset_block<1>(X, rq[Q][1], rq[R][1]);
          if (m > 2) coset_block<2>(X, rq[Q][2], rq[R][2]);
          const double4 sq = qsig[Q], sr = qsig[R];
#define COSET_ST(S, U, CS, CU)                                                                       \
  *reinterpret_cast<double2*>(Gw + coset_off(mq.CS, bq.CS, mr.CU, br.CU)) =                             \
      conj_if(cscale(X[S][U], sq.CS * sr.CU), coset_msk(mq.CS, mr.CU));
#define COSET_ROW(S, CS) COSET_ST(S, 0, CS, x) COSET_ST(S, 1, CS, y) COSET_ST(S, 2, CS, z) COSET_ST(S, 3, CS, w)
          COSET_ROW(0, x) COSET_ROW(1, y) COSET_ROW(2, z) COSET_ROW(3, w)
#undef COSET_ROW
#undef COSET_ST
        }
        step_count += m;
        __syncthreads();
      }
      ++sweeps_done;
      // converged: no off-diagonal entry left that passes the rotation test
      // and reaches the stop ratio
      int big = 0;
      for (int e = threadIdx.x; e < N * N; e += NT) {
        const int i = e >> kk, j = e & (N - 1);
        if (j <= i) continue;
        const int rbi = pidx(i, i, N) - i;
        const double ad = fabs(Gp[rbi + i].x * Gp[pidx(j, j, N)].x);
        const double ab2 = cabs2(Gp[rbi + j]);
        if (ab2 > tol * tol * ad && ab2 > floor2 && ab2 > 0.0 && ab2 >= stop_ratio2 * ad) big = 1;
      }
      if (!__syncthreads_or(big)) break;
    }
  }
  // -- eigenvalues, descending order, truncation --
  for (int i = threadIdx.x; i < n; i += NT) {
    const double l = Gp[pidx(i, i, N)].x;
    lam[i] = (isfinite(l) && l > 0.0) ? l : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += NT) {
    int rk = 0;
    const double li = lam[i];
    for (int j = 0; j < n; ++j) rk += (lam[j] > li) || (lam[j] == li && j < i);
    order_s[rk] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mine = 0.0;
    for (int i = 0; i < n; ++i) mine += lam[i];
    const double tot = d.blocks > 1 ? tr : mine;
    int k = 0;
    double kept = 0.0;
    const int lim = min(min(d.cap, pb.pad), n);
    if (finite && tot > 0.0) {
      while (k < lim && lam[order_s[k]] > d.cutoff * tot) { kept += lam[order_s[k]]; ++k; }
    }
    double scale = 0.0;
    if (d.blocks > 1) {
      scale = finite ? 1.0 / sqrt(tr) : 0.0;
      if (!finite && d.flags) atomicOr(d.flags + t, 1);
      if (d.disc_acc && tot > 0.0) atomicAdd(d.disc_acc + t, (mine - kept) / tot);
    } else {
      if (!(kept > 0.0) || !isfinite(kept)) {
        k = 0;
        if (d.flags) d.flags[t] |= 1;
      } else {
        scale = 1.0 / sqrt(kept);
      }
      if (d.disc_acc && tot > 0.0) d.disc_acc[t] += (tot - kept) / tot;
      if (d.degen_acc && k > 0 && k < n) {
        const double lk1 = lam[order_s[k - 1]], lk = lam[order_s[k]];
        if (lk > d.cutoff * tot && lk1 - lk <= 1e-6 * lk1) d.degen_acc[t] += 1;
      }
      if (d.rank_out) d.rank_out[t * d.rank_stride] = k;
      if (d.rank_max) d.rank_max[t * d.rank_stride] = max(d.rank_max[t * d.rank_stride], k);
    }
    if (d.flops_acc || d.nk_out) {
      // algorithmic work of an n x n complex Hermitian eigen-decomposition
      // with vectors: 36 n^3 real flops, n = the number of non-zero
      // eigenvalues (the actual bond dimension)
      int na = 0;
      for (int i = 0; i < n; ++i) na += lam[i] > 1e-15 * tot;
      const double f = 36.0 * (double)na * na * na;
      if (d.flops_acc) {
        if (d.blocks > 1) atomicAdd(d.flops_acc + t, f);
        else d.flops_acc[t] += f;
      }
      if (d.nk_out) {
        d.nk_out[t * 4 + 2 * pb.k] = na;
        d.nk_out[t * 4 + 2 * pb.k + 1] = k;
        if (d.blocks <= 1) { d.nk_out[t * 4 + 2] = 0; d.nk_out[t * 4 + 3] = 0; }
      }
    }
    if (d.sweeps_out) d.sweeps_out[t] = sweeps_done;
    d.kept[pid] = k;
    d.scale_abs[pid] = scale;
    d.nsteps[pid] = step_count;
  }
  for (int a = threadIdx.x; a < n; a += NT) {
    d.order[pid * pb.n + a] = order_s[a];
    d.lam_sorted[pid * pb.n + a] = lam[order_s[a]];
  }
}

// Kept eigenvectors of a problem of size > 64 from the rotation log of its
// solver (coset-grouped or circle-ordered).  V = J_1 J_2 ... J_S, so column c of V is
// J_1 (J_2 (... (J_S e_c))): the log is replayed in reverse on the unit
// vectors of the kept columns only.  Columns are independent, so each
// wavefront owns a few of them in LDS and runs through the log with no
// workgroup barrier; lane j applies the rotations of pairs j and j + 64 of
// every matching (disjoint index pairs).  One workgroup per problem (a row,
// or one diagonal block of a row).
constexpr int kVecCols = 4;     // columns per wave and pass
template <int NMAX>
__global__ void __launch_bounds__(1024) k_jacobi_vectors(EighDesc d) {
  constexpr int W = NMAX > 128 ? 8 : 16;       // waves: W * 4 columns of NMAX entries in 128 KB
  __shared__ double2 X[W][kVecCols][NMAX];
  __shared__ int order_s[NMAX];
  __shared__ double lam_s[NMAX];
  const long long pid = blockIdx.x;
  if (d.done && d.done[pid]) return;                   // factored by the pivoted Cholesky
  const Problem pb = problem_of(d, pid);
  const long long t = pb.t;
  // the same compaction as the solver's (G is unchanged)
  __shared__ int cidx[NMAX];
  __shared__ int inv[NMAX];
  __shared__ int wcount[W];
  const int n = compact_rows<W>(d, d.G + t * (long long)d.n * d.n, pb, cidx, inv, wcount);
  const bool cos = coset_order(n);
  int kk = 2;
  while ((1 << kk) < n) ++kk;
  const int N = cos ? 1 << kk : n + (n & 1);   // the solver's size
  const int h = N / 2;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;   // launched with W waves
  const int k = d.kept[pid];
  for (int a = threadIdx.x; a < n; a += W * 64) {
    order_s[a] = d.order[pid * pb.n + a];
    lam_s[a] = d.lam_sorted[pid * pb.n + a];
  }
  // the sweep's matchings in LDS: a per-step read from memory would wait
  // for the log entries prefetched for the next step as well
  __shared__ unsigned char dseq_s[256];
  if (cos)
    for (int i = threadIdx.x; i < N - 1; i += W * 64) dseq_s[i] = c_plan.dseq[kk][i];
  __syncthreads();
  const int steps = d.nsteps[pid];
  const double* log = d.rot_log + pid * d.log_stride;
  const double sc = d.scale_abs[pid];
  const bool c128 = d.out_c128 != 0;
  const int per_pass = W * kVecCols;
  for (int base = 0; base < pb.pad; base += per_pass) {
    int ncol = 0;
    for (int cc = 0; cc < kVecCols; ++cc) {
      const int a = base + wave + cc * W;
      if (a < k) ncol = cc + 1;
      for (int i = lane; i < N; i += 64)
        X[wave][cc][i] = make_double2((a < k && i == order_s[a]) ? 1.0 : 0.0, 0.0);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    if (ncol > 0) {
      // lane owns pairs P = lane + 64 j; the log entries of the next
      // (earlier) step are loaded while this step's rotations run
      constexpr int NPL = NMAX / 128;
      double nc[NPL], ns0[NPL], ns1[NPL];
      bool nok[NPL];
      // (unconditional loads from a clamped, valid entry, so that the wait
      // for them can sit in the next step)
      auto fetch = [&](int st) {
#pragma unroll
        for (int j = 0; j < NPL; ++j) {
          const int P = lane + 64 * j;
          nok[j] = P < h && st >= 0;
          const double* e = log + ((long long)(st < 0 ? 0 : st) * h + (P < h ? P : h - 1)) * 3;
          nc[j] = e[0]; ns0[j] = e[1]; ns1[j] = e[2];
        }
      };
      fetch(steps - 1);
      int s = (steps - 1) % (N - 1);            // position in the sweep
      for (int st = steps - 1; st >= 0; --st) {
        double cc_[NPL], s0_[NPL], s1_[NPL];
        bool ok_[NPL];
#pragma unroll
        for (int j = 0; j < NPL; ++j) { cc_[j] = nc[j]; s0_[j] = ns0[j]; s1_[j] = ns1[j]; ok_[j] = nok[j]; }
        fetch(st - 1);
        const int dm = cos ? dseq_s[s] : 1, hb = hibit(dm);
#pragma unroll
        for (int j = 0; j < NPL; ++j) {
          const int P = lane + 64 * j;
          const double c = cc_[j];
          const double2 sv = make_double2(s0_[j], s1_[j]);
          if (ok_[j] && !(c == 1.0 && sv.x == 0.0 && sv.y == 0.0)) {
            int p, q;
            if (cos) { p = insert_zero(P, hb); q = p ^ dm; }
            else pair_of(N, s, P, &p, &q);
            for (int cc = 0; cc < ncol; ++cc) {
              const double2 xp = X[wave][cc][p], xq = X[wave][cc][q];
              X[wave][cc][p] = cadd(cscale(xp, c), cmul(sv, xq));
              X[wave][cc][q] = csub(cscale(xq, c), cmul(cconj(sv), xp));
            }
          }
        }
        // the next (earlier) step touches entries other lanes just wrote
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        s = (s == 0) ? N - 2 : s - 1;
      }
    }
    __syncthreads();
    // rows pad_off + a of W: W_iso[a][off + i] = V[i][order a] / s_a,
    // W_abs[a][off + i] = conj(V[i][order a]) s_a scale; zeros in the other
    // block's columns
    const int rows = min(per_pass, pb.pad - base);
    const int ncols = d.blocks > 1 ? 2 * pb.n : pb.n;
    for (int idx = threadIdx.x; idx < rows * ncols; idx += W * 64) {
      const int al = idx / ncols, ic = idx - (idx / ncols) * ncols;
      const int a = base + al;
      const bool own = ic < pb.n;
      const int i = own ? ic : ic - pb.n;
      double2 wi = make_double2(0.0, 0.0), wa = make_double2(0.0, 0.0);
      if (own && a < k && inv[i] >= 0) {
        const double2 v = X[al % W][al / W][inv[i]];
        const double sv = sqrt(lam_s[a]);
        wi = cscale(v, 1.0 / sv);
        wa = cscale(cconj(v), sv * sc);
      }
      const int col = own ? pb.off + i : (1 - pb.k) * pb.n + i;
      const long long o = t * (long long)d.new_pad * d.n + (long long)(pb.pad_off + a) * d.n + col;
      if (c128) {
        ((double2*)d.W_iso)[o] = wi;
        ((double2*)d.W_abs)[o] = wa;
      } else {
        ((float2*)d.W_iso)[o] = from_d2<float2>(wi);
        ((float2*)d.W_abs)[o] = from_d2<float2>(wa);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Small problems (n <= 16): one wavefront per matrix, the full matrix and V
// in LDS, several matrices per workgroup.  Every step's 2 x 2 blocks (P, Q)
// over all P, Q partition the matrix, so the lanes update disjoint entries;
// a wavefront's LDS operations complete in order, so consecutive steps need
// no workgroup barrier.
template <int NMAX>
__global__ void __launch_bounds__(256) k_jacobi_wave(EighDesc d, long long nprob) {
  constexpr int PER = 4;                       // wavefronts (matrices) per workgroup
  __shared__ double2 Gs[PER][NMAX * NMAX];
  __shared__ double2 Vs[PER][NMAX * NMAX];
  __shared__ Rot rots[PER][NMAX / 2 > 0 ? NMAX / 2 : 1];
  __shared__ double lam_s[PER][NMAX];
  __shared__ int order_s[PER][NMAX];
  __shared__ int cidx_s[PER][NMAX];
  __shared__ int inv_s[PER][NMAX];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long bid = (long long)blockIdx.x * PER + wave;
  if (bid >= nprob) return;                    // whole wavefront leaves; no workgroup barriers below
  const Problem pb = problem_of(d, bid);
  const long long t = pb.t;
  const double2* Gg = d.G + t * (long long)d.n * d.n;
  // compaction to the rows with a non-zero diagonal (as compact_rows)
  int* cidx = cidx_s[wave];
  int* inv = inv_s[wave];
  const bool nz = lane < pb.n && gram_at(d, Gg, (long long)(pb.off + lane) * d.n + pb.off + lane).x > 0.0;
  const unsigned long long mask = __ballot(nz);
  const int n = __popcll(mask);
  if (lane < pb.n) {
    const int c = __popcll(mask & ((1ull << lane) - 1ull));
    inv[lane] = nz ? c : -1;
    if (nz) cidx[c] = lane;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int n2 = n + (n & 1);
  const int h = n2 / 2;
  double2* G = Gs[wave];
  double2* V = Vs[wave];
  for (int idx = lane; idx < n2 * n2; idx += 64) {
    const int i = idx / n2, j = idx - (idx / n2) * n2;
    G[idx] = (i < n && j < n) ? gram_herm(d, Gg, pb.off + cidx[i], pb.off + cidx[j])
                              : make_double2(0.0, 0.0);
    V[idx] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  double part = 0.0;
  for (int i = lane; i < d.n; i += 64) part += gram_at(d, Gg, (long long)i * d.n + i).x;
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
  const double tr = part;
  const bool finite = isfinite(tr) && tr > 0.0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  int sweeps_done = 0;
  const double tol = d.tol > 0.0 ? d.tol : 1e-15;
  const double stop_ratio = d.early_stop ? 0.25 * sqrt(tol) : 0.0;
  if (n2 >= 2 && finite) {
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
      for (int s = 0; s < n2 - 1; ++s) {
        if (lane < h) {
          int p, q;
          pair_of(n2, s, lane, &p, &q);
          const double a = G[p * n2 + p].x, dd = G[q * n2 + q].x;
          const double2 b = G[p * n2 + q];
          const double ab = sqrt(cabs2(b));
          Rot r;
          r.c = 1.0; r.s = make_double2(0.0, 0.0); r.delta = 0.0;
          if (ab > tol * sqrt(fabs(a * dd)) && ab > 0.1 * tol * tr && ab > 0.0) {
            const double th = (dd - a) / (2.0 * ab);
            const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            const double c = 1.0 / sqrt(1.0 + tt * tt);
            const double sn = tt * c;
            r.c = c;
            r.s = make_double2(sn * b.x / ab, sn * b.y / ab);
            r.delta = tt * ab;
          }
          rots[wave][lane] = r;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // G <- J^H G J over every 2x2 block (P, Q)
        for (int idx = lane; idx < h * h; idx += 64) {
          const int P = idx / h, Q = idx - (idx / h) * h;
          const Rot rP = rots[wave][P], rQ = rots[wave][Q];
          if (rP.delta == 0.0 && rQ.delta == 0.0) continue;
          int p, q, pp, qq;
          pair_of(n2, s, P, &p, &q);
          pair_of(n2, s, Q, &pp, &qq);
          if (P == Q) {
            G[p * n2 + p] = make_double2(G[p * n2 + p].x - rP.delta, 0.0);
            G[q * n2 + q] = make_double2(G[q * n2 + q].x + rP.delta, 0.0);
            G[p * n2 + q] = make_double2(0.0, 0.0);
            G[q * n2 + p] = make_double2(0.0, 0.0);
            continue;
          }
          const double2 g00 = G[p * n2 + pp], g01 = G[p * n2 + qq];
          const double2 g10 = G[q * n2 + pp], g11 = G[q * n2 + qq];
          const double2 sQc = cconj(rQ.s);
          const double2 x00 = csub(cscale(g00, rQ.c), cmul(g01, sQc));
          const double2 x01 = cadd(cmul(g00, rQ.s), cscale(g01, rQ.c));
          const double2 x10 = csub(cscale(g10, rQ.c), cmul(g11, sQc));
          const double2 x11 = cadd(cmul(g10, rQ.s), cscale(g11, rQ.c));
          const double2 sPc = cconj(rP.s);
          G[p * n2 + pp] = csub(cscale(x00, rP.c), cmul(rP.s, x10));
          G[p * n2 + qq] = csub(cscale(x01, rP.c), cmul(rP.s, x11));
          G[q * n2 + pp] = cadd(cmul(sPc, x00), cscale(x10, rP.c));
          G[q * n2 + qq] = cadd(cmul(sPc, x01), cscale(x11, rP.c));
        }
        // V <- V J
        for (int idx = lane; idx < n2 * h; idx += 64) {
          const int r = idx / h, P = idx - (idx / h) * h;
          const Rot rP = rots[wave][P];
          if (rP.delta == 0.0) continue;
          int p, q;
          pair_of(n2, s, P, &p, &q);
          const double2 vp = V[r * n2 + p], vq = V[r * n2 + q];
          V[r * n2 + p] = csub(cscale(vp, rP.c), cmul(cconj(rP.s), vq));
          V[r * n2 + q] = cadd(cmul(rP.s, vp), cscale(vq, rP.c));
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
      ++sweeps_done;
      // converged: no off-diagonal entry left that passes the rotation test
      // and reaches the stop ratio
      bool big = false;
      for (int idx = lane; idx < n2 * n2; idx += 64) {
        const int i = idx / n2, j = idx - (idx / n2) * n2;
        if (j <= i) continue;
        const double ad = fabs(G[i * n2 + i].x * G[j * n2 + j].x);
        const double ab = sqrt(cabs2(G[idx]));
        if (ab > tol * sqrt(ad) && ab > 0.1 * tol * tr && ab > 0.0 && ab >= stop_ratio * sqrt(ad)) big = true;
      }
      if (!__any(big)) break;
    }
  }
  // eigenvalues, descending order, truncation
  for (int i = lane; i < n; i += 64) {
    const double l = G[i * n2 + i].x;
    lam_s[wave][i] = (isfinite(l) && l > 0.0) ? l : 0.0;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int i = lane; i < n; i += 64) {
    int rk = 0;
    const double li = lam_s[wave][i];
    for (int j = 0; j < n; ++j) rk += (lam_s[wave][j] > li) || (lam_s[wave][j] == li && j < i);
    order_s[wave][rk] = i;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  double mine = 0.0;
  for (int i = 0; i < n; ++i) mine += lam_s[wave][i];
  const double tot = d.blocks > 1 ? tr : mine;
  int k = 0;
  double kept = 0.0;
  const int lim = min(min(d.cap, pb.pad), n);
  if (finite && tot > 0.0)
    while (k < lim && lam_s[wave][order_s[wave][k]] > d.cutoff * tot) { kept += lam_s[wave][order_s[wave][k]]; ++k; }
  double scale;
  if (d.blocks > 1) {
    scale = finite ? 1.0 / sqrt(tr) : 0.0;
  } else if (!(kept > 0.0) || !isfinite(kept)) {
    k = 0;
    scale = 0.0;
  } else {
    scale = 1.0 / sqrt(kept);
  }
  if (lane == 0) {
    if (d.blocks > 1) {
      if (!finite && d.flags) atomicOr(d.flags + t, 1);
      if (d.disc_acc && tot > 0.0) atomicAdd(d.disc_acc + t, (mine - kept) / tot);
    } else {
      if (k == 0 && d.flags) d.flags[t] |= 1;
      if (d.disc_acc && tot > 0.0) d.disc_acc[t] += (tot - kept) / tot;
      if (d.degen_acc && k > 0 && k < n) {
        const double lk1 = lam_s[wave][order_s[wave][k - 1]], lk = lam_s[wave][order_s[wave][k]];
        if (lk > d.cutoff * tot && lk1 - lk <= 1e-6 * lk1) d.degen_acc[t] += 1;
      }
      if (d.rank_out) d.rank_out[t * d.rank_stride] = k;
      if (d.rank_max) d.rank_max[t * d.rank_stride] = max(d.rank_max[t * d.rank_stride], k);
    }
    if (d.flops_acc || d.nk_out) {
      int na = 0;
      for (int i = 0; i < n; ++i) na += lam_s[wave][i] > 1e-15 * tot;
      const double f = 36.0 * (double)na * na * na;
      if (d.flops_acc) {
        if (d.blocks > 1) atomicAdd(d.flops_acc + t, f);
        else d.flops_acc[t] += f;
      }
      if (d.nk_out) {
        d.nk_out[t * 4 + 2 * pb.k] = na;
        d.nk_out[t * 4 + 2 * pb.k + 1] = k;
        if (d.blocks <= 1) { d.nk_out[t * 4 + 2] = 0; d.nk_out[t * 4 + 3] = 0; }
      }
    }
    if (d.sweeps_out) d.sweeps_out[t] = sweeps_done;
  }
  // factors: own block rows, and zeros in the other block's columns
  const int ncols = d.n;
  const int nr = pb.n;
  for (int idx = lane; idx < pb.pad * nr; idx += 64) {
    const int a = idx / nr, i = idx - (idx / nr) * nr;
    double2 wi = make_double2(0.0, 0.0), wa = make_double2(0.0, 0.0);
    if (a < k && inv[i] >= 0) {
      const double2 v = V[inv[i] * n2 + order_s[wave][a]];
      const double sv = sqrt(lam_s[wave][order_s[wave][a]]);
      wi = cscale(v, 1.0 / sv);
      wa = cscale(cconj(v), sv * scale);
    }
    const long long o = t * (long long)d.new_pad * ncols + (long long)(pb.pad_off + a) * ncols + pb.off + i;
    if (d.out_c128) { ((double2*)d.W_iso)[o] = wi; ((double2*)d.W_abs)[o] = wa; }
    else { ((float2*)d.W_iso)[o] = from_d2<float2>(wi); ((float2*)d.W_abs)[o] = from_d2<float2>(wa); }
    if (d.blocks > 1) {
      const long long o2 = t * (long long)d.new_pad * ncols + (long long)(pb.pad_off + a) * ncols +
                           (1 - pb.k) * pb.n + i;
      if (d.out_c128) { ((double2*)d.W_iso)[o2] = make_double2(0, 0); ((double2*)d.W_abs)[o2] = make_double2(0, 0); }
      else { ((float2*)d.W_iso)[o2] = make_float2(0, 0); ((float2*)d.W_abs)[o2] = make_float2(0, 0); }
    }
  }
}

// ---------------------------------------------------------------------------
// Exact centre moves by a pivoted Cholesky factorisation of the Gram matrix
// (the QR factorisation M P = Q R of the node reshaped with the bond as its
// column, computed through G = M^H M = P R^H R P^T): rank revealing (the
// pivoting stops once the largest remaining diagonal entry falls to
// cutoff x trace), no truncation otherwise.  The factors are
//   W_iso = P_kept R11^-1   (x <- x W_iso = Q, an isometry)
//   W_abs = R P^T           (y absorbs R)
// in the same [new_pad][n] row layout as the eigensolver's, rows >= rank
// zero.  For moves that keep every value above the cutoff (the forward
// moves of a controlled gate, plain moves of the centre); truncation to chi
// stays with the eigensolver.  One workgroup of NW waves per problem (a
// row, or one diagonal block of a row) of size n <= NMAX (16, 32 or 64 by
// the uncompacted size, with one, two or four waves).
//
// The columns z_a of W_iso come out of the same right-looking sweep: with
// y_j = e_j - sum_{c<k} R[c][j] z_c for each remaining column j, the pivot p
// of step k gives z_k = y_p / R_kk, and every remaining y_j loses
// R[k][j] z_k.  y_j lives on the columns pivoted so far, where row j of the
// residual is zero, so each row of A holds the residual on the remaining
// columns and y_j on the pivoted ones, and one update per row and step
// serves both.  After step k, row p holds R[k][c] on the columns pivoted at
// step k or later (R_kk on the diagonal) and z_k[c] on those pivoted before.
//
// Lane j of every wave holds column j.  Each step costs one barrier: every
// wave keeps the residual diagonal in a register and picks the pivot itself
// (a wave maximum of a 32-bit key), reads the pivot row and updates its own
// share of the remaining rows (i = wave mod NW), in one batch of independent LDS
// accesses; the pivot row's final values are written by the wave owning that
// row at the next step, when no wave reads it any more.
__device__ inline unsigned wave_max_u32(unsigned v) {
  // quad_perm(1,0,3,2), quad_perm(2,3,0,1), row_half_mirror, row_mirror:
  // the maximum over each row of 16 lanes, then over the four rows
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)v, 0), b = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)v, 32), e = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  return max(max(a, b), max(c, e));
}
__device__ inline double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ inline double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

template <int NMAX, int NW>
__global__ void __launch_bounds__(64 * NW) k_pchol(EighDesc d) {
  static_assert(NMAX <= 64 && NMAX % NW == 0 && (NW == 1 || NW == 2 || NW == 4 || NW == 8), "one lane per column");
  constexpr int LD = NMAX + 1;
  constexpr int RPW = NMAX / NW;          // rows per wave
  constexpr unsigned long long kRows = NW == 8 ? 0x0101010101010101ull : NW == 4 ? 0x1111111111111111ull
                                     : NW == 2 ? 0x5555555555555555ull : ~0ull;
  __shared__ double2 A[NMAX * LD];
  __shared__ int cidx[64], inv[64], wcount[NW];
  __shared__ int pos[NMAX], order[NMAX];
  __shared__ double red[2][NW];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // (uniform: scalar row bookkeeping)
  const long long pid = blockIdx.x;
  const Problem pb = problem_of(d, pid);
  const long long t = pb.t;
  const double2* G = d.G + t * (long long)d.n * d.n;
  // (compaction: one original row per thread, pb.n <= 64 * NW; the
  // launcher picks NMAX >= pb.n)
  const int n = compact_rows<NW>(d, G, pb, cidx, inv, wcount);
  for (int i = wave; i < n; i += NW)
    if (lane < n) A[i * LD + lane] = gram_herm(d, G, pb.off + cidx[i], pb.off + cidx[lane]);
  if (threadIdx.x < NMAX) pos[threadIdx.x] = -1;
  // trace of the whole matrix (both blocks), and of this problem
  double part = 0.0, own = 0.0;
  for (int i = threadIdx.x; i < d.n; i += blockDim.x) part += gram_at(d, G, (long long)i * d.n + i).x;
  if (threadIdx.x < n) own = gram_at(d, G, (long long)(pb.off + cidx[threadIdx.x]) * d.n + pb.off + cidx[threadIdx.x]).x;
  part = wave_sum_d(part);
  own = wave_sum_d(own);
  if (lane == 0) { red[0][wave] = part; red[1][wave] = own; }
  __syncthreads();
  double tr = 0.0, mine = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) { tr += red[0][w]; mine += red[1][w]; }
  const bool finite = isfinite(tr) && tr > 0.0;
  const double tot = d.blocks > 1 ? tr : mine;
  const double tol = d.cutoff * tot;
  const int lim = min(min(d.cap, pb.pad), n);
  const unsigned long long live = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
  const bool in = lane < n;
  double dj = in ? A[lane * LD + lane].x : 0.0;         // residual diagonal (every wave alike)
  unsigned long long piv = 0;                           // pivoted columns
  double2 prow = make_double2(0.0, 0.0);                // final values of the last pivot row
  int pprev = -1;
  int k = 0;
  if (finite) {
    for (; k < lim; ++k) {
      if (pprev >= 0 && pprev % NW == wave && in) A[pprev * LD + lane] = prow;
      // pivot: the largest remaining diagonal entry (a float key with the
      // lowest index winning near-ties; 0: no column left)
      const bool before = (piv >> lane) & 1ull;         // pivoted at an earlier step
      unsigned key = 0;
      if (in && !before) key = ((__float_as_uint((float)fmax(dj, 0.0)) + 64u) & ~63u) | (unsigned)(63 - lane);
      key = wave_max_u32(key);
      if (key == 0u) break;
      const int p = 63 - (int)(key & 63u);
      const double dm = readlane_d(dj, p);
      if (!(dm > tol) || !isfinite(dm)) break;          // (uniform: every wave alike)
      const double rkk = sqrt(dm);
      const double irkk = 1.0 / rkk;
      piv |= 1ull << p;
      const bool colj = in && !((piv >> lane) & 1ull); // still unpivoted after this step
      const double2 arow = A[p * LD + lane];
      // u = row k of R on the remaining columns; z = z_k on the pivoted ones
      const double2 u = colj ? cscale(arow, irkk) : make_double2(0.0, 0.0);
      const double2 z = before ? cscale(arow, irkk) : make_double2(lane == p ? irkk : 0.0, 0.0);
      const double2 w = colj ? u : z;
      if (colj) dj = fma(-u.x, u.x, fma(-u.y, u.y, dj));
      // each remaining row j: A_jc -= conj(u_j) u_c (remaining c), y_j -= u_j z_k
      unsigned long long rows = live & ~piv & (kRows << wave);
      int ii[RPW];
#pragma unroll
      for (int q = 0; q < RPW; ++q) {
        ii[q] = rows ? __builtin_ctzll(rows) : -1;
        rows &= rows - 1ull;
      }
      double2 v[RPW];
#pragma unroll
      for (int q = 0; q < RPW; ++q)
        if (ii[q] >= 0) v[q] = A[ii[q] * LD + lane];
#pragma unroll
      for (int q = 0; q < RPW; ++q)
        if (ii[q] >= 0) {
          // u_j from the pivot row as loaded (a cross-lane read of a value
          // that no per-lane condition defines)
          const double ujx = readlane_d(arow.x, ii[q]) * irkk;
          const double ujy0 = readlane_d(arow.y, ii[q]) * irkk;
          const double ujy = colj ? -ujy0 : ujy0;        // conj on the residual
          double2 o = lane == p ? make_double2(0.0, 0.0) : v[q];
          o.x = fma(-ujx, w.x, fma(ujy, w.y, o.x));
          o.y = fma(-ujx, w.y, fma(-ujy, w.x, o.y));
          if (in) A[ii[q] * LD + lane] = o;
        }
      if (threadIdx.x == 0) {
        order[k] = p;
        pos[p] = k;
      }
      prow = colj ? u : (lane == p ? make_double2(rkk, 0.0) : z);
      pprev = p;
      __syncthreads();
    }
  }
  if (pprev >= 0 && pprev % NW == wave && in) A[pprev * LD + lane] = prow;
  const int r = k;
  // kept weight, normalisation, counts
  const double resid = wave_sum_d((in && !((piv >> lane) & 1ull)) ? fmax(dj, 0.0) : 0.0);
  const double kept = fmax(mine - resid, 0.0);
  double scale;
  int kk = r;
  if (d.blocks > 1) {
    scale = finite ? 1.0 / sqrt(tr) : 0.0;
  } else if (!(kept > 0.0) || !isfinite(kept) || r == 0) {
    kk = 0;
    scale = 0.0;
  } else {
    scale = 1.0 / sqrt(kept);
  }
  if (threadIdx.x == 0) {
    if (d.blocks > 1) {
      if (!finite && d.flags) atomicOr(d.flags + t, 1);
      if (d.disc_acc && tot > 0.0) atomicAdd(d.disc_acc + t, (mine - kept) / tot);
    } else {
      if (kk == 0 && d.flags) d.flags[t] |= 1;
      if (d.disc_acc && tot > 0.0) d.disc_acc[t] += (tot - kept) / tot;
      if (d.rank_out) d.rank_out[t * d.rank_stride] = kk;
      if (d.rank_max) d.rank_max[t * d.rank_stride] = max(d.rank_max[t * d.rank_stride], kk);
    }
    if (d.flops_acc) {
      // algorithmic work: complex Cholesky r^2 (3n - 2r) / 3 + triangular
      // inverse r^3 / 3 multiply-adds, 8 real flops each
      const double f = 8.0 * ((double)r * r * (3.0 * n - 2.0 * r) / 3.0 + (double)r * r * r / 3.0);
      if (d.blocks > 1) atomicAdd(d.flops_acc + t, f);
      else d.flops_acc[t] += f;
    }
    if (d.nk_out) {
      d.nk_out[t * 4 + 2 * pb.k] = r;
      d.nk_out[t * 4 + 2 * pb.k + 1] = kk;
      if (d.blocks <= 1) { d.nk_out[t * 4 + 2] = 0; d.nk_out[t * 4 + 3] = 0; }
    }
    if (d.sweeps_out) d.sweeps_out[t] = 0;
  }
  __syncthreads();
  // factors: own block rows pad_off + a, columns off + i; zeros in the other
  // block's columns
  const long long base = t * (long long)d.new_pad * d.n;
  const int nr = pb.n;
  for (int idx = threadIdx.x; idx < pb.pad * nr; idx += blockDim.x) {
    const int a = idx / nr, i = idx - (idx / nr) * nr;
    double2 wi = make_double2(0.0, 0.0), wa = make_double2(0.0, 0.0);
    const int c = inv[i];
    if (a < kk && c >= 0) {
      const int pc = pos[c];
      const int ra = order[a];
      const double2 x = A[ra * LD + c];
      // R[a][c] on the columns pivoted at step a or later (and never)
      if (pc < 0 || pc >= a) wa = cscale(x, scale);
      // (P R11^-1)[c][a] = z_a[c]: 1 / R_aa at the pivot, stored before it
      if (pc == a) wi = make_double2(1.0 / x.x, 0.0);
      else if (pc >= 0 && pc < a) wi = x;
    }
    const long long o = base + (long long)(pb.pad_off + a) * d.n + pb.off + i;
    if (d.out_c128) { ((double2*)d.W_iso)[o] = wi; ((double2*)d.W_abs)[o] = wa; }
    else { ((float2*)d.W_iso)[o] = from_d2<float2>(wi); ((float2*)d.W_abs)[o] = from_d2<float2>(wa); }
    if (d.blocks > 1) {
      const long long o2 = base + (long long)(pb.pad_off + a) * d.n + (1 - pb.k) * pb.n + i;
      if (d.out_c128) { ((double2*)d.W_iso)[o2] = make_double2(0, 0); ((double2*)d.W_abs)[o2] = make_double2(0, 0); }
      else { ((float2*)d.W_iso)[o2] = make_float2(0, 0); ((float2*)d.W_abs)[o2] = make_float2(0, 0); }
    }
  }
}

// The same sweep with the rows in registers, for problems of 33 to 128
// columns: NW waves (4 for 64 columns, 8 for 128), wave w holding rows i =
// NW q + w and lane j columns j + 64 s of each.  At each step the wave
// owning the pivot row publishes it through LDS (two buffers by the step's
// parity, one barrier per step), every wave updates its own rows in
// registers, and the owner then keeps the row's final values in place of
// the residual.  Block-diagonal problems (blocks = 2, one workgroup per
// block) as in k_pchol.  With d.done set (the try before a truncating
// eigen-decomposition, no blocks): a problem whose weight above the cutoff
// needs more than the cap's pivots writes done = 0 and nothing else, the
// others write their factors and done = 1.  Without it the factorisation
// stops at the cap.
template <int NMAX, int NW>
__global__ void __launch_bounds__(64 * NW) k_pchol_reg(EighDesc d) {
  static_assert((NMAX == 64 || NMAX == 128) && NMAX % NW == 0 && 64 % NW == 0, "rows over waves, columns over lanes");
  constexpr int RPW = NMAX / NW, CPL = NMAX / 64, KB = NMAX;   // KB: index field of the pivot key
  __shared__ int cidx[NMAX], inv[NMAX], wcount[NW];
  __shared__ int pos[NMAX], order[NMAX];
  __shared__ double2 pbuf[2][NMAX];
  __shared__ double red[2][NW];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long pid = blockIdx.x;
  const Problem pb = problem_of(d, pid);
  const long long t = pb.t;
  const double2* G = d.G + t * (long long)d.n * d.n;
  const int n = compact_rows<NW>(d, G, pb, cidx, inv, wcount);
  if (threadIdx.x < NMAX) pos[threadIdx.x] = -1;
  double2 A[RPW][CPL];
#pragma unroll
  for (int q = 0; q < RPW; ++q)
#pragma unroll
    for (int s = 0; s < CPL; ++s) {
      const int i = NW * q + wave, c = lane + 64 * s;
      A[q][s] = (i < n && c < n) ? gram_herm(d, G, pb.off + cidx[i], pb.off + cidx[c])
                                 : make_double2(0.0, 0.0);
    }
  double dj[CPL];
#pragma unroll
  for (int s = 0; s < CPL; ++s) {
    const int c = lane + 64 * s;
    dj[s] = c < n ? gram_at(d, G, (long long)(pb.off + cidx[c]) * d.n + pb.off + cidx[c]).x : 0.0;
  }
  double part = 0.0, own = 0.0;
  for (int i = threadIdx.x; i < d.n; i += blockDim.x) part += gram_at(d, G, (long long)i * d.n + i).x;
#pragma unroll
  for (int s = 0; s < CPL; ++s) own += dj[s];
  part = wave_sum_d(part);
  own = wave_sum_d(own);
  if (lane == 0) { red[0][wave] = part; red[1][wave] = own; }
  __syncthreads();
  double tr = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) tr += red[0][w];
  const double mine = red[1][0];          // (every wave holds every column's diagonal)
  const bool finite = isfinite(tr) && tr > 0.0;
  const double tot = d.blocks > 1 ? tr : mine;
  const double tol = d.cutoff * tot;
  const int lim = min(min(d.cap, pb.pad), n);
  unsigned long long piv[CPL];                          // pivoted columns (uniform)
#pragma unroll
  for (int s = 0; s < CPL; ++s) piv[s] = 0ull;
  int k = 0;
  bool fail = false;
  if (finite) {
    for (; k <= lim; ++k) {
      unsigned key = 0;
#pragma unroll
      for (int s = 0; s < CPL; ++s) {
        const int c = lane + 64 * s;
        if (c < n && !((piv[s] >> lane) & 1ull))
          key = max(key, ((__float_as_uint((float)fmax(dj[s], 0.0)) + (unsigned)KB) & ~(unsigned)(KB - 1)) |
                             (unsigned)(KB - 1 - c));
      }
      key = wave_max_u32(key);
      if (key == 0u) break;
      const int p = KB - 1 - (int)(key & (unsigned)(KB - 1));
      const double dm = readlane_d(CPL > 1 && p >= 64 ? dj[CPL - 1] : dj[0], p & 63);
      if (!(dm > tol) || !isfinite(dm)) break;         // (uniform: every wave alike)
      if (k == lim) { fail = true; break; }            // weight above the cutoff beyond the cap
      const double rkk = sqrt(dm);
      const double irkk = 1.0 / rkk;
      const int qp = p / NW;
      const bool owner = (p % NW) == wave;
      if (owner) {
#pragma unroll
        for (int q = 0; q < RPW; ++q)
          if (q == qp)
#pragma unroll
            for (int s = 0; s < CPL; ++s) pbuf[k & 1][lane + 64 * s] = A[q][s];
      }
      __syncthreads();
      double2 arow[CPL], u[CPL], z[CPL], w[CPL];
      bool colj[CPL];
#pragma unroll
      for (int s = 0; s < CPL; ++s) {
        const int c = lane + 64 * s;
        arow[s] = pbuf[k & 1][c];
        const bool before = (piv[s] >> lane) & 1ull;
        colj[s] = c < n && !before && c != p;
        u[s] = colj[s] ? cscale(arow[s], irkk) : make_double2(0.0, 0.0);
        z[s] = before ? cscale(arow[s], irkk) : make_double2(c == p ? irkk : 0.0, 0.0);
        w[s] = colj[s] ? u[s] : z[s];
        if (colj[s]) dj[s] = fma(-u[s].x, u[s].x, fma(-u[s].y, u[s].y, dj[s]));
      }
#pragma unroll
      for (int s = 0; s < CPL; ++s)
        if ((p >> 6) == s) piv[s] |= 1ull << (p & 63);
      if (owner) {
#pragma unroll
        for (int q = 0; q < RPW; ++q)
          if (q == qp)
#pragma unroll
            for (int s = 0; s < CPL; ++s)
              A[q][s] = colj[s] ? u[s] : ((lane + 64 * s) == p ? make_double2(rkk, 0.0) : z[s]);
      }
      // each remaining row j: A_jc -= conj(u_j) u_c (remaining c), y_j -= u_j z_k
#pragma unroll
      for (int q = 0; q < RPW; ++q) {
        const int i = NW * q + wave;
        const int wi = (q * NW) / 64;                   // (the word of row i's pivot bit)
        if (i < n && !((piv[wi] >> (i & 63)) & 1ull)) {
          // u_i from the published pivot row (one broadcast LDS read)
          const double2 pi = pbuf[k & 1][i];
          const double ujx = pi.x * irkk;
          const double ujy0 = pi.y * irkk;
#pragma unroll
          for (int s = 0; s < CPL; ++s) {
            const int c = lane + 64 * s;
            const double ujy = colj[s] ? -ujy0 : ujy0;
            double2 o = c == p ? make_double2(0.0, 0.0) : A[q][s];
            o.x = fma(-ujx, w[s].x, fma(ujy, w[s].y, o.x));
            o.y = fma(-ujx, w[s].y, fma(-ujy, w[s].x, o.y));
            if (c < n) A[q][s] = o;
          }
        }
      }
      if (threadIdx.x == 0) {
        order[k] = p;
        pos[p] = k;
      }
    }
  }
  if (d.done) {
    if (threadIdx.x == 0) d.done[pid] = fail ? 0 : 1;
    if (fail) return;                                   // (uniform) left to the eigensolver
  }
  const int r = k;
  double rs = 0.0;
#pragma unroll
  for (int s = 0; s < CPL; ++s)
    if (lane + 64 * s < n && !((piv[s] >> lane) & 1ull)) rs += fmax(dj[s], 0.0);
  const double resid = wave_sum_d(rs);
  const double kept = fmax(mine - resid, 0.0);
  double scale;
  int kk = r;
  if (d.blocks > 1) {
    scale = finite ? 1.0 / sqrt(tr) : 0.0;
  } else if (!(kept > 0.0) || !isfinite(kept) || r == 0) {
    kk = 0;
    scale = 0.0;
  } else {
    scale = 1.0 / sqrt(kept);
  }
  if (threadIdx.x == 0) {
    if (d.blocks > 1) {
      if (!finite && d.flags) atomicOr(d.flags + t, 1);
      if (d.disc_acc && tot > 0.0) atomicAdd(d.disc_acc + t, (mine - kept) / tot);
    } else {
      if (kk == 0 && d.flags) d.flags[t] |= 1;
      if (d.disc_acc && tot > 0.0) d.disc_acc[t] += (tot - kept) / tot;
      if (d.rank_out) d.rank_out[t * d.rank_stride] = kk;
      if (d.rank_max) d.rank_max[t * d.rank_stride] = max(d.rank_max[t * d.rank_stride], kk);
    }
    if (d.flops_acc) {
      const double f = 8.0 * ((double)r * r * (3.0 * n - 2.0 * r) / 3.0 + (double)r * r * r / 3.0);
      if (d.blocks > 1) atomicAdd(d.flops_acc + t, f);
      else d.flops_acc[t] += f;
    }
    if (d.nk_out) {
      d.nk_out[t * 4 + 2 * pb.k] = r;
      d.nk_out[t * 4 + 2 * pb.k + 1] = kk;
      if (d.blocks <= 1) { d.nk_out[t * 4 + 2] = 0; d.nk_out[t * 4 + 3] = 0; }
    }
    if (d.sweeps_out) d.sweeps_out[t] = 0;
  }
  __syncthreads();                                      // pos, order
  // zeros: rows a >= kk, the dead columns of the kept rows, and the other
  // block's columns of every row of this block
  const long long base = t * (long long)d.new_pad * d.n;
  const int nr = pb.n;
  for (int idx = threadIdx.x; idx < pb.pad * nr; idx += blockDim.x) {
    const int a = idx / nr, i = idx - (idx / nr) * nr;
    if (!(a < kk && inv[i] >= 0)) {
      const long long o = base + (long long)(pb.pad_off + a) * d.n + pb.off + i;
      if (d.out_c128) { ((double2*)d.W_iso)[o] = make_double2(0, 0); ((double2*)d.W_abs)[o] = make_double2(0, 0); }
      else { ((float2*)d.W_iso)[o] = make_float2(0, 0); ((float2*)d.W_abs)[o] = make_float2(0, 0); }
    }
    if (d.blocks > 1) {
      const long long o2 = base + (long long)(pb.pad_off + a) * d.n + (1 - pb.k) * pb.n + i;
      if (d.out_c128) { ((double2*)d.W_iso)[o2] = make_double2(0, 0); ((double2*)d.W_abs)[o2] = make_double2(0, 0); }
      else { ((float2*)d.W_iso)[o2] = make_float2(0, 0); ((float2*)d.W_abs)[o2] = make_float2(0, 0); }
    }
  }
  // the kept rows, from the registers of the waves that own their pivots:
  // W_abs row a = R[a] on the columns pivoted at step a or later (scaled),
  // W_iso row a = z_a (1 / R_aa at the pivot, stored on the earlier pivots)
#pragma unroll
  for (int q = 0; q < RPW; ++q) {
    const int i = NW * q + wave;
    const int a = i < n ? pos[i] : -1;
    if (a < 0 || a >= kk) continue;                     // (uniform)
#pragma unroll
    for (int s = 0; s < CPL; ++s) {
      const int c = lane + 64 * s;
      if (c >= n) continue;
      const int pc = pos[c];
      const double2 x = A[q][s];
      const double2 wa = (pc < 0 || pc >= a) ? cscale(x, scale) : make_double2(0.0, 0.0);
      const double2 wi = pc == a ? make_double2(1.0 / x.x, 0.0) : ((pc >= 0 && pc < a) ? x : make_double2(0.0, 0.0));
      const long long o = base + (long long)(pb.pad_off + a) * d.n + pb.off + cidx[c];
      if (d.out_c128) { ((double2*)d.W_iso)[o] = wi; ((double2*)d.W_abs)[o] = wa; }
      else { ((float2*)d.W_iso)[o] = from_d2<float2>(wi); ((float2*)d.W_abs)[o] = from_d2<float2>(wa); }
    }
  }
}

hipError_t launch_pchol(const EighDesc& d, int batch, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  const int nb = d.blocks > 1 ? 2 : 1;
  if (d.n < 1 || d.new_pad < 1 || (nb == 2 && ((d.n & 1) || (d.new_pad & 1))) || d.n / nb > (nb == 2 ? 64 : 128))
    return hipErrorInvalidValue;
  const int nsub = d.n / nb;
  const dim3 grid((unsigned)((long long)batch * nb));
  if (nsub > 64) hipLaunchKernelGGL((k_pchol_reg<128, 8>), grid, dim3(512), 0, st, d);
  else if (nsub <= 16) hipLaunchKernelGGL((k_pchol<16, 1>), grid, dim3(64), 0, st, d);
  else if (nsub <= 32) hipLaunchKernelGGL((k_pchol<32, 2>), grid, dim3(128), 0, st, d);
  else hipLaunchKernelGGL((k_pchol_reg<64, 4>), grid, dim3(256), 0, st, d);
  return hipGetLastError();
}

static bool g_attr_done = false;

// Sweep plans of the coset-grouped solver for N = 2^k, k = 2 .. 8: groups
// {a, b, a ^ b} (two-dimensional subspaces of (Z_2)^k, pairwise meeting only
// in 0), then the left-over matchings two at a time ({a, b}), and at most one
// alone ({a}, with any b != a fixing the cosets).  The triples are chosen
// greedily over a few fixed pseudo-random orders, keeping the plan with the
// fewest groups (a plan covers every d = 1 .. N - 1 exactly once).
static SweepPlan make_sweep_plans() {
  SweepPlan plan{};
  unsigned long long lcg = 0x2545F4914F6CDD1DULL;
  auto next = [&]() { lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL; return (unsigned)(lcg >> 33); };
  for (int k = 2; k <= kPlanMaxK; ++k) {
    const int N = 1 << k;
    std::vector<unsigned> best;
    for (int attempt = 0; attempt < 48; ++attempt) {
      std::vector<int> ord;
      for (int x = 1; x < N; ++x) ord.push_back(x);
      if (attempt > 0)
        for (int i = (int)ord.size() - 1; i > 0; --i) std::swap(ord[i], ord[next() % (unsigned)(i + 1)]);
      std::vector<char> used(N, 0);
      std::vector<unsigned> groups;
      for (int a : ord) {
        if (used[a]) continue;
        for (int b : ord) {
          if (b == a || used[b] || used[a ^ b]) continue;
          used[a] = used[b] = used[a ^ b] = 1;
          groups.push_back((unsigned)a | ((unsigned)b << 8) | (3u << 16));
          break;
        }
      }
      std::vector<int> rest;
      for (int a : ord) if (!used[a]) rest.push_back(a);
      size_t i = 0;
      for (; i + 1 < rest.size(); i += 2) groups.push_back((unsigned)rest[i] | ((unsigned)rest[i + 1] << 8) | (2u << 16));
      if (i < rest.size()) {
        const int a = rest[i];
        groups.push_back((unsigned)a | ((unsigned)(a == 1 ? 2 : 1) << 8) | (1u << 16));
      }
      if (best.empty() || groups.size() < best.size()) best = groups;
    }
    plan.ngroups[k] = (int)best.size();
    int pos = 0;
    for (size_t g = 0; g < best.size(); ++g) {
      plan.grp[k][g] = best[g];
      const int a = best[g] & 0xff, b = (best[g] >> 8) & 0xff, m = (int)(best[g] >> 16);
      const int dd[3] = {a, b, a ^ b};
      for (int j = 0; j < m; ++j) plan.dseq[k][pos++] = (unsigned char)dd[j];
    }
  }
  return plan;
}

const SweepPlan& sweep_plans() {
  static const SweepPlan plan = make_sweep_plans();
  return plan;
}

// the plans in each device's constant memory (once per device)
static hipError_t upload_plans() {
  static bool done[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (done[dev]) return hipSuccess;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_plan), &sweep_plans(), sizeof(SweepPlan));
  if (e == hipSuccess) done[dev] = true;
  return e;
}

int eigh_sweep_plan(int k, unsigned* groups, int cap) {
  if (k < 2 || k > kPlanMaxK || !groups) return -1;
  const SweepPlan& plan = sweep_plans();
  if (cap < plan.ngroups[k]) return -1;
  for (int g = 0; g < plan.ngroups[k]; ++g) groups[g] = plan.grp[k][g];
  return plan.ngroups[k];
}

int eigh_padded_size(int n) {
  int N = 4;
  while (N < n) N <<= 1;
  return N;
}

// Kernel attributes and the coset sweep plans of the current device, set up
// before the first launch (and before any graph capture, which may not copy
// to constant memory)
hipError_t eigh_prepare() {
  if (!g_attr_done) {
    hipError_t e = hipFuncSetAttribute((const void*)k_jacobi<true, kThreadsSmall, double2, 128>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 140 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_jacobi<true, kThreadsSmall, float2, 128>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 140 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_jacobi<false, kThreadsLarge, double2, 128>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 140 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_jacobi_coset<128>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              140 * 1024);
    if (e != hipSuccess) return e;
    g_attr_done = true;
  }
  return upload_plans();
}

hipError_t launch_eigh(const EighDesc& d, int batch, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  const int nb = d.blocks > 1 ? 2 : 1;
  if (d.n < 1 || d.n > 256 || d.new_pad < 1 || (nb == 2 && ((d.n & 1) || (d.new_pad & 1))))
    return hipErrorInvalidValue;
  if (!g_attr_done) {
    hipError_t e = eigh_prepare();
    if (e != hipSuccess) return e;
  }
  const int nsub = d.n / nb;
  const int n2 = nsub + (nsub & 1);
  const size_t gbytes = (size_t)n2 * (n2 + 1) / 2 * sizeof(double2);
  const long long nprob = (long long)batch * nb;
  // one wavefront per matrix for n <= 16; above, the workgroup kernel below
  // spreads each matrix over 8 wavefronts (faster per matrix from n = 24 on,
  // at any batch)
  if (n2 <= 16) {
    const unsigned grid = (unsigned)((nprob + 3) / 4);
    if (n2 <= 8) hipLaunchKernelGGL(k_jacobi_wave<8>, dim3(grid), dim3(256), 0, st, d, nprob);
    else hipLaunchKernelGGL(k_jacobi_wave<16>, dim3(grid), dim3(256), 0, st, d, nprob);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)nprob);
  if (n2 <= kVLdsMax) {
    if (d.out_c128)
      hipLaunchKernelGGL((k_jacobi<true, kThreadsSmall, double2, 128>), grid, dim3(kThreadsSmall),
                         gbytes + (size_t)n2 * n2 * sizeof(double2), st, d);
    else
      hipLaunchKernelGGL((k_jacobi<true, kThreadsSmall, float2, 128>), grid, dim3(kThreadsSmall),
                         gbytes + (size_t)n2 * n2 * sizeof(float2), st, d);
    return hipGetLastError();
  }
  // problems above 64: coset-grouped sweeps on the matrix padded to a power
  // of two, with a rotation log; then the kept columns replayed from it
  if (!d.rot_log || !d.order || !d.lam_sorted || !d.kept || !d.scale_abs || !d.nsteps)
    return hipErrorInvalidValue;
  const int N = eigh_padded_size(n2);
  if ((long long)d.max_steps < (long long)kMaxSweeps * (N - 1) ||
      d.log_stride < (long long)kMaxSweeps * (N - 1) * (N / 2) * 3)
    return hipErrorInvalidValue;
  hipError_t pe = upload_plans();
  if (pe != hipSuccess) return pe;
  // (each solver returns at once on the other's problems; the circle-ordered
  // launch, usually the thinner one, runs on the auxiliary stream beside the
  // coset-ordered one so that neither waits for the other's tail)
  if (N > 256 || (N > 128 && !d.gpk)) return hipErrorInvalidValue;
  const bool fork = d.aux_stream && d.ev_fork && d.ev_join;
  hipStream_t sc = st;
  if (fork) {
    hipError_t e = hipEventRecord(d.ev_fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(d.aux_stream, d.ev_fork, 0);
    if (e != hipSuccess) return e;
    sc = d.aux_stream;
  }
  if (N <= 128)
    hipLaunchKernelGGL((k_jacobi<false, kThreadsLarge, double2, 128>), grid, dim3(kThreadsLarge), gbytes, sc, d);
  else
    hipLaunchKernelGGL((k_jacobi<false, kThreadsLarge, double2, 256>), grid, dim3(kThreadsLarge), 0, sc, d);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (fork) {
    e = hipEventRecord(d.ev_join, sc);
    if (e != hipSuccess) return e;
  }
  if (N <= 128)
    hipLaunchKernelGGL(k_jacobi_coset<128>, grid, dim3(kThreadsCoset), (size_t)N * (N + 1) / 2 * sizeof(double2),
                       st, d);
  else
    hipLaunchKernelGGL(k_jacobi_coset<256>, grid, dim3(kThreadsCoset), 0, st, d);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (fork) {
    e = hipStreamWaitEvent(st, d.ev_join, 0);
    if (e != hipSuccess) return e;
  }
  if (N <= 128) {
    hipLaunchKernelGGL(k_jacobi_vectors<128>, grid, dim3(16 * 64), 0, st, d);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_jacobi_vectors<256>, grid, dim3(8 * 64), 0, st, d);
  return hipGetLastError();
}

}  // namespace ttn
