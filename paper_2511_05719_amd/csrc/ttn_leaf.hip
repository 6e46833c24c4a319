// Bottom-node kernels: single-qubit gates and channels, CNOTs between
// sibling leaves, Born measurements and Kraus jumps; plus the data movement
// of the controlled-gate zip, product-state initialisation and the logical
// readout.
//
// A bottom node holds two physical legs (dims 2 x 2) and its up bond U:
// T[t][a][b][u].  One thread owns one trajectory's node and executes the
// op list in order; probabilities and rescalings are FP64 whatever the
// storage precision.
#include "ttn_device.h"
#include "ttn_kernels.h"

namespace ttn {

template <typename S>
__device__ inline double2 ld(const S* p, int i) { return to_d2(p[i]); }

// apply M (2x2) to physical leg `leg` of T[2][2][U]
template <typename S>
__device__ inline void apply2(S* T, int U, int leg, const double2 m[2][2]) {
  for (int o = 0; o < 2; ++o)
    for (int u = 0; u < U; ++u) {
      const int i0 = (leg == 0 ? (0 * 2 + o) : (o * 2 + 0)) * U + u;
      const int i1 = (leg == 0 ? (1 * 2 + o) : (o * 2 + 1)) * U + u;
      const double2 v0 = ld(T, i0), v1 = ld(T, i1);
      T[i0] = from_d2<S>(cadd(cmul(m[0][0], v0), cmul(m[0][1], v1)));
      T[i1] = from_d2<S>(cadd(cmul(m[1][0], v0), cmul(m[1][1], v1)));
    }
}

// squared norms of the two halves of leg `leg`, in basis Z (xb = 0) or X (xb = 1)
template <typename S>
__device__ inline void half_norms(const S* T, int U, int leg, int xb, double* n0, double* n1) {
  double a = 0.0, b = 0.0;
  const double r = 0.70710678118654752440;
  for (int o = 0; o < 2; ++o)
    for (int u = 0; u < U; ++u) {
      const int i0 = (leg == 0 ? (0 * 2 + o) : (o * 2 + 0)) * U + u;
      const int i1 = (leg == 0 ? (1 * 2 + o) : (o * 2 + 1)) * U + u;
      double2 v0 = ld(T, i0), v1 = ld(T, i1);
      if (xb) {
        const double2 w0 = cscale(cadd(v0, v1), r), w1 = cscale(csub(v0, v1), r);
        v0 = w0; v1 = w1;
      }
      a += cabs2(v0);
      b += cabs2(v1);
    }
  *n0 = a;
  *n1 = b;
}

__device__ inline void set_m(double2 m[2][2], double a, double b, double c, double d) {
  m[0][0] = make_double2(a, 0); m[0][1] = make_double2(b, 0);
  m[1][0] = make_double2(c, 0); m[1][1] = make_double2(d, 0);
}
__device__ inline void matmul2(double2 r[2][2], const double2 a[2][2], const double2 b[2][2]) {
  double2 t[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) t[i][j] = cadd(cmul(a[i][0], b[0][j]), cmul(a[i][1], b[1][j]));
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r[i][j] = t[i][j];
}

template <typename S>
__global__ void __launch_bounds__(256) k_leaf_ops(LeafBatch b) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= b.n_rows) return;
  const double r2 = 0.70710678118654752440;
  const uint64_t traj = (b.traj_offset_dev ? *b.traj_offset_dev : b.traj_offset) + (uint64_t)row;
  for (int k = 0; k < b.n_ops; ++k) {
    const LeafOp op = b.ops[k];
    const int U = b.node_u[k];
    S* T = (S*)b.node_ptr[k] + (long long)row * 4 * U;
    double2 m[2][2];
    if (b.adjoint && op.kind != LOP_SRX && op.kind != LOP_INIT && op.kind != LOP_CNOT && op.kind != LOP_MEAS &&
        op.kind != LOP_KRAUS_AD) {
      b.flags[row] |= 4;
      continue;
    }
    if (b.adjoint && op.kind == LOP_KRAUS_AD) {
      // K_j^T of the recorded branch (both Kraus matrices are real), then
      // back to unit norm (the centre is on this node)
      const double g = b.gamma[(long long)row * b.gamma_row_stride + op.loc];
      const int jump = b.forced_br ? (b.forced_br[(long long)row * b.forced_br_stride + op.branch] ? 1 : 0) : 0;
      if (jump) set_m(m, 0, 0, sqrt(g), 0);
      else set_m(m, 1, 0, 0, sqrt(1.0 - g));
      apply2(T, U, op.leg, m);
      double n0, n1;
      half_norms(T, U, op.leg, 0, &n0, &n1);
      const double tot = n0 + n1;
      if (!(tot > 0.0) || !isfinite(tot)) { b.flags[row] |= 1; continue; }
      const double sc = 1.0 / sqrt(tot);
      set_m(m, sc, 0, 0, sc);
      apply2(T, U, op.leg, m);
      continue;
    }
    switch (op.kind) {
      case LOP_MATRIX: {
        const double* p = b.mat + (long long)row * b.mat_row_stride + (long long)op.loc * 8;
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) m[i][j] = make_double2(p[(i * 2 + j) * 2], p[(i * 2 + j) * 2 + 1]);
        apply2(T, U, op.leg, m);
        break;
      }
      case LOP_SRX: {
        const double th0 = b.theta[(long long)row * b.theta_row_stride + op.loc];
        const double th = b.adjoint ? -th0 : th0;
        const double c = cos(0.5 * th), s = sin(0.5 * th);
        m[0][0] = make_double2(c, 0); m[0][1] = make_double2(0, -s);
        m[1][0] = make_double2(0, -s); m[1][1] = make_double2(c, 0);
        apply2(T, U, op.leg, m);
        break;
      }
      case LOP_PAULI_SRX:
      case LOP_PAULI_AD: {
        double pI, pX, pY;
        if (op.kind == LOP_PAULI_SRX) {
          const double th = b.theta[(long long)row * b.theta_row_stride + op.loc];
          const double c = cos(0.5 * th), s = sin(0.5 * th);
          pI = c * c; pX = s * s; pY = 0.0;
        } else {
          const double g = b.gamma[(long long)row * b.gamma_row_stride + op.loc];
          const double sq = sqrt(1.0 - g);
          pI = 0.25 * (1.0 + sq) * (1.0 + sq); pX = 0.25 * g; pY = 0.25 * g;
        }
        const double u = philox_uniform(b.seed, traj, (uint64_t)op.draw);
        int which = 3;
        if (u < pI) which = 0;
        else if (u < pI + pX) which = 1;
        else if (u < pI + pX + pY) which = 2;
        if (b.probs) {
          const double pz = 1.0 - pI - pX - pY;
          b.probs[(long long)row * b.probs_stride + op.draw] =
              which == 0 ? pI : which == 1 ? pX : which == 2 ? pY : (op.kind == LOP_PAULI_SRX ? 0.0 : pz);
        }
        if (which == 0) break;
        if (which == 1) set_m(m, 0, 1, 1, 0);
        else if (which == 3) set_m(m, 1, 0, 0, -1);
        else { m[0][0] = make_double2(0, 0); m[0][1] = make_double2(0, -1);
               m[1][0] = make_double2(0, 1); m[1][1] = make_double2(0, 0); }
        apply2(T, U, op.leg, m);
        break;
      }
      case LOP_INIT: {
        double2 prep[2][2], undo[2][2];
        set_m(undo, 1, 0, 0, 1);
        const int mbit = (op.prev >= 0) ? (int)b.records[(long long)row * b.rec_stride + op.rec] : 0;
        if (op.prev == 0 && mbit) set_m(undo, 0, 1, 1, 0);          // |1> -> |0>
        if (op.prev == 1 && mbit) set_m(undo, 1, 0, 0, -1);         // |-> -> |+>
        const bool had_x = (op.prev == 1);
        // from |0> (prev none / Z) or |+> (prev X) to the requested basis state
        if ((op.arg == 1) != had_x) set_m(prep, r2, r2, r2, -r2);
        else set_m(prep, 1, 0, 0, 1);
        // both factors are real symmetric: the adjoint is the reversed product
        if (b.adjoint) matmul2(m, undo, prep);
        else matmul2(m, prep, undo);
        apply2(T, U, op.leg, m);
        break;
      }
      case LOP_CNOT: {
        // control on leg `leg`, target on the other physical leg
        for (int u = 0; u < U; ++u) {
          const int i0 = (op.leg == 0 ? (1 * 2 + 0) : (0 * 2 + 1)) * U + u;
          const int i1 = (1 * 2 + 1) * U + u;
          const S a = T[i0];
          T[i0] = T[i1];
          T[i1] = a;
        }
        break;
      }
      case LOP_GATE4: {
        const double* p = b.mat + (long long)row * b.mat_row_stride + (long long)op.loc * 32;
        for (int u = 0; u < U; ++u) {
          double2 v[4], w[4];
          for (int i = 0; i < 4; ++i) v[i] = ld(T, i * U + u);
          for (int i = 0; i < 4; ++i) {
            w[i] = make_double2(0, 0);
            for (int j = 0; j < 4; ++j)
              w[i] = cadd(w[i], cmul(make_double2(p[(i * 4 + j) * 2], p[(i * 4 + j) * 2 + 1]), v[j]));
          }
          for (int i = 0; i < 4; ++i) T[i * U + u] = from_d2<S>(w[i]);
        }
        break;
      }
      case LOP_MEAS: {
        double n0, n1;
        half_norms(T, U, op.leg, op.arg, &n0, &n1);
        const double tot = n0 + n1;
        if (!(tot > 0.0) || !isfinite(tot)) { b.flags[row] |= 1; break; }
        double p0 = n0 / tot;
        p0 = p0 < 0.0 ? 0.0 : (p0 > 1.0 ? 1.0 : p0);
        int mres;
        if (b.forced_rec) mres = b.forced_rec[(long long)row * b.forced_rec_stride + op.rec] ? 1 : 0;
        else mres = (philox_uniform(b.seed, traj, (uint64_t)op.draw) >= p0) ? 1 : 0;
        const double p = mres ? 1.0 - p0 : p0;
        if (p < 1e-300) { b.flags[row] |= 2; if (!b.adjoint) b.logp[row] = -INFINITY; }
        else if (!b.adjoint) b.logp[row] += log(p);
        if (b.probs && !b.adjoint) b.probs[(long long)row * b.probs_stride + op.draw] = p;
        const double sc = (p > 0.0) ? 1.0 / sqrt(p * tot) : 0.0;
        // projector onto the outcome, rescaled to unit norm
        if (op.arg == 0) {
          if (mres == 0) set_m(m, sc, 0, 0, 0); else set_m(m, 0, 0, 0, sc);
        } else {
          const double hs = 0.5 * sc;
          if (mres == 0) set_m(m, hs, hs, hs, hs); else set_m(m, hs, -hs, -hs, hs);
        }
        apply2(T, U, op.leg, m);
        if (b.records && !b.adjoint) b.records[(long long)row * b.rec_stride + op.rec] = (uint8_t)mres;
        break;
      }
      case LOP_KRAUS_AD:
      case LOP_KRAUS_MAT: {
        double2 K0[2][2], K1[2][2];
        if (op.kind == LOP_KRAUS_AD) {
          const double g = b.gamma[(long long)row * b.gamma_row_stride + op.loc];
          set_m(K0, 1, 0, 0, sqrt(1.0 - g));
          set_m(K1, 0, sqrt(g), 0, 0);
        } else {
          const double* p = b.mat + (long long)row * b.mat_row_stride + (long long)op.loc * 16;
          for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
              K0[i][j] = make_double2(p[(i * 2 + j) * 2], p[(i * 2 + j) * 2 + 1]);
              K1[i][j] = make_double2(p[8 + (i * 2 + j) * 2], p[8 + (i * 2 + j) * 2 + 1]);
            }
        }
        // p1 = |K1 v|^2 / |v|^2
        double tot = 0.0, j1 = 0.0;
        for (int o = 0; o < 2; ++o)
          for (int u = 0; u < U; ++u) {
            const int i0 = (op.leg == 0 ? (0 * 2 + o) : (o * 2 + 0)) * U + u;
            const int i1 = (op.leg == 0 ? (1 * 2 + o) : (o * 2 + 1)) * U + u;
            const double2 v0 = ld(T, i0), v1 = ld(T, i1);
            tot += cabs2(v0) + cabs2(v1);
            j1 += cabs2(cadd(cmul(K1[0][0], v0), cmul(K1[0][1], v1))) +
                  cabs2(cadd(cmul(K1[1][0], v0), cmul(K1[1][1], v1)));
          }
        if (!(tot > 0.0) || !isfinite(tot)) { b.flags[row] |= 1; break; }
        double p1 = j1 / tot;
        p1 = p1 < 0.0 ? 0.0 : (p1 > 1.0 ? 1.0 : p1);
        int jump;
        if (b.forced_br) jump = b.forced_br[(long long)row * b.forced_br_stride + op.branch] ? 1 : 0;
        else jump = (philox_uniform(b.seed, traj, (uint64_t)op.draw) < p1) ? 1 : 0;
        const double p = jump ? p1 : 1.0 - p1;
        if (p < 1e-300) { b.flags[row] |= 2; b.logp[row] = -INFINITY; }
        else b.logp[row] += log(p);
        if (b.probs) b.probs[(long long)row * b.probs_stride + op.draw] = p;
        double sc = (p > 0.0) ? 1.0 / sqrt(p * tot) : 0.0;
        if (b.ad_trotter && op.kind == LOP_KRAUS_AD && !jump) {
          // the Trotterised no-jump gate diag(1, e^{-g/2}): its norm is not
          // (1 - p1) |psi|^2, so rescale by the norm it leaves
          const double g = b.gamma[(long long)row * b.gamma_row_stride + op.loc];
          set_m(K0, 1, 0, 0, exp(-0.5 * g));
          double j0 = 0.0;
          for (int o = 0; o < 2; ++o)
            for (int u = 0; u < U; ++u) {
              const int i0 = (op.leg == 0 ? (0 * 2 + o) : (o * 2 + 0)) * U + u;
              const int i1 = (op.leg == 0 ? (1 * 2 + o) : (o * 2 + 1)) * U + u;
              j0 += cabs2(cmul(K0[0][0], ld(T, i0))) + cabs2(cmul(K0[1][1], ld(T, i1)));
            }
          sc = (j0 > 0.0) ? 1.0 / sqrt(j0) : 0.0;
        }
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) m[i][j] = cscale(jump ? K1[i][j] : K0[i][j], sc);
        apply2(T, U, op.leg, m);
        if (b.branches) b.branches[(long long)row * b.br_stride + op.branch] = (int8_t)jump;
        break;
      }
      default:
        b.flags[row] |= 4;
    }
  }
}

hipError_t launch_leaf_ops(const LeafBatch& b, hipStream_t st) {
  if (b.n_rows <= 0 || b.n_ops <= 0) return hipSuccess;
  dim3 grid((b.n_rows + 255) / 256);
  if (b.c128) hipLaunchKernelGGL(k_leaf_ops<double2>, grid, dim3(256), 0, st, b);
  else hipLaunchKernelGGL(k_leaf_ops<float2>, grid, dim3(256), 0, st, b);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Each thread owns two consecutive entries of a row (their source offsets
// are the same for every trajectory) and writes them for the rows
// blockIdx.y, blockIdx.y + gridDim.y, ... as one 2-element store; per-row
// element indices fit 32 bits (a node holds at most 2^31 entries per row).
template <typename S>
__device__ inline void extend_source(const ExtendDesc& d, int rr, int* src_off, int* src_off2, int* k, int* row) {
  int D[3] = {d.d0, d.d1, d.d2};
  int E[3] = {d.d0, d.d1, d.d2};
  E[d.leg_in] *= 2;
  if (d.leg_out >= 0) E[d.leg_out] *= 2;
  int idx[3];
  idx[2] = rr % E[2];
  const int r1 = rr / E[2];
  idx[1] = r1 % E[1];
  idx[0] = r1 / E[1];
  *src_off = -1; *src_off2 = -1; *k = 0; *row = 0;
  if (d.mode == 0) {
    const int kin = idx[d.leg_in] / D[d.leg_in];
    const int kout = idx[d.leg_out] / D[d.leg_out];
    if (kin == kout) {
      int j[3] = {idx[0], idx[1], idx[2]};
      j[d.leg_in] -= kin * D[d.leg_in];
      j[d.leg_out] -= kout * D[d.leg_out];
      *src_off = (j[0] * D[1] + j[1]) * D[2] + j[2];
    }
  } else {
    // doubled leg_in = (k, u); block k = bmat[k] applied on physical leg ctrl_leg
    // (the projector at the start of a controlled gate, or B_k at its end)
    *k = idx[d.leg_in] / D[d.leg_in];
    int j[3] = {idx[0], idx[1], idx[2]};
    j[d.leg_in] -= *k * D[d.leg_in];
    *row = j[d.ctrl_leg];
    j[d.ctrl_leg] = 0;
    *src_off = (j[0] * D[1] + j[1]) * D[2] + j[2];
    j[d.ctrl_leg] = 1;
    *src_off2 = (j[0] * D[1] + j[1]) * D[2] + j[2];
  }
}

template <typename S>
__device__ inline double2 extend_value(const ExtendDesc& d, const S* src, int so, int so2, int k, int row) {
  if (d.mode == 0) return so >= 0 ? to_d2(src[so]) : make_double2(0.0, 0.0);
  const double2 b0 = make_double2(d.bmat[k][row][0][0], d.bmat[k][row][0][1]);
  const double2 b1 = make_double2(d.bmat[k][row][1][0], d.bmat[k][row][1][1]);
  return cadd(cmul(b0, to_d2(src[so])), cmul(b1, to_d2(src[so2])));
}

// Extended tensors are written once and read back only by the next launches
// (far beyond the caches at batch sizes that fill the GPU): non-temporal
// stores stream them to HBM without allocating in the caches
__device__ inline void nt_store(float2* p, float2 v) {
  double w;
  __builtin_memcpy(&w, &v, 8);
  __builtin_nontemporal_store(w, reinterpret_cast<double*>(p));
}
__device__ inline void nt_store(double2* p, double2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}
template <typename S>
__global__ void __launch_bounds__(256) k_extend(ExtendDesc d, int batch, int per) {
  const int r0 = 2 * (blockIdx.x * blockDim.x + threadIdx.x);
  if (r0 >= per) return;
  const bool two = r0 + 1 < per;
  int a0, a1, ka, rowa, b0, b1, kb, rowb;
  extend_source<S>(d, r0, &a0, &a1, &ka, &rowa);
  if (two) extend_source<S>(d, r0 + 1, &b0, &b1, &kb, &rowb);
  for (long long t = blockIdx.y; t < batch; t += gridDim.y) {
    const S* src = (const S*)d.src + t * d.src_stride;
    S* dst = (S*)d.dst + t * d.dst_stride;
    const S va = from_d2<S>(extend_value<S>(d, src, a0, a1, ka, rowa));
    if (two) {
      const S vb = from_d2<S>(extend_value<S>(d, src, b0, b1, kb, rowb));
      nt_store(dst + r0, va);
      nt_store(dst + r0 + 1, vb);
    } else {
      nt_store(dst + r0, va);
    }
  }
}

hipError_t launch_extend(const ExtendDesc& d, int batch, hipStream_t st) {
  int E[3] = {d.d0, d.d1, d.d2};
  E[d.leg_in] *= 2;
  if (d.leg_out >= 0) E[d.leg_out] *= 2;
  const long long per = (long long)E[0] * E[1] * E[2];
  if (per <= 0 || batch <= 0) return hipSuccess;
  if (per >= (1ll << 31)) return hipErrorInvalidValue;
  // rows per workgroup: enough workgroups to fill the chip several times
  const long long pairs = (per + 1) / 2;
  const long long xblocks = (pairs + 255) / 256;
  const int ry = (int)std::max<long long>(1, std::min<long long>(batch, std::max<long long>(1, 65536 / xblocks)));
  dim3 grid((unsigned)xblocks, (unsigned)std::min(ry, 65535));
  if (d.c128) hipLaunchKernelGGL(k_extend<double2>, grid, dim3(256), 0, st, d, batch, (int)per);
  else hipLaunchKernelGGL(k_extend<float2>, grid, dim3(256), 0, st, d, batch, (int)per);
  return hipGetLastError();
}

__global__ void k_fill_zero(uint4* p, long long n16) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) p[i] = make_uint4(0, 0, 0, 0);
}

hipError_t launch_fill_zero(void* p, long long bytes, hipStream_t st) {
  if (bytes <= 0) return hipSuccess;
  if (bytes % 16) return hipErrorInvalidValue;
  const long long n16 = bytes / 16;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, st, (uint4*)p, n16);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <typename S>
__global__ void k_init_product(InitDesc d, int batch) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= batch) return;
  if (!d.bottom) {
    ((S*)d.ptr)[t] = from_d2<S>(make_double2(1.0, 0.0));
    return;
  }
  S* T = (S*)d.ptr + (long long)t * 4;
  const double r = 0.70710678118654752440;
  const double a0 = d.basis0 ? r : 1.0, a1 = d.basis0 ? r : 0.0;
  const double b0 = d.basis1 ? r : 1.0, b1 = d.basis1 ? r : 0.0;
  T[0] = from_d2<S>(make_double2(a0 * b0, 0.0));
  T[1] = from_d2<S>(make_double2(a0 * b1, 0.0));
  T[2] = from_d2<S>(make_double2(a1 * b0, 0.0));
  T[3] = from_d2<S>(make_double2(a1 * b1, 0.0));
}

hipError_t launch_init_product(const InitDesc& d, int batch, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  dim3 grid((batch + 255) / 256);
  if (d.c128) hipLaunchKernelGGL(k_init_product<double2>, grid, dim3(256), 0, st, d, batch);
  else hipLaunchKernelGGL(k_init_product<float2>, grid, dim3(256), 0, st, d, batch);
  return hipGetLastError();
}

// ------------------------------------------------------ work ledger ----
// adim[t][node][leg]: actual (unpadded) leg dimensions of row t.  The flops of
// a centre move from x to y, with na_b non-zero Gram eigenvalues and k_b kept
// values in block b (one block unless the move is block diagonal):
//   Gram          8 sum_b na_b^2 rest_x
//   contractions  8 sum_b k_b na_b (rest_x + rest_y)
// where rest_x, rest_y are the products of the other two leg dimensions of x
// and y (dense complex products, 8 real flops per complex multiply-add).
__global__ void k_ledger_hop(LedgerHop d, int batch) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= batch) return;
  int* ax = d.adim + ((long long)t * d.L + d.x) * 3;
  int* ay = d.adim + ((long long)t * d.L + d.y) * 3;
  const int* nk = d.nk + (long long)t * 4;
  double rx = 1.0, ry = 1.0;
  for (int l = 0; l < 3; ++l) {
    if (l != d.lx) rx *= ax[l];
    if (l != d.ly) ry *= ay[l];
  }
  const double na0 = nk[0], k0 = nk[1], na1 = nk[2], k1 = nk[3];
  d.gram_acc[t] += 8.0 * (na0 * na0 + na1 * na1) * rx;
  d.contract_acc[t] += 8.0 * (k0 * na0 + k1 * na1) * (rx + ry);
  // Gram: the node's rows of the bond read once, G written once (FP64
  // complex); contraction, per diagonal block and per side: the node block,
  // the factor block and the result
  d.gram_bytes[t] += d.es * (na0 + na1) * rx + 16.0 * (na0 * na0 + na1 * na1);
  d.contract_bytes[t] += d.es * ((na0 + k0 + na1 + k1) * (rx + ry) + 2.0 * (k0 * na0 + k1 * na1));
  ax[d.lx] = nk[1] + nk[3];
  ay[d.ly] = nk[1] + nk[3];
}
__global__ void k_ledger_double(int* adim, int L, int node, int l0, int l1, int batch) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= batch) return;
  int* a = adim + ((long long)t * L + node) * 3;
  a[l0] *= 2;
  if (l1 >= 0) a[l1] *= 2;
}
__global__ void k_ledger_reset(int* adim, int L, int batch) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)batch * L * 3) return;
  const int leg = (int)(i % 3);
  const int node = (int)((i / 3) % L);
  adim[i] = (node >= L / 2 && leg < 2) ? 2 : 1;
}
hipError_t launch_ledger_hop(const LedgerHop& d, int batch, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  if (d.x < 1 || d.x >= d.L || d.y < 1 || d.y >= d.L || d.lx < 0 || d.lx > 2 || d.ly < 0 || d.ly > 2)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ledger_hop, dim3((batch + 255) / 256), dim3(256), 0, st, d, batch);
  return hipGetLastError();
}
hipError_t launch_ledger_double(int* adim, int L, int node, int l0, int l1, int batch, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  if (node < 1 || node >= L || l0 < 0 || l0 > 2 || l1 > 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ledger_double, dim3((batch + 255) / 256), dim3(256), 0, st, adim, L, node, l0, l1, batch);
  return hipGetLastError();
}
hipError_t launch_ledger_reset(int* adim, int L, int batch, hipStream_t st) {
  const long long n = (long long)batch * L * 3;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ledger_reset, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, adim, L, batch);
  return hipGetLastError();
}

// the batch's largest value of each of the four per-row counts: one 16-byte
// load per row, a wavefront maximum by lane exchange, then across the
// sixteen wavefronts through LDS
__global__ void __launch_bounds__(1024) k_nk_max(const int* nk, int batch, int* out) {
  __shared__ int red[16][4];
  const int4* v = reinterpret_cast<const int4*>(nk);
  int m0 = 0, m1 = 0, m2 = 0, m3 = 0;
  for (int t = threadIdx.x; t < batch; t += 1024) {
    const int4 x = v[t];
    m0 = max(m0, x.x); m1 = max(m1, x.y); m2 = max(m2, x.z); m3 = max(m3, x.w);
  }
  for (int o = 32; o > 0; o >>= 1) {
    m0 = max(m0, __shfl_xor(m0, o)); m1 = max(m1, __shfl_xor(m1, o));
    m2 = max(m2, __shfl_xor(m2, o)); m3 = max(m3, __shfl_xor(m3, o));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { red[w][0] = m0; red[w][1] = m1; red[w][2] = m2; red[w][3] = m3; }
  __syncthreads();
  if (threadIdx.x < 4) {
    int r = 0;
    for (int k = 0; k < 16; ++k) r = max(r, red[k][threadIdx.x]);
    out[threadIdx.x] = r;
  }
}
hipError_t launch_nk_max(const int* nk, int batch, int* out, hipStream_t st) {
  if (batch <= 0) return hipErrorInvalidValue;
  if (reinterpret_cast<size_t>(nk) & 15) return hipErrorInvalidValue;   // rows are read as int4
  hipLaunchKernelGGL(k_nk_max, dim3(1), dim3(1024), 0, st, nk, batch, out);
  return hipGetLastError();
}

// dst[t * dst_stride] = src[t * src_stride] for every row t
__global__ void __launch_bounds__(256) k_set_ext(int* dst, long long dst_stride, const int* src,
                                                 long long src_stride, int batch) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < batch) dst[t * dst_stride] = src[t * src_stride];
}
hipError_t launch_set_ext(int* dst, long long dst_stride, const int* src, long long src_stride, int batch,
                          hipStream_t st) {
  if (batch <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_set_ext, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, st, dst, dst_stride, src,
                     src_stride, batch);
  return hipGetLastError();
}

__global__ void k_fill_cone(void* p, int c128, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (c128) ((double2*)p)[i] = make_double2(1.0, 0.0);
  else ((float2*)p)[i] = make_float2(1.0f, 0.0f);
}
hipError_t launch_fill_cone(void* p, int c128, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_cone, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, c128, n);
  return hipGetLastError();
}

__global__ void k_fill_i32(int* p, int v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f64(double* p, double v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, uint64_t v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
hipError_t launch_fill_u64(uint64_t* p, uint64_t value, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, value, n);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int* p, int value, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, value, n);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, double value, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, value, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ void k_decode(const uint8_t* records, long long rec_stride, const int* data_rec, int n_data,
                         const uint32_t* check_masks, int n_checks, const uint8_t* leader_parity,
                         uint8_t* fail, int batch) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= batch) return;
  const uint8_t* r = records + (long long)t * rec_stride;
  // check_masks: n_checks x 2 words (data index < 64)
  uint64_t bits = 0;
  int par = 0;
  for (int k = 0; k < n_data; ++k) {
    const int v = r[data_rec[k]] & 1;
    bits |= (uint64_t)v << k;
    par ^= v;
  }
  uint32_t syn = 0;
  for (int p = 0; p < n_checks; ++p) {
    const uint64_t m = (uint64_t)check_masks[2 * p] | ((uint64_t)check_masks[2 * p + 1] << 32);
    syn |= (uint32_t)(__popcll(bits & m) & 1) << p;
  }
  fail[t] = (uint8_t)(par ^ leader_parity[syn]);
}

hipError_t launch_decode(const uint8_t* records, long long rec_stride, const int* data_rec, int n_data,
                         const uint32_t* check_masks, int n_checks, const uint8_t* leader_parity,
                         uint8_t* fail, int batch, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_decode, dim3((batch + 255) / 256), dim3(256), 0, st, records, rec_stride, data_rec,
                     n_data, check_masks, n_checks, leader_parity, fail, batch);
  return hipGetLastError();
}

__global__ void k_philox(uint64_t seed, uint64_t off, int n_draws, double* out, int batch) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)batch * n_draws) return;
  const long long t = i / n_draws;
  const int k = (int)(i % n_draws);
  out[i] = philox_uniform(seed, off + (uint64_t)t, (uint64_t)k);
}

hipError_t launch_philox_uniforms(uint64_t seed, uint64_t traj_offset, int n_draws, double* out, int batch,
                                  hipStream_t st) {
  const long long total = (long long)batch * n_draws;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, seed, traj_offset,
                     n_draws, out, batch);
  return hipGetLastError();
}

}  // namespace ttn
