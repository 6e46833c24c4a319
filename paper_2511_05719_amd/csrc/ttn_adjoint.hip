// Bottom-node kernels of the adjoint gradient of log P.
//
// For a forced record the unnormalised final state is psi_N = A_N ... A_1
// psi_0 and P = <psi_N|psi_N>.  A layer of noise ops between two structural
// ops acts on distinct qubits as (x)_q N_q, N_q the ordered product of that
// qubit's SRX unitaries and recorded Kraus operators (Eq. 1-3).  With psi the
// state before the layer and lambda = A_>^dagger psi_N the adjoint state after
// it, P = <lambda| (x)_q N_q |psi> and, for a parameter p of one op of N_q,
//   d log P / dp = 2 Re <lambda| dN_q (x)_{q' != q} N_q' |psi> / P.
// Both are contractions of the two trees with the 2 x 2 operators on their
// physical legs.  The runtime contracts the internal nodes into up and down
// environments (GEMMs); these kernels handle the bottom nodes: their up
// environment, and the environment E_q of each leaf, from which
// P = sum_ii' E_q[i][i'] N_q[i][i'] and the derivatives follow.
#include "ttn_device.h"
#include "ttn_kernels.h"

namespace ttn {

// 2 x 2 complex helpers (row-major)
struct M2 { double2 a[2][2]; };
__device__ inline M2 m2_id() {
  M2 m;
  m.a[0][0] = make_double2(1, 0); m.a[0][1] = make_double2(0, 0);
  m.a[1][0] = make_double2(0, 0); m.a[1][1] = make_double2(1, 0);
  return m;
}
__device__ inline M2 m2_mul(const M2& x, const M2& y) {
  M2 r;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r.a[i][j] = cadd(cmul(x.a[i][0], y.a[0][j]), cmul(x.a[i][1], y.a[1][j]));
  return r;
}

// op j of a leaf's noise list and its derivative by its own parameter
__device__ inline void noise_op(const LeafNoise& nz, int j, const EnvParams& p, long long row, M2* op, M2* dop) {
  const long long o = row * p.pstride + nz.loc[j];
  M2 m, d;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) { m.a[a][b] = make_double2(0, 0); d.a[a][b] = make_double2(0, 0); }
  if (nz.kind[j] == NOISE_SRX) {
    // U = cos(t/2) I - i sin(t/2) X,  dU/dt = -sin(t/2)/2 I - i cos(t/2)/2 X
    const double th = p.theta[o];
    const double c = cos(0.5 * th), s = sin(0.5 * th);
    m.a[0][0] = m.a[1][1] = make_double2(c, 0);
    m.a[0][1] = m.a[1][0] = make_double2(0, -s);
    d.a[0][0] = d.a[1][1] = make_double2(-0.5 * s, 0);
    d.a[0][1] = d.a[1][0] = make_double2(0, -0.5 * c);
  } else {
    // recorded Kraus operator of amplitude damping and its gamma derivative
    const double g = p.gamma[o];
    const int jump = p.branches[row * p.br_stride + nz.branch[j]] ? 1 : 0;
    if (jump) {
      const double sg = sqrt(fmax(g, 0.0));
      m.a[0][1] = make_double2(sg, 0);
      d.a[0][1] = make_double2(0.5 / fmax(sg, 1e-300), 0);
    } else {
      const double s1 = sqrt(fmax(1.0 - g, 0.0));
      m.a[0][0] = make_double2(1, 0);
      m.a[1][1] = make_double2(s1, 0);
      d.a[1][1] = make_double2(-0.5 / fmax(s1, 1e-300), 0);
    }
  }
  *op = m;
  *dop = d;
}

// N_q = O_{n-1} ... O_0 (O_0 applied first)
__device__ inline M2 noise_product(const LeafNoise& nz, const EnvParams& p, long long row) {
  M2 r = m2_id();
  for (int j = 0; j < nz.n; ++j) {
    M2 o, d;
    noise_op(nz, j, p, row, &o, &d);
    r = m2_mul(o, r);
  }
  return r;
}

template <typename S>
__device__ inline double2 at(const S* T, int i, int j, int u, int U) { return to_d2(T[(i * 2 + j) * U + u]); }

// U[t][u][u'] = sum conj(lam[i][j][u]) N0[i][i'] N1[j][j'] psi[i'][j'][u']
template <typename S>
__global__ void __launch_bounds__(256) k_env_bottom_up(EnvBottom d, int batch) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= batch) return;
  const S* lam = (const S*)d.lam + (long long)row * 4 * d.ul;
  const S* psi = (const S*)d.psi + (long long)row * 4 * d.up;
  S* out = (S*)d.out + (long long)row * d.ul * d.up;
  const M2 N0 = noise_product(d.nz[0], d.par, row), N1 = noise_product(d.nz[1], d.par, row);
  for (int u = 0; u < d.ul; ++u)
    for (int v = 0; v < d.up; ++v) {
      double2 acc = make_double2(0, 0);
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          double2 w = make_double2(0, 0);      // ((N0 (x) N1) psi)[i][j][v]
          for (int i2 = 0; i2 < 2; ++i2)
            for (int j2 = 0; j2 < 2; ++j2)
              w = cadd(w, cmul(cmul(N0.a[i][i2], N1.a[j][j2]), at(psi, i2, j2, v, d.up)));
          acc = cadd(acc, cmul(cconj(at(lam, i, j, u, d.ul)), w));
        }
      out[u * d.up + v] = from_d2<S>(acc);
    }
}

// Leaf environments of a bottom node from its down environment D[u][u'],
// and the log-derivatives of every noise op on its two leaves.
template <typename S>
__global__ void __launch_bounds__(256) k_env_leaf_grad(EnvBottom d, int batch) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= batch) return;
  const S* lam = (const S*)d.lam + (long long)row * 4 * d.ul;
  const S* psi = (const S*)d.psi + (long long)row * 4 * d.up;
  const S* D = (const S*)d.down + (long long)row * d.ul * d.up;
  M2 N[2];
  N[0] = noise_product(d.nz[0], d.par, row);
  N[1] = noise_product(d.nz[1], d.par, row);
  for (int q = 0; q < 2; ++q) {
    const LeafNoise& nz = d.nz[q];
    if (nz.n == 0) continue;
    const M2& No = N[1 - q];
    // E[i][i'] = sum conj(lam[..i..][u]) No[j][j'] psi[..i'..j'..][u'] D[u][u'] (leaf q carries i)
    double2 E[2][2];
    for (int i = 0; i < 2; ++i)
      for (int i2 = 0; i2 < 2; ++i2) {
        double2 acc = make_double2(0, 0);
        for (int j = 0; j < 2; ++j)
          for (int j2 = 0; j2 < 2; ++j2) {
            const double2 nj = No.a[j][j2];
            if (nj.x == 0.0 && nj.y == 0.0) continue;
            for (int u = 0; u < d.ul; ++u) {
              const double2 l = cconj(q == 0 ? at(lam, i, j, u, d.ul) : at(lam, j, i, u, d.ul));
              double2 s = make_double2(0, 0);
              for (int v = 0; v < d.up; ++v)
                s = cadd(s, cmul(to_d2(D[u * d.up + v]), q == 0 ? at(psi, i2, j2, v, d.up) : at(psi, j2, i2, v, d.up)));
              acc = cadd(acc, cmul(cmul(l, nj), s));
            }
          }
        E[i][i2] = acc;
      }
    double2 P = make_double2(0, 0);
    for (int i = 0; i < 2; ++i)
      for (int i2 = 0; i2 < 2; ++i2) P = cadd(P, cmul(E[i][i2], N[q].a[i][i2]));
    const double pn = cabs2(P);
    if (!(pn > 0.0) || !isfinite(pn)) {
      if (d.flags) d.flags[row] |= 8;
      continue;
    }
    // derivative of N_q by the parameter of op j
    for (int j = 0; j < nz.n; ++j) {
      M2 dN = m2_id();
      for (int k = 0; k < nz.n; ++k) {
        M2 o, dd;
        noise_op(nz, k, d.par, row, &o, &dd);
        dN = m2_mul(k == j ? dd : o, dN);
      }
      double2 z = make_double2(0, 0);
      for (int i = 0; i < 2; ++i)
        for (int i2 = 0; i2 < 2; ++i2) z = cadd(z, cmul(E[i][i2], dN.a[i][i2]));
      // 2 Re(z / P)
      const double g = 2.0 * (z.x * P.x + z.y * P.y) / pn;
      double* out = nz.kind[j] == NOISE_SRX ? d.dtheta : d.dgamma;
      out[(long long)row * d.gstride + nz.loc[j]] += g;
    }
  }
}

hipError_t launch_env_bottom_up(const EnvBottom& d, int batch, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  if (d.ul < 1 || d.up < 1 || d.ul > 4 || d.up > 4 || d.nz[0].n > kMaxLeafNoise || d.nz[1].n > kMaxLeafNoise)
    return hipErrorInvalidValue;
  dim3 grid((batch + 255) / 256);
  if (d.c128) hipLaunchKernelGGL(k_env_bottom_up<double2>, grid, dim3(256), 0, st, d, batch);
  else hipLaunchKernelGGL(k_env_bottom_up<float2>, grid, dim3(256), 0, st, d, batch);
  return hipGetLastError();
}

hipError_t launch_env_leaf_grad(const EnvBottom& d, int batch, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  if (d.ul < 1 || d.up < 1 || d.ul > 4 || d.up > 4 || d.nz[0].n > kMaxLeafNoise || d.nz[1].n > kMaxLeafNoise ||
      !d.down || !d.dtheta || !d.dgamma)
    return hipErrorInvalidValue;
  dim3 grid((batch + 255) / 256);
  if (d.c128) hipLaunchKernelGGL(k_env_leaf_grad<double2>, grid, dim3(256), 0, st, d, batch);
  else hipLaunchKernelGGL(k_env_leaf_grad<float2>, grid, dim3(256), 0, st, d, batch);
  return hipGetLastError();
}

}  // namespace ttn
