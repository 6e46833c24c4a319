// Batched strided complex GEMM on MFMA (gfx950).
//
// Every tensor contraction of the engine is one of
//   * applying a small matrix W to one leg of a 3-leg node tensor
//     T'[.., a, ..] = sum_i W[a][i] T[.., i, ..]            (absorb / isometrise)
//   * the Gram matrix of one leg,  G[i][j] = sum_rest conj(T[..i..]) T[..j..]
// Both are C[t,g,h][i][j] = sum_l op(A)[t,g,h][i][l] op(B)[t,g,h][l][j]
// with per-operand element strides, a trajectory batch index t, a block
// index g (the two diagonal blocks of a block-diagonal problem), an inner
// batch index h, and a K index that may be split in two strided parts
// (l / Kin, l % Kin) so the middle-leg Gram needs no transpose.
//
// Tiling: a 256-thread workgroup (4 wave64) owns a 64 x 64 output tile; each
// wave owns a 32 x 32 quadrant built from 2 x 2 MFMA 16x16x4 tiles.  A complex
// multiply-accumulate is four real MFMAs (re*re, -im*im, re*im, im*re).
// K is staged through LDS in chunks of 16, with the contiguous operand
// dimension mapped to consecutive lanes on the global load.
#include "ttn_device.h"
#include "ttn_kernels.h"

namespace ttn {

typedef float  f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

template <typename R> struct MfmaAcc;
// Output lane layout of the 16x16x4 MFMAs on gfx950 (lane l, register r):
// f32 holds D[4 (l / 16) + r][l % 16], f64 holds D[l / 16 + 4 r][l % 16].
template <> struct MfmaAcc<float> {
  typedef f4v type;
  __device__ static inline int row(int lk, int r) { return 4 * lk + r; }
  __device__ static inline f4v mma(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct MfmaAcc<double> {
  typedef d4v type;
  __device__ static inline int row(int lk, int r) { return lk + 4 * r; }
  __device__ static inline d4v mma(double a, double b, d4v c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

constexpr int TM = 64, TN = 64, TK = 16, PADL = 1;

template <typename S> __device__ inline void load_c(const S* p, long long off, double& re, double& im) {
  S v = p[off];
  re = (double)v.x;
  im = (double)v.y;
}

template <typename SA, typename SB, typename SC, typename R>
__global__ void __launch_bounds__(256) k_zgemm(GemmDesc d) {
  __shared__ R As[2][TK][TM + PADL];   // [re/im][k][m]
  __shared__ R Bs[2][TK][TN + PADL];   // [re/im][k][n]
  typedef typename MfmaAcc<R>::type acc_t;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const long long bx = blockIdx.x;
  const int tile_n = (int)(bx % d.tilesN);
  const long long bh = bx / d.tilesN;            // flattened (t, g, h)
  const int h = (int)(bh % d.H);
  const int g = (int)((bh / d.H) % d.G2);
  const long long t = bh / ((long long)d.H * d.G2);
  const int tile_m = blockIdx.y;
  const int m0 = tile_m * TM, n0 = tile_n * TN;

  const SA* A = (const SA*)d.A + t * d.sAt + h * d.sAh + g * d.sAg;
  const SB* B = (const SB*)d.B + t * d.sBt + h * d.sBh + g * d.sBg;
  SC* C = (SC*)d.C + t * d.sCt + h * d.sCh + g * d.sCg;
  const R sgnA = d.conjA ? (R)-1 : (R)1;
  const R sgnB = d.conjB ? (R)-1 : (R)1;

  acc_t acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc_re[a][b] = (acc_t){0, 0, 0, 0};
      acc_im[a][b] = (acc_t){0, 0, 0, 0};
    }

  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lk = lane >> 4;

  for (int k0 = 0; k0 < d.K; k0 += TK) {
    // ---- stage A tile [TM x TK] and B tile [TK x TN] ----
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int mm, kk;
      if (d.a_m_fast) { mm = tid & 63; kk = (tid >> 6) + 4 * r; }
      else            { mm = (tid >> 4) + 16 * r; kk = tid & 15; }
      const int gm = m0 + mm, gk = k0 + kk;
      double re = 0.0, im = 0.0;
      if (gm < d.M && gk < d.K) {
        long long off = (long long)gm * d.sAi + (long long)(gk / d.Kin) * d.sAl1 +
                        (long long)(gk % d.Kin) * d.sAl2;
        load_c(A, off, re, im);
      }
      As[0][kk][mm] = (R)re;
      As[1][kk][mm] = (R)im * sgnA;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int nn, kk;
      if (d.b_n_fast) { nn = tid & 63; kk = (tid >> 6) + 4 * r; }
      else            { nn = (tid >> 4) + 16 * r; kk = tid & 15; }
      const int gn = n0 + nn, gk = k0 + kk;
      double re = 0.0, im = 0.0;
      if (gn < d.N && gk < d.K) {
        long long off = (long long)(gk / d.Kin) * d.sBl1 + (long long)(gk % d.Kin) * d.sBl2 +
                        (long long)gn * d.sBj;
        load_c(B, off, re, im);
      }
      Bs[0][kk][nn] = (R)re;
      Bs[1][kk][nn] = (R)im * sgnB;
    }
    __syncthreads();
    // ---- 4 k-steps of the 16x16x4 MFMA per chunk ----
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      R a_re[2], a_im[2], b_re[2], b_im[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int mi = wm * 32 + s * 16 + li;
        const int nj = wn * 32 + s * 16 + li;
        a_re[s] = As[0][ks + lk][mi];
        a_im[s] = As[1][ks + lk][mi];
        b_re[s] = Bs[0][ks + lk][nj];
        b_im[s] = Bs[1][ks + lk][nj];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc_re[a][b] = MfmaAcc<R>::mma(a_re[a], b_re[b], acc_re[a][b]);
          acc_re[a][b] = MfmaAcc<R>::mma(-a_im[a], b_im[b], acc_re[a][b]);
          acc_im[a][b] = MfmaAcc<R>::mma(a_re[a], b_im[b], acc_im[a][b]);
          acc_im[a][b] = MfmaAcc<R>::mma(a_im[a], b_re[b], acc_im[a][b]);
        }
    }
    __syncthreads();
  }
  // ---- write back each 16x16 tile in the MFMA's output lane layout ----
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = m0 + wm * 32 + a * 16 + MfmaAcc<R>::row(lk, r);
        const int gj = n0 + wn * 32 + b * 16 + li;
        if (gi < d.M && gj < d.N) {
          double2 v = make_double2((double)acc_re[a][b][r], (double)acc_im[a][b][r]);
          C[(long long)gi * d.sCi + (long long)gj * d.sCj] = from_d2<SC>(v);
        }
      }
}

template <typename SA, typename SB, typename SC, typename R>
hipError_t launch_zgemm_t(GemmDesc d, int batch, hipStream_t st) {
  d.tilesN = (d.N + TN - 1) / TN;
  const int tilesM = (d.M + TM - 1) / TM;
  if (d.M <= 0 || d.N <= 0 || batch <= 0) return hipSuccess;
  if (d.K <= 0) return hipErrorInvalidValue;
  if (d.Kin <= 0) d.Kin = d.K;
  if (d.G2 < 1) d.G2 = 1;
  if (d.H < 1) return hipErrorInvalidValue;
  dim3 grid((unsigned)((long long)batch * d.G2 * d.H * d.tilesN), (unsigned)tilesM, 1);
  hipLaunchKernelGGL((k_zgemm<SA, SB, SC, R>), grid, dim3(256), 0, st, d);
  return hipGetLastError();
}

hipError_t launch_zgemm(const GemmDesc& d, int batch, int kind, hipStream_t st) {
  switch (kind) {
    case GEMM_C64:        return launch_zgemm_t<float2, float2, float2, float>(d, batch, st);
    case GEMM_C128:       return launch_zgemm_t<double2, double2, double2, double>(d, batch, st);
    case GEMM_GRAM_C64:   return launch_zgemm_t<float2, float2, double2, double>(d, batch, st);
    case GEMM_GRAM_C128:  return launch_zgemm_t<double2, double2, double2, double>(d, batch, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ttn
