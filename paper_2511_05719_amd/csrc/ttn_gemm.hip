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
// (l / Kin, l % Kin) so the middle-leg Gram needs no transpose.  With
// ksplit > 1 the K range is cut into ksplit slices whose partial products
// go to ksplit copies of C (stride sCz); the consumer sums them.
//
// Tiling: a 256-thread workgroup (4 wave64).  Each wave owns a (16 FA) x
// (16 FB) output block built from FA x FB MFMA 16x16x4 tiles (2 x 2: 32 x 32;
// 1 x 1 and 1 x 2 for problems of at most 16 rows); a complex
// multiply-accumulate is three real MFMAs with FP32 accumulation (re*re,
// im*im, (re+im)*(re+im)) and four with FP64 (re*re, -im*im, re*im, im*re;
// three on the diagonal tiles of a Gram matrix, whose imaginary part is
// antisymmetric).  The waves are arranged WM x WN over the output tile, or,
// for outputs of at most 32 x 32 (KW = 4), all four share one block and each
// takes a quarter of every K chunk, reduced through LDS at the end.  K is
// staged through LDS in chunks of 16 KW; the next chunk's global loads are
// issued before the current chunk's MFMAs, and the contiguous operand
// dimension is mapped to consecutive lanes on the global load.
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

// LDS row padding of the staged tiles: a 4-byte row stride of 17 (mod 32
// banks) keeps both the 16 x 4 read pattern of the MFMA operands and a
// column of 16 staged stores free of bank conflicts; 8-byte elements use 1
template <typename R> struct Pad { static constexpr int value = 17; };
template <> struct Pad<double> { static constexpr int value = 1; };

template <typename SA, typename SB, typename SC, typename R, int WM, int WN, int KW, int FA, int FB>
__global__ void __launch_bounds__(256, 2) k_zgemm(GemmDesc d) {
  static_assert(WM * WN * KW == 4, "four waves per workgroup");
  static_assert(FA * FB <= 4, "at most four 16 x 16 MFMA tiles per wave");
  constexpr int KPW = 16;                                  // K values per wave and chunk
  constexpr int TM = 16 * FA * WM, TN = 16 * FB * WN, TK = KPW * KW;
  constexpr int AE = TM * TK / 256, BE = TN * TK / 256;   // staged elements per thread
  constexpr int PADL = Pad<R>::value;
  constexpr int STAGE = 2 * TK * (TM + PADL) + 2 * TK * (TN + PADL);
  constexpr int RED = (KW > 1) ? (KW - 1) * FA * FB * 8 * 64 : 0;   // partial accumulators of waves kw > 0
  __shared__ R smem[STAGE > RED ? STAGE : RED];
  R (*As)[TK][TM + PADL] = reinterpret_cast<R (*)[TK][TM + PADL]>(smem);                 // [re/im][k][m]
  R (*Bs)[TK][TN + PADL] = reinterpret_cast<R (*)[TK][TN + PADL]>(smem + 2 * TK * (TM + PADL));
  typedef typename MfmaAcc<R>::type acc_t;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int kw = wave / (WM * WN);
  const int wm = (wave % (WM * WN)) / WN, wn = wave % WN;
  // XCD-aware order: the chip deals consecutive workgroups out to its 8
  // XCDs in turn, so workgroup x is given logical tile (x % 8) * (nx / 8) +
  // x / 8 and each XCD runs a contiguous range of tiles, the N tiles of a
  // row together: the row's W block stays in that XCD's L2
  long long bx = blockIdx.x;
  {
    const long long nx = gridDim.x;
    if (nx % 8 == 0) bx = (bx & 7) * (nx >> 3) + (bx >> 3);
  }
  const int tile_n = (int)(bx % d.tilesN);
  const long long bh = bx / d.tilesN;            // flattened (t, g, h)
  const int h = (int)(bh % d.H);
  const int g = (int)((bh / d.H) % d.G2);
  const long long t = bh / ((long long)d.H * d.G2);
  const int tile_m = blockIdx.y;
  const int z = blockIdx.z;
  const int m0 = tile_m * TM, n0 = tile_n * TN;
  if (d.herm && m0 >= n0 + TN) return;           // (uniform) a tile wholly below the diagonal

  const SA* A = (const SA*)d.A + t * d.sAt + h * d.sAh + g * d.sAg;
  const SB* B = (const SB*)d.B + t * d.sBt + h * d.sBh + g * d.sBg;
  SC* C = (SC*)d.C + t * d.sCt + h * d.sCh + g * d.sCg + z * d.sCz;
  const R sgnA = d.conjA ? (R)-1 : (R)1;
  const R sgnB = d.conjB ? (R)-1 : (R)1;
  const R bsg = sgnA * sgnB;        // staged A's imaginary part as B's (same_ab)

  // this trajectory's extents: rows, columns and K terms that can be
  // non-zero; a tile beyond them only writes its zeros.  A split N index
  // bounds its inner part by Nt and its outer part by No.
  const bool nsplit = d.Nin > 0 && d.Nin < d.N;
  int Mt = d.M, Nt = nsplit ? d.Nin : d.N, No = nsplit ? d.N / d.Nin : 1, Kt = d.K, Kin = d.Kin;
  if (d.ext) {
    const int* ex = d.ext + t * d.ext_stride;
    const int kn = d.knew ? d.knew[t * 4] : 0;
    auto extent = [&](int e) { return e < 0 ? kn : ex[e]; };
    int ht = d.H, ko = d.K / d.Kin, ki = d.Kin;
    if (d.eM) Mt = min(Mt, extent(d.eM) * d.mM);
    if (d.eN) Nt = min(Nt, extent(d.eN) * d.mN);
    if (nsplit && d.eNo) No = min(No, extent(d.eNo));
    if (d.eH) ht = min(ht, extent(d.eH));
    if (d.eKo) ko = min(ko, extent(d.eKo));
    if (d.eKi) ki = min(ki, extent(d.eKi));
    Kin = max(ki, 1);
    Kt = max(ko, 0) * max(ki, 0);
    if (h >= ht || m0 >= Mt || n0 >= (nsplit ? No * d.Nin : Nt)) Kt = 0;
  }
  if (d.band) {
    bool out = m0 >= d.bM1 || m0 + TM <= d.bM0 || h < d.bH0 || h >= d.bH1;
    if (nsplit) {
      const int qlo = n0 / d.Nin, qhi = (min(n0 + TN, d.N) - 1) / d.Nin;
      out = out || qhi < d.bNo0 || qlo >= d.bNo1;
    } else {
      out = out || n0 >= d.bN1 || n0 + TN <= d.bN0;
    }
    if (out) Kt = 0;
  }
  // K slice of this split (an empty slice still writes its zero partials)
  const int nchunks = (Kt + TK - 1) / TK;
  const int per = (nchunks + d.ksplit - 1) / d.ksplit;
  const int kbeg = z * per * TK;
  const int kend = min(Kt, kbeg + per * TK);

  // complex64 products accumulated in FP32 take the three-product form of
  // the complex product (Gauss; Higham, "Stability of a method for
  // multiplying complex matrices with three real matrix multiplications",
  // 1992): a quarter fewer MFMAs, an imaginary part with about twice the
  // conventional rounding bound.  FP64 accumulation (Gram matrices,
  // complex128) keeps the four-product form: its third accumulator set
  // would cost a wave per SIMD, which ate the saving.
  constexpr bool M3 = sizeof(R) == 4;
  acc_t acc_re[FA][FB], acc_im[FA][FB], acc_ii[FA][FB];
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int b = 0; b < FB; ++b) {
      acc_re[a][b] = (acc_t){0, 0, 0, 0};
      acc_im[a][b] = (acc_t){0, 0, 0, 0};
      acc_ii[a][b] = (acc_t){0, 0, 0, 0};
    }
  const int li = lane & 15, lk = lane >> 4;

  // Per-thread staging coordinates.  Element r of this thread's share of a
  // chunk sits at (row, k) = (base + r * step) of A (B), one of the two steps
  // zero (TM, TN and TK divide the 256 threads' stride), so row, k and LDS
  // slot are affine in r and only their bases live in registers; B keeps
  // each element's column offset (-1 beyond the row's extent), which a split
  // column index makes non-affine.  In-row offsets and strides fit 24 bits x
  // 24 bits products below 2^31 (checked by the launcher), so the K loop runs
  // on 32-bit full-rate integer arithmetic.
  static_assert(256 % TM == 0 && 256 % TN == 0 && 256 % TK == 0, "affine staging coordinates");
  const int am0 = d.a_m_fast ? tid % TM : tid / TK, ak0 = d.a_m_fast ? tid / TM : tid % TK;
  const int adm = d.a_m_fast ? 0 : 256 / TK, adk = d.a_m_fast ? 256 / TM : 0;
  const int als0 = ak0 * (TM + PADL) + am0, alsd = adk * (TM + PADL) + adm;
  const int bn0 = d.b_n_fast ? tid % TN : tid / TK, bk0 = d.b_n_fast ? tid / TN : tid % TK;
  const int bdn = d.b_n_fast ? 0 : 256 / TK, bdk = d.b_n_fast ? 256 / TN : 0;
  const int bls0 = bk0 * (TN + PADL) + bn0, blsd = bdk * (TN + PADL) + bdn;
  int b_co[BE];
#pragma unroll
  for (int r = 0; r < BE; ++r) {
    const int gn = n0 + bn0 + r * bdn;
    if (nsplit) {
      const int q = gn / d.Nin, rj = gn - q * d.Nin;
      const bool ok = gn < d.N && q < No && rj < Nt &&
                      (!d.band || (rj >= d.bN0 && rj < d.bN1 && q >= d.bNo0 && q < d.bNo1));
      b_co[r] = ok ? q * (int)d.sBj1 + rj * (int)d.sBj : -1;
    } else {
      b_co[r] = gn < Nt ? __umul24((unsigned)gn, (unsigned)d.sBj) : -1;
    }
  }
  const int gm0 = m0 + am0;
  // the K index l splits into (l / Kin, l % Kin); within one leg (Kin >= K
  // range) the quotient is 0; otherwise a float reciprocal and one
  // correction step give the exact quotient (l < 2^22)
  const bool kflat = Kin >= kend;
  const float kinv = 1.0f / (float)Kin;
  const unsigned sA1 = (unsigned)d.sAl1, sA2 = (unsigned)d.sAl2, sB1 = (unsigned)d.sBl1, sB2 = (unsigned)d.sBl2;
  auto kpart = [&](int gk, unsigned s1, unsigned s2) -> int {
    if (kflat) return __umul24((unsigned)gk, s2);
    int q = (int)((float)gk * kinv);
    if (q * Kin > gk) --q;
    else if ((q + 1) * Kin <= gk) ++q;
    return __umul24((unsigned)q, s1) + __umul24((unsigned)(gk - q * Kin), s2);
  };

  // a diagonal tile of a Gram matrix reads its B fragments from the staged
  // A (same rows, the conjugation undone by the sign), so B is neither
  // fetched nor staged
  const bool same = TM == TN && d.same_ab && tile_m == tile_n;
  // the fetched elements stay as loaded until they are staged: no
  // arithmetic on them between the load and the MFMAs of the current chunk,
  // so the wave does not wait for the next chunk's loads before computing
  SA ra[AE];
  SB rb[BE];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < AE; ++r) {
      const int gk = k0 + ak0 + r * adk, gm = gm0 + r * adm;
      SA v;
      v.x = 0;
      v.y = 0;
      if (gm < Mt && gk < kend) v = A[__umul24((unsigned)gm, (unsigned)d.sAi) + kpart(gk, sA1, sA2)];
      ra[r] = v;
    }
    if (same) return;
#pragma unroll
    for (int r = 0; r < BE; ++r) {
      const int gk = k0 + bk0 + r * bdk;
      SB v;
      v.x = 0;
      v.y = 0;
      if (b_co[r] >= 0 && gk < kend) v = B[b_co[r] + kpart(gk, sB1, sB2)];
      rb[r] = v;
    }
  };
  R* As0 = &As[0][0][0];
  R* As1 = &As[1][0][0];
  R* Bs0 = &Bs[0][0][0];
  R* Bs1 = &Bs[1][0][0];
  auto stage = [&]() {
#pragma unroll
    for (int r = 0; r < AE; ++r) {
      As0[als0 + r * alsd] = (R)ra[r].x;
      As1[als0 + r * alsd] = (R)ra[r].y * sgnA;
    }
    if (same) return;
#pragma unroll
    for (int r = 0; r < BE; ++r) {
      Bs0[bls0 + r * blsd] = (R)rb[r].x;
      Bs1[bls0 + r * blsd] = (R)rb[r].y * sgnB;
    }
  };
  // B fragments: from the staged B, or for a diagonal Gram tile from the
  // staged A with the conjugation undone by the sign (no branch in the loop)
  const R* Bf = same ? As0 : Bs0;
  const int bplane = same ? TK * (TM + PADL) : TK * (TN + PADL);
  const R bfs = same ? bsg : (R)1;
  // A diagonal tile of a Gram matrix conj(X + iY)^T (X + iY) (64 x 64 tiles):
  // the real part takes both products, the imaginary part X^T Y - Y^T X is
  // antisymmetric, so only P = X^T Y is accumulated (three MFMAs instead of
  // four, every product exact) and im = P - P^T is formed through LDS at
  // the end.  The conjugation must sit on exactly one operand.
  constexpr bool SYMOK = !M3 && TM == TN;
  const bool sym = SYMOK && same && (d.conjA != d.conjB);

  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += TK) {
    stage();
    __syncthreads();
    if (k0 + TK < kend) fetch(k0 + TK);      // in flight during the MFMAs below
    // ---- this wave's KPW k values of the chunk, 4 per MFMA ----
#pragma unroll
    for (int ks = 0; ks < KPW; ks += 4) {
      if (k0 + KPW * kw + ks >= kend) break;  // (uniform) only zeros staged from here on
      const int kr = KPW * kw + ks + lk;
      R a_re[FA], a_im[FA], b_re[FB], b_im[FB];
#pragma unroll
      for (int s = 0; s < (FA > FB ? FA : FB); ++s) {
        if (s < FA) {
          const int mi = wm * 16 * FA + s * 16 + li;
          a_re[s] = As[0][kr][mi];
          a_im[s] = As[1][kr][mi];
        }
        if (s < FB) {
          const int nj = wn * 16 * FB + s * 16 + li;
          b_re[s] = Bf[kr * (TN + PADL) + nj];
          b_im[s] = bfs * Bf[bplane + kr * (TN + PADL) + nj];
        }
      }
      // the accumulators are independent: issue each real product for all
      // of them before the next, so that consecutive MFMAs never wait on one
      // another's result
      if constexpr (M3) {
        // three real products: re.re, im.im and (re+im).(re+im)
        R sa[FA], sb[FB];
#pragma unroll
        for (int a = 0; a < FA; ++a) sa[a] = a_re[a] + a_im[a];
#pragma unroll
        for (int b = 0; b < FB; ++b) sb[b] = b_re[b] + b_im[b];
#pragma unroll
        for (int a = 0; a < FA; ++a)
#pragma unroll
          for (int b = 0; b < FB; ++b) acc_re[a][b] = MfmaAcc<R>::mma(a_re[a], b_re[b], acc_re[a][b]);
#pragma unroll
        for (int a = 0; a < FA; ++a)
#pragma unroll
          for (int b = 0; b < FB; ++b) acc_ii[a][b] = MfmaAcc<R>::mma(a_im[a], b_im[b], acc_ii[a][b]);
#pragma unroll
        for (int a = 0; a < FA; ++a)
#pragma unroll
          for (int b = 0; b < FB; ++b) acc_im[a][b] = MfmaAcc<R>::mma(sa[a], sb[b], acc_im[a][b]);
      } else {
        R na_im[FA];
#pragma unroll
        for (int a = 0; a < FA; ++a) na_im[a] = -a_im[a];
#pragma unroll
        for (int a = 0; a < FA; ++a)
#pragma unroll
          for (int b = 0; b < FB; ++b) acc_re[a][b] = MfmaAcc<R>::mma(a_re[a], b_re[b], acc_re[a][b]);
#pragma unroll
        for (int a = 0; a < FA; ++a)
#pragma unroll
          for (int b = 0; b < FB; ++b) acc_im[a][b] = MfmaAcc<R>::mma(a_re[a], b_im[b], acc_im[a][b]);
#pragma unroll
        for (int a = 0; a < FA; ++a)
#pragma unroll
          for (int b = 0; b < FB; ++b) acc_re[a][b] = MfmaAcc<R>::mma(na_im[a], b_im[b], acc_re[a][b]);
        if (!sym) {
#pragma unroll
          for (int a = 0; a < FA; ++a)
#pragma unroll
            for (int b = 0; b < FB; ++b) acc_im[a][b] = MfmaAcc<R>::mma(a_im[a], b_re[b], acc_im[a][b]);
        }
      }
    }
    __syncthreads();
  }
  if constexpr (SYMOK) {
    if (sym) {
      // acc_im holds sgnB P: im[i][j] = acc_im[i][j] - acc_im[j][i] (with the
      // K chunk split over the waves, each wave's partial P on its own)
      static_assert(KW * TM * TN <= (STAGE > RED ? STAGE : RED), "P tiles fit the staging buffer");
      R* P = smem + (KW > 1 ? kw * TM * TN : 0);
#pragma unroll
      for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            P[(wm * 16 * FA + a * 16 + MfmaAcc<R>::row(lk, r)) * TN + wn * 16 * FB + b * 16 + li] = acc_im[a][b][r];
      __syncthreads();
#pragma unroll
      for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            acc_im[a][b][r] -= P[(wn * 16 * FB + b * 16 + li) * TN + wm * 16 * FA + a * 16 + MfmaAcc<R>::row(lk, r)];
      if (KW > 1) __syncthreads();          // the reduction below reuses the buffer
    }
  }
  if constexpr (M3) {
    // re = re.re - im.im, im = (re+im).(re+im) - re.re - im.im
#pragma unroll
    for (int a = 0; a < FA; ++a)
#pragma unroll
      for (int b = 0; b < FB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const R p1 = acc_re[a][b][r], p2 = acc_ii[a][b][r];
          acc_re[a][b][r] = p1 - p2;
          acc_im[a][b][r] = acc_im[a][b][r] - p1 - p2;
        }
  }
  if (KW > 1) {
    // waves kw > 0 hand their partial sums to wave 0 (the staging buffers
    // are free after the last barrier of the loop)
    if (kw > 0) {
      R* red = smem + (kw - 1) * FA * FB * 8 * 64;
#pragma unroll
      for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            red[((a * FB + b) * 8 + r) * 64 + lane] = acc_re[a][b][r];
            red[((a * FB + b) * 8 + 4 + r) * 64 + lane] = acc_im[a][b][r];
          }
    }
    __syncthreads();
    if (kw > 0) return;
#pragma unroll
    for (int w = 0; w < KW - 1; ++w) {
      const R* red = smem + w * FA * FB * 8 * 64;
#pragma unroll
      for (int a = 0; a < FA; ++a)
#pragma unroll
        for (int b = 0; b < FB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            acc_re[a][b][r] += red[((a * FB + b) * 8 + r) * 64 + lane];
            acc_im[a][b][r] += red[((a * FB + b) * 8 + 4 + r) * 64 + lane];
          }
    }
  }
  // ---- write back each 16x16 tile in the MFMA's output lane layout ----
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int b = 0; b < FB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = m0 + wm * 16 * FA + a * 16 + MfmaAcc<R>::row(lk, r);
        const int gj = n0 + wn * 16 * FB + b * 16 + li;
        if (gi < d.M && gj < d.N) {
          double2 v = make_double2((double)acc_re[a][b][r], (double)acc_im[a][b][r]);
          if (d.herm && gi == gj) v.y = 0.0;    // a Hermitian matrix's real diagonal
          long long oj = (long long)gj * d.sCj;
          if (nsplit) {
            const int q = gj / d.Nin;
            oj = (long long)q * d.sCj1 + (long long)(gj - q * d.Nin) * d.sCj;
          }
          C[(long long)gi * d.sCi + oj] = from_d2<SC>(v);
        }
      }
}

// Output tile shape of a problem by the fixed rule: 64 x 64 in general,
// 128 x 32 or 32 x 128 when one side is at most 32 (16 x 128 when M is at
// most 16), and with the K chunk split over the four waves 32 x 32 when both
// are at most 32, 16 x 16 when both are at most 16 (the runtime's tuner may
// pick another shape by measurement).
enum TileCfg { TILE_64x64 = 0, TILE_128x32 = 1, TILE_32x128 = 2, TILE_32x32 = 3, TILE_16x16 = 4, TILE_16x128 = 5 };
static int tile_cfg(int M, int N) {
  if (M <= 16 && N <= 16) return TILE_16x16;
  if (M <= 32 && N <= 32) return TILE_32x32;
  if (N <= 32) return TILE_128x32;
  if (M <= 16) return TILE_16x128;
  if (M <= 32) return TILE_32x128;
  return TILE_64x64;
}
static void tile_dims(int cfg, int* tm, int* tn) {
  switch (cfg) {
    case TILE_128x32: *tm = 128; *tn = 32; return;
    case TILE_32x128: *tm = 32; *tn = 128; return;
    case TILE_32x32: *tm = 32; *tn = 32; return;
    case TILE_16x16: *tm = 16; *tn = 16; return;
    case TILE_16x128: *tm = 16; *tn = 128; return;
    default: *tm = 64; *tn = 64; return;
  }
}

int zgemm_rule_cfg(const GemmDesc& d) { return tile_cfg(d.M, d.N); }

// the 16-row shapes are only worth measuring for problems of at most 16 rows
// (and 16 columns for the 16 x 16 one)
bool zgemm_cfg_useful(const GemmDesc& d, int cfg) {
  if (cfg == TILE_16x16) return d.M <= 16 && d.N <= 16;
  if (cfg == TILE_16x128) return d.M <= 16;
  return cfg >= 0 && cfg < kZgemmCfgs;
}

long long zgemm_tiles(const GemmDesc& d) {
  int tm, tn;
  tile_dims(tile_cfg(d.M, d.N), &tm, &tn);
  return (long long)((d.M + tm - 1) / tm) * ((d.N + tn - 1) / tn);
}

template <typename SA, typename SB, typename SC, typename R, int WM, int WN, int KW, int FA, int FB>
hipError_t launch_cfg(GemmDesc d, int batch, hipStream_t st) {
  constexpr int TM = 16 * FA * WM, TN = 16 * FB * WN;
  d.tilesN = (d.N + TN - 1) / TN;
  const int tilesM = (d.M + TM - 1) / TM;
  dim3 grid((unsigned)((long long)batch * d.G2 * d.H * d.tilesN), (unsigned)tilesM, (unsigned)d.ksplit);
  hipLaunchKernelGGL((k_zgemm<SA, SB, SC, R, WM, WN, KW, FA, FB>), grid, dim3(256), 0, st, d);
  return hipGetLastError();
}

template <typename SA, typename SB, typename SC, typename R>
hipError_t launch_zgemm_t(GemmDesc d, int batch, hipStream_t st, int cfg) {
  if (d.M <= 0 || d.N <= 0 || batch <= 0) return hipSuccess;
  if (d.K <= 0) return hipErrorInvalidValue;
  if (d.Kin <= 0) d.Kin = d.K;
  if (d.G2 < 1) d.G2 = 1;
  if (d.ksplit < 1) d.ksplit = 1;
  if (d.H < 1 || d.ksplit > 64) return hipErrorInvalidValue;
  if (d.ext && (d.K % d.Kin != 0 || d.ext_stride < 1)) return hipErrorInvalidValue;
  {
    // the kernel's in-row offsets: 24-bit factors, sums below 2^31
    const long long lim24 = 1ll << 24;
    const long long kq = (d.K - 1) / d.Kin, kr = (d.K >= d.Kin) ? d.Kin - 1 : d.K - 1;
    const long long sA[4] = {d.sAi, d.sAl1, d.sAl2, 0}, sB[4] = {d.sBj, d.sBl1, d.sBl2, 0};
    for (int i = 0; i < 3; ++i)
      if (sA[i] < 0 || sA[i] >= lim24 || sB[i] < 0 || sB[i] >= lim24) return hipErrorInvalidValue;
    if (d.M >= lim24 || d.N >= lim24 || d.K >= (1 << 22)) return hipErrorInvalidValue;
    const long long ea = (long long)(d.M - 1) * d.sAi + kq * d.sAl1 + kr * d.sAl2;
    const bool nsplit = d.Nin > 0 && d.Nin < d.N;
    if (nsplit && (d.N % d.Nin != 0 || d.sBj1 < 0)) return hipErrorInvalidValue;
    const long long eb = (nsplit ? (long long)(d.N / d.Nin - 1) * d.sBj1 + (long long)(d.Nin - 1) * d.sBj
                                 : (long long)(d.N - 1) * d.sBj) + kq * d.sBl1 + kr * d.sBl2;
    if (ea >= (1ll << 31) || eb >= (1ll << 31)) return hipErrorInvalidValue;
  }
  if (d.ext && (d.eM < 0 || d.eN < 0 || d.eH < 0 || d.eKo < 0 || d.eKi < 0) && !d.knew) return hipErrorInvalidValue;
  if (cfg < 0 || cfg >= kZgemmCfgs) cfg = tile_cfg(d.M, d.N);
  switch (cfg) {
    case TILE_128x32: return launch_cfg<SA, SB, SC, R, 4, 1, 1, 2, 2>(d, batch, st);
    case TILE_32x128: return launch_cfg<SA, SB, SC, R, 1, 4, 1, 2, 2>(d, batch, st);
    case TILE_32x32: return launch_cfg<SA, SB, SC, R, 1, 1, 4, 2, 2>(d, batch, st);
    case TILE_16x16: return launch_cfg<SA, SB, SC, R, 1, 1, 4, 1, 1>(d, batch, st);
    case TILE_16x128: return launch_cfg<SA, SB, SC, R, 1, 4, 1, 1, 2>(d, batch, st);
    default: return launch_cfg<SA, SB, SC, R, 2, 2, 1, 2, 2>(d, batch, st);
  }
}

hipError_t launch_zgemm(const GemmDesc& d, int batch, int kind, hipStream_t st, int cfg) {
  switch (kind) {
    case GEMM_C64:        return launch_zgemm_t<float2, float2, float2, float>(d, batch, st, cfg);
    case GEMM_C128:       return launch_zgemm_t<double2, double2, double2, double>(d, batch, st, cfg);
    case GEMM_GRAM_C64:   return launch_zgemm_t<float2, float2, double2, double>(d, batch, st, cfg);
    case GEMM_GRAM_C128:  return launch_zgemm_t<double2, double2, double2, double>(d, batch, st, cfg);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ttn
