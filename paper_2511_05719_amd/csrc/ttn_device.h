// Device-side helpers of the TTN trajectory engine (gfx950).
//
// Complex numbers are stored interleaved (re, im) as float2 (complex64) or
// double2 (complex128).  Contractions accumulate in the MFMA type of the
// instantiation; every probability, norm and eigen-decomposition is FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ttn {

template <typename T> struct cplx;
template <> struct cplx<float>  { typedef float2  type; };
template <> struct cplx<double> { typedef double2 type; };

__host__ __device__ inline double2 to_d2(float2 v) { return make_double2((double)v.x, (double)v.y); }
__host__ __device__ inline double2 to_d2(double2 v) { return v; }
template <typename S> __host__ __device__ inline S from_d2(double2 v);
template <> __host__ __device__ inline float2 from_d2<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
template <> __host__ __device__ inline double2 from_d2<double2>(double2 v) { return v; }

__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).  One trajectory's
// stream is keyed by (seed, global trajectory id); draw k is 64-bit word
// k mod 4 of the block computed at counter (k/4 + 1, 0, 0, 0), mapped to
// [0, 1) with 53 random bits.
// ---------------------------------------------------------------------------
__host__ __device__ inline void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
#if defined(__HIP_DEVICE_COMPILE__)
  *lo = a * b;
  *hi = __umul64hi(a, b);
#else
  unsigned __int128 p = (unsigned __int128)a * b;
  *lo = (uint64_t)p;
  *hi = (uint64_t)(p >> 64);
#endif
}

__host__ __device__ inline void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c[0], &hi0, &lo0);
    mulhilo64(M1, c[2], &hi1, &lo1);
    uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += W0; k1 += W1;
  }
}

__host__ __device__ inline double philox_uniform(uint64_t seed, uint64_t traj, uint64_t draw) {
  uint64_t c[4] = {draw / 4 + 1, 0, 0, 0};
  philox4x64_10(c, seed, traj);
  uint64_t w = c[draw % 4];
  return (double)(w >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace ttn
