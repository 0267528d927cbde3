// Shared device/host helpers for libls (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/ls.h"

#define LS_WAVE 64

// ---------------------------------------------------------------- status plumbing
#define LS_HIP_TRY(expr)                                  \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return LS_E_HIP;                \
  } while (0)

#define LS_TRY(expr)                                      \
  do {                                                    \
    int s_ = (expr);                                      \
    if (s_ < 0) return s_;                                \
  } while (0)

__host__ __device__ static inline size_t ls_align256(size_t x) { return (x + 255) & ~(size_t)255; }
__host__ __device__ static inline int64_t ls_cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- Philox4x32-10
// Salmon et al. (SC'11): ten rounds of two 32x32->64 multiplications on
// counter words 0 and 2, XOR of the high halves with the other two words and
// the round key, word permutation; the key advances by the Weyl constants.
__device__ __forceinline__ void ls_philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                                 uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    // three-input XORs in one instruction each (truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Uniform in (0, 1) from the top 23 bits of a word: (2 (w >> 9) + 1) 2^-24.
__device__ __forceinline__ double ls_u01d(uint32_t w) {
  return (double)((w >> 9) * 2u + 1u) * 5.9604644775390625e-8;
}

// Box-Muller in binary64 (library log/sqrt/sincospi).
__device__ __forceinline__ void ls_box_muller_f64(uint32_t w0, uint32_t w1, double& z0, double& z1) {
  const double u0 = ls_u01d(w0);
  const double u1 = ls_u01d(w1);
  const double rad = sqrt(-2.0 * log(u0));
  double s, c;
  sincospi(2.0 * u1, &s, &c);
  z0 = rad * c;
  z1 = rad * s;
}

// Round binary32 to bf16 (nearest, ties to even); returns the bit pattern.
__device__ __forceinline__ uint16_t ls_f32_to_bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float ls_bf16_bits_to_f32(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}

// ---------------------------------------------------------------- narrow formats
// Nearest value of a format with t mantissa bits after the point and minimum
// normal exponent emin (ties to even), computed exactly: the quantum at x's
// exponent (clamped to emin, so subnormals are kept) is a power of two, so
// x / quantum is exact and rint rounds it; beyond fmax the result saturates
// (e4m3) or becomes infinite.
struct LsFmt {
  int t, emin;
  double fmax;
  bool saturate;
};
__host__ __device__ constexpr LsFmt ls_fmt_bf16() { return {7, -126, 0x1.fep127, false}; }
__host__ __device__ constexpr LsFmt ls_fmt_f16() { return {10, -14, 65504.0, false}; }
__host__ __device__ constexpr LsFmt ls_fmt_e4m3() { return {3, -6, 448.0, true}; }

__device__ __forceinline__ double ls_round_fmt(double x, LsFmt f) {
  if (x == 0.0 || !isfinite(x)) return x;
  int e;
  (void)frexp(fabs(x), &e);   // |x| = g 2^e, g in [0.5, 1): leading bit 2^(e-1)
  int ex = e - 1;
  if (ex < f.emin) ex = f.emin;
  // the spacing 2^(ex - t) is a power of two: scaling by it is exact
  double r = ldexp(rint(ldexp(x, f.t - ex)), ex - f.t);
  if (fabs(r) > f.fmax) r = f.saturate ? copysign(f.fmax, r) : copysign((double)INFINITY, r);
  return r;
}
__device__ __forceinline__ float ls_round_fmt_f(float x, LsFmt f) {
  if (x == 0.0f || !isfinite(x)) return x;
  int e;
  (void)frexpf(fabsf(x), &e);
  int ex = e - 1;
  if (ex < f.emin) ex = f.emin;
  float r = ldexpf(rintf(ldexpf(x, f.t - ex)), ex - f.t);
  if (fabsf(r) > (float)f.fmax) r = f.saturate ? copysignf((float)f.fmax, r) : copysignf(INFINITY, r);
  return r;
}
// OCP e4m3 bits of a value already representable in e4m3 (|v| <= 448); a
// NaN or an infinity (which the format lacks) becomes its NaN, 0x7f.
__device__ __forceinline__ uint8_t ls_e4m3_bits(double v) {
  if (!isfinite(v)) return 0x7f;
  const uint8_t sgn = (v < 0.0 || (v == 0.0 && signbit(v))) ? 0x80 : 0x00;
  const double a = fabs(v);
  if (a == 0.0) return sgn;
  int e;
  const double g = frexp(a, &e);        // a = g 2^e, leading bit 2^(e-1)
  if (e - 1 < -6) return (uint8_t)(sgn | (uint8_t)(a * 512.0));   // subnormal: a = m 2^-9
  const int mant = (int)((2.0 * g - 1.0) * 8.0);
  return (uint8_t)(sgn | (uint8_t)((e - 1 + 7) << 3) | (uint8_t)mant);
}
// IEEE binary16 bits of a value already representable in binary16.
__device__ __forceinline__ uint16_t ls_f16_bits(double v) {
  return __builtin_bit_cast(uint16_t, (_Float16)(float)v);
}

// ---------------------------------------------------------------- reductions
template <typename T>
__device__ __forceinline__ T ls_wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a block of NT threads (NT multiple of 64); result valid in all threads.
template <typename T, int NT>
__device__ __forceinline__ T ls_block_sum(T v, T* sh /* NT/64 entries */) {
  v = ls_wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += sh[i];
  return s;
}

// Upper-triangular matrix-vector product out = U f, rows of one block of
// kUtThreads threads: thread (r = t % 32, g = t / 32) sums the columns
// j = row + g + 32 k, sixteen of them (and their f) loaded together per
// round, then the 32 column-group sums of each row are added in a fixed
// order.  The row value is returned in the threads with g == 0 (zero
// elsewhere).  Launch with ceil(n / 32) blocks of kUtThreads threads; red
// holds 32 x 33 doubles.
constexpr int kUtThreads = 1024;
template <typename TU, typename F>
__device__ __forceinline__ double ls_utmv_row(const TU* __restrict__ U, int64_t ldu, int64_t n, F f,
                                              double* red) {
  const int r = threadIdx.x & 31, g = threadIdx.x >> 5;
  const int64_t row = (int64_t)blockIdx.x * 32 + r;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  if (row < n) {
    for (int64_t j0 = row + g; j0 < n; j0 += 32 * 16) {
      double u[16], x[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t j = j0 + 32 * q;
        u[q] = (j < n) ? (double)U[row + j * ldu] : 0.0;
        x[q] = (j < n) ? f(j) : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) a[q & 3] += u[q] * x[q];
    }
  }
  red[g * 33 + r] = (a[0] + a[1]) + (a[2] + a[3]);
  __syncthreads();
  double s = 0.0;
  if (g == 0)
    for (int q = 0; q < 32; ++q) s += red[q * 33 + r];
  return s;
}

// Double-double helpers (Knuth's two-sum and an FMA two-product).  These
// error-free transformations need every product and sum rounded exactly as
// written, so floating-point contraction is switched off inside them.
struct ls_dd {
  double hi, lo;
};
__device__ __forceinline__ ls_dd ls_two_sum(double a, double b) {
#pragma clang fp contract(off)
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ __forceinline__ ls_dd ls_dd_add(ls_dd a, ls_dd b) {
#pragma clang fp contract(off)
  ls_dd s = ls_two_sum(a.hi, b.hi);
  double lo = s.lo + a.lo + b.lo;
  return ls_two_sum(s.hi, lo);
}
__device__ __forceinline__ ls_dd ls_dd_fma(ls_dd acc, double a, double b) {
#pragma clang fp contract(off)
  double p = a * b;
  double pe = fma(a, b, -p);
  ls_dd s = ls_two_sum(acc.hi, p);
  double lo = s.lo + acc.lo + pe;
  return ls_two_sum(s.hi, lo);
}
