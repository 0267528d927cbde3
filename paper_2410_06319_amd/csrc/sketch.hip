// Algorithm 1, the sketch: the Gaussian sketch Y = Omega [A b] on gfx950.
//
// Omega = S / sqrt(s) is never stored: S entries are regenerated from
// Philox4x32-10 (key = seed) where they are multiplied.  Narrow formats: the
// entry of S row k and column i is the 16-bit uniform U in half i % 2 of word
// (i % 8) / 2 of the block with counter (i / 8, k, prob, 2), mapped to the
// format's rounding of Phi^-1((U + 1/2) / 2^16) by a 2^15-entry table held in
// LDS (one Philox block serves eight entries).  Binary64: Box-Muller on the
// words of the block (i / 4, k, prob, 0).  [A b] is first packed into a zero-padded operand of the sketch
// format (Algorithm 1 takes A in the sketch's precision); it may be split into
// up to five parts of that format whose sum reproduces the data more closely.
// Products run on MFMA with binary32 (narrow formats) or binary64 (f64 path)
// accumulation over a chunk of rows of A; the chunk partial sums are added in
// binary64.
//
// bf16 and fp16 path: a block of 8 waves owns 128 rows of S and BN columns of [A b].
// Every K-step of 32 rows, the block generates its 128 x 32 tile of S once
// (each Gaussian is drawn once per column tile) and stages the TERMS x BN x 32
// operand tile, both in LDS.  With BN = 512 each wave multiplies all 128 rows
// by 64 columns (eight S fragments and the wave's operand fragments read from
// LDS per step); with narrower BN, wave (wr, wc) takes rows 64 wr .. +64 and
// columns wc BN/4 .. +BN/4.  LDS rows of 32 bf16 (four 16-byte quarters) are
// stored with the quarter index XORed with bits 2..3 of the row, so that the
// 16 lanes of each MFMA operand read hit distinct banks.
//
// e4m3 path: the same block shape on the 32x32x64 f8f6f4 MFMA with 64-row
// K-steps (k_sketch_e4m3), twice the product rate of the fp8 form of the
// 16x16x32 instruction.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <vector>

#include "common.h"
#include "kernels.h"

typedef __bf16 ls_bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef _Float16 ls_f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t ls_u32x2 __attribute__((ext_vector_type(2)));
typedef float ls_floatx4 __attribute__((ext_vector_type(4)));
typedef double ls_doublex4 __attribute__((ext_vector_type(4)));
typedef double ls_double2v __attribute__((ext_vector_type(2)));
typedef uint32_t ls_u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ narrow-format operand
// Column exponents (Section 3.2 column scaling, power-of-two constant):
// e_j = the largest integer with max_i |[A b]_ij| 2^e_j <= the format's
// largest finite value (0 for a zero column).  One block per column.
template <typename TA>
__global__ __launch_bounds__(256) void k_colexp(const TA* __restrict__ A, int64_t lda, const TA* __restrict__ b,
                                                int64_t m, int64_t n, double fmaxv, int32_t* __restrict__ e) {
  __shared__ double red[4];
  const int64_t j = blockIdx.x;
  const TA* col = (j < n) ? A + j * lda : b;
  // the largest magnitude (exact in TA), eight loads per thread in flight:
  // 16-byte vectors where the column is aligned to them, then the tail
  using V = typename std::conditional<sizeof(TA) == 4, ls_floatx4, ls_double2v>::type;
  constexpr int PV = 16 / (int)sizeof(TA);
  TA mt = 0;
  int64_t done = 0;
  if ((reinterpret_cast<uintptr_t>(col) & 15) == 0) {
    const V* cv = reinterpret_cast<const V*>(col);
    const int64_t nv = m / PV;
    for (int64_t i0 = threadIdx.x; i0 < nv; i0 += 256 * 8) {
      V v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t i = i0 + 256 * u;
        v[u] = (i < nv) ? cv[i] : V{};
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int k = 0; k < PV; ++k) mt = fmax(mt, fabs(v[u][k]));
    }
    done = nv * PV;
  }
  for (int64_t i0 = done + threadIdx.x; i0 < m; i0 += 256 * 8) {
    TA v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = i0 + 256 * u;
      v[u] = (i < m) ? col[i] : TA(0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) mt = fmax(mt, fabs(v[u]));
  }
  double mx = (double)mt;
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    int32_t ej = 0;
    if (mx > 0.0) {
      int E, G;
      const double f = frexp(mx, &E);
      const double F = frexp(fmaxv, &G);
      ej = (f <= F) ? G - E : G - E - 1;
    }
    e[j] = ej;
  }
}

// Two binary32 values rounded to nearest even in bf16 by the hardware
// conversion, packed (the first value in the lowest bits).
typedef __bf16 ls_bf16x2v __attribute__((ext_vector_type(2)));
typedef float ls_f32x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t sk_pack2_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((ls_f32x2v){a, b}, ls_bf16x2v));
}
// Values of packed elements (exact in binary64).
__device__ __forceinline__ double sk_bf16_at(uint32_t w, int i) {
  return (double)__uint_as_float(((w >> (16 * i)) & 0xffffu) << 16);
}
__device__ __forceinline__ double sk_f16_at(uint32_t w, int i) {
  return (double)__builtin_bit_cast(_Float16, (uint16_t)((w >> (16 * i)) & 0xffffu));
}
__device__ __forceinline__ double sk_e4m3_at(uint32_t w, int i) {
  const uint32_t b = (w >> (8 * i)) & 0xffu;
  const uint32_t e = (b >> 3) & 15u, mnt = b & 7u;
  double v;
  if (e == 15u && mnt == 7u) v = __builtin_nan("");
  else if (e == 0u) v = ldexp((double)mnt, -9);
  else v = ldexp((double)(8u + mnt), (int)e - 10);
  return (b & 0x80u) ? -v : v;
}

// ------------------------------------------------------------------ quantile tables
// Narrow-format entries of S: for v = 0 .. 2^15 - 1, the format's bits of
// a_v = -Phi^-1((v + 1/2) / 2^16) > 0 (round to nearest even); U < 2^15 maps
// to -a_U, U >= 2^15 to a_{2^16 - 1 - U}.  One table per format in device
// memory, filled once per device by k_icdf_init.
constexpr int kIcdfHalf = 32768;
static __device__ __align__(256) uint16_t g_icdf_bf16[kIcdfHalf];
static __device__ __align__(256) uint16_t g_icdf_f16[kIcdfHalf];
static __device__ __align__(256) uint8_t g_icdf_e4m3[kIcdfHalf];

// a_v by bisection on 0.5 erfc(a / sqrt 2) = p (its left side decreases in a)
// to about 1e-7, then Newton steps, which converge quadratically from there.
__global__ __launch_bounds__(256) void k_icdf_init(uint16_t* __restrict__ tb, uint16_t* __restrict__ th,
                                                   uint8_t* __restrict__ te) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v >= kIcdfHalf) return;
  const double p = ((double)v + 0.5) * (1.0 / 65536.0);
  const double r2 = 0.70710678118654752440;   // 1 / sqrt(2)
  double lo = 0.0, hi = 9.0;
  for (int it = 0; it < 27; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (0.5 * erfc(mid * r2) > p) lo = mid;
    else hi = mid;
  }
  double a = 0.5 * (lo + hi);
  for (int it = 0; it < 5; ++it) {
    const double f = 0.5 * erfc(a * r2) - p;
    const double dens = 0.39894228040143267794 * exp(-0.5 * a * a);   // the normal density at a
    a += f / dens;
  }
  tb[v] = ls_f32_to_bf16_bits((float)ls_round_fmt(a, ls_fmt_bf16()));
  th[v] = ls_f16_bits(ls_round_fmt(a, ls_fmt_f16()));
  te[v] = ls_e4m3_bits(ls_round_fmt(a, ls_fmt_e4m3()));
}

// Format bits of entry U (16-bit uniform) from the table of magnitudes.
__device__ __forceinline__ uint32_t sk_icdf16(const uint16_t* tab, uint32_t U) {
  const uint32_t neg = (U >> 15) ^ 1u;                 // U < 2^15: negative
  const uint32_t v = (U ^ (0xffffu * (1u - neg))) & 0x7fffu;
  return (uint32_t)tab[v] | (neg << 15);
}
__device__ __forceinline__ uint32_t sk_icdf8(const uint8_t* tab, uint32_t U) {
  const uint32_t neg = (U >> 15) ^ 1u;
  const uint32_t v = (U ^ (0xffffu * (1u - neg))) & 0x7fffu;
  return (uint32_t)tab[v] | (neg << 7);
}

// Table indices of the low and high 16-bit uniforms of a word: U below 2^15,
// 2^16 - 1 - U from 2^15 on (the sign-extended top bit flips the rest).
__device__ __forceinline__ uint32_t sk_ix_lo(uint32_t w) { return (w ^ (uint32_t)((int32_t)(w << 16) >> 31)) & 0x7fffu; }
__device__ __forceinline__ uint32_t sk_ix_hi(uint32_t w) { return ((w >> 16) ^ (uint32_t)((int32_t)w >> 31)) & 0x7fffu; }

// Formats of the narrow sketch: element bits, S rounding, MFMA.  An operand
// fragment is 8 consecutive K elements: what one lane supplies to a 16x16x32
// MFMA in the 16-bit formats (16 bytes); in e4m3 (8 bytes) four of them make
// a lane's operand of the 32x32x64 f8f6f4 MFMA.
// Eight 16-bit entries (K order: low half of word 0 first) from four words:
// the magnitudes of a word's two entries side by side, and the sign bits
// (set where the uniform is below 2^15) from the complemented top bits.
__device__ __forceinline__ ls_u32x4 sk_words16(const uint16_t* tab, uint32_t w0, uint32_t w1, uint32_t w2,
                                               uint32_t w3) {
  const uint32_t w[4] = {w0, w1, w2, w3};
  ls_u32x4 f;
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const uint32_t mag = __builtin_amdgcn_perm((uint32_t)tab[sk_ix_hi(w[h])], (uint32_t)tab[sk_ix_lo(w[h])], 0x05040100u);
    f[h] = mag | (~w[h] & 0x80008000u);
  }
  return f;
}

template <int FMT>
struct SkFmt;
template <>
struct SkFmt<LS_BF16> {
  using E = uint16_t;
  using frag = ls_u32x4;
  static constexpr LsFmt fmt() { return ls_fmt_bf16(); }
  static __device__ __forceinline__ frag from_words(const E* tab, uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3) {
    return sk_words16(tab, w0, w1, w2, w3);
  }
  static __device__ __forceinline__ E from_exact(double v) { return ls_f32_to_bf16_bits((float)v); }
  static __device__ __forceinline__ ls_floatx4 mma(frag a, frag b, ls_floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(ls_bf16x8, a), __builtin_bit_cast(ls_bf16x8, b),
                                                   c, 0, 0, 0);
  }
};
template <>
struct SkFmt<LS_FP16> {
  using E = uint16_t;
  using frag = ls_u32x4;
  static constexpr LsFmt fmt() { return ls_fmt_f16(); }
  static __device__ __forceinline__ frag from_words(const E* tab, uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3) {
    return sk_words16(tab, w0, w1, w2, w3);
  }
  static __device__ __forceinline__ E from_exact(double v) { return ls_f16_bits(v); }
  static __device__ __forceinline__ ls_floatx4 mma(frag a, frag b, ls_floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(ls_f16x8, a), __builtin_bit_cast(ls_f16x8, b), c,
                                                  0, 0, 0);
  }
};
template <>
struct SkFmt<LS_FP8E4M3> {
  using E = uint8_t;
  using frag = ls_u32x2;
  static constexpr LsFmt fmt() { return ls_fmt_e4m3(); }
  static __device__ __forceinline__ E from_exact(double v) { return ls_e4m3_bits(v); }
};

// K-panel layout of the narrow operand: for term t and K-block kb (rows
// 32 kb .. 32 kb + 31 of [A b]) the n_pad columns follow each other with
// their 32 elements contiguous: element (i, j) of term t sits at
// ((t nkb + i / 32) n_pad + j) 32 + i % 32, nkb = m_pad / 32.  Zero outside
// i < m, j <= n.  With column exponents e the column is first scaled by 2^e_j
// (exact).  The parts satisfy x = T_0 + T_1 + ... + rest, each T_t the
// format's rounding of what is left (differences exact in binary64).
// One thread per 8 consecutive rows of one column (one operand fragment):
// every part of the fragment leaves with one vector store.
template <int EB>
struct SkPackVec;
template <>
struct SkPackVec<2> {
  using type = uint4;
};
template <>
struct SkPackVec<1> {
  using type = uint2;
};
template <typename TA, int FMT>
__global__ __launch_bounds__(256) void k_pack_lp(const TA* __restrict__ A, int64_t lda, const TA* __restrict__ b,
                                                 int64_t m, int64_t n, int terms, const int32_t* __restrict__ e,
                                                 typename SkFmt<FMT>::E* __restrict__ Tt, int64_t m_pad,
                                                 int64_t n_pad) {
  using F = SkFmt<FMT>;
  using E = typename F::E;
  using V = typename SkPackVec<sizeof(E)>::type;
  // block (kb, cb): K-block kb (32 rows) of 64 columns; thread t takes rows
  // 8 (t % 4) .. +7 of column 64 cb + t / 4, so that a wave's stores of one
  // part are one contiguous run (16 columns x 32 elements)
  const int64_t i0 = (int64_t)blockIdx.x * 32 + 8 * (threadIdx.x & 3);
  const int64_t j = (int64_t)blockIdx.y * 64 + (threadIdx.x >> 2);
  if (i0 >= m_pad || j >= n_pad) return;
  const TA* col = (j < n) ? A + j * lda : b;
  TA xa[8];
  if (j <= n && i0 + 8 <= m && ((uintptr_t)(col + i0) & 15) == 0) {   // 16-byte loads
    constexpr int VW = 16 / sizeof(TA);
    using LV = typename std::conditional<sizeof(TA) == 4, ls_floatx4, ls_double2v>::type;
#pragma unroll
    for (int q = 0; q < 8; q += VW) {
      const LV v = *reinterpret_cast<const LV*>(col + i0 + q);
#pragma unroll
      for (int e2 = 0; e2 < VW; ++e2) xa[q + e2] = v[e2];
    }
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r) xa[r] = (i0 + r < m && j <= n) ? col[i0 + r] : TA(0);
  }
  const int64_t nkb = m_pad / 32;
  const int64_t pos = ((i0 >> 5) * n_pad + j) * 32 + (i0 & 31);
  if constexpr (FMT == LS_BF16 && sizeof(TA) == 4) {
    if (!e) {
      // binary32 data: each part is the hardware's round-to-nearest-even of what
      // is left, and what is left stays exact in binary32
#pragma unroll 1
      for (int t = 0; t < terms; ++t) {
        ls_u32x4 w;
#pragma unroll
        for (int p2 = 0; p2 < 4; ++p2) {
          w[p2] = sk_pack2_bf16(xa[2 * p2], xa[2 * p2 + 1]);
          xa[2 * p2] -= __uint_as_float(w[p2] << 16);
          xa[2 * p2 + 1] -= __uint_as_float(w[p2] & 0xffff0000u);
        }
        *reinterpret_cast<ls_u32x4*>(Tt + t * nkb * n_pad * 32 + pos) = w;
      }
      return;
    }
  }
  if constexpr (sizeof(TA) == 4 && (FMT == LS_FP8E4M3 || FMT == LS_FP16)) {
    if (e) {
      // binary32 data scaled by 2^e_j (exact: the scaled column lies within
      // the format's range): each part is the hardware's round-to-nearest-even
      // of what is left, and what is left stays exact in binary32
      const int ej = (j <= n) ? e[j] : 0;
      float xs[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) xs[r] = ldexpf(xa[r], ej);
#pragma unroll 1
      for (int t = 0; t < terms; ++t) {
        if constexpr (FMT == LS_FP8E4M3) {
          ls_u32x2 w;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            int wd = __builtin_amdgcn_cvt_pk_fp8_f32(xs[4 * h], xs[4 * h + 1], 0, false);
            wd = __builtin_amdgcn_cvt_pk_fp8_f32(xs[4 * h + 2], xs[4 * h + 3], wd, true);
            w[h] = (uint32_t)wd;
            xs[4 * h] -= __builtin_amdgcn_cvt_f32_fp8(wd, 0);
            xs[4 * h + 1] -= __builtin_amdgcn_cvt_f32_fp8(wd, 1);
            xs[4 * h + 2] -= __builtin_amdgcn_cvt_f32_fp8(wd, 2);
            xs[4 * h + 3] -= __builtin_amdgcn_cvt_f32_fp8(wd, 3);
          }
          *reinterpret_cast<ls_u32x2*>(Tt + t * nkb * n_pad * 32 + pos) = w;
        } else {
          ls_u32x4 w;
#pragma unroll
          for (int p2 = 0; p2 < 4; ++p2) {
            const _Float16 h0 = (_Float16)xs[2 * p2], h1 = (_Float16)xs[2 * p2 + 1];
            w[p2] = (uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
            xs[2 * p2] -= (float)h0;
            xs[2 * p2 + 1] -= (float)h1;
          }
          *reinterpret_cast<ls_u32x4*>(Tt + t * nkb * n_pad * 32 + pos) = w;
        }
      }
      return;
    }
  }
  const int ej = (e && j <= n) ? e[j] : 0;
  double x[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) x[r] = ldexp((double)xa[r], ej);
  for (int t = 0; t < terms; ++t) {
    E v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const double q = ls_round_fmt(x[r], F::fmt());
      v[r] = F::from_exact(q);
      x[r] -= q;
    }
    *reinterpret_cast<V*>(Tt + t * nkb * n_pad * 32 + pos) = __builtin_bit_cast(V, v);
  }
}

template <typename TA>
__global__ __launch_bounds__(256) void k_pack_f64(const TA* __restrict__ A, int64_t lda,
                                                  const TA* __restrict__ b, int64_t m, int64_t n,
                                                  double* __restrict__ M, int64_t m_pad, int64_t n_pad) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= m_pad || j >= n_pad) return;
  double x = 0.0;
  if (i < m) {
    if (j < n) x = (double)A[i + j * lda];
    else if (j == n) x = (double)b[i];
  }
  M[j * m_pad + i] = x;
}

// ------------------------------------------------------------------ narrow MFMA sketch
// v_mfma_f32_16x16x32_{bf16,f16} operands: lane l supplies row (l % 16)
// of S and column (l % 16) of the packed operand, at the 8 consecutive K
// indices 8 (l / 16) .. +7 of the step (one fragment); the product sums over
// the same K set on both sides.  Result: lane l holds D[4 (l/16) + r][l % 16].
constexpr int kSkThreads = 512;
constexpr int kSkRows = 128;   // rows of S per block

// Fragment slot of quarter q of LDS row r (rows of 32 elements = 4
// fragments); the XOR with bits of r makes the 16 lanes of an operand read hit
// distinct banks (16-byte fragments: bits 2..3; 8-byte fragments: bits 3..4).
template <int FB>
__device__ __forceinline__ int sk_slot(int r, int q) {
  return r * 4 + (q ^ ((r >> ((FB == 16) ? 2 : 3)) & 3));
}

// Block b of one problem's sketch (the kernels below give b).
template <int FMT, int BN, int TERMS>
__device__ __forceinline__ void sk_lp_body(const typename SkFmt<FMT>::E* __restrict__ Tt, int64_t nkb, int64_t n_pad,
                                           int64_t kb_per_split, int ns, int nn, uint32_t key0, uint32_t key1,
                                           uint32_t prob, const typename SkFmt<FMT>::E* __restrict__ icdf,
                                           float* __restrict__ Yp, int64_t s_pad, int b) {
  using F = SkFmt<FMT>;
  using frag = typename F::frag;
  constexpr int FB = sizeof(frag);
  // wave layout: WRG groups of rows x (8 / WRG) groups of columns; with 512
  // columns every wave takes all 128 rows (fewer operand reads from LDS per
  // product), otherwise two row groups of 64
  constexpr int WRG = (BN >= 512) ? 1 : 2;
  constexpr int RT = 8 / WRG;                  // 16-row tiles per wave
  constexpr int CT = BN / (16 * (8 / WRG));    // 16-column tiles per wave
  // column tiles whose operand fragments are held in registers at once
  constexpr int HALF = (CT * TERMS <= 8) ? CT : (TERMS >= 3 && CT >= 4) ? CT / 4 : (CT >= 2) ? CT / 2 : 1;
  constexpr int BQ = TERMS * BN * 4;           // fragments of the operand tile
  constexpr int BPT = (BQ + kSkThreads - 1) / kSkThreads;
  // one LDS block, the table at its start: an entry's LDS address is then
  // its index times the entry's size
  using E = typename F::E;
  __shared__ __align__(16) uint8_t lds[kIcdfHalf * sizeof(E) + (kSkRows * 4 + TERMS * BN * 4) * sizeof(frag)];
  E* const tab = reinterpret_cast<E*>(lds);
  frag* const As = reinterpret_cast<frag*>(lds + kIcdfHalf * sizeof(E));
  frag* const Bs = As + kSkRows * 4;
  const int t = threadIdx.x;
  {   // the quantile table, 16-byte pieces
    const uint4* src = reinterpret_cast<const uint4*>(icdf);
    uint4* dst = reinterpret_cast<uint4*>(tab);
    constexpr int nq = (int)(kIcdfHalf * sizeof(typename F::E) / 16);
    for (int i = t; i < nq; i += kSkThreads) dst[i] = src[i];
  }
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wr = wave % WRG, wc = wave / WRG;
  // blocks of one (K-split, column tile) group run on one XCD (block b -> XCD
  // b % 8; a grouped launch starts each problem at a multiple of 8)
  const int rest = b >> 3;
  const int grp = (rest / ns) * 8 + (b & 7);
  const int st = rest % ns;
  const int z = grp / nn;
  const int ntile = grp % nn;
  const int64_t row0 = (int64_t)st * kSkRows;
  const int64_t col0 = (int64_t)ntile * BN;
  const int64_t kb0 = (int64_t)z * kb_per_split;
  const int64_t kb1 = (kb0 + kb_per_split < nkb) ? kb0 + kb_per_split : nkb;

  // S generation: thread t draws row t % 128, quarter t / 128 of the K-step:
  // the eight entries of one Philox block (counter (i / 8, row, prob, 2))
  const int grow = t & (kSkRows - 1);
  const int gq = t >> 7;
  const uint32_t srow = (uint32_t)(row0 + grow);
  auto gen = [&](int64_t kb) -> frag {
    uint32_t a0 = (uint32_t)(kb * 4 + gq), a1 = srow, a2 = prob, a3 = 2u;
    ls_philox4x32_10(a0, a1, a2, a3, key0, key1);
    return F::from_words(tab, a0, a1, a2, a3);
  };
  // operand tile: fragment p = t + 512 u is (term, column, quarter) = (p / (4 BN), (p / 4) % BN, p % 4)
  const frag* Tf = reinterpret_cast<const frag*>(Tt);
  const int64_t term_stride = nkb * n_pad * 4;   // fragments
  auto loadb = [&](int64_t kb, frag (&reg)[BPT]) {
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
      const int p = t + kSkThreads * u;
      if (p < BQ) {
        const int term = p / (4 * BN);
        const int c = (p >> 2) % BN;
        const int q = p & 3;
        reg[u] = Tf[term * term_stride + (kb * n_pad + col0 + c) * 4 + q];
      }
    }
  };
  auto storeb = [&](const frag (&reg)[BPT]) {
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
      const int p = t + kSkThreads * u;
      if (p < BQ) {
        const int term = p / (4 * BN);
        const int c = (p >> 2) % BN;
        Bs[term * BN * 4 + sk_slot<FB>(c, p & 3)] = reg[u];
      }
    }
  };

  ls_floatx4 acc[RT][CT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = ls_floatx4{0.f, 0.f, 0.f, 0.f};

  frag sreg{};
  frag breg[BPT];
  __syncthreads();   // the table is in LDS
  if (kb0 < kb1) {
    sreg = gen(kb0);
    loadb(kb0, breg);
  }
  const int fq = lane >> 4;   // operand quarter of this lane
  for (int64_t kb = kb0; kb < kb1; ++kb) {
    __syncthreads();   // the previous step's operands have been read
    As[sk_slot<FB>(grow, gq)] = sreg;
    storeb(breg);
    __syncthreads();
    if (kb + 1 < kb1) {   // next step's operand loads in flight and its S drawn during the products
      loadb(kb + 1, breg);
      sreg = gen(kb + 1);
    }
#pragma unroll
    for (int h = 0; h < CT; h += HALF) {
      frag bf[HALF][TERMS];
#pragma unroll
      for (int ct = 0; ct < HALF; ++ct) {
        const int c = wc * (16 * CT) + (h + ct) * 16 + (lane & 15);
#pragma unroll
        for (int tm = 0; tm < TERMS; ++tm) bf[ct][tm] = Bs[tm * BN * 4 + sk_slot<FB>(c, fq)];
      }
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int r = wr * (16 * RT) + rt * 16 + (lane & 15);
        const frag af = As[sk_slot<FB>(r, fq)];
#pragma unroll
        for (int ct = 0; ct < HALF; ++ct)
#pragma unroll
          for (int tm = 0; tm < TERMS; ++tm) acc[rt][h + ct] = F::mma(af, bf[ct][tm], acc[rt][h + ct]);
      }
    }
  }
  float* out = Yp + (int64_t)z * s_pad * n_pad;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int64_t r = row0 + wr * (16 * RT) + rt * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int64_t c = col0 + wc * (16 * CT) + ct * 16 + (lane & 15);
      *reinterpret_cast<ls_floatx4*>(out + r + c * s_pad) = acc[rt][ct];
    }
  }
}

// ------------------------------------------------------------------ e4m3 sketch, 32x32x64 MFMA
// v_mfma_scale_f32_32x32x64_f8f6f4 (unit scales): lane l supplies row (or
// column) l % 32 of a 32-row (32-column) tile at the 32 K indices of K-group
// l / 32, here one whole 32-row K-block of the packed operand and of S; the
// result's lane l holds column l % 32, rows 8 (r / 4) + 4 (l / 32) + r % 4 in
// its register r (the same dot-product rounding as four chained 16x16x32 fp8
// steps, measured).  64-row steps keep the operand tile small enough that
// three parts' 512-column tiles fit in LDS beside the table, so that each S
// tile serves 512 columns.  LDS: the quantile table at offset 0, S tile [2 groups][128 rows]
// [32 bytes], operand tile [parts][2 groups][BN columns][32 bytes] (16-byte
// halves swapped in rows / columns 8..15 of each 16).  Waves: two groups of 64
// rows x four groups of BN / 4 columns.
constexpr size_t sk_e4m3_lds_bytes(int terms, int bn) {
  return (size_t)kIcdfHalf + (size_t)(kSkRows * 64) + (size_t)terms * bn * 64;
}

// 16-byte half h of row (column) rc of a tile: the halves are swapped in rows
// 8..15 of each 16, so that a 16-lane read covers every bank once.
__device__ __forceinline__ int sk_half(int rc, int h) { return h ^ ((rc >> 3) & 1); }

template <int BN, int TERMS>
__device__ __forceinline__ void sk_e4m3_body(const uint8_t* __restrict__ Tt, int64_t nkb, int64_t n_pad,
                                            int64_t kb_per_split, int ns, int nn, uint32_t key0, uint32_t key1,
                                            uint32_t prob, const uint8_t* __restrict__ icdf, float* __restrict__ Yp,
                                            int64_t s_pad, int b) {
  using F = SkFmt<LS_FP8E4M3>;
  typedef int v8i __attribute__((ext_vector_type(8)));
  typedef float v16f __attribute__((ext_vector_type(16)));
  constexpr int RT = 2;                    // 32-row tiles per wave (64 rows)
  constexpr int CT = BN / 128;             // 32-column tiles per wave (BN / 4 columns)
  constexpr int BQ = TERMS * 2 * BN * 2;   // 16-byte pieces of the operand tile
  constexpr int BPT = (BQ + kSkThreads - 1) / kSkThreads;
  static_assert(CT >= 1, "tile width");
  __shared__ __align__(16) uint8_t lds[kIcdfHalf + (2 * kSkRows * 2 + BQ) * 16];
  uint8_t* const tab = lds;
  ls_u32x4* const As = reinterpret_cast<ls_u32x4*>(lds + kIcdfHalf);
  ls_u32x4* const Bs = As + 2 * kSkRows * 2;
  const int t = threadIdx.x;
  {
    const ls_u32x4* src = reinterpret_cast<const ls_u32x4*>(icdf);
    ls_u32x4* dst = reinterpret_cast<ls_u32x4*>(tab);
    for (int i = t; i < kIcdfHalf / 16; i += kSkThreads) dst[i] = src[i];
  }
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int rest = b >> 3;
  const int grp = (rest / ns) * 8 + (b & 7);
  const int st = rest % ns;
  const int z = grp / nn;
  const int ntile = grp % nn;
  const int64_t row0 = (int64_t)st * kSkRows;
  const int64_t col0 = (int64_t)ntile * BN;
  // 64-row steps [ks0, ks1) of this K-split (kb_per_split and nkb are even)
  const int64_t ks0 = (int64_t)z * (kb_per_split / 2);
  const int64_t ks1 = ks0 + kb_per_split / 2 < nkb / 2 ? ks0 + kb_per_split / 2 : nkb / 2;

  // S: thread t draws row t % 128 of K-block 2 ks + (t / 128) % 2, entries
  // 16 h .. 16 h + 15 (h = t / 256): two Philox blocks
  const int grow = t & (kSkRows - 1);
  const int gg = (t >> 7) & 1;
  const int gh = t >> 8;
  const uint32_t srow = (uint32_t)(row0 + grow);
  auto gen = [&](int64_t ks) -> ls_u32x4 {
    uint32_t w[8];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      uint32_t a0 = (uint32_t)((ks * 2 + gg) * 4 + gh * 2 + i), a1 = srow, a2 = prob, a3 = 2u;
      ls_philox4x32_10(a0, a1, a2, a3, key0, key1);
      w[4 * i] = a0;
      w[4 * i + 1] = a1;
      w[4 * i + 2] = a2;
      w[4 * i + 3] = a3;
    }
    // all sixteen table reads issued together, then combined
    uint32_t v[16];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      v[2 * k] = tab[sk_ix_lo(w[k])];
      v[2 * k + 1] = tab[sk_ix_hi(w[k])];
    }
    ls_u32x4 f;
#pragma unroll
    for (int h = 0; h < 4; ++h) {   // entries 4h .. 4h+3 from words 2h, 2h+1
      const uint32_t a = w[2 * h], b2 = w[2 * h + 1];
      // magnitudes: the low then the high uniform of each word, byte by byte
      const uint32_t lo = __builtin_amdgcn_perm(v[4 * h + 1], v[4 * h], 0x0c0c0400u);
      const uint32_t hi = __builtin_amdgcn_perm(v[4 * h + 3], v[4 * h + 2], 0x0c0c0400u);
      // sign bits: bytes 1 and 3 of a and b hold the uniforms' top bits at bit 7
      const uint32_t top = __builtin_amdgcn_perm(b2, a, 0x07050301u);
      f[h] = (lo | (hi << 16)) | (~top & 0x80808080u);
    }
    return f;
  };
  // operand piece p = t + 512 u: (part, group, column, half) = (p / 4BN, (p / 2BN) % 2, (p / 2) % BN, p % 2)
  const ls_u32x4* T16 = reinterpret_cast<const ls_u32x4*>(Tt);
  const int64_t term_stride = nkb * n_pad * 2;   // pieces
  auto loadb = [&](int64_t ks, ls_u32x4 (&reg)[BPT]) {
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
      const int p = t + kSkThreads * u;
      if (p < BQ) {
        const int term = p / (4 * BN);
        const int g = (p / (2 * BN)) & 1;
        const int c = (p >> 1) % BN;
        reg[u] = T16[term * term_stride + ((ks * 2 + g) * n_pad + col0 + c) * 2 + (p & 1)];
      }
    }
  };
  auto storeb = [&](const ls_u32x4 (&reg)[BPT]) {
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
      const int p = t + kSkThreads * u;
      if (p < BQ) {
        const int c = (p >> 1) % BN;
        Bs[(p & ~(2 * BN - 1)) + c * 2 + sk_half(c, p & 1)] = reg[u];
      }
    }
  };
  auto frag_at = [&](const ls_u32x4* base, int rc) -> v8i {
    const ls_u32x4 lo = base[rc * 2 + sk_half(rc, 0)];
    const ls_u32x4 hi = base[rc * 2 + sk_half(rc, 1)];
    return v8i{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
  };

  v16f acc[RT][CT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = v16f{};

  ls_u32x4 sreg{};
  ls_u32x4 breg[BPT];
  __syncthreads();   // the table is in LDS
  if (ks0 < ks1) {
    sreg = gen(ks0);
    loadb(ks0, breg);
  }
  const int g = lane >> 5;   // K-group of this lane
  for (int64_t ks = ks0; ks < ks1; ++ks) {
    __syncthreads();   // the previous step's tiles have been read
    As[((gg * kSkRows + grow) * 2) + sk_half(grow, gh)] = sreg;
    storeb(breg);
    __syncthreads();
    {   // the next step's operand loads in flight and its S drawn during the products
      const int64_t kn = (ks + 1 < ks1) ? ks + 1 : ks;
      loadb(kn, breg);
      sreg = gen(kn);
    }
    v8i af[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) af[rt] = frag_at(As + g * kSkRows * 2, wr * 64 + rt * 32 + (lane & 31));
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int c = wc * (BN / 4) + ct * 32 + (lane & 31);
#pragma unroll
      for (int tm = 0; tm < TERMS; ++tm) {
        const v8i bf = frag_at(Bs + (tm * 2 + g) * BN * 2, c);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          acc[rt][ct] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(af[rt], bf, acc[rt][ct], 0, 0, 0, 127, 0, 127);
      }
    }
  }
  float* out = Yp + (int64_t)z * s_pad * n_pad;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int64_t c = col0 + wc * (BN / 4) + ct * 32 + (lane & 31);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = row0 + wr * 64 + rt * 32 + 8 * q + 4 * (lane >> 5);
        *reinterpret_cast<ls_floatx4*>(out + r + c * s_pad) =
            ls_floatx4{acc[rt][ct][4 * q], acc[rt][ct][4 * q + 1], acc[rt][ct][4 * q + 2], acc[rt][ct][4 * q + 3]};
      }
    }
  }
}

// One problem's sketch: block b = blockIdx.x.
template <int FMT, int BN, int TERMS>
__global__ __launch_bounds__(kSkThreads) void k_sketch_lp(const typename SkFmt<FMT>::E* __restrict__ Tt, int64_t nkb,
                                                          int64_t n_pad, int64_t kb_per_split, int ns, int nn,
                                                          uint32_t key0, uint32_t key1, uint32_t prob,
                                                          const typename SkFmt<FMT>::E* __restrict__ icdf,
                                                          float* __restrict__ Yp, int64_t s_pad) {
  sk_lp_body<FMT, BN, TERMS>(Tt, nkb, n_pad, kb_per_split, ns, nn, key0, key1, prob, icdf, Yp, s_pad, (int)blockIdx.x);
}
template <int BN, int TERMS>
__global__ __launch_bounds__(kSkThreads) void k_sketch_e4m3(const uint8_t* __restrict__ Tt, int64_t nkb,
                                                            int64_t n_pad, int64_t kb_per_split, int ns, int nn,
                                                            uint32_t key0, uint32_t key1, uint32_t prob,
                                                            const uint8_t* __restrict__ icdf,
                                                            float* __restrict__ Yp, int64_t s_pad) {
  sk_e4m3_body<BN, TERMS>(Tt, nkb, n_pad, kb_per_split, ns, nn, key0, key1, prob, icdf, Yp, s_pad, (int)blockIdx.x);
}

// Grouped sketches: one launch over the blocks of several problems of the
// same tile width and part count, problem i owning blocks [block0_i,
// block0_{i+1}) (block0 a multiple of 8); each block runs the single-problem
// code on its problem's arguments, so every result is the one the problem's
// own launch gives.
struct SkItem {
  const void* Tt;
  float* Yp;
  int64_t nkb, n_pad, kb_per_split, s_pad;
  int ns, nn;
  uint32_t key0, key1, prob;
  int block0;
};

__device__ __forceinline__ const SkItem& sk_item(const SkItem* __restrict__ items, int nitems, int b) {
  int lo = 0, hi = nitems - 1;   // the last item with block0 <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].block0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return items[lo];
}

template <int FMT, int BN, int TERMS>
__global__ __launch_bounds__(kSkThreads) void k_sketch_lp_grouped(const SkItem* __restrict__ items, int nitems,
                                                                  const typename SkFmt<FMT>::E* __restrict__ icdf) {
  using E = typename SkFmt<FMT>::E;
  const SkItem& it = sk_item(items, nitems, (int)blockIdx.x);
  sk_lp_body<FMT, BN, TERMS>(static_cast<const E*>(it.Tt), it.nkb, it.n_pad, it.kb_per_split, it.ns, it.nn, it.key0,
                             it.key1, it.prob, icdf, it.Yp, it.s_pad, (int)blockIdx.x - it.block0);
}
template <int BN, int TERMS>
__global__ __launch_bounds__(kSkThreads) void k_sketch_e4m3_grouped(const SkItem* __restrict__ items, int nitems,
                                                                    const uint8_t* __restrict__ icdf) {
  const SkItem& it = sk_item(items, nitems, (int)blockIdx.x);
  sk_e4m3_body<BN, TERMS>(static_cast<const uint8_t*>(it.Tt), it.nkb, it.n_pad, it.kb_per_split, it.ns, it.nn,
                         it.key0, it.key1, it.prob, icdf, it.Yp, it.s_pad, (int)blockIdx.x - it.block0);
}

// ------------------------------------------------------------------ f64 MFMA sketch
// v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// result lane l holds D[(l/16) + 4 r][l % 16] (rows interleaved, unlike the
// bf16 layout above).  Within a 16-row block of A the
// four steps t use K index kb + 4 (l/16) + t, so one Philox block (4 samples
// of one S row) serves the lane's four steps.
template <int NB>
__global__ __launch_bounds__(256) void k_sketch_f64(const double* __restrict__ M, int64_t m_pad,
                                                    int64_t n_pad, int64_t kchunk, uint32_t key0,
                                                    uint32_t key1, uint32_t prob,
                                                    double* __restrict__ Yp, int64_t s_pad) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint32_t srow = (uint32_t)(blockIdx.x * 64 + wave * 16 + (lane & 15));
  const int64_t col0 = (int64_t)blockIdx.y * (16 * NB);
  const int64_t kb0 = (int64_t)blockIdx.z * kchunk;
  const int64_t kb1 = (kb0 + kchunk < m_pad) ? kb0 + kchunk : m_pad;
  const int kq = (lane >> 4) * 4;
  const double* colp = M + (col0 + (lane & 15)) * m_pad + kq;

  ls_doublex4 acc[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc[nb] = ls_doublex4{0.0, 0.0, 0.0, 0.0};

  for (int64_t k = kb0; k < kb1; k += 16) {
    uint32_t a0 = (uint32_t)((k + kq) >> 2), a1 = srow, a2 = prob, a3 = 0u;
    ls_philox4x32_10(a0, a1, a2, a3, key0, key1);
    double z[4];
    ls_box_muller_f64(a0, a1, z[0], z[1]);
    ls_box_muller_f64(a2, a3, z[2], z[3]);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const double* p = colp + nb * 16 * m_pad + k;
      const double b0 = p[0], b1 = p[1], b2 = p[2], b3 = p[3];
      acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(z[0], b0, acc[nb], 0, 0, 0);
      acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(z[1], b1, acc[nb], 0, 0, 0);
      acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(z[2], b2, acc[nb], 0, 0, 0);
      acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(z[3], b3, acc[nb], 0, 0, 0);
    }
  }
  double* out = Yp + (int64_t)blockIdx.z * s_pad * n_pad;
  const int64_t r0 = (int64_t)blockIdx.x * 64 + wave * 16 + (lane >> 4);
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int64_t c = col0 + nb * 16 + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) out[(r0 + 4 * r) + c * s_pad] = acc[nb][r];
  }
}

// ------------------------------------------------------------------ chunk combine
// Y[k + j ldy] = scale 2^-e_j sum_z Yp[z][k + j s_pad], summed in binary64 in
// chunk order (deterministic).
template <typename TP>
__global__ __launch_bounds__(256) void k_sketch_combine(const TP* __restrict__ Yp, int64_t s_pad,
                                                        int64_t n_pad, int nsplit, int64_t s,
                                                        int64_t ncols, double scale,
                                                        const int32_t* __restrict__ e,
                                                        double* __restrict__ Y, int64_t ldy) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (k >= s || j >= ncols) return;
  double acc = 0.0;
  for (int z = 0; z < nsplit; ++z) acc += (double)Yp[(int64_t)z * s_pad * n_pad + k + j * s_pad];
  acc *= scale;
  if (e) acc = ldexp(acc, -e[j]);   // undo the column scaling (exact)
  Y[k + j * ldy] = acc;
}

// ------------------------------------------------------------------ Omega itself
// S[k + i lds] for k < s, i < m: one Philox block per thread (4 consecutive i).
// The sketch's S (unscaled) as binary64 values, S[k + i lds]: Box-Muller
// values for LS_FP64, the narrow formats' table entries otherwise.
__global__ __launch_bounds__(256) void k_omega(uint32_t key0, uint32_t key1, uint32_t prob,
                                               int64_t s, int64_t m, int fmt, const void* __restrict__ icdf,
                                               double* __restrict__ S, int64_t lds) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;   // index of 8 columns along m
  const int64_t k = blockIdx.y;
  if (8 * q >= m || k >= s) return;
  double z[8];
  if (fmt == LS_FP64) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint32_t c0 = (uint32_t)(2 * q + h), c1 = (uint32_t)k, c2 = prob, c3 = 0u;
      ls_philox4x32_10(c0, c1, c2, c3, key0, key1);
      ls_box_muller_f64(c0, c1, z[4 * h], z[4 * h + 1]);
      ls_box_muller_f64(c2, c3, z[4 * h + 2], z[4 * h + 3]);
    }
  } else {
    uint32_t c0 = (uint32_t)q, c1 = (uint32_t)k, c2 = prob, c3 = 2u;
    ls_philox4x32_10(c0, c1, c2, c3, key0, key1);
    const uint32_t w[4] = {c0, c1, c2, c3};
    for (int t = 0; t < 8; ++t) {
      const uint32_t U = (w[t / 2] >> (16 * (t % 2))) & 0xffffu;
      if (fmt == LS_FP8E4M3) {
        z[t] = sk_e4m3_at(sk_icdf8(static_cast<const uint8_t*>(icdf), U), 0);
      } else if (fmt == LS_FP16) {
        z[t] = sk_f16_at(sk_icdf16(static_cast<const uint16_t*>(icdf), U), 0);
      } else {
        z[t] = sk_bf16_at(sk_icdf16(static_cast<const uint16_t*>(icdf), U), 0);
      }
    }
  }
  for (int t = 0; t < 8; ++t) {
    const int64_t i = 8 * q + t;
    if (i < m) S[k + i * lds] = z[t];
  }
}

__global__ __launch_bounds__(256) void k_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1, int64_t count,
                                                uint32_t* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= count) return;
  uint32_t a = c0 + (uint32_t)t, b = c1, c = c2, d = c3;
  ls_philox4x32_10(a, b, c, d, k0, k1);
  out[4 * t + 0] = a;
  out[4 * t + 1] = b;
  out[4 * t + 2] = c;
  out[4 * t + 3] = d;
}

// ------------------------------------------------------------------ host side
namespace ls {

// Device address of the quantile table of a narrow format on the current
// device, filled on first use: the filling kernel runs on a stream of its
// own, which is synchronised before any sketch can read the table.
int icdf_table(int fmt, const void** out) {
  struct Tabs {
    bool ready = false;
    void* p[3] = {nullptr, nullptr, nullptr};
  };
  static std::mutex mu;
  static Tabs tabs[64];
  int dev = 0;
  LS_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return LS_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(mu);
  Tabs& t = tabs[dev];
  if (!t.ready) {
    LS_HIP_TRY(hipGetSymbolAddress(&t.p[0], HIP_SYMBOL(g_icdf_bf16)));
    LS_HIP_TRY(hipGetSymbolAddress(&t.p[1], HIP_SYMBOL(g_icdf_f16)));
    LS_HIP_TRY(hipGetSymbolAddress(&t.p[2], HIP_SYMBOL(g_icdf_e4m3)));
    hipStream_t st;
    LS_HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    hipLaunchKernelGGL(k_icdf_init, dim3(kIcdfHalf / 256), dim3(256), 0, st, (uint16_t*)t.p[0], (uint16_t*)t.p[1],
                       (uint8_t*)t.p[2]);
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipStreamSynchronize(st);
    const hipError_t e3 = hipStreamDestroy(st);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return LS_E_HIP;
    t.ready = true;
  }
  *out = (fmt == LS_BF16) ? t.p[0] : (fmt == LS_FP16) ? t.p[1] : t.p[2];
  return LS_OK;
}

static bool sk_narrow(ls_prec_t u) { return u == LS_BF16 || u == LS_FP16 || u == LS_FP8E4M3; }

// Launch shapes the planner can take (plan = index + 1).  Narrow formats:
// columns per block (0: the narrowest of 128 / 256 / 512 that holds n + 1)
// and the blocks the K-splits aim at, in 1/4 of the compute units.  Binary64:
// the blocks the K-splits aim at, in 1/4 of the compute units.  The first
// entry is the untuned rule; the tuned table picks per shape.
struct SkCand {
  int bn;
  int quarter_cus;
};
constexpr SkCand kNarrowCands[] = {{0, 4}, {0, 2}, {0, 1}, {0, 8}, {128, 4}, {256, 4}, {512, 4}};
constexpr SkCand kF64Cands[] = {{0, 8}, {0, 4}, {0, 16}, {0, 2}};
constexpr int kNarrowCandCount = (int)(sizeof(kNarrowCands) / sizeof(kNarrowCands[0]));
constexpr int kF64CandCount = (int)(sizeof(kF64Cands) / sizeof(kF64Cands[0]));

// Tuned choices: for each (format, parts) the first entry with n + 1 <=
// ncols_max and m <= m_max gives the plan (written by the package's
// autotune module from timings on the device).
struct SkTuned {
  int fmt, terms;
  int64_t ncols_max, m_max;
  int plan;
};
static const SkTuned kSkTuned[] = {
#include "sketch_tuned.inc"
    {-1, 0, 0, 0, 0}};

int sketch_plan_count(ls_prec_t u_s) {
  if (sk_narrow(u_s)) return kNarrowCandCount;
  if (u_s == LS_FP64) return kF64CandCount;
  return 0;
}

int sketch_plan_shape(ls_prec_t u_s, int plan, int* bn, int* quarter_cus) {
  if (plan < 1 || plan > sketch_plan_count(u_s)) return LS_E_ARG;
  const SkCand c = sk_narrow(u_s) ? kNarrowCands[plan - 1] : kF64Cands[plan - 1];
  *bn = c.bn;
  *quarter_cus = c.quarter_cus;
  return LS_OK;
}

static int sketch_tuned_plan(ls_prec_t u_s, int terms, int64_t ncols, int64_t m) {
  for (const SkTuned& t : kSkTuned) {
    if (t.fmt < 0) break;
    if (t.fmt == (int)u_s && t.terms == terms && ncols <= t.ncols_max && m <= t.m_max) {
      return (t.plan >= 1 && t.plan <= sketch_plan_count(u_s)) ? t.plan : 1;
    }
  }
  return 1;
}

// LDS of one block of k_sketch_lp: the 128 x 32 S tile and the parts' BN x 32
// operand tile, in fragments of 8 elements, and the quantile table.
static constexpr size_t sk_lds_bytes(int ebytes, int terms, int bn) {
  return (size_t)(kSkRows * 4 + terms * bn * 4) * (size_t)(8 * ebytes) + (size_t)kIcdfHalf * ebytes;
}

// Largest K-split, in 32-row K-blocks, for a terms-part sketch in u_s.
static int64_t sk_chunk_kblocks_max(ls_prec_t u_s, int terms) {
  const double u = (u_s == LS_BF16) ? 0x1p-8 : (u_s == LS_FP16) ? 0x1p-11 : 0x1p-4;
  const double us = std::pow(u, (double)terms);
  const double q = us / (4.0 * 0x1p-24);
  const double rows = 32.0 * q * q;
  if (rows >= 1e15) return (int64_t)1 << 40;
  return std::max<int64_t>(8192 / 32, (int64_t)(rows / 32.0));
}

SketchPlan sketch_plan(const ls_problem_t* P, const ls_sketch_opts_t* so, int64_t s, ls_prec_t u_s) {
  const int64_t m = P->m, n = P->n;
  const int terms = so->terms;
  SketchPlan p{};
  p.ncols = n + 1;
  if (so->zeta > 0) {   // sparse sign embedding: its workspace in place of the operand
    p.zeta = so->zeta;
    p.terms = 1;
    p.operand_bytes = ls_align256(sparse_workspace(m, n, so->zeta, s, (P->store == LS_FP64) ? 8 : 4));
    return p;
  }
  p.terms = sk_narrow(u_s) ? terms : 1;
  p.exp_bytes = ls_align256(4 * (size_t)p.ncols);
  int plan = (so->plan > 0) ? so->plan : sketch_tuned_plan(u_s, p.terms, p.ncols, m);
  if (plan > sketch_plan_count(u_s)) plan = 1;
  p.plan = plan;
  const int64_t target = (int64_t)device_cu_count() *
                         (sk_narrow(u_s) ? kNarrowCands[plan - 1].quarter_cus : kF64Cands[plan - 1].quarter_cus) / 4;
  if (sk_narrow(u_s)) {
    p.ebytes = (u_s == LS_FP8E4M3) ? 1 : 2;
    const int bn = kNarrowCands[plan - 1].bn;
    p.bn = bn ? bn : (p.ncols <= 128) ? 128 : (p.ncols <= 256) ? 256 : 512;
    // the automatic width stays at 256 columns where 512 would spill the
    // accumulators' registers (three or more 16-bit parts)
    if (!bn && p.ebytes == 2 && p.terms >= 3 && p.bn > 256) p.bn = 256;
    // the block's S tile and its parts' operand tile must fit in LDS
    const bool e4m3 = (u_s == LS_FP8E4M3);
    auto lds = [&](int w) { return e4m3 ? sk_e4m3_lds_bytes(p.terms, w) : sk_lds_bytes(p.ebytes, p.terms, w); };
    while (p.bn > 128 && lds(p.bn) > (size_t)device_lds_bytes()) p.bn /= 2;
    p.nn = ls_cdiv(p.ncols, p.bn);
    p.n_pad = p.nn * p.bn;
    p.ns = ls_cdiv(s, kSkRows);
    p.s_pad = p.ns * kSkRows;
    p.kstep = 32;
    // about `target` blocks; (column tiles x K-splits) a multiple of 8 so
    // that each XCD receives whole groups
    const int64_t kbn = ls_cdiv(m, 32);
    int64_t nsplit = ls_cdiv(target, p.ns * p.nn);
    // accuracy: each K-split sums its rows in binary32, one MFMA accumulation
    // per 32 rows, an error of about u32 sqrt(L / 32) relative to the sums for
    // L rows; splits of at most L_max = 32 (u_s / (4 u32))^2 rows (not below
    // 8192) keep it under a quarter of the parts' own accuracy u_s = u^terms
    const int64_t kb_max = sk_chunk_kblocks_max(u_s, p.terms);
    if (nsplit < ls_cdiv(kbn, kb_max)) nsplit = ls_cdiv(kbn, kb_max);
    if (nsplit > kbn) nsplit = kbn;
    if (nsplit < 1) nsplit = 1;
    while ((p.nn * nsplit) % 8) ++nsplit;
    p.kb_per_split = ls_cdiv(kbn, nsplit);
    if (e4m3) p.kb_per_split = ls_cdiv(p.kb_per_split, 2) * 2;   // whole 64-row steps
    p.nsplit = nsplit;
    p.nkb = p.kb_per_split * nsplit;
    p.m_pad = p.nkb * 32;
    p.kchunk = p.kb_per_split * 32;
    p.operand_bytes = ls_align256((size_t)p.terms * p.m_pad * p.n_pad * p.ebytes);
    p.partial_bytes = ls_align256((size_t)p.nsplit * p.s_pad * p.n_pad * 4);
    return p;
  }
  p.ebytes = 8;
  p.s_pad = ls_cdiv(s, 64) * 64;
  p.nb = 8;
  p.kstep = 16;
  p.n_pad = ls_cdiv(p.ncols, 16 * p.nb) * 16 * p.nb;
  // split K so that the grid holds about `target` blocks
  const int64_t tiles = (p.s_pad / 64) * (p.n_pad / (16 * p.nb));
  int64_t nsplit = ls_cdiv(target, tiles);
  const int64_t ksteps = ls_cdiv(m, p.kstep);
  if (nsplit > ksteps) nsplit = ksteps;
  if (nsplit < 1) nsplit = 1;
  if (nsplit > 64) nsplit = 64;
  p.kchunk = ls_cdiv(ksteps, nsplit) * p.kstep;
  p.nsplit = ls_cdiv(m, p.kchunk);
  if (p.nsplit < 1) p.nsplit = 1;
  p.m_pad = p.kchunk * p.nsplit;
  p.operand_bytes = ls_align256((size_t)p.m_pad * p.n_pad * 8);
  p.partial_bytes = ls_align256((size_t)p.nsplit * p.s_pad * p.n_pad * 8);
  return p;
}

namespace {
// Arguments of one k_sketch_lp launch.
template <typename E>
struct SkLaunchT {
  dim3 grid;
  hipStream_t st;
  ProfEv ev;
  const E* Tt;
  int64_t nkb, n_pad, kb_per_split;
  int ns, nn;
  uint32_t key0, key1, prob;
  const E* icdf;
  float* Yp;
  int64_t s_pad;
};

// Launch k_sketch_lp<FMT, BN, TERMS>; shapes whose tiles exceed the LDS of a
// compute unit are not instantiated (the planner narrows BN first).
template <int FMT, int BN, int TERMS>
int sk_launch(const SkLaunchT<typename SkFmt<FMT>::E>& L) {
  if constexpr (sk_lds_bytes(sizeof(typename SkFmt<FMT>::E), TERMS, BN) <= 160 * 1024) {
    hipExtLaunchKernelGGL((k_sketch_lp<FMT, BN, TERMS>), L.grid, dim3(kSkThreads), 0, L.st, L.ev.a, L.ev.b, 0, L.Tt,
                          L.nkb, L.n_pad, L.kb_per_split, L.ns, L.nn, L.key0, L.key1, L.prob, L.icdf, L.Yp,
                          L.s_pad);
    return LS_OK;
  } else {
    return LS_E_UNSUPPORTED;
  }
}

// Launch k_sketch_e4m3<BN, TERMS> (e4m3); shapes beyond the LDS are not instantiated.
template <int BN, int TERMS>
int sk_e4m3_launch(const SkLaunchT<uint8_t>& L) {
  if constexpr (sk_e4m3_lds_bytes(TERMS, BN) <= 160 * 1024) {
    hipExtLaunchKernelGGL((k_sketch_e4m3<BN, TERMS>), L.grid, dim3(kSkThreads), 0, L.st, L.ev.a, L.ev.b, 0, L.Tt, L.nkb,
                          L.n_pad, L.kb_per_split, L.ns, L.nn, L.key0, L.key1, L.prob, L.icdf, L.Yp, L.s_pad);
    return LS_OK;
  } else {
    return LS_E_UNSUPPORTED;
  }
}

template <int FMT, int BN>
int sk_launch_terms(const SkLaunchT<typename SkFmt<FMT>::E>& L, int terms) {
  if constexpr (FMT == LS_FP8E4M3) {
    switch (terms) {
      case 1: return sk_e4m3_launch<BN, 1>(L);
      case 2: return sk_e4m3_launch<BN, 2>(L);
      case 3: return sk_e4m3_launch<BN, 3>(L);
      case 4: return sk_e4m3_launch<BN, 4>(L);
      case 5: return sk_e4m3_launch<BN, 5>(L);
      default: return LS_E_ARG;
    }
  } else {
    switch (terms) {
      case 1: return sk_launch<FMT, BN, 1>(L);
      case 2: return sk_launch<FMT, BN, 2>(L);
      case 3: return sk_launch<FMT, BN, 3>(L);
      case 4: return sk_launch<FMT, BN, 4>(L);
      case 5: return sk_launch<FMT, BN, 5>(L);
      default: return LS_E_ARG;
    }
  }
}

// The operand of a narrow sketch: column exponents (column scaling) and the
// packed parts, in ws (operand, then partials, then exponents).
template <int FMT, typename TA>
void sk_prepare(const ls_problem_t* P, const SketchPlan& p, char* ws, bool colscale, hipStream_t st) {
  using F = SkFmt<FMT>;
  using E = typename F::E;
  E* Tt = reinterpret_cast<E*>(ws);
  int32_t* e = colscale ? reinterpret_cast<int32_t*>(ws + p.operand_bytes + p.partial_bytes) : nullptr;
  const TA* A = static_cast<const TA*>(P->A);
  const TA* b = static_cast<const TA*>(P->b);
  if (e)
    hipLaunchKernelGGL((k_colexp<TA>), dim3((unsigned)p.ncols), dim3(256), 0, st, A, P->lda, b, P->m, P->n,
                       F::fmt().fmax, e);
  hipLaunchKernelGGL((k_pack_lp<TA, FMT>), dim3((unsigned)(p.m_pad / 32), (unsigned)ls_cdiv(p.n_pad, 64)), dim3(256), 0, st,
                     A, P->lda, b, P->m, P->n, p.terms, e, Tt, p.m_pad, p.n_pad);
}

template <int FMT>
int sk_prepare_store(const ls_problem_t* P, const SketchPlan& p, char* ws, bool colscale, hipStream_t st) {
  if (P->store == LS_FP32) sk_prepare<FMT, float>(P, p, ws, colscale, st);
  else if (P->store == LS_FP64) sk_prepare<FMT, double>(P, p, ws, colscale, st);
  else return LS_E_UNSUPPORTED;
  return LS_OK;
}

// Y = the binary64 sum of the K-splits' partials, scaled by 1/sqrt(s) and
// 2^-e_j; the column exponents to so->col_exp when asked.
int sk_finish(const ls_problem_t* P, const ls_sketch_opts_t* so, const SketchPlan& p, int64_t s, double* Y,
              int64_t ldy, char* ws, bool colscale, hipStream_t st) {
  const float* Yp = reinterpret_cast<const float*>(ws + p.operand_bytes);
  const int32_t* e = colscale ? reinterpret_cast<const int32_t*>(ws + p.operand_bytes + p.partial_bytes) : nullptr;
  hipLaunchKernelGGL(k_sketch_combine<float>, dim3((unsigned)ls_cdiv(s, 256), (unsigned)p.ncols), dim3(256), 0, st, Yp,
                     p.s_pad, p.n_pad, (int)p.nsplit, s, p.ncols, 1.0 / sqrt((double)s), e, Y, ldy);
  LS_HIP_TRY(hipGetLastError());
  if (so->col_exp) {
    if (e)
      LS_HIP_TRY(hipMemcpyAsync(so->col_exp, e, 4 * (size_t)p.ncols, hipMemcpyDeviceToDevice, st));
    else
      LS_HIP_TRY(hipMemsetAsync(so->col_exp, 0, 4 * (size_t)p.ncols, st));
  }
  return LS_OK;
}

size_t sk_block_lds(int fmt, int terms, int bn) {
  return (fmt == LS_FP8E4M3) ? sk_e4m3_lds_bytes(terms, bn) : sk_lds_bytes(fmt == LS_BF16 || fmt == LS_FP16 ? 2 : 1, terms, bn);
}

template <int FMT, typename TA>
int sketch_narrow(const ls_problem_t* P, const ls_sketch_opts_t* so, const SketchPlan& p, int64_t s, double* Y,
                  int64_t ldy, char* ws, bool colscale, hipStream_t st) {
  using F = SkFmt<FMT>;
  using E = typename F::E;
  using SkLaunch = SkLaunchT<E>;
  const uint32_t key0 = (uint32_t)(so->seed & 0xffffffffu);
  const uint32_t key1 = (uint32_t)(so->seed >> 32);
  E* Tt = reinterpret_cast<E*>(ws);
  float* Yp = reinterpret_cast<float*>(ws + p.operand_bytes);
  if (sk_block_lds(FMT, p.terms, (int)p.bn) > (size_t)device_lds_bytes()) return LS_E_UNSUPPORTED;
  const E* icdf = nullptr;
  LS_TRY(icdf_table(FMT, reinterpret_cast<const void**>(&icdf)));
  sk_prepare<FMT, TA>(P, p, ws, colscale, st);
  const dim3 gb((unsigned)(p.ns * p.nn * p.nsplit));
  const ProfEv ev = prof_events(kProfSketch);
  const SkLaunch L{gb, st, ev, Tt, p.nkb, p.n_pad, p.kb_per_split, (int)p.ns, (int)p.nn, key0, key1, so->prob_id,
                  icdf, Yp, p.s_pad};
  int rc = LS_E_UNSUPPORTED;
  if (p.bn == 128) rc = sk_launch_terms<FMT, 128>(L, p.terms);
  else if (p.bn == 256) rc = sk_launch_terms<FMT, 256>(L, p.terms);
  else if (p.bn == 512) rc = sk_launch_terms<FMT, 512>(L, p.terms);
  LS_TRY(rc);
  prof_commit(kProfSketch, 2.0 * (double)s * (double)P->m * (double)(P->n + 1));
  return sk_finish(P, so, p, s, Y, ldy, ws, colscale, st);
}

// One grouped launch (problems of one tile width and part count).
template <int FMT, int TERMS>
int sk_grouped_launch_bn(int bn, unsigned blocks, hipStream_t st, const SkItem* items, int nitems, const void* icdf) {
  using E = typename SkFmt<FMT>::E;
  auto go = [&](auto bn_c) -> int {
    constexpr int BN = decltype(bn_c)::value;
    if constexpr (FMT == LS_FP8E4M3) {
      if constexpr (sk_e4m3_lds_bytes(TERMS, BN) <= 160 * 1024) {
        hipLaunchKernelGGL((k_sketch_e4m3_grouped<BN, TERMS>), dim3(blocks), dim3(kSkThreads), 0, st, items, nitems,
                           static_cast<const uint8_t*>(icdf));
        return LS_OK;
      }
    } else {
      if constexpr (sk_lds_bytes(sizeof(E), TERMS, BN) <= 160 * 1024) {
        hipLaunchKernelGGL((k_sketch_lp_grouped<FMT, BN, TERMS>), dim3(blocks), dim3(kSkThreads), 0, st, items,
                           nitems, static_cast<const E*>(icdf));
        return LS_OK;
      }
    }
    return LS_E_UNSUPPORTED;
  };
  if (bn == 128) return go(std::integral_constant<int, 128>{});
  if (bn == 256) return go(std::integral_constant<int, 256>{});
  if (bn == 512) return go(std::integral_constant<int, 512>{});
  return LS_E_UNSUPPORTED;
}

template <int FMT>
int sk_grouped_launch(int bn, int terms, unsigned blocks, hipStream_t st, const SkItem* items, int nitems,
                      const void* icdf) {
  switch (terms) {
    case 1: return sk_grouped_launch_bn<FMT, 1>(bn, blocks, st, items, nitems, icdf);
    case 2: return sk_grouped_launch_bn<FMT, 2>(bn, blocks, st, items, nitems, icdf);
    case 3: return sk_grouped_launch_bn<FMT, 3>(bn, blocks, st, items, nitems, icdf);
    case 4: return sk_grouped_launch_bn<FMT, 4>(bn, blocks, st, items, nitems, icdf);
    case 5: return sk_grouped_launch_bn<FMT, 5>(bn, blocks, st, items, nitems, icdf);
    default: return LS_E_ARG;
  }
}

template <int FMT>
int sketch_narrow_store(const ls_problem_t* P, const ls_sketch_opts_t* so, const SketchPlan& p, int64_t s, double* Y,
                        int64_t ldy, char* ws, bool colscale, hipStream_t st) {
  if (P->store == LS_FP32) return sketch_narrow<FMT, float>(P, so, p, s, Y, ldy, ws, colscale, st);
  if (P->store == LS_FP64) return sketch_narrow<FMT, double>(P, so, p, s, Y, ldy, ws, colscale, st);
  return LS_E_UNSUPPORTED;
}
}  // namespace

bool sketch_colscale(ls_prec_t u_s, int32_t col_scale) {
  if (col_scale < 0) return false;
  if (col_scale > 0) return sk_narrow(u_s);
  return u_s == LS_FP16 || u_s == LS_FP8E4M3;
}

int sketch_run(const ls_problem_t* P, const ls_sketch_opts_t* so, ls_prec_t u_s, const SketchPlan& p,
               int64_t s, double* Y, int64_t ldy, char* ws, hipStream_t st) {
  if (p.zeta > 0) {
    if (so->col_exp) LS_HIP_TRY(hipMemsetAsync(so->col_exp, 0, 4 * (size_t)(P->n + 1), st));
    return sparse_run(P, so, s, Y, ldy, ws, st);
  }
  if (p.terms < 1 || p.terms > kMaxSketchTerms) return LS_E_ARG;
  const bool cs = sketch_colscale(u_s, so->col_scale);
  if (u_s == LS_BF16) return sketch_narrow_store<LS_BF16>(P, so, p, s, Y, ldy, ws, cs, st);
  if (u_s == LS_FP16) return sketch_narrow_store<LS_FP16>(P, so, p, s, Y, ldy, ws, cs, st);
  if (u_s == LS_FP8E4M3) return sketch_narrow_store<LS_FP8E4M3>(P, so, p, s, Y, ldy, ws, cs, st);
  if (u_s != LS_FP64) return LS_E_UNSUPPORTED;
  const uint32_t key0 = (uint32_t)(so->seed & 0xffffffffu);
  const uint32_t key1 = (uint32_t)(so->seed >> 32);
  char* operand = ws;
  char* partial = ws + p.operand_bytes;
  const dim3 gpack((unsigned)ls_cdiv(p.m_pad, 256), (unsigned)p.n_pad);
  const dim3 gsk((unsigned)(p.s_pad / 64), (unsigned)(p.n_pad / (16 * p.nb)), (unsigned)p.nsplit);
  const dim3 gcomb((unsigned)ls_cdiv(s, 256), (unsigned)p.ncols);
  const double scale = 1.0 / sqrt((double)s);
  double* M = reinterpret_cast<double*>(operand);
  if (P->store == LS_FP64)
    hipLaunchKernelGGL(k_pack_f64<double>, gpack, dim3(256), 0, st, (const double*)P->A, P->lda,
                       (const double*)P->b, P->m, P->n, M, p.m_pad, p.n_pad);
  else
    hipLaunchKernelGGL(k_pack_f64<float>, gpack, dim3(256), 0, st, (const float*)P->A, P->lda,
                       (const float*)P->b, P->m, P->n, M, p.m_pad, p.n_pad);
  double* Yp = reinterpret_cast<double*>(partial);
  const ProfEv ev = prof_events(kProfSketch);
  hipExtLaunchKernelGGL((k_sketch_f64<8>), gsk, dim3(256), 0, st, ev.a, ev.b, 0, M, p.m_pad, p.n_pad, p.kchunk,
                        key0, key1, so->prob_id, Yp, p.s_pad);
  prof_commit(kProfSketch, 2.0 * (double)s * (double)P->m * (double)(P->n + 1));
  hipLaunchKernelGGL(k_sketch_combine<double>, gcomb, dim3(256), 0, st, Yp, p.s_pad, p.n_pad,
                     (int)p.nsplit, s, p.ncols, scale, (const int32_t*)nullptr, Y, ldy);
  LS_HIP_TRY(hipGetLastError());
  if (so->col_exp) LS_HIP_TRY(hipMemsetAsync(so->col_exp, 0, 4 * (size_t)p.ncols, st));
  return LS_OK;
}

bool sketch_groupable(const ls_sketch_opts_t* so, ls_prec_t u_s) {
  return sk_narrow(u_s) && so->zeta == 0 && so->terms >= 1 && so->terms <= kMaxSketchTerms;
}

size_t sketch_grouped_bytes(const ls_problem_t* P, const ls_sketch_opts_t* so, ls_prec_t u_s, int64_t s) {
  const SketchPlan p = sketch_plan(P, so, s, u_s);
  return p.operand_bytes + p.partial_bytes + p.exp_bytes;
}

size_t sketch_grouped_items_bytes(int nprob) { return ls_align256(sizeof(SkItem) * (size_t)nprob); }

int sketch_grouped(int nprob, const ls_problem_t* P, const ls_sketch_opts_t* so, ls_prec_t u_s, const int64_t* s,
                   double* const* Y, char* const* ws, void* items_dev, hipStream_t st) {
  std::vector<SketchPlan> pl((size_t)nprob);
  for (int i = 0; i < nprob; ++i) {
    if (!sketch_groupable(&so[i], u_s)) return LS_E_UNSUPPORTED;
    pl[i] = sketch_plan(&P[i], &so[i], s[i], u_s);
    if (sk_block_lds(u_s, pl[i].terms, (int)pl[i].bn) > (size_t)device_lds_bytes()) return LS_E_UNSUPPORTED;
  }
  const void* icdf = nullptr;
  LS_TRY(icdf_table(u_s, &icdf));
  // groups of one tile width and part count; within a group each problem's
  // blocks follow the previous problem's (its block count is a multiple of 8)
  std::vector<int> order((size_t)nprob);
  for (int i = 0; i < nprob; ++i) order[i] = i;
  auto key = [&](int i) { return pl[i].bn * 16 + pl[i].terms; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
  std::vector<SkItem> items((size_t)nprob);
  struct Group {
    int first, count, bn, terms;
    int64_t blocks;
  };
  std::vector<Group> groups;
  for (int k = 0; k < nprob; ++k) {
    const int i = order[k];
    const SketchPlan& p = pl[i];
    if (groups.empty() || key(order[groups.back().first]) != key(i))
      groups.push_back(Group{k, 0, (int)p.bn, p.terms, 0});
    Group& g = groups.back();
    SkItem& it = items[k];
    it.Tt = ws[i];
    it.Yp = reinterpret_cast<float*>(ws[i] + p.operand_bytes);
    it.nkb = p.nkb;
    it.n_pad = p.n_pad;
    it.kb_per_split = p.kb_per_split;
    it.s_pad = p.s_pad;
    it.ns = (int)p.ns;
    it.nn = (int)p.nn;
    it.key0 = (uint32_t)(so[i].seed & 0xffffffffu);
    it.key1 = (uint32_t)(so[i].seed >> 32);
    it.prob = so[i].prob_id;
    it.block0 = (int)g.blocks;
    g.blocks += p.ns * p.nn * p.nsplit;
    ++g.count;
    if (g.blocks > INT32_MAX) return LS_E_UNSUPPORTED;
  }
  // the work list to the device (the host copy is released after the copy)
  LS_HIP_TRY(hipMemcpyAsync(items_dev, items.data(), sizeof(SkItem) * items.size(), hipMemcpyHostToDevice, st));
  LS_HIP_TRY(hipStreamSynchronize(st));
  for (int i = 0; i < nprob; ++i) {
    const bool cs = sketch_colscale(u_s, so[i].col_scale);
    char* w = ws[i];
    if (u_s == LS_BF16) LS_TRY(sk_prepare_store<LS_BF16>(&P[i], pl[i], w, cs, st));
    else if (u_s == LS_FP16) LS_TRY(sk_prepare_store<LS_FP16>(&P[i], pl[i], w, cs, st));
    else LS_TRY(sk_prepare_store<LS_FP8E4M3>(&P[i], pl[i], w, cs, st));
  }
  const SkItem* dev = static_cast<const SkItem*>(items_dev);
  for (const Group& g : groups) {
    const unsigned blocks = (unsigned)g.blocks;
    if (u_s == LS_BF16) LS_TRY(sk_grouped_launch<LS_BF16>(g.bn, g.terms, blocks, st, dev + g.first, g.count, icdf));
    else if (u_s == LS_FP16) LS_TRY(sk_grouped_launch<LS_FP16>(g.bn, g.terms, blocks, st, dev + g.first, g.count, icdf));
    else LS_TRY(sk_grouped_launch<LS_FP8E4M3>(g.bn, g.terms, blocks, st, dev + g.first, g.count, icdf));
  }
  for (int i = 0; i < nprob; ++i)
    LS_TRY(sk_finish(&P[i], &so[i], pl[i], s[i], Y[i], s[i], ws[i], sketch_colscale(u_s, so[i].col_scale), st));
  return LS_OK;
}

int omega_run(uint64_t seed, uint32_t prob, int64_t s, int64_t m, ls_prec_t fmt, double* S, int64_t lds,
              hipStream_t st) {
  const void* icdf = nullptr;
  if (fmt != LS_FP64) LS_TRY(icdf_table((int)fmt, &icdf));
  const dim3 g((unsigned)ls_cdiv(ls_cdiv(m, 8), 256), (unsigned)s);
  hipLaunchKernelGGL(k_omega, g, dim3(256), 0, st, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32),
                     prob, s, m, (int)fmt, icdf, S, lds);
  LS_HIP_TRY(hipGetLastError());
  return LS_OK;
}

int philox_run(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1, int64_t count,
               uint32_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_philox, dim3((unsigned)ls_cdiv(count, 256)), dim3(256), 0, st, c0, c1, c2, c3, k0, k1,
                     count, out);
  LS_HIP_TRY(hipGetLastError());
  return LS_OK;
}

}  // namespace ls
