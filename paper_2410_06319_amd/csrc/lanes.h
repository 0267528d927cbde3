// Cross-lane sums within a 64-lane wave on gfx950 without LDS traffic:
// permlane swaps for lane bits 5 and 4, DPP for the bits below.
#pragma once
#include <type_traits>
#include <utility>

#include <hip/hip_runtime.h>

namespace {

// Sum each of v[0..NB) over the 64 lanes of a wave with a transposed
// butterfly: after it, the returned value is the full sum of index `idx`.
// The loops run over a compile-time step count so that every register index
// is a constant after unrolling.
template <int NB>
struct Log2 {
  static constexpr int value = (NB <= 1) ? 0 : 1 + Log2<NB / 2>::value;
};
template <>
struct Log2<1> {
  static constexpr int value = 0;
};

// f(std::integral_constant<int, 0>{}), ..., f(std::integral_constant<int, N - 1>{}):
// an unrolled loop whose index is a compile-time constant in every copy.
template <typename F, int... C>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, C...>) {
  (f(std::integral_constant<int, C>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Cross-lane moves within a wave without LDS.  v_permlane32_swap(x, y)
// returns {x on lanes 0..31 with y's lanes 0..31 on lanes 32..63, x's lanes
// 32..63 on lanes 0..31 with y on lanes 32..63}; v_permlane16_swap does the
// same for the 16-lane halves of each 32-lane half.  DPP row_ror:8 reads lane
// l ^ 8, row_half_mirror lane l ^ 7, quad_perm [2,3,0,1] and [1,0,3,2] lanes
// l ^ 2 and l ^ 1 (all within rows of 16 lanes).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f(double x) {
  const long long u = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// r0 + r1 of the 32- or 16-lane swap of (a, b): on lanes with the bit clear
// a summed with its partner's a, on the others b summed with its partner's b.
template <int BIT>
__device__ __forceinline__ float swap_add(float a, float b) {
  const unsigned int ua = __builtin_bit_cast(unsigned int, a), ub = __builtin_bit_cast(unsigned int, b);
  const auto r = (BIT == 5) ? __builtin_amdgcn_permlane32_swap(ua, ub, false, false)
                            : __builtin_amdgcn_permlane16_swap(ua, ub, false, false);
  return __builtin_bit_cast(float, (unsigned int)r[0]) + __builtin_bit_cast(float, (unsigned int)r[1]);
}
template <int BIT>
__device__ __forceinline__ double swap_add(double a, double b) {
  const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
  const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
  const unsigned int alo = (unsigned int)ua, ahi = (unsigned int)(ua >> 32);
  const unsigned int blo = (unsigned int)ub, bhi = (unsigned int)(ub >> 32);
  const auto rl = (BIT == 5) ? __builtin_amdgcn_permlane32_swap(alo, blo, false, false)
                             : __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
  const auto rh = (BIT == 5) ? __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false)
                             : __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
  const double r0 = __builtin_bit_cast(double, ((unsigned long long)(unsigned int)rh[0] << 32) | (unsigned int)rl[0]);
  const double r1 = __builtin_bit_cast(double, ((unsigned long long)(unsigned int)rh[1] << 32) | (unsigned int)rl[1]);
  return r0 + r1;
}
// DPP control of the partner lane for a lane bit below 4 (xor 8, xor 7, xor 2, xor 1).
template <int BIT>
struct DppCtrl {
  static constexpr int value = (BIT == 3) ? 0x128 : (BIT == 2) ? 0x141 : (BIT == 1) ? 0x4E : 0xB1;
};

// Sum each of v[0..NB) over the 64 lanes of a wave with a transposed
// butterfly: the halving steps pair lanes that differ in bit 5, 4, 3, then
// (through the 8-lane mirror) bit 2; the kept half follows the lane's bit,
// so lane l ends with index idx = its bits 5.. as a binary number.  The
// remaining low bits are plain sums.  Every pairing is an exchange between
// the two lanes, so both see the same two addends.
template <typename T, int NB>
__device__ __forceinline__ T wave_multi_sum(T (&v)[NB], int lane, int& idx) {
  constexpr int L = Log2<NB>::value;
  static_assert(L <= 4, "at most 16 values");
  int base = 0;
  static_for<L>([&](auto stc) {
    constexpr int step = decltype(stc)::value;
    constexpr int bit = 5 - step;
    constexpr int h = NB >> (step + 1);
    const bool up = ((lane >> bit) & 1) != 0;
    if constexpr (bit >= 4) {
#pragma unroll
      for (int q = 0; q < h; ++q) v[q] = swap_add<bit>(v[q], v[q + h]);
    } else {
      // exact blend (factors 1 and 0) rather than a select, which the compiler
      // would turn into a run-time register index
      const T fu = up ? T(1) : T(0);
      const T fl = T(1) - fu;
#pragma unroll
      for (int q = 0; q < h; ++q) {
        const T send = v[q] * fu + v[q + h] * fl;
        const T keep = v[q + h] * fu + v[q] * fl;
        v[q] = keep + dpp_f<DppCtrl<bit>::value>(send);
      }
    }
    if (up) base += h;
  });
  T s = v[0];
  static_for<6 - L>([&](auto stc) {
    constexpr int bit = 5 - L - decltype(stc)::value;
    if constexpr (bit >= 4) s = swap_add<bit>(s, s);
    else s = s + dpp_f<DppCtrl<bit>::value>(s);
  });
  idx = base;
  return s;
}

}  // namespace
