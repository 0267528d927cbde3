// Algorithm 1, the QR: economic Householder QR of the sketch, R factor only,
// plus the explicit inverse R^-1 used to apply the preconditioner.
//
// Blocked right-looking Householder QR (compact WY, LAPACK's forward
// column-wise convention H = I - V T V^T):
//   * a panel of NB columns is factored by one 512-thread block that keeps
//     the panel in registers (RPT rows per thread), with one block-wide
//     reduction per column, and forms T from the stored inner products after
//     the column loop;
//   * trailing columns are updated as C <- C - V (T^T (V^T C)) on MFMA
//     straight from registers, 16 columns per block;
//   * one launch per panel with look-ahead: while block 0 updates and
//     factors the next panel, the other blocks update the rest.
// Reflectors follow the usual choice beta = -sign(x_1) ||x||; at the end
// the rows of R are multiplied by the signs of its diagonal so diag(R) > 0.
#include <type_traits>
#include <utility>

#include "common.h"
#include "kernels.h"
#include "lanes.h"

typedef float ls_qr_f4 __attribute__((ext_vector_type(4)));
typedef double ls_qr_d4 __attribute__((ext_vector_type(4)));
typedef double ls_qr_d2 __attribute__((ext_vector_type(2)));

namespace {

constexpr int kQrThreads = 512;      // block size of the QR kernels
constexpr int kPanelThreads = 512;   // threads that hold the panel (all of the block)


// Panel factorisation with one block reduction per column.  For column c
// with x = its rows li >= c (x0 = row c), one reduction gives
//   d[c] = sum_{li > c} x_li^2  and  d[q] = sum_{li > c} P(li, q) x_li  (q != c);
// with row c of the panel broadcast through LDS this is everything the step
// needs: beta = -sign(x0) sqrt(x0^2 + d[c]), tau = (beta - x0) / beta,
// v = [1; x_{>c} / (x0 - beta)], and since v(li) = x_li scal below row c,
//   v . y_b = y_b(c) + scal d[b]   (later columns b > c),
//   v_a . v = v_a(c) + scal d[a]   (earlier reflectors a < c, for T).
// The kPanelThreads panel threads hold RPT consecutive rows each (li =
// RPT tid + r), read and written as 16-byte vectors; Y is the internal
// working copy, whose leading dimension is a multiple of 4 with zero rows
// between s and ldy.
template <typename T>
struct QrVec;
template <>
struct QrVec<float> {
  using type = ls_qr_f4;
  static constexpr int W = 4;
};
template <>
struct QrVec<double> {
  using type = ls_qr_d2;
  static constexpr int W = 2;
};

// Value of lane `src` (a constant after unrolling) on every lane of the wave.
__device__ __forceinline__ float qr_bcast(float v, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}
__device__ __forceinline__ double qr_bcast(double v, int src) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float qr_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double qr_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float qr_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double qr_rcp(double x) { return 1.0 / x; }

template <typename T, int RPT, int NB>
__device__ __forceinline__ void qr_panel_body(T* __restrict__ Y, int64_t ldy, int64_t s, int64_t j0, int nb,
                                              T* __restrict__ tau, T* __restrict__ Tm) {
  constexpr int PW = kPanelThreads / 64;
  using vec_t = typename QrVec<T>::type;
  constexpr int VW = QrVec<T>::W;
  static_assert(RPT % VW == 0, "rows per thread must fill whole vectors");
  __shared__ __align__(16) T red[2][PW][NB];   // wave partials, by column parity
  __shared__ T rowc[2][NB];                    // row c of the panel, by column parity
  __shared__ T Gs[NB][NB];                     // Gs[c][b] = v_b . v_c (b < c)
  __shared__ T taus[NB];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const bool act = tid < kPanelThreads;
  constexpr int lowmask = 64 / NB - 1;
  const int64_t i0 = j0 + (int64_t)RPT * tid;   // first row of this thread

  T P[RPT][NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
#pragma unroll
    for (int r = 0; r < RPT; r += VW) {
      vec_t v{};
      if (act && c < nb && i0 + r < ldy) v = *reinterpret_cast<const vec_t*>(Y + (i0 + r) + (j0 + c) * ldy);
#pragma unroll
      for (int e = 0; e < VW; ++e) P[r + e][c] = v[e];
    }
  }

  static_for<NB>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    constexpr int cown = c / RPT, cslot = c % RPT;   // thread and slot holding row c
    if (c < nb) {
      const int par = c & 1;
      if (act) {
        T part[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) part[q] = 0;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
          const int li = RPT * tid + r;
          if (li > c) {
            const T x = P[r][c];
#pragma unroll
            for (int q = 0; q < NB; ++q) part[q] += P[r][q] * x;
          }
        }
        if (tid == cown) {
#pragma unroll
          for (int q = 0; q < NB; ++q) rowc[par][q] = P[cslot][q];
        }
        int idx;
        const T wsum = wave_multi_sum<T, NB>(part, lane, idx);
        if ((lane & lowmask) == 0) red[par][wv][idx] = wsum;
      }
      __syncthreads();
      if (act) {
        // lane q (mod NB) of each wave adds the wave partials of index q, in
        // wave order, and reads entry q of row c; the values then reach every
        // lane by cross-lane reads (one LDS read per lane instead of all of
        // the partials on every thread)
        const int lq = lane % NB;
        T mine = red[par][0][lq];
#pragma unroll
        for (int w = 1; w < PW; ++w) mine += red[par][w][lq];
        const T rmine = rowc[par][lq];
        T dots[NB], rc[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          dots[q] = qr_bcast(mine, q);
          rc[q] = qr_bcast(rmine, q);
        }
        const T ss = dots[c];
        const T x0 = rc[c];
        T beta, tauc, scal;
        if (ss == T(0)) {
          tauc = 0;
          beta = x0;
          scal = 0;
        } else {
          const T nrm = qr_sqrt(x0 * x0 + ss);
          beta = (x0 >= T(0)) ? -nrm : nrm;
          tauc = (beta - x0) * qr_rcp(beta);
          scal = qr_rcp(x0 - beta);
        }
        // inner products with the earlier reflectors, for T after the loop
        if (tid < c) Gs[c][tid] = rmine + scal * mine;
        if (tid == 0) {
          tau[j0 + c] = tauc;
          taus[c] = tauc;
        }
        // v_c in place of x, then H_c applied to the later panel columns
        T coef[NB];
#pragma unroll
        for (int bq = c + 1; bq < NB; ++bq) coef[bq] = tauc * (rc[bq] + scal * dots[bq]);
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
          const int li = RPT * tid + r;
          if (li > c) P[r][c] *= scal;
          if (li >= c) {
            const T vc = (li == c) ? T(1) : P[r][c];
#pragma unroll
            for (int bq = c + 1; bq < NB; ++bq) P[r][bq] -= coef[bq] * vc;
          }
        }
        if (tid == cown) P[cslot][c] = beta;
      }
    }
  });
  if (act) {
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c < nb) {
#pragma unroll
        for (int r = 0; r < RPT; r += VW) {
          if (i0 + r < ldy) {
            vec_t v;
#pragma unroll
            for (int e = 0; e < VW; ++e) v[e] = P[r + e][c];
            *reinterpret_cast<vec_t*>(Y + (i0 + r) + (j0 + c) * ldy) = v;
          }
        }
      }
    }
  }
  __syncthreads();
  // T (upper triangular, H_0 ... H_{nb-1} = I - V T V^T): lane a of wave 0
  // computes row a, T(a, a) = tau_a and, for c > a,
  // T(a, c) = -tau_c sum_{b = a}^{c-1} T(a, b) (v_b . v_c); row a needs only itself.
  if (tid < NB) {
    const int a = tid;
    T row[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      T v = 0;
      if (c < nb && a < nb) {
        if (c == a) {
          v = taus[c];
        } else if (c > a) {
          T acc = 0;
#pragma unroll
          for (int bq = 0; bq < NB; ++bq)
            if (bq >= a && bq < c) acc += row[bq] * Gs[c][bq];
          v = -taus[c] * acc;
        }
      }
      row[c] = v;
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) Tm[a + c * NB] = row[c];
  }
}

template <typename T, int RPT, int NB>
__global__ __launch_bounds__(kQrThreads) void k_qr_panel(T* __restrict__ Y, int64_t ldy, int64_t s, int64_t j0,
                                                          int nb, T* __restrict__ tau, T* __restrict__ Tm) {
  qr_panel_body<T, RPT, NB>(Y, ldy, s, j0, nb, tau, Tm);
}

__device__ __forceinline__ ls_qr_f4 qr_mfma(float a, float b, ls_qr_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ ls_qr_d4 qr_mfma(double a, double b, ls_qr_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Row of the 16 x 16 MFMA result held in slot r of lane l (binary32 rows are
// blocked, binary64 rows interleaved); the column is l % 16.
template <typename T>
__device__ __forceinline__ int qr_drow(int lane, int r) {
  return (sizeof(T) == 4) ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r;
}

// Apply the nb0 reflectors of the panel starting at j0 (V unit lower
// trapezoidal below row j0, T upper triangular, Tm[a + c NB] = T(a, c)) to the
// cw <= 16 columns c0.. of Y: C <- C - V (T^T (V^T C)).  One block of
// kQrThreads threads; both products on MFMA 16x16x4 straight from registers.
//   W = V^T C: lane l (column l % 16, row group l / 16) loads VW consecutive
//   rows of its column of V and of C as one vector; product step e pairs row
//   e of every lane's vector, so the K index of the MFMA runs over the same
//   rows for both operands.  Wave w takes the row groups w, w + 8, ... (8 in
//   flight); the wave partials are added in wave order through LDS.
//   W2 = T^T W.
//   C <- C - V W2 by 16-row tiles (wave w: tiles w, w + 8, ...): lane l reads
//   V(row l % 16, columns 4q + l / 16) for the A operand, and the rows of C
//   that the MFMA result places in lane l (4 consecutive rows for binary32).
// Rows from s up to ldy are zero in the working copy and stay zero.
template <typename T, int NB>
__device__ __forceinline__ void qr_update16(T* __restrict__ Y, int64_t ldy, int64_t s, int64_t j0, int nb0,
                                            const T* __restrict__ Tm, int64_t c0, int cw) {
  using acc_t = typename std::conditional<sizeof(T) == 4, ls_qr_f4, ls_qr_d4>::type;
  using vec_t = typename QrVec<T>::type;
  constexpr int VW = QrVec<T>::W;
  constexpr int NW = kQrThreads / 64;
  constexpr int GR = 4 * VW;   // rows of one row group (4 lane groups x VW)
  constexpr int UG = 8;        // row groups in flight per wave
  constexpr int UT = 4;        // 16-row tiles in flight per wave
  __shared__ T part[NW][16][17];
  __shared__ T Ws[16][17];
  __shared__ T W2s[16][17];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int cl = lane & 15;
  const int kq = lane >> 4;
  const bool vok = cl < nb0;
  const bool cok = cl < cw;
  const int64_t vcol = j0 + cl;                       // this lane's column of V (if vok)
  const T* __restrict__ Vc = Y + (vok ? vcol : j0) * ldy;
  T* __restrict__ Cc = Y + (c0 + (cok ? cl : 0)) * ldy;
  const int64_t rows = s - j0;

  // W = V^T C
  const int64_t ng = ls_cdiv(rows, GR);
  acc_t acc = acc_t{0, 0, 0, 0};
  for (int64_t g0 = wave; g0 < ng; g0 += (int64_t)NW * UG) {
    vec_t va[UG], ca[UG];
#pragma unroll
    for (int u = 0; u < UG; ++u) {
      const int64_t g = g0 + (int64_t)NW * u;
      const int64_t rs = j0 + GR * g + VW * kq;
      const bool in = g < ng && rs < ldy;
      va[u] = (in && vok) ? *reinterpret_cast<const vec_t*>(Vc + rs) : vec_t{};
      ca[u] = (in && cok) ? *reinterpret_cast<const vec_t*>(Cc + rs) : vec_t{};
    }
#pragma unroll
    for (int u = 0; u < UG; ++u) {
      const int64_t rs = j0 + GR * (g0 + (int64_t)NW * u) + VW * kq;
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const int64_t i = rs + e;
        const T v = !vok ? T(0) : ((i > vcol) ? va[u][e] : ((i == vcol) ? T(1) : T(0)));
        acc = qr_mfma(v, ca[u][e], acc);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) part[wave][qr_drow<T>(lane, r)][cl] = acc[r];
  __syncthreads();
  if (tid < 256) {
    const int a = tid >> 4, c = tid & 15;
    T w = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) w += part[q][a][c];
    Ws[a][c] = w;
  }
  __syncthreads();
  if (tid < 256) {
    const int a = tid >> 4, c = tid & 15;
    T w2 = 0;
    if (a < nb0)
      for (int q = 0; q <= a; ++q) w2 += Tm[q + a * NB] * Ws[q][c];
    W2s[a][c] = w2;
  }
  __syncthreads();

  // C <- C - V W2
  T wb[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) wb[q] = W2s[4 * q + kq][cl];
  const int64_t nt = ls_cdiv(rows, 16);
  for (int64_t t0 = wave; t0 < nt; t0 += (int64_t)NW * UT) {
    T av[UT][4], cv[UT][4];
#pragma unroll
    for (int u = 0; u < UT; ++u) {
      const int64_t r0 = j0 + 16 * (t0 + (int64_t)NW * u);
      const bool tin = t0 + (int64_t)NW * u < nt;
      const int64_t i = r0 + cl;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = 4 * q + kq;
        const int64_t d = j0 + k;
        T v = 0;
        if (tin && k < nb0 && i < ldy) v = (i > d) ? Y[i + d * ldy] : ((i == d) ? T(1) : T(0));
        av[u][q] = v;
      }
      if constexpr (sizeof(T) == 4) {
        const int64_t rc = r0 + 4 * kq;
        vec_t c4 = vec_t{};
        if (tin && cok && rc < ldy) c4 = *reinterpret_cast<const vec_t*>(Cc + rc);
#pragma unroll
        for (int r = 0; r < 4; ++r) cv[u][r] = c4[r];
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t ir = r0 + qr_drow<T>(lane, r);
          cv[u][r] = (tin && cok && ir < ldy) ? Cc[ir] : T(0);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < UT; ++u) {
      const int64_t r0 = j0 + 16 * (t0 + (int64_t)NW * u);
      const bool tin = t0 + (int64_t)NW * u < nt;
      acc_t d = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < 4; ++q) d = qr_mfma(av[u][q], wb[q], d);
      if (tin && cok) {
        if constexpr (sizeof(T) == 4) {
          const int64_t rc = r0 + 4 * kq;
          if (rc < ldy) {
            vec_t c4;
#pragma unroll
            for (int r = 0; r < 4; ++r) c4[r] = cv[u][r] - d[r];
            *reinterpret_cast<vec_t*>(Cc + rc) = c4;
          }
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t ir = r0 + qr_drow<T>(lane, r);
            if (ir < ldy) Cc[ir] = cv[u][r] - d[r];
          }
        }
      }
    }
  }
}

// One step of the blocked factorisation with look-ahead.  The panel at j0
// (nb0 columns, T in Tprev) is factored already.  Block 0 applies it to the
// next panel (columns j1 .. j1 + nb1 - 1) and factors that panel (T into
// Tnext); blocks b >= 1 apply it to the 16 columns jt + 16 (b - 1) .. of the
// trailing matrix, which the next panel's reflectors reach in the next step.

template <typename T, int RPT, int NB>
__global__ __launch_bounds__(kQrThreads) void k_qr_step(T* __restrict__ Y, int64_t ldy, int64_t s, int64_t ncols,
                                                         int64_t j0, int nb0, const T* __restrict__ Tprev,
                                                         int64_t j1, int nb1, T* __restrict__ tau,
                                                         T* __restrict__ Tnext, int64_t jt) {
  if (blockIdx.x == 0) {
    qr_update16<T, NB>(Y, ldy, s, j0, nb0, Tprev, j1, nb1);
    __syncthreads();   // the next panel's updated columns are read back below
    qr_panel_body<T, RPT, NB>(Y, ldy, s, j1, nb1, tau, Tnext);
  } else {
    const int64_t c0 = jt + 16 * (int64_t)(blockIdx.x - 1);
    const int cw = (int)((ncols - c0 < 16) ? ncols - c0 : 16);
    qr_update16<T, NB>(Y, ldy, s, j0, nb0, Tprev, c0, cw);
  }
}

// Z(0:rows, 0:cols) = X, rows >= valid set to zero.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_copy_cols(const TI* __restrict__ X, int64_t ldx, TO* __restrict__ Z,
                                                   int64_t ldz, int64_t rows, int64_t valid, int64_t cols) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i < rows && j < cols) Z[i + j * ldz] = (i < valid) ? (TO)X[i + j * ldx] : TO(0);
}

// R = diag(sign(diag)) * triu(Y(0:ncols, 0:ncols)); flags a zero or non-finite
// diagonal entry among the first check_cols.
template <typename T>
__global__ __launch_bounds__(256) void k_qr_finish(const T* __restrict__ Y, int64_t ldy, int64_t ncols,
                                                   int64_t check_cols, double* __restrict__ R, int64_t ldr,
                                                   int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= ncols || j >= ncols) return;
  const double d = (double)Y[i + i * ldy];
  const double sg = (d < 0.0) ? -1.0 : 1.0;
  R[i + j * ldr] = (i <= j) ? sg * (double)Y[i + j * ldy] : 0.0;
  // bit 0: a zero diagonal entry (rank deficient), bit 1: a non-finite one
  // (NaN or Inf reached the sketch)
  if (i == j && i < check_cols) {
    if (!isfinite(d))
      atomicOr(flag, 2);
    else if (d == 0.0)
      atomicOr(flag, 1);
  }
}

// W = R^-1, one block per column j: back substitution R w = e_j in binary64,
// rows taken in chunks of 64 from the diagonal up.  Wave 0 solves a chunk's
// triangle with one row per lane (the chunk's rows of R in registers, each
// solved entry broadcast from its lane through a scalar register, the
// diagonal applied as a precomputed reciprocal); then every thread subtracts
// the chunk's contribution from the rows above it.  With fro != nullptr the
// block also stores fro[2j] = ||W[:, j]||^2 and fro[2j+1] = ||R[0:j+1, j]||^2.
__device__ __forceinline__ double trinv_bcast(double v, int lane) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__global__ __launch_bounds__(256) void k_trinv(const double* __restrict__ R, int64_t ldr, int64_t n,
                                               double* __restrict__ W, int64_t ldw, int* __restrict__ flag,
                                               double* __restrict__ fro) {
  extern __shared__ double bsh[];
  __shared__ double red[4];
  const int64_t j = blockIdx.x;
  const int t = threadIdx.x;
  const int lane = t & 63;
  double wsq = 0.0;   // wave 0: squares of the solved entries of its lanes
  for (int64_t i = t; i <= j; i += 256) bsh[i] = (i == j) ? 1.0 : 0.0;
  for (int64_t i = j + 1 + t; i < n; i += 256) W[i + j * ldw] = 0.0;
  for (int64_t c0 = (j / 64) * 64; c0 >= 0; c0 -= 64) {
    const int cn = (int)((j + 1 - c0 < 64) ? j + 1 - c0 : 64);   // rows c0 .. c0 + cn - 1
    __syncthreads();
    if (t < 64) {
      const int64_t i = c0 + lane;
      const bool act = lane < cn;
      double rrow[64];
#pragma unroll
      for (int kk = 0; kk < 64; ++kk) rrow[kk] = (act && kk < cn && kk >= lane) ? R[i + (c0 + kk) * ldr] : 0.0;
      double bi = act ? bsh[i] : 0.0;
      const double rinv = act ? 1.0 / R[i + i * ldr] : 0.0;
#pragma unroll
      for (int kk = 63; kk >= 0; --kk) {
        if (kk < cn) {
          const double wk = trinv_bcast(bi * rinv, kk);
          if (lane == kk) bi = wk;
          else if (lane < kk) bi -= rrow[kk] * wk;
        }
      }
      if (act) {
        bsh[i] = bi;
        W[i + j * ldw] = bi;
        wsq += bi * bi;
        if (!isfinite(bi)) atomicOr(flag, 1);
      }
    }
    __syncthreads();
    // rows above the chunk: b_i -= sum_kk R(i, c0 + kk) w(c0 + kk)
    for (int64_t i = t; i < c0; i += 256) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int kb = 0; kb < cn; kb += 16) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = (kb + q < cn) ? R[i + (c0 + kb + q) * ldr] : 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q & 3] += v[q] * ((kb + q < cn) ? bsh[c0 + kb + q] : 0.0);
      }
      bsh[i] -= (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
  }
  if (fro) {
    double rsq = 0.0;
    for (int64_t i = t; i <= j; i += 256) {
      const double v = R[i + j * ldr];
      rsq += v * v;
    }
    const double rs = ls_block_sum<double, 256>(rsq, red);
    const double ws = ls_wave_sum(wsq);   // nonzero in wave 0 only
    if (t == 0) {
      fro[2 * j] = ws;
      fro[2 * j + 1] = rs;
    }
  }
}

__global__ __launch_bounds__(256) void k_to_f32(const double* __restrict__ W, int64_t ldw, int64_t n,
                                                float* __restrict__ W32) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i < n && j < n) W32[i + j * n] = (float)W[i + j * ldw];
}

// Wt = W^T (n x n, ld n), 32 x 32 tiles through LDS: coalesced reads and writes.
__global__ __launch_bounds__(256) void k_transpose_f64(const double* __restrict__ W, int64_t ldw, int64_t n,
                                                       double* __restrict__ Wt) {
  __shared__ double tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 8 rows of threads
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + tx, j = j0 + r;
    tile[r][tx] = (i < n && j < n) ? W[i + j * ldw] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = j0 + tx, i = i0 + r;
    if (i < n && j < n) Wt[j + i * n] = tile[tx][r];
  }
}

template <typename T, int RPT, int NB>
int qr_blocked(T* Y, int64_t ldy, int64_t s, int64_t ncols, char* ws, hipStream_t st) {
  T* tau = reinterpret_cast<T*>(ws);
  T* Tm = reinterpret_cast<T*>(ws + ls_align256(sizeof(T) * ncols));   // two NB x NB buffers
  const int nbf = (int)((ncols < NB) ? ncols : NB);
  hipLaunchKernelGGL((k_qr_panel<T, RPT, NB>), dim3(1), dim3(kQrThreads), 0, st, Y, ldy, s, (int64_t)0, nbf, tau, Tm);
  int k = 0;
  for (int64_t j0 = 0; j0 + NB < ncols; j0 += NB, ++k) {
    const int nb0 = NB;
    const int64_t j1 = j0 + NB;
    const int nb1 = (int)((ncols - j1 < NB) ? ncols - j1 : NB);
    const int64_t jt = j1 + nb1;
    const unsigned ntr = (unsigned)ls_cdiv(ncols - jt, 16);
    hipLaunchKernelGGL((k_qr_step<T, RPT, NB>), dim3(1 + ntr), dim3(kQrThreads), 0, st, Y, ldy, s, ncols, j0, nb0,
                       Tm + (k & 1) * NB * NB, j1, nb1, tau, Tm + ((k + 1) & 1) * NB * NB, jt);
  }
  LS_HIP_TRY(hipGetLastError());
  return LS_OK;
}

template <typename T>
int qr_dispatch(T* Y, int64_t ldy, int64_t s, int64_t ncols, char* ws, hipStream_t st) {
  // Panel width chosen so that RPT x NB panel values stay in registers of the
  // kPanelThreads panel threads (512-thread blocks allow 256 VGPRs per lane).
  const int64_t rpt = ls_cdiv(s, kPanelThreads);
  // (RPT = 8 would spill at this width of the panel: such s use RPT = 16.)
  if constexpr (sizeof(T) == 4) {
    if (rpt <= 4) return qr_blocked<T, 4, 16>(Y, ldy, s, ncols, ws, st);
    if (rpt <= 16) return qr_blocked<T, 16, 8>(Y, ldy, s, ncols, ws, st);
    if (rpt <= 32) return qr_blocked<T, 32, 4>(Y, ldy, s, ncols, ws, st);
  } else {
    if (rpt <= 4) return qr_blocked<T, 4, 8>(Y, ldy, s, ncols, ws, st);
    if (rpt <= 8) return qr_blocked<T, 8, 8>(Y, ldy, s, ncols, ws, st);
    if (rpt <= 16) return qr_blocked<T, 16, 4>(Y, ldy, s, ncols, ws, st);
    if (rpt <= 32) return qr_blocked<T, 32, 2>(Y, ldy, s, ncols, ws, st);
  }
  return LS_E_UNSUPPORTED;
}

}  // namespace

namespace ls {

// Leading dimension of the internal working copy of Y.
static int64_t qr_ldw(int64_t s) { return ls_cdiv(s, 4) * 4; }

size_t qr_workspace(int64_t s, int64_t ncols, ls_prec_t u_qr) {
  const size_t elt = (u_qr == LS_FP32) ? 4 : 8;
  size_t b = 0;
  b += ls_align256(elt * (size_t)qr_ldw(s) * ncols);                    // working copy
  b += ls_align256(elt * ncols);                                         // tau
  b += ls_align256(elt * 2 * 16 * 16);                                   // T of two consecutive panels
  return b;
}

int qr_run(int64_t s, int64_t ncols, ls_prec_t u_qr, const double* Y, int64_t ldy, double* R, int64_t ldr, char* ws,
           size_t ws_bytes, int* d_flag, int64_t check_cols, hipStream_t st) {
  if (ws_bytes < qr_workspace(s, ncols, u_qr)) return LS_E_WORKSPACE;
  if (s > 32 * (int64_t)kPanelThreads) return LS_E_UNSUPPORTED;
  const int64_t ldw = qr_ldw(s);
  const dim3 gfin((unsigned)ls_cdiv(ncols, 256), (unsigned)ncols);
  const dim3 gcp((unsigned)ls_cdiv(ldw, 256), (unsigned)ncols);
  if (u_qr == LS_FP32) {
    float* Yw = reinterpret_cast<float*>(ws);
    char* rest = ws + ls_align256(4 * (size_t)ldw * ncols);
    hipLaunchKernelGGL((k_copy_cols<double, float>), gcp, dim3(256), 0, st, Y, ldy, Yw, ldw, ldw, s, ncols);
    LS_TRY(qr_dispatch<float>(Yw, ldw, s, ncols, rest, st));
    hipLaunchKernelGGL(k_qr_finish<float>, gfin, dim3(256), 0, st, Yw, ldw, ncols, check_cols, R, ldr, d_flag);
  } else if (u_qr == LS_FP64) {
    double* Yw = reinterpret_cast<double*>(ws);
    char* rest = ws + ls_align256(8 * (size_t)ldw * ncols);
    hipLaunchKernelGGL((k_copy_cols<double, double>), gcp, dim3(256), 0, st, Y, ldy, Yw, ldw, ldw, s, ncols);
    LS_TRY(qr_dispatch<double>(Yw, ldw, s, ncols, rest, st));
    hipLaunchKernelGGL(k_qr_finish<double>, gfin, dim3(256), 0, st, Yw, ldw, ncols, check_cols, R, ldr, d_flag);
  } else {
    return LS_E_UNSUPPORTED;
  }
  LS_HIP_TRY(hipGetLastError());
  return LS_OK;
}

int trinv_run(const double* R, int64_t ldr, int64_t n, double* W, int64_t ldw, float* W32, int* d_flag,
              hipStream_t st, double* fro) {
  hipLaunchKernelGGL(k_trinv, dim3((unsigned)n), dim3(256), (size_t)n * sizeof(double), st, R, ldr, n, W, ldw,
                     d_flag, fro);
  if (W32)
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)ls_cdiv(n, 256), (unsigned)n), dim3(256), 0, st, W, ldw, n, W32);
  // W^T right after W (ld n): row r of W is then contiguous
  hipLaunchKernelGGL(k_transpose_f64, dim3((unsigned)ls_cdiv(n, 32), (unsigned)ls_cdiv(n, 32)), dim3(256), 0, st, W,
                     ldw, n, W + ldw * n);
  LS_HIP_TRY(hipGetLastError());
  return LS_OK;
}

}  // namespace ls
