// Algorithm 2 on gfx950: LSQR right-preconditioned with R and the
// augmented-system refinement loop with split-preconditioned FGMRES.
//
// The preconditioned operator B = A R^-1 is formed once per call (an MFMA
// GEMM with the explicit upper-triangular W = R^-1).  LSQR then works on
// min ||b - B z|| with x = W z, and FGMRES on the split-preconditioned
// augmented matrix, which is exactly [I B; B^T 0]; R^-1 is applied only to
// the final corrections.  The refinement residuals use A itself.
//
// Every iteration reads B once: a block of RB rows (all n columns) is
// prefetched into registers while the previous block, staged in LDS, is used
// for both the row products (B v) and the column products (B^T u).  Each
// block of threads owns a contiguous range of row blocks.  Column products
// are per-block partial sums, stored column-major (partial[c * G + block]) so
// that a wave reduces one column with coalesced loads, in a fixed order.
//
// Scalars live in device memory; kernels of one iteration are enqueued back
// to back and the host reads a convergence flag every few iterations.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "lanes.h"

namespace ls {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxKrylov = 96;     // Arnoldi columns per FGMRES cycle (kmax + 1)
constexpr int kMaxPanQ = 32;       // 16-byte loads per lane for one panel of B (n <= 2048)
// The panel passes load the next panel while using the current one, except at
// the widest panels (n > 1024), where one panel is already 32 loads per lane
// in flight and a second set would not fit the register file.
template <int Q>
constexpr bool kPanPrefetch = Q < 32;

typedef float ls_float4v __attribute__((ext_vector_type(4)));
typedef double ls_double4v __attribute__((ext_vector_type(4)));
typedef double ls_double2v __attribute__((ext_vector_type(2)));

// Panel layout of B: panels of PR = 16 / sizeof(T) rows, one 16-byte vector per
// column.  Panel p holds rows [PR p, PR p + PR) of all n columns, column after
// column: row i of column c is element PR n (i / PR) + PR c + i % PR.  Rows
// past m in the last panel are zero.  A wave reads a panel with fully
// coalesced 1 KB loads (lane l, load q: column l + 64 q).
template <typename T>
struct PanVec;
template <>
struct PanVec<float> {
  static constexpr int PR = 4;
  using type = ls_float4v;
};
template <>
struct PanVec<double> {
  static constexpr int PR = 2;
  using type = ls_double2v;
};

// The value of lane src on every lane (through a scalar register).
__device__ __forceinline__ float lane_value(float v, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}
__device__ __forceinline__ double lane_value(double v, int src) {
  const long long u = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Butterfly sum over the wave; every lane ends with the same bits (each step
// adds the same two numbers in every lane of a pair).
template <typename T>
__device__ __forceinline__ T wave_allsum(T v) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double* align8(void* p) {
  return reinterpret_cast<double*>(((uintptr_t)p + 7) & ~(uintptr_t)7);
}

template <typename T>
__device__ __forceinline__ T block_sum256(T v, T* sh) {
  return ls_block_sum<T, kThreads>(v, sh);
}

// Sum of part[0..G) by one wave (all lanes get the result); each lane adds
// its elements lane, lane + 64, ... in order, eight loads in flight.
__device__ __forceinline__ double wave_sum_array(const double* __restrict__ part, int G, int lane) {
  double s = 0.0;
  for (int g0 = 0; g0 < G; g0 += 512) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int g = g0 + 64 * q + lane;
      v[q] = (g < G) ? part[g] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) s += v[q];
  }
  return ls_wave_sum(s);
}

// wave_sum_array with all of a lane's loads in flight at once (G <= 64 NL):
// the same values added in the same order, one memory round trip.
template <int NL>
__device__ __forceinline__ double wave_sum_array_all(const double* __restrict__ part, int G, int lane) {
  double v[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    const int g = 64 * q + lane;
    v[q] = (g < G) ? part[g] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < NL; ++q) s += v[q];
  return ls_wave_sum(s);
}

// wave_sum_array of two arrays at once (their loads issued together); each
// sum is added in the same order as by wave_sum_array alone.
__device__ __forceinline__ void wave_sum_array2(const double* __restrict__ pa, int Ga,
                                                const double* __restrict__ pb, int Gb, int lane, double& sa,
                                                double& sb) {
  double s0 = 0.0, s1 = 0.0;
  const int Gm = (Ga > Gb) ? Ga : Gb;
  for (int g0 = 0; g0 < Gm; g0 += 512) {
    double va[8], vb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int g = g0 + 64 * q + lane;
      va[q] = (g < Ga) ? pa[g] : 0.0;
      vb[q] = (g < Gb) ? pb[g] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) s0 += va[q];
#pragma unroll
    for (int q = 0; q < 8; ++q) s1 += vb[q];
  }
  sa = ls_wave_sum(s0);
  sb = ls_wave_sum(s1);
}

// Range of row blocks owned by block `bx` of G.
__device__ __forceinline__ void row_range(int64_t nrb, int G, int bx, int64_t& b0, int64_t& b1) {
  b0 = (nrb * bx) / G;
  b1 = (nrb * (bx + 1)) / G;
}

// ================================================================== B = A W
// MFMA 16x16x4 (binary32 or binary64).  Block tile 64 x 64, K step 32 with the
// next step's tiles loaded into registers while the current one is multiplied;
// wave w owns rows 32 (w & 1) .. +32 and columns 32 (w >> 1) .. +32 (2 x 2 MFMA
// tiles).  W is upper triangular: column tile [j0, j0+64) needs K < j0 + 64 only.
__device__ __forceinline__ ls_float4v mfma4(float a, float b, ls_float4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ ls_double4v mfma4(double a, double b, ls_double4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Row of the D element held in slot r of lane l: binary32 rows are blocked,
// binary64 rows interleaved.
template <typename T>
__device__ __forceinline__ int mfma_drow(int lane, int r) {
  return (sizeof(T) == 4) ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r;
}

template <typename TA, typename T>
__global__ __launch_bounds__(kThreads) void k_form_b(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                     const T* __restrict__ W, T* __restrict__ B) {
  using acc_t = typename std::conditional<sizeof(T) == 4, ls_float4v, ls_double4v>::type;
  constexpr int KS = 32;                   // K step
  constexpr int LPT = KS * 64 / kThreads;  // tile elements per thread (A and W each)
  __shared__ T As[KS][64 + 1];   // As[k][i]
  __shared__ T Ws[KS][64 + 1];   // Ws[k][j]
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int64_t j0 = (int64_t)blockIdx.y * 64;
  const int64_t kend = (j0 + 64 < n) ? j0 + 64 : n;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  // element u of this thread: A tile column kk = idx / 64, row ii = idx % 64
  // (coalesced over ii); W tile column jj = idx / KS, row k2 = idx % KS
  T ra[LPT], rw[LPT];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      const int idx = t + kThreads * u;
      const int kk = idx / 64, ii = idx % 64;
      const int64_t gi = i0 + ii, gk = k0 + kk;
      ra[u] = (gi < m && gk < n) ? (T)A[gi + gk * lda] : T(0);
      const int jj = idx / KS, k2 = idx % KS;
      const int64_t gj = j0 + jj, gk2 = k0 + k2;
      rw[u] = (gj < n && gk2 < n) ? W[gk2 + gj * n] : T(0);
    }
  };
  load(0);
  for (int64_t k0 = 0; k0 < kend; k0 += KS) {
    __syncthreads();   // the previous step's tiles have been read
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      const int idx = t + kThreads * u;
      As[idx / 64][idx % 64] = ra[u];
      Ws[idx % KS][idx / KS] = rw[u];
    }
    __syncthreads();
    if (k0 + KS < kend) load(k0 + KS);   // in flight during the products
#pragma unroll
    for (int ks = 0; ks < KS / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const T av = As[kk][wr + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma4(av, Ws[kk][wc + b * 16 + (lane & 15)], acc[a][b]);
      }
    }
  }
  // panel layout; rows in [m, mp) of the last panel are written as zeros
  constexpr int PR = PanVec<T>::PR;
  const int64_t mp = ls_cdiv(m, PR) * PR;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t gj = j0 + wc + b * 16 + (lane & 15);
      if (gj >= n) continue;
      if constexpr (sizeof(T) == 4) {
        // binary32: the lane's four rows are one aligned group of PR = 4 rows
        const int64_t gi = i0 + wr + a * 16 + mfma_drow<T>(lane, 0);
        if (gi < mp) *reinterpret_cast<ls_float4v*>(B + (gi / PR) * PR * n + gj * PR) = acc[a][b];
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gi = i0 + wr + a * 16 + mfma_drow<T>(lane, r);
          if (gi < mp) B[(gi / PR) * PR * n + gj * PR + (gi % PR)] = acc[a][b][r];
        }
      }
    }
}

// out = W v for upper-triangular W (n x n, ld).
__global__ __launch_bounds__(kUtThreads) void k_trmv(const double* __restrict__ W, int64_t ldw, int64_t n,
                                                     const double* __restrict__ v, double* __restrict__ out) {
  __shared__ double red[32 * 33];
  const double s = ls_utmv_row(W, ldw, n, [&](int64_t j) { return v[j]; }, red);
  const int64_t row = (int64_t)blockIdx.x * 32 + threadIdx.x;
  if (threadIdx.x < 32 && row < n) out[row] = s;
}

template <typename TO, typename TI>
__global__ __launch_bounds__(kThreads) void k_cast(const TI* __restrict__ a, TO* __restrict__ b, int64_t n, TO sign) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) b[i] = sign * (TO)a[i];
}

// The start of an FGMRES cycle: a zeroed state holding the cycle's tolerance.
__global__ void k_fg_begin(FgState* st, double tol) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    FgState S{};
    S.tol = tol;
    *st = S;
  }
}

__global__ void k_zero_bytes(char* p, size_t nbytes) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < nbytes; i += (size_t)gridDim.x * kThreads) p[i] = 0;
}

// ================================================================== LSQR on B
// Carried state C_i (written by the column kernel of iteration i-1).
// Iteration i:  pass:   u_{i+1} = B v_i / alpha_i - (alpha_i / beta_i) u_i  (unnormalised u)
//               column: beta_{i+1}, rotation i, w_i, y, v_{i+1} = B^T u / beta - (beta/alpha) v_i
struct LsqrRec {
  double c, s;        // rotation of iteration i-1 (init: c = -1, s = 0)
  double rho;         // rho_{i-1}
  double phibar;      // phibar_i
  double normB2;      // sum over k < i of alpha_k^2 + beta_{k+1}^2
  double beta;        // beta_i
  double alpha_prev;  // alpha_{i-1}
  double normr, normar, normB;
  int32_t its, done, stop, pad;
};
struct LsqrState {
  LsqrRec rec[2];
  double normb;
  int32_t flag, pad;
};

// Progress of a call, written by the kernels that test convergence into
// pinned host memory and polled by the host (so that it can keep a few
// iterations queued instead of synchronising to read the state).
struct Progress {
  int32_t lsqr_it, lsqr_done, fg_j, fg_done;
  int32_t pad[12];
};

__device__ __forceinline__ void progress_put(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Pass of iteration i over the panels of B (one wave streams a contiguous
// range of panels, the next panel in flight while the current one is used):
// per panel, the row sums B v are reduced across the wave, giving the panel's
// rows of u_{i+1}; every lane then adds those rows' contribution to its own
// columns of B^T u_{i+1}.  Column partials are summed over the block's waves
// in a fixed order.  Init: u_1 = b - B z0 (v = -z0, coef = -1).
template <typename T, int Q>
__global__ __launch_bounds__(kThreads) void k_lsqr_pan(const T* __restrict__ Bp, int64_t npan, int64_t m, int64_t n,
                                                       const T* __restrict__ v, const double* __restrict__ nvpart,
                                                       int Gv, T* __restrict__ u, const LsqrState* __restrict__ st,
                                                       int par, int init, T* __restrict__ tpart,
                                                       double* __restrict__ nupart, double* __restrict__ nbpart) {
  if (!init && st->rec[par].done) return;
  using vec_t = typename PanVec<T>::type;
  constexpr int PR = PanVec<T>::PR;
  __shared__ T cred[64 * Q];
  __shared__ double dsh[8];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t nw = (int64_t)gridDim.x * 4;
  int64_t p0, p1;
  row_range(npan, (int)nw, blockIdx.x * 4 + wave, p0, p1);
  double nu = 0.0, nb = 0.0;
  vec_t cur[Q];
  vec_t uo;
  auto load = [&](int64_t p, vec_t* dst, vec_t& uu) {
    const T* base = Bp + p * (PR * n);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t c = lane + 64 * q;
      dst[q] = (c < n) ? *reinterpret_cast<const vec_t*>(base + c * PR) : vec_t{};
    }
    const int64_t i0 = p * PR;
    if (i0 + PR <= m) {
      uu = *reinterpret_cast<const vec_t*>(u + i0);
    } else {
#pragma unroll
      for (int k = 0; k < PR; ++k) uu[k] = (i0 + k < m) ? u[i0 + k] : T(0);
    }
  };
  // the first panel of B and its rows of u do not depend on alpha: their
  // loads go out before alpha's partials are summed
  if (p0 < p1) load(p0, cur, uo);
  T scale = 1, coef = -1;
  if (!init) {
    const double alpha = sqrt(wave_sum_array(nvpart, Gv, lane));
    scale = (T)(1.0 / alpha);
    coef = (T)(alpha / st->rec[par].beta);
  }
  T vl[Q], creg[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t c = lane + 64 * q;
    vl[q] = (c < n) ? v[c] * scale : T(0);
    creg[q] = 0;
  }
  constexpr int GP = 64 / PR;   // panels per group of 64 rows
  T ukeep = 0, bkeep = 0;
  for (int64_t p = p0; p < p1; ++p) {
    vec_t nxt[kPanPrefetch<Q> ? Q : 1];
    vec_t un_o;
    if (kPanPrefetch<Q> && p + 1 < p1) load(p + 1, nxt, un_o);
    const int64_t i0 = p * PR;
    T s[PR];
#pragma unroll
    for (int k = 0; k < PR; ++k) s[k] = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int k = 0; k < PR; ++k) s[k] += cur[q][k] * vl[q];
    // the panel's row sums: a transposed butterfly leaves row idx's on lanes
    // (64 / PR) idx .., then each row's sum reaches every lane
    int idx;
    const T tot = wave_multi_sum<T, PR>(s, lane, idx);
    vec_t un;
#pragma unroll
    for (int k = 0; k < PR; ++k) {
      const T sk = lane_value(tot, k * (64 / PR));
      un[k] = (i0 + k < m) ? sk - coef * uo[k] : T(0);
    }
    // lane l keeps row l % PR of panel l / PR of an aligned group of GP
    // panels; the group's 64 rows of u go out as one store
    const int pp = (int)(p % GP);
    if (lane / PR == pp) {
#pragma unroll
      for (int k = 0; k < PR; ++k)
        if (k == lane % PR) {
          ukeep = un[k];
          bkeep = uo[k];
        }
    }
    if (pp == GP - 1 || p + 1 == p1) {
      const int64_t i = (p - pp) * PR + lane;
      if (i >= p0 * PR && i < i0 + PR && i < m) {
        u[i] = ukeep;
        nu += (double)ukeep * (double)ukeep;
        if (init) nb += (double)bkeep * (double)bkeep;
      }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int k = 0; k < PR; ++k) creg[q] += cur[q][k] * un[k];
    if (p + 1 < p1) {
      if constexpr (kPanPrefetch<Q>) {
#pragma unroll
        for (int q = 0; q < Q; ++q) cur[q] = nxt[q];
        uo = un_o;
      } else {
        load(p + 1, cur, uo);
      }
    }
  }
  // column partials of the block's four waves, summed in wave order
  for (int wv = 0; wv < 4; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int q = 0; q < Q; ++q) cred[lane + 64 * q] = (wv ? cred[lane + 64 * q] : T(0)) + creg[q];
    }
    __syncthreads();
  }
  for (int64_t c = threadIdx.x; c < n; c += kThreads) tpart[c * gridDim.x + blockIdx.x] = cred[c];
  nu = ls_wave_sum(nu);
  if (init) nb = ls_wave_sum(nb);
  if (lane == 0) {
    dsh[wave] = nu;
    dsh[4 + wave] = nb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    nupart[blockIdx.x] = (dsh[0] + dsh[1]) + (dsh[2] + dsh[3]);
    if (init) nbpart[blockIdx.x] = (dsh[4] + dsh[5]) + (dsh[6] + dsh[7]);
  }
}

// Column kernel, one wave per column (4 per block).  Reads rec[par] (C_i),
// block 0 writes rec[par ^ 1] (C_{i+1}).  Init: v_1 = B^T u_1 / beta_1.
// tpart: Gt partials per column of B^T u; nupart, nbpart: the pass's G partials.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_lsqr_col(int64_t n, const T* __restrict__ tpart, int Gt, int G,
                                                       const double* __restrict__ nupart,
                                                       const double* __restrict__ nbpart,
                                                       const double* __restrict__ nvpart_in, int Gv,
                                                       double* __restrict__ nvpart_out, LsqrState* st, int par,
                                                       int init, int it, double tol, T* __restrict__ v,
                                                       T* __restrict__ w, double* __restrict__ y,
                                                       Progress* prog) {
  __shared__ double dsh[4];
  const LsqrRec R = st->rec[par];
  if (!init && R.done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->rec[par ^ 1] = R;
      if (prog) {
        progress_put(&prog->lsqr_done, 1);
        progress_put(&prog->lsqr_it, it);
      }
    }
    return;
  }
  const int lane = threadIdx.x & 63;
  const int64_t col = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  double beta, alpha2 = 0.0;
  if (init) {
    beta = sqrt(wave_sum_array(nupart, G, lane));                     // beta_{i+1}
  } else {
    double beta2;
    wave_sum_array2(nupart, G, nvpart_in, Gv, lane, beta2, alpha2);
    beta = sqrt(beta2);
  }
  LsqrRec N = R;
  double alpha = 0.0, xw = 0.0, yw = 0.0, vcoef = 0.0;
  bool done = false;
  if (init) {
    N.c = -1.0;
    N.s = 0.0;
    N.rho = 1.0;
    N.phibar = beta;
    N.normB2 = 0.0;
    N.beta = beta;
    N.alpha_prev = 0.0;
    N.its = 0;
    N.stop = (beta == 0.0) ? 4 : 0;
    done = N.stop != 0;
    N.done = done ? 1 : 0;
  } else {
    alpha = sqrt(alpha2);                                             // alpha_i
    const double rhobar = -R.c * alpha;
    const double theta = R.s * alpha;
    // stopping tests of iteration i-1 (they need alpha_i)
    if (it > 1) {
      N.normr = R.phibar;
      N.normar = R.phibar * alpha * fabs(R.c);
      N.normB = sqrt(R.normB2);
      N.its = it - 1;
      int stop = 0;
      if (N.normr <= tol * st->normb) stop = 1;
      else if (N.normar <= tol * N.normB * N.normr) stop = 2;
      else if (alpha == 0.0) stop = 4;
      if (stop) {
        N.stop = stop;
        N.done = 1;
        done = true;
      }
    }
    if (!done) {
      N.normB2 = R.normB2 + alpha * alpha + beta * beta;
      const double rho = hypot(rhobar, beta);
      const double c = rhobar / rho;
      const double sn = beta / rho;
      const double phi = c * R.phibar;
      N.phibar = sn * R.phibar;
      N.c = c;
      N.s = sn;
      N.rho = rho;
      N.beta = beta;
      N.alpha_prev = alpha;
      N.its = it;
      xw = (it == 1) ? 0.0 : theta / R.rho;        // w_i = v_i - (theta_i / rho_{i-1}) w_{i-1}
      yw = phi / rho;                              // y += (phi_i / rho_i) w_i
      vcoef = beta / alpha;                        // v_{i+1} = t - (beta_{i+1} / alpha_i) v_i
      if (!isfinite(yw) || !isfinite(xw) || !isfinite(vcoef)) {
        N.stop = 5;
        N.done = 1;
        done = true;
      } else if (beta == 0.0) {
        N.stop = 4;   // exact solution reached after this update
      }
    }
  }
  double contrib = 0.0;
  if (!done && col < n) {
    const T* tp = tpart + col * Gt;
    T acc = 0;
    for (int g0 = 0; g0 < Gt; g0 += 512) {   // eight loads per lane in flight
      T pv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int g = g0 + 64 * q + lane;
        pv[q] = (g < Gt) ? tp[g] : T(0);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) acc += pv[q];
    }
    acc = ls_wave_sum(acc);
    if (lane == 0) {
      const T t = (beta > 0.0) ? (T)(acc / (T)beta) : T(0);
      T vn;
      if (init) {
        vn = t;
      } else {
        const T vo = v[col];
        const T wi = vo * (T)(1.0 / alpha) - (T)xw * w[col];
        w[col] = wi;
        y[col] += yw * (double)wi;
        vn = t - (T)vcoef * vo;
      }
      v[col] = vn;
      contrib = (double)vn * (double)vn;
    }
  }
  contrib = block_sum256(contrib, dsh);
  if (threadIdx.x == 0) nvpart_out[blockIdx.x] = contrib;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (init) {
      double sb = 0.0;
      for (int g = 0; g < G; ++g) sb += nbpart[g];
      st->normb = sqrt(sb);
    }
    if (N.stop == 4 && !init) N.done = 1;
    if (N.stop == 5) st->flag = 1;
    st->rec[par ^ 1] = N;
    if (prog) {
      progress_put(&prog->lsqr_done, N.done ? 1 : 0);
      progress_put(&prog->lsqr_it, it);
    }
  }
}

// LSQR over A's panels with W = R^-1 applied on either side of the pass
// (B = A W is then never formed): before the pass, vz = W v (binary64
// products, rounded to the working precision); after it, the column partials
// of A^T u are summed (k_lsqr_colsum) and t = W^T (A^T u) is formed
// (k_lsqr_wt), which the column kernel reads as a single partial per column.
template <typename T>
__global__ __launch_bounds__(1024) void k_lsqr_zx(const double* __restrict__ W, int64_t n, const T* __restrict__ v,
                                                  const LsqrState* __restrict__ st, int par, int init,
                                                  T* __restrict__ vz) {
  if (!init && st->rec[par].done) return;
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* wr = W + n * n + row * n;   // W[row, :] from W^T, which follows W
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t c0 = row + lane; c0 < n; c0 += 64 * 8) {
    double wv[8], xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t c = c0 + 64 * q;
      wv[q] = (c < n) ? wr[c] : 0.0;
      xv[q] = (c < n) ? (double)v[c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q & 3] += wv[q] * xv[q];
  }
  const double z = ls_wave_sum((a[0] + a[1]) + (a[2] + a[3]));
  if (lane == 0) vz[row] = (T)z;
}

// a[c] = sum over the pass's G blocks of the column partials (one wave per
// column, eight loads per lane in flight), in binary64.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_lsqr_colsum(int64_t n, const T* __restrict__ tpart, int G,
                                                          const LsqrState* __restrict__ st, int par, int init,
                                                          double* __restrict__ a) {
  if (!init && st->rec[par].done) return;
  const int lane = threadIdx.x & 63;
  const int64_t col = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= n) return;
  const T* tp = tpart + col * G;
  double acc = 0.0;
  for (int g0 = 0; g0 < G; g0 += 512) {
    T pv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int g = g0 + 64 * q + lane;
      pv[q] = (g < G) ? tp[g] : T(0);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc += (double)pv[q];
  }
  acc = ls_wave_sum(acc);
  if (lane == 0) a[col] = acc;
}

// t = W^T a (column c of W is row c of W^T; one wave per column, 16 per
// block), rounded to the working precision.
template <typename T>
__global__ __launch_bounds__(1024) void k_lsqr_wt(const double* __restrict__ W, int64_t n,
                                                  const double* __restrict__ a, const LsqrState* __restrict__ st,
                                                  int par, int init, T* __restrict__ t) {
  if (!init && st->rec[par].done) return;
  const int lane = threadIdx.x & 63;
  const int64_t col = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 6);
  if (col >= n) return;
  const double* wc = W + col * n;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i0 = lane; i0 <= col; i0 += 64 * 8) {   // eight loads per lane in flight
    double wv[8], av[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t i = i0 + 64 * q;
      wv[q] = (i <= col) ? wc[i] : 0.0;
      av[q] = (i <= col) ? a[i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q & 3] += wv[q] * av[q];
  }
  const double val = ls_wave_sum((acc[0] + acc[1]) + (acc[2] + acc[3]));
  if (lane == 0) t[col] = (T)val;
}

// Final: stopping data of the last iteration (needs alpha_{k+1}) and x = W (z0 + y).
template <typename T>
__global__ __launch_bounds__(kUtThreads) void k_lsqr_finish(const double* __restrict__ W, int64_t n,
                                                          const double* __restrict__ z0,
                                                          const double* __restrict__ y,
                                                          const double* __restrict__ nvpart, int Gv,
                                                          LsqrState* st, int par, int it, double* __restrict__ x) {
  __shared__ double red[32 * 33];
  const int lane = threadIdx.x & 63;
  if (blockIdx.x == 0 && threadIdx.x < 64) {
    const double alpha = sqrt(wave_sum_array(nvpart, Gv, lane));
    if (lane == 0) {
      LsqrRec R = st->rec[par];
      if (!R.done) {
        R.normr = R.phibar;
        R.normar = R.phibar * alpha * fabs(R.c);
        R.normB = sqrt(R.normB2);
        R.its = it;
        R.stop = 3;
      }
      st->rec[par] = R;
    }
  }
  const double v = ls_utmv_row(W, n, n, [&](int64_t j) { return z0[j] + y[j]; }, red);
  const int64_t row = (int64_t)blockIdx.x * 32 + threadIdx.x;
  if (threadIdx.x < 32 && row < n) x[row] = (double)(T)v;
}

// ================================================================== refinement
// Passes over A itself (column-major, as stored).  A block of 256 threads
// owns 256 rows: lane l of every wave holds rows 4 l .. 4 l + 3 (one 16-byte
// load of binary32 A per column, two of binary64), and wave w takes the
// columns of the w-th quarter of [0, n), sixteen at a time (sixteen loads in
// flight).  Row sums are added over the four waves in LDS at the end.
constexpr int kResRows = 256;
constexpr int kResWaves = 8;                  // column groups of a residual block
constexpr int kResThreads = 64 * kResWaves;

// Rows i0 .. i0 + 3 of column j of A in its storage type, zero where ok is
// false or past m.
template <typename TA>
__device__ __forceinline__ void load_rows4_st(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t i0,
                                              int64_t j, bool vec, bool ok, TA (&a)[4]) {
  const TA* p = A + i0 + j * lda;
  if (ok && vec) {
    if constexpr (sizeof(TA) == 4) {
      const ls_float4v v = *reinterpret_cast<const ls_float4v*>(p);
#pragma unroll
      for (int k = 0; k < 4; ++k) a[k] = v[k];
    } else {
      const ls_double2v v0 = *reinterpret_cast<const ls_double2v*>(p);
      const ls_double2v v1 = *reinterpret_cast<const ls_double2v*>(p + 2);
      a[0] = v0[0];
      a[1] = v0[1];
      a[2] = v1[0];
      a[3] = v1[1];
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = (ok && i0 + k < m) ? p[k] : TA(0);
  }
}

template <typename TA>
__device__ __forceinline__ void load_rows4(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t i0, int64_t j,
                                           bool vec, double (&a)[4]) {
  const TA* p = A + i0 + j * lda;
  if (vec) {
    if constexpr (sizeof(TA) == 4) {
      const ls_float4v v = *reinterpret_cast<const ls_float4v*>(p);
      a[0] = v[0];
      a[1] = v[1];
      a[2] = v[2];
      a[3] = v[3];
    } else {
      const ls_double2v v0 = *reinterpret_cast<const ls_double2v*>(p);
      const ls_double2v v1 = *reinterpret_cast<const ls_double2v*>(p + 2);
      a[0] = v0[0];
      a[1] = v0[1];
      a[2] = v1[0];
      a[3] = v1[1];
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = (i0 + k < m) ? (double)p[k] : 0.0;
  }
}

// Accumulator of the refinement residual: binary64, or double-double.
template <bool DD>
struct RAcc {
  double hi = 0.0, lo = 0.0;
  __device__ __forceinline__ void fma(double a, double b) {
    if constexpr (DD) {
      const ls_dd t = ls_dd_fma(ls_dd{hi, lo}, a, b);
      hi = t.hi;
      lo = t.lo;
    } else {
      hi += a * b;
    }
  }
  __device__ __forceinline__ void add(const RAcc& o) {
    if constexpr (DD) {
      const ls_dd t = ls_dd_add(ls_dd{hi, lo}, ls_dd{o.hi, o.lo});
      hi = t.hi;
      lo = t.lo;
    } else {
      hi += o.hi;
    }
  }
  __device__ __forceinline__ RAcc xor_lane(int m) const {
    RAcc r;
    r.hi = __shfl_xor(hi, m, 64);
    if constexpr (DD) r.lo = __shfl_xor(lo, m, 64);
    return r;
  }
  // this value if f == 1, o if f == 0 (exact for finite values)
  __device__ __forceinline__ RAcc blend(const RAcc& o, double f) const {
    RAcc r;
    r.hi = hi * f + o.hi * (1.0 - f);
    if constexpr (DD) r.lo = lo * f + o.lo * (1.0 - f);
    return r;
  }
};

// Transposed butterfly over the wave for 16 accumulators: lane l ends with
// the wave total of index ((l >> 5) & 1) 8 + ((l >> 4) & 1) 4 + ((l >> 3) & 1) 2 + ((l >> 2) & 1).
template <bool DD>
__device__ __forceinline__ RAcc<DD> racc_multi_sum16(RAcc<DD> (&v)[16], int lane, int& idx) {
  int base = 0;
#pragma unroll
  for (int step = 0; step < 4; ++step) {
    const int off = 32 >> step;
    const int h = 8 >> step;
    const double fu = (lane & off) ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q < h) {
        const RAcc<DD> send = v[q].blend(v[q + h], fu);
        RAcc<DD> keep = v[q + h].blend(v[q], fu);
        keep.add(send.xor_lane(off));
        v[q] = keep;
      }
    }
    if (lane & off) base += h;
  }
  RAcc<DD> s = v[0];
  s.add(s.xor_lane(2));
  s.add(s.xor_lane(1));
  idx = base;
  return s;
}

// r = b - A x in precision T (the refinement's starting residual).
template <typename TA, typename T>
__global__ __launch_bounds__(kResThreads) void k_resid_u(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                         int vec_ok, const TA* __restrict__ b,
                                                         const double* __restrict__ x, double* __restrict__ r) {
  __shared__ T rs[kResWaves][kResRows];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * kResRows + 4 * lane;
  const bool vec = vec_ok && i0 + 4 <= m;
  const int64_t jq = ls_cdiv(n, kResWaves);
  const int64_t j0 = wave * jq, j1 = (j0 + jq < n) ? j0 + jq : n;
  T acc[4] = {0, 0, 0, 0};
  constexpr int NQ = 8;   // columns whose loads are in flight together
  for (int64_t jb = j0; jb < j1; jb += NQ) {
    TA av[NQ][4];
    double xv[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int64_t j = jb + q;
      const bool ok = j < j1 && i0 < m;
      load_rows4_st(A, lda, m, i0, j, vec, ok, av[q]);
      xv[q] = (j < j1) ? x[j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if (jb + q < j1 && i0 < m) {
        const T xj = (T)xv[q];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += (T)(double)av[q][k] * xj;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) rs[wave][4 * lane + k] = acc[k];
  __syncthreads();
  const int t = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kResRows + t;
  if (t < kResRows && i < m) {
    T q = rs[0][t];
#pragma unroll
    for (int w = 1; w < kResWaves; ++w) q += rs[w][t];
    r[i] = (double)((T)b[i] - q);
  }
}

// Refinement residuals in u_r: f = b - r - A x (rows, written to V[:, 0]) and g = A^T r as
// per-block column partials (tpart[c G + block], hi and lo parts), binary64
// or double-double; A and b are used exactly as stored.
template <typename TA, bool DD>
__global__ __launch_bounds__(kResThreads) __attribute__((amdgpu_waves_per_eu(DD ? 2 : 3))) void k_lsir_resid(const TA* __restrict__ A, int64_t lda, int64_t m,
                                                            int64_t n, int vec_ok, const TA* __restrict__ b,
                                                            const double* __restrict__ r, const double* __restrict__ x,
                                                            double* __restrict__ V, double* __restrict__ tpart_hi,
                                                            double* __restrict__ tpart_lo, double* __restrict__ fpart) {
  __shared__ double rsh[kResWaves][kResRows], rsl[kResWaves][kResRows];
  __shared__ double dsh[kResWaves];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int G = gridDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * kResRows + 4 * lane;
  const bool vec = vec_ok && i0 + 4 <= m;
  const int64_t jq = ls_cdiv(n, kResWaves);
  const int64_t j0 = wave * jq, j1 = (j0 + jq < n) ? j0 + jq : n;
  double rv[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) rv[k] = (i0 + k < m) ? r[i0 + k] : 0.0;
  RAcc<DD> racc[4];
  constexpr int NQ = (sizeof(TA) == 4 || DD) ? 8 : 4;   // columns whose loads are in flight together
  for (int64_t jb = j0; jb < j1; jb += 16) {
    RAcc<DD> cp[16];
#pragma unroll
    for (int h = 0; h < 16; h += NQ) {
      // NQ columns' loads first, then the products (same order of addition)
      TA av[NQ][4];
      double xv[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int64_t j = jb + h + q;
        const bool ok = j < j1 && i0 < m;
        load_rows4_st(A, lda, m, i0, j, vec, ok, av[q]);
        xv[q] = (j < j1) ? x[j] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (jb + h + q < j1 && i0 < m) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const double a = (double)av[q][k];
            racc[k].fma(a, xv[q]);
            cp[h + q].fma(a, rv[k]);
          }
        }
      }
    }
    int idx;
    const RAcc<DD> tot = racc_multi_sum16<DD>(cp, lane, idx);
    const int64_t c = jb + idx;
    if ((lane & 3) == 0 && c < j1) {
      tpart_hi[c * G + blockIdx.x] = tot.hi;
      if (DD) tpart_lo[c * G + blockIdx.x] = tot.lo;
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    rsh[wave][4 * lane + k] = racc[k].hi;
    rsl[wave][4 * lane + k] = racc[k].lo;
  }
  __syncthreads();
  const int t = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kResRows + t;
  double fn = 0.0;
  if (t < kResRows && i < m) {
    RAcc<DD> q;
    q.hi = rsh[0][t];
    q.lo = rsl[0][t];
#pragma unroll
    for (int w = 1; w < kResWaves; ++w) {
      RAcc<DD> o;
      o.hi = rsh[w][t];
      o.lo = rsl[w][t];
      q.add(o);
    }
    const double ri = r[i];
    double f;
    if (DD) {
      ls_dd fb = ls_two_sum((double)b[i], -ri);
      fb = ls_dd_add(fb, ls_dd{-q.hi, -q.lo});
      f = fb.hi + fb.lo;
    } else {
      f = ((double)b[i] - ri) - q.hi;
    }
    V[i] = f;
    fn = f * f;
  }
  fn = ls_block_sum<double, kResThreads>(fn, dsh);
  if (threadIdx.x == 0) fpart[blockIdx.x] = fn;
}

// g = -(A^T r) from the column partials; one wave per column.
template <bool DD>
__global__ __launch_bounds__(kThreads) void k_lsir_g(const double* __restrict__ tpart_hi,
                                                     const double* __restrict__ tpart_lo, int G, int64_t n,
                                                     double* __restrict__ g) {
  const int lane = threadIdx.x & 63;
  const int64_t col = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= n) return;
  ls_dd acc{0.0, 0.0};
  for (int q = lane; q < G; q += 64) {
    if (DD) acc = ls_dd_add(acc, ls_dd{tpart_hi[col * G + q], tpart_lo[col * G + q]});
    else acc.hi += tpart_hi[col * G + q];
  }
  for (int off = 32; off > 0; off >>= 1) {
    const ls_dd o{__shfl_xor(acc.hi, off, 64), __shfl_xor(acc.lo, off, 64)};
    if (DD) acc = ls_dd_add(acc, o);
    else acc.hi += o.hi;
  }
  if (lane == 0) g[col] = -(acc.hi + acc.lo);
}

// h = W^T g (the preconditioned residual) into V[m:, 0]; partial ||h||^2.  One wave per column.
template <bool DD>
__global__ __launch_bounds__(kThreads) void k_lsir_h(const double* __restrict__ W, int64_t n, int64_t m,
                                                     const double* __restrict__ g, double* __restrict__ V,
                                                     double* __restrict__ hpart) {
  __shared__ double dsh[4];
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  double contrib = 0.0;
  if (j < n) {
    const double* wc = W + j * n;
    ls_dd acc{0.0, 0.0};
    for (int64_t i = lane; i <= j; i += 64) {
      if (DD) acc = ls_dd_fma(acc, wc[i], g[i]);
      else acc.hi += wc[i] * g[i];
    }
    for (int off = 32; off > 0; off >>= 1) {
      const ls_dd o{__shfl_xor(acc.hi, off, 64), __shfl_xor(acc.lo, off, 64)};
      if (DD) acc = ls_dd_add(acc, o);
      else acc.hi += o.hi;
    }
    if (lane == 0) {
      const double h = acc.hi + acc.lo;
      V[m + j] = h;
      contrib = h * h;
    }
  }
  contrib = block_sum256(contrib, dsh);
  if (threadIdx.x == 0) hpart[blockIdx.x] = contrib;
}

// The same residuals in binary64 over A's binary32 panel copy (rows 4p..4p+3
// of panel p, entry (i, c) at p 4n + 4c + i % 4), where the FGMRES pass
// streams it: one wave per contiguous panel range, contiguous 16-byte loads
// instead of n column segments per row block.  f = (b - r) - A x -> f, ||f||^2
// per block -> fpart[block], the column partials of A^T r -> tpart[c G + block].
template <int Q>
__global__ __launch_bounds__(kThreads) void k_resid_pan(const float* __restrict__ Ap, int64_t npan, int64_t m,
                                                        int64_t n, const float* __restrict__ b,
                                                        const double* __restrict__ r, const double* __restrict__ x,
                                                        double* __restrict__ f, double* __restrict__ tpart,
                                                        double* __restrict__ fpart) {
  constexpr int PR = 4;
  __shared__ double cred[64 * Q];
  __shared__ double dsh[kThreads / 64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int64_t p0, p1;
  row_range(npan, (int)gridDim.x * 4, blockIdx.x * 4 + wave, p0, p1);
  double xl[Q], creg[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t c = lane + 64 * q;
    xl[q] = (c < n) ? x[c] : 0.0;
    creg[q] = 0.0;
  }
  double fn = 0.0, skeep = 0.0;
  ls_float4v cur[Q];
  auto load = [&](int64_t p) {
    const float* base = Ap + p * (PR * n);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t c = lane + 64 * q;
      cur[q] = (c < n) ? *reinterpret_cast<const ls_float4v*>(base + c * PR) : ls_float4v{};
    }
  };
  if (p0 < p1) load(p0);
  for (int64_t p = p0; p < p1; ++p) {
    const int64_t i0 = p * PR;
    double rv[PR], s[PR];
#pragma unroll
    for (int k = 0; k < PR; ++k) {
      rv[k] = (i0 + k < m) ? r[i0 + k] : 0.0;
      s[k] = 0.0;
    }
    // both products of an entry while its binary64 conversion is live
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
      for (int k = 0; k < PR; ++k) {
        const double a = (double)cur[q][k];
        s[k] += a * xl[q];
        creg[q] += a * rv[k];
      }
      asm volatile("" : "+v"(creg[q]), "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]));
      __builtin_amdgcn_sched_barrier(0);
    }
    if (p + 1 < p1) load(p + 1);
    // row sums to lane l = PR (p % 16) + row; the group's 64 rows of f
    // are formed and stored by one instruction each
    int idx;
    const double sk = wave_multi_sum<double, PR>(s, lane, idx);
    const double skl = __shfl(sk, 16 * (lane % PR));
    const int pp = (int)(p % 16);
    if (lane / PR == pp) skeep = skl;
    if (pp == 15 || p + 1 == p1) {
      const int64_t i = (p - pp) * PR + lane;
      if (i >= p0 * PR && i < i0 + PR && i < m) {
        const double fi = ((double)b[i] - r[i]) - skeep;
        f[i] = fi;
        fn += fi * fi;
      }
    }
  }
  for (int wv = 0; wv < 4; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int q = 0; q < Q; ++q) cred[lane + 64 * q] = (wv ? cred[lane + 64 * q] : 0.0) + creg[q];
    }
    __syncthreads();
  }
  for (int64_t c = threadIdx.x; c < n; c += kThreads) tpart[c * gridDim.x + blockIdx.x] = cred[c];
  fn = block_sum256(fn, dsh);
  if (threadIdx.x == 0) fpart[blockIdx.x] = fn;
}

// ------------------------------------------------------------------ FGMRES on [I B; B^T 0]
struct FgPtrs {
  double* V;        // (m + n) x (kmax + 1), ld ldv; column j stored unnormalised until iteration j
  int64_t ldv;
  double* H;        // (kmax + 1) x kmax, ld kmax + 1
  double* cs;
  double* sn;
  double* g;
  double* hj;       // norm used to normalise the current column
  FgState* st;
};

// Column j: h = ||u_j|| from partials (j = 0: beta = ||s||, and block 0
// starts the cycle's state); h is stored for the kernels after the pass, and
// a zero or non-finite h ends the pass (the Gram-Schmidt stage then closes the
// cycle).  Then, per panel of P (one wave per contiguous panel range, next
// panel in flight):
// v_r = V_r[:, j] / h (written back normalised), w_r = v_r + P y ->
// V_r[:, j+1], and the lanes' column partials of t = P^T v_r, with products
// and sums in TC.  B-path: P = B = A W in its precision TB, y = v_x = V_x[:, j] / h
// (xin null), TC = TB.  A-path: P = A in its storage precision (panel copy),
// y = W v_x = xin / h with xin = W V_x[:, j], TC = binary64: the products with
// the preconditioned operator in binary64 over the stored data.
template <typename TB, typename TC, int Q>
__global__ __launch_bounds__(kThreads) void k_fg_pan(const TB* __restrict__ Bp, int64_t npan, int64_t m, int64_t n,
                                                     FgPtrs F, int j, const double* __restrict__ w2part, int Gw,
                                                     TC* __restrict__ tpart, const double* __restrict__ xin) {
  if (F.st->done) return;
  using vec_t = typename PanVec<TB>::type;
  constexpr int PR = PanVec<TB>::PR;
  __shared__ TC cred[64 * Q];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double* vj = F.V + (int64_t)j * F.ldv;
  double* w = F.V + (int64_t)(j + 1) * F.ldv;
  const int64_t nw = (int64_t)gridDim.x * 4;
  int64_t p0, p1;
  row_range(npan, (int)nw, blockIdx.x * 4 + wave, p0, p1);
  vec_t cur[Q];
  double vro[PR];
  // v_j's rows of a panel: 16-byte loads where the column is aligned to them
  const bool vvec = (((uintptr_t)vj | (uintptr_t)w) & 15) == 0;
  auto load = [&](int64_t p, vec_t* dst, double* vr_) {
    const TB* base = Bp + p * (PR * n);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t c = lane + 64 * q;
      dst[q] = (c < n) ? *reinterpret_cast<const vec_t*>(base + c * PR) : vec_t{};
    }
    const int64_t i0 = p * PR;
    if (vvec && i0 + PR <= m) {
#pragma unroll
      for (int k = 0; k < PR; k += 2) {
        const ls_double2v t2 = *reinterpret_cast<const ls_double2v*>(vj + i0 + k);
        vr_[k] = t2[0];
        vr_[k + 1] = t2[1];
      }
    } else {
#pragma unroll
      for (int k = 0; k < PR; ++k) vr_[k] = (i0 + k < m) ? vj[i0 + k] : 0.0;
    }
  };
  // the first panel of B, its rows of v_j and the lane's entries of y do not
  // depend on ||w||: their loads go out before the norm's partials are summed
  if (p0 < p1) load(p0, cur, vro);
  const double* xs = xin ? xin : vj + m;
  double xraw[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t c = lane + 64 * q;
    xraw[q] = (c < n) ? xs[c] : 0.0;
  }
  constexpr int kNl = (Q >= 32) ? 0 : 32;   // the widest rows keep the looped sum (registers)
  const double h = sqrt((kNl > 0 && Gw <= 64 * kNl) ? wave_sum_array_all<(kNl > 0 ? kNl : 1)>(w2part, Gw, lane)
                                                   : wave_sum_array(w2part, Gw, lane));
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *F.hj = h;
    if (j == 0) {
      FgState S = *F.st;
      S.beta = h;
      F.g[0] = h;
      S.relres = 1.0;
      S.k = 0;
      if (h == 0.0 || !isfinite(h)) {
        S.done = 1;
        S.breakdown = (h == 0.0) ? 0 : 2;
      }
      *F.st = S;
    }
  }
  if (h == 0.0 || !isfinite(h)) return;
  const double inv = 1.0 / h;
  constexpr int GP = 64 / PR;   // panels per group of 64 rows
  double wkeep = 0.0, vkeep = 0.0;
  TC vl[Q], creg[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t c = lane + 64 * q;
    vl[q] = (c < n) ? (TC)(xraw[q] * inv) : TC(0);
    creg[q] = 0;
  }
  for (int64_t p = p0; p < p1; ++p) {
    // binary64 products of binary32 entries: converting a whole panel at once
    // would take the registers of a second panel, so the next panel is loaded
    // after the current one is used (faster than prefetching, measured at one
    // wave per SIMD)
    constexpr bool kConv = sizeof(TC) > sizeof(TB);
    constexpr bool PF = kPanPrefetch<Q> && !kConv;
    vec_t nxt[PF ? Q : 1];
    double vrn[PR];
    if (PF && p + 1 < p1) load(p + 1, nxt, vrn);
    const int64_t i0 = p * PR;
    double vr[PR];
    TC vrt[PR], s[PR];
#pragma unroll
    for (int k = 0; k < PR; ++k) {
      vr[k] = vro[k] * inv;
      vrt[k] = (TC)vr[k];
      s[k] = 0;
    }
    if constexpr (kConv) {
      // both products of an entry while its binary64 conversion is live; the
      // scheduling barrier keeps the compiler from converting every entry first
#pragma unroll
      for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int k = 0; k < PR; ++k) {
          const TC a = (TC)cur[q][k];
          s[k] += a * vl[q];
          creg[q] += a * vrt[k];
        }
        // the empty asm takes both sums as they stand, so neither product can
        // be moved past it (else every converted entry stays live to the end)
        asm volatile("" : "+v"(creg[q]), "+v"(s[0]), "+v"(s[1]), "+v"(s[2]), "+v"(s[3]));
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int k = 0; k < PR; ++k) s[k] += (TC)cur[q][k] * vl[q];
    }
    // the panel's row sums: a transposed butterfly leaves row idx's on lanes
    // GP idx .. GP (idx + 1) - 1.  Lane l keeps row l % PR of panel l / PR of
    // an aligned group of GP panels; the group's 64 rows of w and v_j then go
    // out as one 512-byte store each
    int idx;
    const TC sk = wave_multi_sum<TC, PR>(s, lane, idx);
    const TC skl = __shfl(sk, GP * (lane % PR));
    const int pp = (int)(p % GP);
    if (lane / PR == pp) {
#pragma unroll
      for (int k2 = 0; k2 < PR; ++k2)
        if (k2 == lane % PR) {
          wkeep = (double)(vrt[k2] + skl);
          vkeep = vr[k2];
        }
    }
    if (pp == GP - 1 || p + 1 == p1) {
      const int64_t i = (p - pp) * PR + lane;
      if (i >= p0 * PR && i < i0 + PR && i < m) {
        w[i] = wkeep;
        vj[i] = vkeep;
      }
    }
    if constexpr (!kConv) {
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int k = 0; k < PR; ++k) creg[q] += (TC)cur[q][k] * vrt[k];
    }
    if (p + 1 < p1) {
      if constexpr (PF) {
#pragma unroll
        for (int q = 0; q < Q; ++q) cur[q] = nxt[q];
#pragma unroll
        for (int k = 0; k < PR; ++k) vro[k] = vrn[k];
      } else {
        load(p + 1, cur, vro);
      }
    }
  }
  for (int wv = 0; wv < 4; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int q = 0; q < Q; ++q) cred[lane + 64 * q] = (wv ? cred[lane + 64 * q] : TC(0)) + creg[q];
    }
    __syncthreads();
  }
  for (int64_t c = threadIdx.x; c < n; c += kThreads) tpart[c * gridDim.x + blockIdx.x] = cred[c];
}

// One wave per column (16 per block): t = P^T v_r from the pass's column
// partials; V_x[:, j] normalised by the pass's h; B-path (tout null): w_x = t
// -> V[m:, j+1]; A-path: t -> tout (k_fg_wt forms w_x = W^T t).
template <typename TB>
__global__ __launch_bounds__(1024) void k_fg_col(int64_t m, int64_t n, const TB* __restrict__ tpart, int G, FgPtrs F,
                                                 int j, double* __restrict__ tout) {
  if (F.st->done) return;
  const double h = *F.hj;
  if (h == 0.0 || !isfinite(h)) return;   // the Gram-Schmidt stage closes the cycle
  const int lane = threadIdx.x & 63;
  const int wvi = threadIdx.x >> 6;
  const int64_t col = (int64_t)blockIdx.x * 16 + wvi;
  if (col >= n) return;
  const double inv = 1.0 / h;
  const TB* tp = tpart + col * G;
  TB acc = 0;
  for (int g0 = 0; g0 < G; g0 += 512) {   // eight loads per lane in flight
    TB v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int g = g0 + 64 * q + lane;
      v[q] = (g < G) ? tp[g] : TB(0);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc += v[q];
  }
  acc = ls_wave_sum(acc);
  if (lane == 0) {
    double* vj = F.V + (int64_t)j * F.ldv;
    vj[m + col] *= inv;
    if (tout) tout[col] = (double)acc;
    else F.V[m + col + (int64_t)(j + 1) * F.ldv] = (double)acc;
  }
}

// A-path, before the pass of column j: xin = W V[m:, j] (the x part of v_j
// before its normalisation, which the pass applies).  W^T follows W in memory:
// row r of W is column r of W^T, contiguous; one wave per row, 16 per block.
__global__ __launch_bounds__(1024) void k_fg_zx(const double* __restrict__ W, int64_t n, FgPtrs F, int64_t m, int j,
                                                double* __restrict__ xin) {
  if (F.st->done) return;
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* wr = W + n * n + row * n;   // W[row, :] = W^T[:, row]
  const double* vx = F.V + (int64_t)j * F.ldv + m;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t c0 = row + lane; c0 < n; c0 += 64 * 8) {   // eight loads per lane in flight
    double wv[8], xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t c = c0 + 64 * q;
      wv[q] = (c < n) ? wr[c] : 0.0;
      xv[q] = (c < n) ? vx[c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q & 3] += wv[q] * xv[q];
  }
  const double z = ls_wave_sum((a[0] + a[1]) + (a[2] + a[3]));
  if (lane == 0) xin[row] = z;
}

// A-path, after the pass: w_x = W^T t -> V[m:, j+1] (one wave per column,
// 16 columns per block, column c of W being row c of W^T).
__global__ __launch_bounds__(1024) void k_fg_wt(const double* __restrict__ W, int64_t m, int64_t n,
                                                const double* __restrict__ t, FgPtrs F, int j) {
  if (F.st->done) return;
  const double h = *F.hj;
  if (h == 0.0 || !isfinite(h)) return;
  const int lane = threadIdx.x & 63;
  const int wvi = threadIdx.x >> 6;
  const int64_t col = (int64_t)blockIdx.x * 16 + wvi;
  if (col >= n) return;
  const double* wc = W + col * n;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i0 = lane; i0 <= col; i0 += 64 * 8) {   // eight loads per lane in flight
    double wv[8], tv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t i = i0 + 64 * q;
      wv[q] = (i <= col) ? wc[i] : 0.0;
      tv[q] = (i <= col) ? t[i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q & 3] += wv[q] * tv[q];
  }
  const double val = ls_wave_sum((a[0] + a[1]) + (a[2] + a[3]));
  if (lane == 0) F.V[m + col + (int64_t)(j + 1) * F.ldv] = val;
}

// A copied into the panel layout of B, in its storage precision (the A-path's
// operand): a block moves 64 rows x 64 columns through LDS, reading each
// column's rows with coalesced 16-byte loads and writing each panel's 64
// columns as one contiguous 1 KB run.  Rows of the last panel past m are zero.
template <typename TA>
__global__ __launch_bounds__(kThreads) void k_a_panels(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                       int vec_ok, TA* __restrict__ Ap) {
  using vec_t = typename PanVec<TA>::type;
  constexpr int PR = PanVec<TA>::PR;
  constexpr int NP = 64 / PR;   // panels in the tile
  __shared__ vec_t tile[64][NP + 1];
  const int t = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int64_t c0 = (int64_t)blockIdx.y * 64;
  const int64_t npan = ls_cdiv(m, PR);
  for (int u = t; u < 64 * NP; u += kThreads) {
    const int c = u / NP, pq = u % NP;
    const int64_t gc = c0 + c, gi = i0 + (int64_t)pq * PR;
    vec_t v{};
    if (gc < n && gi < m) {
      const TA* src = A + gi + gc * lda;
      if (vec_ok && gi + PR <= m) {
        v = *reinterpret_cast<const vec_t*>(src);
      } else {
#pragma unroll
        for (int k = 0; k < PR; ++k) v[k] = (gi + k < m) ? src[k] : TA(0);
      }
    }
    tile[c][pq] = v;
  }
  __syncthreads();
  for (int u = t; u < 64 * NP; u += kThreads) {
    const int pq = u / 64, c = u % 64;
    const int64_t gp = i0 / PR + pq, gc = c0 + c;
    if (gp < npan && gc < n) *reinterpret_cast<vec_t*>(Ap + gp * PR * n + gc * PR) = tile[c][pq];
  }
}

// sum_{c <= j} V[i + c ldv] h[c] with NL independent loads in flight: the
// columns in groups of NL, the last group guarded (its loads issued together
// like the others; columns beyond j add zero).
template <int NL = 8>
__device__ __forceinline__ double vrow_dot(const double* __restrict__ V, int64_t ldv, int64_t i, int j,
                                           const double* __restrict__ h) {
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int c = 0; c <= j; c += NL) {
    double v[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) v[q] = (c + q <= j) ? V[i + (int64_t)(c + q) * ldv] : 0.0;
#pragma unroll
    for (int q = 0; q < NL; ++q) a[q & 7] += v[q] * ((c + q <= j) ? h[c + q] : 0.0);
  }
  return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// Arnoldi orthogonalisation: classical Gram-Schmidt with the second pass
// (reorthogonalisation) of each vector delayed to the next iteration, so that
// one sweep over V computes every inner product an iteration needs and one
// more sweep applies every update (V is read twice per iteration).
//
// Entering iteration j, V[:, 0:j] are final (orthonormal) and V[:, j] holds
// u_j, the previous iteration's vector after one Gram-Schmidt pass; the pass
// normalises it to q_j = u_j / beta_j and writes w = M q_j to V[:, j+1] (M the
// split-preconditioned augmented operator).  Then:
//   sweep 1 (k_dcgs_dots): s = V_{<j}^T q_j, b = V_{<j}^T w, q_j . w, q_j . q_j;
//   the stage (every block of sweep 2): the second pass of q_j, v_j = (q_j - V s) / nu
//     with nu^2 = q_j . q_j - |s|^2, makes column j-1 of the Hessenberg matrix
//     final (H[<j, j-1] += beta_j s, H[j, j-1] = beta_j nu; the Givens
//     rotations and the convergence test are applied to it); M v_j follows
//     from w and the Arnoldi relation of the earlier columns,
//     M v_j = (w - V_{<=j} t) / nu with t = H[0:j+1, 0:j] s, whose first-pass
//     coefficients h'_j = V_{<=j}^T M v_j come from s, b and t alone; u_{j+1} =
//     M v_j - V_{<=j} h'_j = w / nu - V_{<j} d - (gamma / nu) q_j;
//   sweep 2 (k_dcgs_update): writes v_j and u_{j+1} and the partials of
//     |u_{j+1}|^2.
// H keeps the rotated columns (the triangular factor of the least-squares
// problem), Hraw the unrotated final ones (t needs them), pend the pending
// first-pass column.  A cycle that reaches its iteration limit closes with a
// sweep and a stage of the same kind for its last column (closing = 1: no w).
constexpr int kSweepThreads = 512;   // rows of V per block of the sweeps (one per thread)
constexpr int kSweepWaves = kSweepThreads / 64;
// Above this many row blocks the sweep's partials are summed by a launch of
// their own (k_colsum_parts, once) rather than by the one-block stage.
constexpr int kSweepSumAbove = 512;
constexpr int kMaxDots = 2 * kMaxKrylov + 2;   // quantities of sweep 1

// out[e] = sum of the G partials part[e G + g], one block per quantity e.
__global__ __launch_bounds__(kThreads) void k_colsum_parts(const FgState* __restrict__ st,
                                                           const double* __restrict__ part, int G,
                                                           double* __restrict__ out) {
  if (st->done) return;
  __shared__ double dsh[4];
  const double* pc = part + (int64_t)blockIdx.x * G;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int g0 = threadIdx.x; g0 < G; g0 += 4 * kThreads) {
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int g = g0 + q * kThreads;
      v[q] = (g < G) ? pc[g] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] += v[q];
  }
  const double t = block_sum256((a[0] + a[1]) + (a[2] + a[3]), dsh);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// Sweep 1 over rows [512 b, 512 b + 512): partials part[e G + b] of
// e = c < j: V[:, c] . q;  e = j + c (c < j): V[:, c] . w;  e = 2j: q . w;
// e = 2j + 1: q . q;  q = V[:, j], w = V[:, j+1] (closing: no w, q = u_j).
__global__ __launch_bounds__(kSweepThreads) void k_dcgs_dots(FgPtrs F, int64_t rows, int j, int closing,
                                                             double* __restrict__ part) {
  if (F.st->done) return;
  if (!closing) {
    const double h = *F.hj;
    if (h == 0.0 || !isfinite(h)) return;   // the stage closes the cycle without the partials
  }
  __shared__ double qs[kSweepThreads];
  __shared__ double ws[kSweepThreads];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int G = gridDim.x;
  const int64_t base = (int64_t)blockIdx.x * kSweepThreads;
  const int64_t i = base + threadIdx.x;
  const double* q = F.V + (int64_t)j * F.ldv;
  qs[threadIdx.x] = (i < rows) ? q[i] : 0.0;
  ws[threadIdx.x] = (!closing && i < rows) ? q[F.ldv + i] : 0.0;
  __syncthreads();
  // wave per Krylov column, the loads of kCols columns (kSweepWaves rows per
  // lane each) issued together
  constexpr int kCols = 4;
  for (int c0 = wave; c0 < j; c0 += kCols * kSweepWaves) {
    double as[kCols], ab[kCols];
#pragma unroll
    for (int cc = 0; cc < kCols; ++cc) {
      const int c = c0 + kSweepWaves * cc;
      as[cc] = 0.0;
      ab[cc] = 0.0;
      if (c < j) {
        const double* vc = F.V + (int64_t)c * F.ldv + base;
        double v[kSweepWaves];
#pragma unroll
        for (int u = 0; u < kSweepWaves; ++u) {
          const int li = u * 64 + lane;
          v[u] = (base + li < rows) ? vc[li] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSweepWaves; ++u) {
          as[cc] += v[u] * qs[u * 64 + lane];
          ab[cc] += v[u] * ws[u * 64 + lane];
        }
      }
    }
#pragma unroll
    for (int cc = 0; cc < kCols; ++cc) {
      const int c = c0 + kSweepWaves * cc;
      const double t1 = ls_wave_sum(as[cc]);
      const double t2 = ls_wave_sum(ab[cc]);
      if (c < j && lane == 0) {
        part[(int64_t)c * G + blockIdx.x] = t1;
        if (!closing) part[(int64_t)(j + c) * G + blockIdx.x] = t2;
      }
    }
  }
  if (wave == kSweepWaves - 1 || wave == kSweepWaves - 2) {
    const bool qq = (wave == kSweepWaves - 1);
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < kSweepWaves; ++u) {
      const int li = u * 64 + lane;
      a += qs[li] * (qq ? qs[li] : ws[li]);
    }
    a = ls_wave_sum(a);
    if (lane == 0 && (qq || !closing)) part[(int64_t)(2 * j + (qq ? 1 : 0)) * G + blockIdx.x] = a;
  }
}

// The stage of iteration j, computed by every block of sweep 2 (each from the
// same data in the same order, so that all hold the same coefficients):
// sums the sweep's partials (Gp per quantity; 1 when k_colsum_parts has summed
// them); stages Hraw's final columns 0 .. j-2 and the pending first-pass
// column j-1 (pend[(j-1) % 2]); completes column j-1 (H[<j, j-1] += beta s,
// H[j, j-1] = beta nu) and, unless the cycle closes, forms column j's
// first-pass coefficients h'_j and sweep 2's coefficients s, d, 1/nu,
// gamma/nu.  The writer block (block 0) stores the final column j-1 in Hraw,
// applies the Givens rotations to it (the convergence test) and stores h'_j in
// pend[j % 2]; no block reads what the writer stores in the same launch.
constexpr int kTriMax = kMaxKrylov * (kMaxKrylov + 3) / 2;   // columns 0 .. j-1, rows <= k + 1
struct DcgsLds {
  double e[kMaxDots];
  double tri[kTriMax];   // column k at k (k + 3) / 2, rows 0 .. k + 1
  double sv[kMaxKrylov + 1];
  double dv[kMaxKrylov + 1];
  double tv[kMaxKrylov + 1];
  double css[kMaxKrylov], sns[kMaxKrylov];
  double sc[8];          // beta, nu, s . b, 1/nu, gamma/nu
};

// Returns true when sweep 2 should run (a regular iteration whose vector did
// not break down).
template <int NT>
__device__ bool dcgs_stage(const FgPtrs& F, double* __restrict__ Hraw, double* __restrict__ pend, int kmax, int j,
                           int closing, const double* __restrict__ part, int Gp, double tol, Progress* prog,
                           bool writer, DcgsLds& L) {
  constexpr int nwaves = NT / 64;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t ldh = kmax + 1;
  const double hj = closing ? 0.0 : *F.hj;
  const bool skip = !closing && (hj == 0.0 || !isfinite(hj));   // no sweep ran: nothing to read
  const int ne = 2 * j + 2;
  auto wanted = [&](int q) { return !(closing && q >= j && q < 2 * j + 1); };   // the closing sweep has no w
  if (!skip) {
    if (Gp == 1) {
      for (int q = tid; q < ne; q += NT)
        if (wanted(q)) L.e[q] = part[q];
    } else {
      // wave per quantity, four quantities' loads (up to eight per lane each) in flight
      for (int q0 = wave; q0 < ne; q0 += 4 * nwaves) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        for (int g0 = lane; g0 < Gp; g0 += 64 * 8) {
          double v[4][8];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int q = q0 + nwaves * u;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const int g = g0 + 64 * k;
              v[u][k] = (q < ne && wanted(q) && g < Gp) ? part[(int64_t)q * Gp + g] : 0.0;
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < 8; ++k) a[u] += v[u][k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = q0 + nwaves * u;
          const double t = ls_wave_sum(a[u]);
          if (lane == 0 && q < ne) L.e[q] = t;
        }
      }
    }
  }
  // final columns 0 .. j-2 from Hraw, pending column j-1 from pend
  const int ntri = j * (j + 3) / 2;
  const double* pj = pend + (int64_t)((j - 1) & 1) * ldh;
  for (int idx = tid; idx < ntri; idx += NT) {
    int k = (int)((sqrt(8.0 * idx + 9.0) - 3.0) * 0.5);   // column of idx: k (k + 3) / 2 <= idx
    while (k > 0 && k * (k + 3) / 2 > idx) --k;
    while ((k + 1) * (k + 4) / 2 <= idx) ++k;
    const int r = idx - k * (k + 3) / 2;
    L.tri[idx] = (k == j - 1) ? ((r < j) ? pj[r] : 0.0) : Hraw[r + (int64_t)k * ldh];
  }
  if (writer)
    for (int i = tid; i < j - 1; i += NT) {
      L.css[i] = F.cs[i];
      L.sns[i] = F.sn[i];
    }
  __syncthreads();
  // s, beta and nu (wave 0)
  if (wave == 0) {
    const double beta = closing ? sqrt(L.e[2 * j + 1]) : hj;
    double nu = 1.0;   // j = 0: v_0 is final
    if (j > 0) {
      if (skip || !isfinite(beta) || beta == 0.0) {
        nu = 0.0;
      } else {
        const double inv = closing ? 1.0 / beta : 1.0;
        double ss = 0.0;
        for (int c = lane; c < j; c += 64) {
          const double v = L.e[c] * inv;
          L.sv[c] = v;
          ss += v * v;
        }
        ss = ls_wave_sum(ss);
        const double sig = closing ? 1.0 : L.e[2 * j + 1];
        const double nu2 = sig - ss;
        nu = (nu2 > 0.0) ? sqrt(nu2) : 0.0;
      }
    }
    if (lane == 0) {
      L.sc[0] = beta;
      L.sc[1] = nu;
    }
  }
  __syncthreads();
  const double beta = L.sc[0], nu = L.sc[1];
  const bool ok = (j == 0) || (isfinite(beta) && beta > 0.0 && nu > 0.0);
  if (j > 0) {
    // column j - 1 becomes final
    double* tc = L.tri + (j - 1) * (j + 2) / 2;
    for (int c = tid; c <= j; c += NT) {
      double v = tc[c];
      if (c < j) {
        if (ok) v += beta * L.sv[c];
      } else {
        v = ok ? beta * nu : 0.0;
      }
      tc[c] = v;
      if (writer) Hraw[c + (int64_t)(j - 1) * ldh] = v;
    }
    __syncthreads();
    if (writer && tid == 0) {
      // Givens rotations of the earlier columns, then a new one for this column
      FgState S = *F.st;
      const double sub = tc[j];
      double* Hc = F.H + (int64_t)(j - 1) * ldh;
      double x = tc[0];
      for (int i = 0; i < j - 1; ++i) {
        const double y = tc[i + 1];
        Hc[i] = L.css[i] * x + L.sns[i] * y;
        x = -L.sns[i] * x + L.css[i] * y;
      }
      const double dd = hypot(x, sub);
      const double cc = (dd > 0.0) ? x / dd : 1.0;
      const double sn = (dd > 0.0) ? sub / dd : 0.0;
      F.cs[j - 1] = cc;
      F.sn[j - 1] = sn;
      Hc[j - 1] = dd;
      Hc[j] = 0.0;
      const double gl = F.g[j - 1];
      F.g[j] = -sn * gl;
      F.g[j - 1] = cc * gl;
      S.relres = fabs(sn * gl) / S.beta;
      S.k = j;
      int done = 0;
      if (!isfinite(S.relres) || !isfinite(beta)) {
        done = 1;
        S.breakdown = 2;
      } else if (S.relres <= tol || sub == 0.0 || closing || j >= kmax) {
        done = 1;
        if (sub == 0.0) S.breakdown = 1;
      }
      if (done) S.done = 1;
      *F.st = S;
      if (prog) {
        progress_put(&prog->fg_done, done);
        progress_put(&prog->fg_j, j);
      }
    }
  }
  if (closing || !ok) return false;
  // t = Hraw[0:j+1, 0:j] s (column k holding rows <= k + 1)
  for (int c = tid; c <= j; c += NT) {
    double a = 0.0;
    for (int k = (c > 0 ? c - 1 : 0); k < j; ++k) a += L.tri[k * (k + 3) / 2 + c] * L.sv[k];
    L.tv[c] = a;
  }
  if (wave == nwaves - 1) {
    double sb = 0.0;
    for (int c = lane; c < j; c += 64) sb += L.sv[c] * L.e[j + c];
    sb = ls_wave_sum(sb);
    if (lane == 0) L.sc[2] = sb;
  }
  __syncthreads();
  const double inu = 1.0 / nu;
  double* pn = pend + (int64_t)(j & 1) * ldh;
  for (int c = tid; c <= j; c += NT) {
    const double h = (c < j) ? (L.e[j + c] - L.tv[c]) * inu : ((L.e[2 * j] - L.sc[2]) * inu - L.tv[j]) * inu;
    if (writer) pn[c] = h;
    L.tv[c] = L.tv[c] * inu + h;   // c < j: the coefficient of V[:, c]; c = j: gamma
  }
  __syncthreads();
  const double gq = L.tv[j] * inu;   // gamma / nu
  for (int c = tid; c < j; c += NT) L.dv[c] = L.tv[c] - gq * L.sv[c];
  if (tid == 0) {
    L.sc[3] = inu;
    L.sc[4] = gq;
  }
  __syncthreads();
  return true;
}

// A cycle at its iteration limit: the second pass of u_kmax makes column
// kmax - 1 final (one block).
__global__ __launch_bounds__(kSweepThreads) void k_dcgs_close(FgPtrs F, double* __restrict__ Hraw,
                                                              double* __restrict__ pend, int kmax,
                                                              const double* __restrict__ part, int Gp) {
  if (F.st->done) return;
  __shared__ DcgsLds L;
  dcgs_stage<kSweepThreads>(F, Hraw, pend, kmax, kmax, 1, part, Gp, F.st->tol, nullptr, true, L);
}

// Sweep 2 over the block's rows: v_j = (q - V_{<j} s) / nu -> V[:, j] and
// u_{j+1} = w / nu - V_{<j} d - (gamma / nu) q -> V[:, j+1]; partial
// |u_{j+1}|^2 -> w2part.
__device__ __forceinline__ void dcgs_rows(const FgPtrs& F, int64_t rows, int j, const double* sv, const double* dv,
                                          double inu, double gq, double* __restrict__ w2part, double* dsh) {
  const int64_t i = (int64_t)blockIdx.x * kSweepThreads + threadIdx.x;
  double nrm = 0.0;
  if (i < rows) {
    double as[8] = {0, 0, 0, 0, 0, 0, 0, 0}, ad[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    constexpr int NL = 16;   // loads of V in flight per thread
    for (int c = 0; c < j; c += NL) {
      double v[NL];
#pragma unroll
      for (int q = 0; q < NL; ++q) v[q] = (c + q < j) ? F.V[i + (int64_t)(c + q) * F.ldv] : 0.0;
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const bool in = (c + q < j);
        as[q & 7] += v[q] * (in ? sv[c + q] : 0.0);
        ad[q & 7] += v[q] * (in ? dv[c + q] : 0.0);
      }
    }
    const double vs = ((as[0] + as[1]) + (as[2] + as[3])) + ((as[4] + as[5]) + (as[6] + as[7]));
    const double vd = ((ad[0] + ad[1]) + (ad[2] + ad[3])) + ((ad[4] + ad[5]) + (ad[6] + ad[7]));
    double* q = F.V + (int64_t)j * F.ldv;
    const double qi = q[i], wi = q[F.ldv + i];
    const double u = wi * inu - vd - gq * qi;
    q[i] = (qi - vs) * inu;
    q[F.ldv + i] = u;
    nrm = u * u;
  }
  nrm = ls_block_sum<double, kSweepThreads>(nrm, dsh);
  if (threadIdx.x == 0) w2part[blockIdx.x] = nrm;
}

// Sweep 2 with the stage in every block (few row blocks: the stage's reads are
// cheap and its launch is saved).
__global__ __launch_bounds__(kSweepThreads) void k_dcgs_update(FgPtrs F, int64_t rows, int j, double* __restrict__ Hraw,
                                                               double* __restrict__ pend, int kmax,
                                                               const double* __restrict__ part, int Gp,
                                                               Progress* prog, double* __restrict__ w2part) {
  if (F.st->done) return;
  __shared__ DcgsLds L;
  __shared__ double dsh[kSweepWaves];
  if (!dcgs_stage<kSweepThreads>(F, Hraw, pend, kmax, j, 0, part, Gp, F.st->tol, prog, blockIdx.x == 0, L)) return;
  dcgs_rows(F, rows, j, L.sv, L.dv, L.sc[3], L.sc[4], w2part, dsh);
}

// Many row blocks: the stage runs once (one block) and stores sweep 2's
// coefficients coef = [s (j), d (j), 1/nu, gamma/nu, go], go = 0 when sweep 2
// is not needed; k_dcgs_apply then reads them.
__global__ __launch_bounds__(kSweepThreads) void k_dcgs_stage(FgPtrs F, int j, double* __restrict__ Hraw,
                                                              double* __restrict__ pend, int kmax,
                                                              const double* __restrict__ part, int Gp,
                                                              Progress* prog, double* __restrict__ coef) {
  if (F.st->done) return;
  __shared__ DcgsLds L;
  const bool go = dcgs_stage<kSweepThreads>(F, Hraw, pend, kmax, j, 0, part, Gp, F.st->tol, prog, true, L);
  for (int c = threadIdx.x; c < j; c += kSweepThreads) {
    coef[c] = L.sv[c];
    coef[j + c] = L.dv[c];
  }
  if (threadIdx.x == 0) {
    coef[2 * j] = L.sc[3];
    coef[2 * j + 1] = L.sc[4];
    coef[2 * j + 2] = go ? 1.0 : 0.0;
  }
}

__global__ __launch_bounds__(kSweepThreads) void k_dcgs_apply(FgPtrs F, int64_t rows, int j,
                                                              const double* __restrict__ coef,
                                                              double* __restrict__ w2part) {
  if (F.st->done) return;
  __shared__ double cs_[2 * kMaxKrylov + 3];
  __shared__ double dsh[kSweepWaves];
  for (int t = threadIdx.x; t < 2 * j + 3; t += kSweepThreads) cs_[t] = coef[t];
  __syncthreads();
  if (cs_[2 * j + 2] == 0.0) return;
  dcgs_rows(F, rows, j, cs_, cs_ + j, cs_[2 * j], cs_[2 * j + 1], w2part, dsh);
}

// Correction of one refinement step: y = H(0:k,0:k)^-1 g(0:k) (every block);
// rows < m: dr = V_r y, r += dr (working precision TU), partial norms of dr
// and r (and, with r_ref, of r - r_ref and r_ref), four per block;
// rows >= m: dz = V_x y -> dz buffer.
template <typename TU>
__global__ __launch_bounds__(kThreads) void k_fg_update(FgPtrs F, int64_t m, int64_t n, int kmax,
                                                        double* __restrict__ r, double* __restrict__ dz,
                                                        double* __restrict__ part, const double* __restrict__ r_ref) {
  __shared__ double y[128];
  __shared__ double dsh[16];
  __shared__ double Hs[kMaxKrylov * (kMaxKrylov + 1) / 2];   // upper triangle, column c at c (c + 1) / 2
  const int k = F.st->k;
  const int64_t ldh = kmax + 1;
  for (int i = threadIdx.x; i < k; i += kThreads) y[i] = F.g[i];
  // stage H(0:k, 0:k)'s upper triangle in LDS (eight loads per thread in
  // flight), so that the substitution below waits on no global load
  const int kk = k * k;
  for (int b0 = 0; b0 < kk; b0 += 8 * kThreads) {
    double hv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = b0 + (int)threadIdx.x + kThreads * u;
      hv[u] = 0.0;
      if (idx < kk) {
        const int c = idx / k, t = idx - c * k;
        if (t <= c) hv[u] = F.H[t + (int64_t)c * ldh];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = b0 + (int)threadIdx.x + kThreads * u;
      if (idx < kk) {
        const int c = idx / k, t = idx - c * k;
        if (t <= c) Hs[c * (c + 1) / 2 + t] = hv[u];
      }
    }
  }
  for (int i = k - 1; i >= 0; --i) {
    __syncthreads();
    const double* hc = Hs + i * (i + 1) / 2;
    const double yi = y[i] / hc[i];
    __syncthreads();
    if (threadIdx.x == 0) y[i] = yi;
    for (int t = threadIdx.x; t < i; t += kThreads) y[t] -= hc[t] * yi;
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (i < m + n) {
    const double d = (k > 0) ? vrow_dot(F.V, F.ldv, i, k - 1, y) : 0.0;
    if (i < m) {
      const double rn = (double)((TU)r[i] + (TU)d);
      r[i] = rn;
      a0 = d * d;
      a1 = rn * rn;
      if (r_ref) {
        const double rr = r_ref[i];
        a2 = (rn - rr) * (rn - rr);
        a3 = rr * rr;
      }
    } else {
      dz[i - m] = d;
    }
  }
  a0 = block_sum256(a0, dsh);
  a1 = block_sum256(a1, dsh + 4);
  a2 = block_sum256(a2, dsh + 8);
  a3 = block_sum256(a3, dsh + 12);
  if (threadIdx.x == 0) {
    double* p = part + 4 * (int64_t)blockIdx.x;
    p[0] = a0;
    p[1] = a1;
    p[2] = a2;
    p[3] = a3;
  }
}

// dx = W dz (R^-1 on the x part of the correction), x += dx (TU); partial
// norms of dx and x (and, with x_ref, of x - x_ref and x_ref), four per block.
template <typename TU>
__global__ __launch_bounds__(kUtThreads) void k_fg_dx(const double* __restrict__ W, int64_t n,
                                                      const double* __restrict__ dz, double* __restrict__ x,
                                                      double* __restrict__ part, const double* __restrict__ x_ref) {
  __shared__ double red[32 * 33];
  const double d = ls_utmv_row(W, n, n, [&](int64_t j) { return dz[j]; }, red);
  const int64_t row = (int64_t)blockIdx.x * 32 + threadIdx.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (threadIdx.x < 32 && row < n) {
    const double xn = (double)((TU)x[row] + (TU)d);
    x[row] = xn;
    a0 = d * d;
    a1 = xn * xn;
    if (x_ref) {
      const double xr = x_ref[row];
      a2 = (xn - xr) * (xn - xr);
      a3 = xr * xr;
    }
  }
  if (threadIdx.x < 64) {   // rows of the block live in the first wave
    a0 = ls_wave_sum(a0);
    a1 = ls_wave_sum(a1);
    a2 = ls_wave_sum(a2);
    a3 = ls_wave_sum(a3);
    if (threadIdx.x == 0) {
      double* p = part + 4 * (int64_t)blockIdx.x;
      p[0] = a0;
      p[1] = a1;
      p[2] = a2;
      p[3] = a3;
    }
  }
}

// ------------------------------------------------------------------ host helpers
// Device properties are read once (thread-safe static initialisation); the
// library assumes the devices of one process are alike.
size_t device_lds_limit() {
  static const size_t cached = [] {
    size_t v = 0;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) v = prop.sharedMemPerBlock;
    return v ? v : (size_t)64 * 1024;
  }();
  return cached;
}

// 16-byte vector loads of a column-major matrix are possible (base aligned,
// leading dimension a multiple of the vector length).
bool vec_aligned(const void* M, int64_t ld, size_t elt) {
  const size_t v = 16 / elt;
  return ((uintptr_t)M % 16 == 0) && (ld % (int64_t)v == 0);
}

// Loads per lane for one panel: the smallest power of two with 64 Q >= n.
int pan_q(int64_t n) {
  int q = 1;
  while (64 * (int64_t)q < n) q *= 2;
  return q;
}

int64_t pan_count(int64_t m, size_t elt) { return ls_cdiv(m, (int64_t)(16 / elt)); }

// Resident waves per SIMD targeted by the panel passes (LS_PASS_WAVES, 1..8).
int pan_occ() {
  static const int occ = [] {
    if (const char* e = getenv("LS_PASS_WAVES")) {
      const int v = atoi(e);
      if (v >= 1 && v <= 8) return v;
    }
    return 2;
  }();
  return occ;
}

// Blocks of four waves for a pass over npan panels of n columns: at most
// pan_occ() waves per SIMD (one from n > 512 on, where a wave's registers
// take the whole file), every wave given the same number of panels (k or k - 1).
int pan_grid(int64_t npan, int64_t n, int ncu) {
  const int occ = (pan_q(n) >= 16) ? 1 : pan_occ();
  const int64_t nwmax = (int64_t)occ * 4 * ncu;
  const int64_t k = ls_cdiv(npan, nwmax);
  const int64_t nw = ls_cdiv(npan, k);
  const int64_t g = ls_cdiv(nw, 4);
  return (int)(g < 1 ? 1 : g);
}

}  // namespace

int device_lds_bytes() { return (int)device_lds_limit(); }

int device_cu_count() {
  static const int cached = [] {
    int v = 0;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) v = prop.multiProcessorCount;
    return v > 0 ? v : 256;
  }();
  return cached;
}

namespace {
// ------------------------------------------------------------------ progress slots
// One page of pinned, device-mapped, coherent host memory per device, split
// into slots.  A driver call owns one slot from its start to its end (calls on
// other host threads, e.g. the workers of a batched solve, get other slots).
// Kernels store into the slot with system-scope stores; the host polls it.
// Without such memory, or with every slot taken, the drivers synchronise to
// read the state instead.
constexpr int kProgressSlots = 64;
constexpr int kMaxDevices = 64;
struct ProgressPool {
  std::mutex mu;
  bool tried = false;
  Progress* host = nullptr;
  Progress* dev = nullptr;
  uint64_t used = 0;   // bit k: slot k is owned by a call
};

ProgressPool& progress_pool(int dev) {
  static ProgressPool pools[kMaxDevices];
  return pools[(dev >= 0 && dev < kMaxDevices) ? dev : 0];
}

class ProgressSlot {
 public:
  explicit ProgressSlot(hipStream_t st) : st_(st) {
    if (hipGetDevice(&dev_) != hipSuccess || dev_ < 0 || dev_ >= kMaxDevices) return;
    ProgressPool& p = progress_pool(dev_);
    std::lock_guard<std::mutex> g(p.mu);
    if (!p.tried) {
      p.tried = true;
      void* h = nullptr;
      if (hipHostMalloc(&h, sizeof(Progress) * kProgressSlots,
                        hipHostMallocMapped | hipHostMallocPortable | hipHostMallocCoherent) == hipSuccess) {
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) == hipSuccess && d) {
          memset(h, 0, sizeof(Progress) * kProgressSlots);
          p.host = static_cast<Progress*>(h);
          p.dev = static_cast<Progress*>(d);
        } else {
          (void)hipHostFree(h);
        }
      } else {
        (void)hipGetLastError();   // clear the failed allocation's error
      }
    }
    if (!p.host) return;
    for (int k = 0; k < kProgressSlots; ++k) {
      if (!(p.used >> k & 1u)) {
        p.used |= uint64_t{1} << k;
        slot_ = k;
        host = p.host + k;
        dev = p.dev + k;
        return;
      }
    }
  }
  // The slot goes back to the pool once no queued kernel of this call can
  // still store into it; if the stream cannot be drained it stays taken.
  ~ProgressSlot() {
    if (slot_ < 0) return;
    if (hipStreamSynchronize(st_) != hipSuccess) return;
    ProgressPool& p = progress_pool(dev_);
    std::lock_guard<std::mutex> g(p.mu);
    p.used &= ~(uint64_t{1} << slot_);
  }
  ProgressSlot(const ProgressSlot&) = delete;
  ProgressSlot& operator=(const ProgressSlot&) = delete;
  Progress* host = nullptr;
  Progress* dev = nullptr;

 private:
  hipStream_t st_;
  int dev_ = 0;
  int slot_ = -1;
};

// Streams on which graphs are captured (capture records without running, and
// the caller's stream may be the legacy default stream, which cannot be
// captured): a pool per device, each stream held by one call at a time,
// created at the default priority and kept until the process ends.
struct CapturePool {
  std::mutex mu;
  std::vector<hipStream_t> idle;
};
CapturePool& capture_pool(int dev) {
  static CapturePool pools[64];
  return pools[(dev >= 0 && dev < 64) ? dev : 0];
}
struct CaptureStream {
  int dev = 0;
  hipStream_t s = nullptr;
  int acquire() {
    LS_HIP_TRY(hipGetDevice(&dev));
    CapturePool& p = capture_pool(dev);
    std::lock_guard<std::mutex> g(p.mu);
    if (!p.idle.empty()) {
      s = p.idle.back();
      p.idle.pop_back();
      return LS_OK;
    }
    LS_HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    return LS_OK;
  }
  ~CaptureStream() {
    if (!s) return;
    CapturePool& p = capture_pool(dev);
    std::lock_guard<std::mutex> g(p.mu);
    p.idle.push_back(s);
  }
};

// Instantiated graphs of one call, destroyed once the stream has drained.
struct GraphChunks {
  hipStream_t st;
  std::vector<hipGraphExec_t> v;
  ~GraphChunks() {
    if (v.empty()) return;
    (void)hipStreamSynchronize(st);
    for (hipGraphExec_t e : v) (void)hipGraphExecDestroy(e);
  }
};

void progress_set(int32_t* f, int32_t v) { __atomic_store_n(f, v, __ATOMIC_RELEASE); }

// Waits until *val >= target or *done.  Returns 1 when done was seen, 0 when
// the target was reached, -1 when the stream went idle with neither (the slot
// is not being updated).
int progress_wait(int32_t* val, int32_t* done, int target, hipStream_t st) {
  // The stream is queried only after 2 ms without progress (an iteration
  // takes tens of microseconds): a query can place a marker in the stream,
  // which the device then processes between two kernels.
  const auto t0 = std::chrono::steady_clock::now();
  for (unsigned spin = 0;; ++spin) {
    if (__atomic_load_n(done, __ATOMIC_ACQUIRE)) return 1;
    if (__atomic_load_n(val, __ATOMIC_ACQUIRE) >= target) return 0;
    if ((spin & 255u) == 255u && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2) &&
        hipStreamQuery(st) == hipSuccess) {
      if (__atomic_load_n(done, __ATOMIC_ACQUIRE)) return 1;
      return (__atomic_load_n(val, __ATOMIC_ACQUIRE) >= target) ? 0 : -1;
    }
  }
}
}  // namespace

// B = A W (W binary64 n x n, ld n; W32 its binary32 copy), binary32 or binary64.
int form_b(const ls_problem_t* P, const double* W, const float* W32, ls_prec_t tb, void* Bout, hipStream_t st) {
  const dim3 g((unsigned)ls_cdiv(P->m, 64), (unsigned)ls_cdiv(P->n, 64));
  if (tb == LS_FP32) {
    if (P->store == LS_FP32)
      hipLaunchKernelGGL((k_form_b<float, float>), g, dim3(kThreads), 0, st, (const float*)P->A, P->lda, P->m, P->n,
                         W32, (float*)Bout);
    else
      hipLaunchKernelGGL((k_form_b<double, float>), g, dim3(kThreads), 0, st, (const double*)P->A, P->lda, P->m, P->n,
                         W32, (float*)Bout);
  } else {
    if (P->store == LS_FP32)
      hipLaunchKernelGGL((k_form_b<float, double>), g, dim3(kThreads), 0, st, (const float*)P->A, P->lda, P->m, P->n,
                         W, (double*)Bout);
    else
      hipLaunchKernelGGL((k_form_b<double, double>), g, dim3(kThreads), 0, st, (const double*)P->A, P->lda, P->m,
                         P->n, W, (double*)Bout);
  }
  LS_HIP_TRY(hipGetLastError());
  return LS_OK;
}

size_t b_bytes(const ls_problem_t* P, ls_prec_t tb) {
  const size_t elt = (tb == LS_FP32) ? 4 : 8;
  return ls_align256((size_t)pan_count(P->m, elt) * (16 / elt) * P->n * elt);
}

// ================================================================== LSQR driver
namespace {
struct LsqrWs {
  LsqrState* st;
  char* v;
  char* u;
  char* w;
  double* y;
  double* z0;
  char* tpart;
  double* nupart;
  double* nbpart;
  double* nvpart[2];
  char* vz;       // W v (LSQR over A's panels)
  char* tw;       // W^T A^T u
  double* asum;   // A^T u
  size_t bytes;
};

LsqrWs lsqr_carve(char* ws, const ls_problem_t* P, size_t elt, int G, int Gv) {
  LsqrWs w{};
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = ws ? ws + off : nullptr;
    off += ls_align256(b);
    return q;
  };
  w.st = reinterpret_cast<LsqrState*>(take(sizeof(LsqrState)));
  w.v = take(elt * P->n);
  w.u = take(elt * P->m);
  w.w = take(elt * P->n);
  w.y = reinterpret_cast<double*>(take(8 * (size_t)P->n));
  w.z0 = reinterpret_cast<double*>(take(8 * (size_t)P->n));
  w.tpart = take(elt * P->n * (size_t)G);
  w.nupart = reinterpret_cast<double*>(take(8 * (size_t)G));
  w.nbpart = reinterpret_cast<double*>(take(8 * (size_t)G));
  w.nvpart[0] = reinterpret_cast<double*>(take(8 * (size_t)Gv));
  w.nvpart[1] = reinterpret_cast<double*>(take(8 * (size_t)Gv));
  w.vz = take(elt * P->n);
  w.tw = take(elt * P->n);
  w.asum = reinterpret_cast<double*>(take(8 * (size_t)P->n));
  w.bytes = off;
  return w;
}

template <typename T, int Q>
void lsqr_pan_launch(int G, hipStream_t st, ProfEv ev, const T* Bm, int64_t npan, int64_t m, int64_t n, const T* v,
                     const double* nvp, int Gv, T* u, const LsqrState* S, int par, int init, T* tpart,
                     double* nupart, double* nbpart) {
  hipExtLaunchKernelGGL((k_lsqr_pan<T, Q>), dim3(G), dim3(kThreads), 0, st, ev.a, ev.b, 0, Bm, npan, m, n, v, nvp,
                        Gv, u, S, par, init, tpart, nupart, nbpart);
}

template <typename T>
int lsqr_typed(const ls_problem_t* P, const double* R, int64_t ldr, const double* W, const T* Bm, int apply_w,
               double* x, const ls_iter_opts_t* io, ls_stats_t* stats, char* ws, size_t ws_bytes, hipStream_t st) {
  const int64_t m = P->m, n = P->n;
  if (n > 64 * kMaxPanQ) return LS_E_UNSUPPORTED;
  const int ncu = device_cu_count();
  const int64_t npan = pan_count(m, sizeof(T));
  const int G = pan_grid(npan, n, ncu);
  const int Gv = (int)ls_cdiv(n, 4);
  LsqrWs w = lsqr_carve(ws, P, sizeof(T), G, Gv);
  if (w.bytes > ws_bytes) return LS_E_WORKSPACE;
  T* v = reinterpret_cast<T*>(w.v);
  T* u = reinterpret_cast<T*>(w.u);
  T* wv = reinterpret_cast<T*>(w.w);
  T* tpart = reinterpret_cast<T*>(w.tpart);
  T* vz = reinterpret_cast<T*>(w.vz);
  T* tw = reinterpret_cast<T*>(w.tw);
  const int q = pan_q(n);
  const int maxit = io->lsqr_maxit;
  const double tol = io->lsqr_tol;
  const int check = io->check_every > 0 ? io->check_every : 8;
  const dim3 gcol((unsigned)Gv);
  const dim3 gut((unsigned)ls_cdiv(n, 32));

  hipLaunchKernelGGL(k_zero_bytes, dim3(4), dim3(kThreads), 0, st, reinterpret_cast<char*>(w.st), sizeof(LsqrState));
  hipLaunchKernelGGL(k_zero_bytes, dim3(4), dim3(kThreads), 0, st, reinterpret_cast<char*>(w.y), 8 * (size_t)n);
  hipLaunchKernelGGL(k_zero_bytes, dim3(4), dim3(kThreads), 0, st, w.w, sizeof(T) * (size_t)n);
  // z0 = R x0 (so that A x0 = B z0), v <- -z0, u <- b
  hipLaunchKernelGGL(k_trmv, gut, dim3(kUtThreads), 0, st, R, ldr, n, x, w.z0);
  hipLaunchKernelGGL((k_cast<T, double>), dim3((unsigned)ls_cdiv(n, kThreads)), dim3(kThreads), 0, st, w.z0, v, n,
                     T(-1));
  if (P->store == LS_FP32)
    hipLaunchKernelGGL((k_cast<T, float>), dim3((unsigned)ls_cdiv(m, kThreads)), dim3(kThreads), 0, st,
                       (const float*)P->b, u, m, T(1));
  else
    hipLaunchKernelGGL((k_cast<T, double>), dim3((unsigned)ls_cdiv(m, kThreads)), dim3(kThreads), 0, st,
                       (const double*)P->b, u, m, T(1));
  // Bm is B = A W, or with apply_w A's panels, W applied before and after the pass
  const T* vin = apply_w ? vz : v;
  auto pass = [&](int par, int init, const double* nvp) {
    if (apply_w)
      hipLaunchKernelGGL(k_lsqr_zx<T>, dim3((unsigned)ls_cdiv(n, 16)), dim3(1024), 0, st, W, n, v, w.st, par, init,
                         vz);
    const ProfEv ev = prof_events(kProfLsqrPass);
#define LS_LSQR_PAN(QQ)                                                                                              \
  lsqr_pan_launch<T, QQ>(G, st, ev, Bm, npan, m, n, vin, nvp, Gv, u, w.st, par, init, tpart, w.nupart, w.nbpart); \
  break
    switch (q) {
      case 1: LS_LSQR_PAN(1);
      case 2: LS_LSQR_PAN(2);
      case 4: LS_LSQR_PAN(4);
      case 8: LS_LSQR_PAN(8);
      case 16: LS_LSQR_PAN(16);
      default: LS_LSQR_PAN(32);
    }
#undef LS_LSQR_PAN
    // B once, u read and written, v read, t written
    prof_commit(kProfLsqrPass, (double)m * n * sizeof(T) + 2.0 * m * sizeof(T) + 2.0 * n * sizeof(T));
    if (apply_w) {
      hipLaunchKernelGGL(k_lsqr_colsum<T>, gcol, dim3(kThreads), 0, st, n, tpart, G, w.st, par, init, w.asum);
      hipLaunchKernelGGL(k_lsqr_wt<T>, dim3((unsigned)ls_cdiv(n, 16)), dim3(1024), 0, st, W, n, w.asum, w.st, par,
                         init, tw);
    }
  };
  // the column kernel's partials of B^T u: the pass's, or W^T A^T u as one per column
  const T* tcol = apply_w ? tw : tpart;
  const int Gcol = apply_w ? 1 : G;
  // init: u_1 = b - B z0, beta_1, v_1 = B^T u_1 / beta_1; C_1 -> rec[1]
  const size_t pmark = prof_mark();
  pass(1, 1, w.nvpart[0]);
  ProgressSlot slot(st);
  Progress *prog = slot.host, *dprog = slot.dev;
  if (prog) {
    progress_set(&prog->lsqr_it, -1);
    progress_set(&prog->lsqr_done, 0);
  }
  hipLaunchKernelGGL(k_lsqr_col<T>, gcol, dim3(kThreads), 0, st, n, tcol, Gcol, G, w.nupart, w.nbpart,
                     w.nvpart[1], Gv, w.nvpart[0], w.st, 0, 1, 0, tol, v, wv, w.y, dprog);
  int it = 1, cur = 0;   // nvpart[cur] holds ||v_it||^2 partials
  int last = 0;          // last column kernel launched
  LsqrRec rec{};
  for (; it <= maxit; ++it) {
    const int par = it & 1;
    pass(par, 0, w.nvpart[cur]);
    hipLaunchKernelGGL(k_lsqr_col<T>, gcol, dim3(kThreads), 0, st, n, tcol, Gcol, G, w.nupart, w.nbpart,
                       w.nvpart[cur], Gv, w.nvpart[cur ^ 1], w.st, par, 0, it, tol, v, wv, w.y, dprog);
    cur ^= 1;
    last = it;
    // at most `check` iterations in flight; stop queueing once converged
    if (prog) {
      const int rc = progress_wait(&prog->lsqr_it, &prog->lsqr_done, it - check + 1, st);
      if (rc == 1) break;
      if (rc == 0) continue;
      prog = nullptr;   // the slot is not updated: read the state instead from now on
    }
    if (it % check == 0) {
      LS_HIP_TRY(hipMemcpyAsync(&rec, &w.st->rec[par ^ 1], sizeof(LsqrRec), hipMemcpyDeviceToHost, st));
      LS_HIP_TRY(hipStreamSynchronize(st));
      if (rec.done) break;
    }
  }
  const int fpar = (last + 1) & 1;         // rec written by it
  hipLaunchKernelGGL(k_lsqr_finish<T>, gut, dim3(kUtThreads), 0, st, W, n, w.z0, w.y,
                     w.nvpart[cur], Gv, w.st, fpar, last, x);
  LsqrState S;
  LS_HIP_TRY(hipMemcpyAsync(&S, w.st, sizeof(LsqrState), hipMemcpyDeviceToHost, st));
  LS_HIP_TRY(hipStreamSynchronize(st));
  LS_HIP_TRY(hipGetLastError());
  rec = S.rec[fpar];
  // full passes: the first one, then iterations 1 .. its + 1 (the column
  // kernel of the last of them finds the stop)
  prof_keep(kProfLsqrPass, pmark, rec.its + 2);
  if (stats) {
    stats->lsqr_its = rec.its;
    stats->lsqr_normr = rec.normr;
    stats->lsqr_normar = rec.normar;
    stats->lsqr_normB = rec.normB;
  }
  if (S.flag || rec.stop == 5) return LS_E_NONFINITE;
  return (rec.stop == 1 || rec.stop == 2 || rec.stop == 4) ? LS_OK : LS_NOT_CONVERGED;
}
}  // namespace

size_t lsqr_workspace(const ls_problem_t* P, ls_prec_t u, int ncu) {
  const size_t elt = (u == LS_FP32) ? 4 : 8;
  return lsqr_carve(nullptr, P, elt, pan_grid(pan_count(P->m, elt), P->n, ncu), (int)ls_cdiv(P->n, 4)).bytes;
}

int lsqr_device(const ls_problem_t* P, const double* R, int64_t ldr, const double* W, const void* Bm, int apply_w,
                ls_prec_t u, double* x, const ls_iter_opts_t* io, ls_stats_t* stats, char* ws, size_t ws_bytes,
                hipStream_t st) {
  if (u == LS_FP32)
    return lsqr_typed<float>(P, R, ldr, W, (const float*)Bm, apply_w, x, io, stats, ws, ws_bytes, st);
  if (u == LS_FP64)
    return lsqr_typed<double>(P, R, ldr, W, (const double*)Bm, apply_w, x, io, stats, ws, ws_bytes, st);
  return LS_E_UNSUPPORTED;
}

// ================================================================== refinement driver
namespace {
struct LsirWs {
  FgState* st;
  double* V;
  int64_t ldv;
  double* H;
  double* cs;
  double* sn;
  double* g;
  double* hj;
  char* tpart;        // n x G (TB), column-major partials
  double* Hraw;       // (kmax + 1) x kmax: the Hessenberg columns before rotation
  double* dots;       // (2 kmax + 2) x Gs: sweep 1's partials
  double* dsum;       // 2 kmax + 2: their sums (many row blocks)
  double* pend;       // 2 x (kmax + 1): the pending first-pass column, by parity of j
  double* coef;       // 2 kmax + 3: sweep 2's coefficients (many row blocks)
  double* w2part;     // max(Gr + Gh, Gs)
  double* rt_hi;      // n x Gr
  double* rt_lo;      // n x Gr
  double* gvec;       // n
  double* dz;         // n
  double* upart;      // 4 x (Gd + Gn)
  double* xin;        // n: W V_x[:, j] (A-path)
  double* tbuf;       // n: A^T v_r (A-path)
  size_t bytes;
};

struct LsirDims {
  int kmax, G, Gr, Gc, Gd, Gs, Gh, Gn;
  int64_t npan;   // panels of B
};

template <typename TB, typename TC, int Q>
void fg_pan_launch(int G, hipStream_t st, ProfEv ev, const TB* Bm, int64_t npan, int64_t m, int64_t n,
                   const FgPtrs& F, int j, const double* w2part, int Gw, TC* tpart, const double* xin) {
  if (ev.a)
    hipExtLaunchKernelGGL((k_fg_pan<TB, TC, Q>), dim3(G), dim3(kThreads), 0, st, ev.a, ev.b, 0, Bm, npan, m, n, F, j,
                          w2part, Gw, tpart, xin);
  else   // no timing events: a plain launch (the form a graph capture records)
    hipLaunchKernelGGL((k_fg_pan<TB, TC, Q>), dim3(G), dim3(kThreads), 0, st, Bm, npan, m, n, F, j, w2part, Gw, tpart,
                       xin);
}

LsirDims lsir_dims(const ls_problem_t* P, size_t tb_elt, size_t ta_elt, int fgmres_maxit, int ncu) {
  LsirDims d{};
  d.kmax = fgmres_maxit;

  d.npan = pan_count(P->m, tb_elt);
  d.G = pan_grid(d.npan, P->n, ncu);
  d.Gr = (int)ls_cdiv(P->m, kResRows);
  d.Gc = (int)ls_cdiv(P->n, 16);
  d.Gs = (int)ls_cdiv(P->m + P->n, kSweepThreads);
  d.Gd = (int)ls_cdiv(P->m + P->n, kThreads);
  d.Gh = (int)ls_cdiv(P->n, 4);
  d.Gn = (int)ls_cdiv(P->n, 32);
  return d;
}

LsirWs lsir_carve(char* ws, const ls_problem_t* P, const LsirDims& d, size_t tb_elt) {
  LsirWs w{};
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = ws ? ws + off : nullptr;
    off += ls_align256(b);
    return q;
  };
  const int64_t m = P->m, n = P->n;
  const int kmax = d.kmax;
  w.ldv = m + n;
  w.st = reinterpret_cast<FgState*>(take(sizeof(FgState)));
  // right after the state: the host reads both back with one copy per step
  w.upart = reinterpret_cast<double*>(take(8 * 4 * (size_t)(d.Gd + d.Gn)));
  w.V = reinterpret_cast<double*>(take(8 * (size_t)w.ldv * (kmax + 1)));
  w.H = reinterpret_cast<double*>(take(8 * (size_t)(kmax + 1) * kmax));
  w.cs = reinterpret_cast<double*>(take(8 * (size_t)kmax));
  w.sn = reinterpret_cast<double*>(take(8 * (size_t)kmax));
  w.g = reinterpret_cast<double*>(take(8 * (size_t)(kmax + 1)));
  w.hj = reinterpret_cast<double*>(take(8));
  w.tpart = take(tb_elt * (size_t)d.G * n);
  w.Hraw = reinterpret_cast<double*>(take(8 * (size_t)(kmax + 1) * kmax));
  w.dots = reinterpret_cast<double*>(take(8 * (size_t)(2 * kmax + 2) * d.Gs));
  w.dsum = reinterpret_cast<double*>(take(8 * (size_t)(2 * kmax + 2)));
  w.pend = reinterpret_cast<double*>(take(8 * 2 * (size_t)(kmax + 1)));
  w.coef = reinterpret_cast<double*>(take(8 * (size_t)(2 * kmax + 3)));
  // partials of ||f||^2 (row blocks of the residual pass, at most max(Gr, G)) and of ||h||^2
  const int gf = (d.Gr > d.G) ? d.Gr : d.G;
  const int w2n = (gf + d.Gh > d.Gs) ? gf + d.Gh : d.Gs;
  w.w2part = reinterpret_cast<double*>(take(8 * (size_t)w2n));
  w.rt_hi = reinterpret_cast<double*>(take(8 * (size_t)d.Gr * n));
  w.rt_lo = reinterpret_cast<double*>(take(8 * (size_t)d.Gr * n));
  w.gvec = reinterpret_cast<double*>(take(8 * (size_t)n));
  w.dz = reinterpret_cast<double*>(take(8 * (size_t)n));
  w.xin = reinterpret_cast<double*>(take(8 * (size_t)n));
  w.tbuf = reinterpret_cast<double*>(take(8 * (size_t)n));
  w.bytes = off;
  return w;
}

template <int Q>
void resid_pan_launch(int G, hipStream_t st, ProfEv ev, const float* Ap, int64_t npan, int64_t m, int64_t n,
                      const float* b, const double* r, const double* x, double* f, double* tpart, double* fpart) {
  hipExtLaunchKernelGGL((k_resid_pan<Q>), dim3(G), dim3(kThreads), 0, st, ev.a, ev.b, 0, Ap, npan, m, n, b, r, x, f,
                        tpart, fpart);
}

// TB: element type of the panels the FGMRES pass streams; TC: its arithmetic
// (TB on the B-path, binary64 on the A-path, AP, where the panels are A's).
template <typename TA, typename TB, typename TU, bool DD, bool AP>
int lsir_typed(const ls_problem_t* P, const double* W, const TB* Bm, double* x, double* r, int r_given,
               const ls_iter_opts_t* io, ls_stats_t* stats, char* ws, size_t ws_bytes, hipStream_t st,
               int fg_maxit) {
  using TC = typename std::conditional<AP, double, TB>::type;
  const int64_t m = P->m, n = P->n;
  const int ncu = device_cu_count();
  const LsirDims d = lsir_dims(P, sizeof(TB), sizeof(TA), fg_maxit, ncu);
  if (d.kmax > kMaxKrylov - 1) return LS_E_ARG;
  if (n > 64 * kMaxPanQ) return LS_E_UNSUPPORTED;
  LsirWs w = lsir_carve(ws, P, d, sizeof(TC));
  if (w.bytes > ws_bytes) return LS_E_WORKSPACE;
  FgPtrs F{w.V, w.ldv, w.H, w.cs, w.sn, w.g, w.hj, w.st};
  const TA* A = static_cast<const TA*>(P->A);
  const TA* b = static_cast<const TA*>(P->b);
  const int vec_a = vec_aligned(A, P->lda, sizeof(TA)) ? 1 : 0;
  const int q = pan_q(n);
  TC* tpart = reinterpret_cast<TC*>(w.tpart);
  const int check = io->check_every > 0 ? io->check_every : 8;
  double tol = io->fgmres_tol;   // FGMRES tolerance of the current step
  const double lsir_tol = io->lsir_tol;
  const int ncb = (int)d.Gc;
  // binary64 residuals on the A-path: the residual pass streams A's panel copy
  // (G blocks, the column partials in tpart); otherwise A as stored (Gr blocks)
  // (rows of up to 1024 columns: wider ones spill its registers)
  constexpr bool kResPan = AP && !DD && std::is_same<TA, float>::value && std::is_same<TB, float>::value;
  const bool res_pan = kResPan && q <= 16;
  const int Gf = res_pan ? d.G : d.Gr;

  if (!r_given)
    hipLaunchKernelGGL((k_resid_u<TA, TU>), dim3((unsigned)d.Gr), dim3(kResThreads), 0, st, A, P->lda, m, n, vec_a, b, x,
                       r);
  ProgressSlot slot(st);
  Progress *prog = slot.host, *dprog = slot.dev;
  // graph replay of the FGMRES iterations (not with per-kernel timing events)
  const bool use_graph = io->graph != 0 && io->profile == 0;
  GraphChunks chunks{st, {}};
  CaptureStream cap;
  if (use_graph) LS_TRY(cap.acquire());
  hipStream_t lst = st;   // the stream the iterations' launches go to (the capture stream while capturing)
  auto fg_pass = [&](int j, int Gw, ProfEv ev) {
#define LS_FG_PAN(QQ)                                                                                           \
  fg_pan_launch<TB, TC, QQ>(d.G, lst, ev, Bm, d.npan, m, n, F, j, w.w2part, Gw, tpart, AP ? w.xin : nullptr); \
  break
    switch (q) {
      case 1: LS_FG_PAN(1);
      case 2: LS_FG_PAN(2);
      case 4: LS_FG_PAN(4);
      case 8: LS_FG_PAN(8);
      case 16: LS_FG_PAN(16);
      default: LS_FG_PAN(32);
    }
#undef LS_FG_PAN
  };
  // sweep 1, then sweep 2 with the stage (closing: the last column's second
  // pass only)
  auto gram_schmidt = [&](int j, int closing) {
    const int64_t rows = m + n;
    hipLaunchKernelGGL(k_dcgs_dots, dim3((unsigned)d.Gs), dim3(kSweepThreads), 0, lst, F, rows, j, closing, w.dots);
    const double* parts = w.dots;
    int Gp = d.Gs;
    if (d.Gs > kSweepSumAbove) {   // summed once rather than by the stage's waves
      hipLaunchKernelGGL(k_colsum_parts, dim3((unsigned)(2 * j + 2)), dim3(kThreads), 0, lst, w.st, w.dots, d.Gs,
                         w.dsum);
      parts = w.dsum;
      Gp = 1;
    }
    if (closing) {
      hipLaunchKernelGGL(k_dcgs_close, dim3(1), dim3(kSweepThreads), 0, lst, F, w.Hraw, w.pend, d.kmax, parts, Gp);
    } else if (d.Gs > kSweepSumAbove) {   // the stage once, then the sweep
      hipLaunchKernelGGL(k_dcgs_stage, dim3(1), dim3(kSweepThreads), 0, lst, F, j, w.Hraw, w.pend, d.kmax, parts, Gp,
                         dprog, w.coef);
      hipLaunchKernelGGL(k_dcgs_apply, dim3((unsigned)d.Gs), dim3(kSweepThreads), 0, lst, F, rows, j, w.coef, w.w2part);
    } else {
      hipLaunchKernelGGL(k_dcgs_update, dim3((unsigned)d.Gs), dim3(kSweepThreads), 0, lst, F, rows, j, w.Hraw, w.pend,
                         d.kmax, parts, Gp, dprog, w.w2part);
    }
  };
  int total_fg = 0, its = 0, status = LS_NOT_CONVERGED;
  double dx_rel = 0.0, dr_rel = 0.0;
  std::vector<double> up(4 * (size_t)(d.Gd + d.Gn));
  std::vector<char> rb((size_t)(reinterpret_cast<char*>(w.upart) - reinterpret_cast<char*>(w.st)) +
                       8 * 4 * (size_t)(d.Gd + d.Gn));
  const bool with_ref = io->x_ref && io->r_ref;
  double err_x = -1.0, err_r = -1.0;
  for (its = 1; its <= io->lsir_maxit; ++its) {
    if (io->inner_adapt && its > 1) {
      const double rho = std::max(dx_rel, dr_rel);
      tol = (rho > 0.0) ? 0.1 * lsir_tol / rho : 1e-2;
      tol = std::min(1e-2, std::max(io->fgmres_tol, tol));
    }
    // residuals f, g and h = R^-T g in u_r
    const ProfEv ev = prof_events(kProfResidPass);
    if constexpr (kResPan) {
      if (res_pan) {
#define LS_RES_PAN(QQ) \
  resid_pan_launch<QQ>(d.G, st, ev, Bm, d.npan, m, n, b, r, x, w.V, tpart, w.w2part); \
  break
        switch (q) {
          case 1: LS_RES_PAN(1);
          case 2: LS_RES_PAN(2);
          case 4: LS_RES_PAN(4);
          case 8: LS_RES_PAN(8);
          default: LS_RES_PAN(16);
        }
#undef LS_RES_PAN
        hipLaunchKernelGGL(k_lsir_g<DD>, dim3((unsigned)ls_cdiv(n, 4)), dim3(kThreads), 0, st, tpart, tpart, d.G, n,
                           w.gvec);
      }
    }
    if (!res_pan) {
      hipExtLaunchKernelGGL((k_lsir_resid<TA, DD>), dim3((unsigned)d.Gr), dim3(kResThreads), 0, st, ev.a, ev.b, 0, A,
                            P->lda, m, n, vec_a, b, r, x, w.V, w.rt_hi, w.rt_lo, w.w2part);
      hipLaunchKernelGGL(k_lsir_g<DD>, dim3((unsigned)ls_cdiv(n, 4)), dim3(kThreads), 0, st, w.rt_hi, w.rt_lo, d.Gr, n,
                         w.gvec);
    }
    // A and b once, r read, f written, x read, g written
    prof_commit(kProfResidPass, (double)m * n * sizeof(TA) + (double)m * sizeof(TA) + 16.0 * m + 16.0 * n);
    hipLaunchKernelGGL(k_lsir_h<DD>, dim3((unsigned)d.Gh), dim3(kThreads), 0, st, W, n, m, w.gvec, w.V,
                       w.w2part + Gf);
    hipLaunchKernelGGL(k_fg_begin, dim3(1), dim3(64), 0, st, w.st, tol);
    // the correction: FGMRES on [I B; B^T 0]
    const size_t pmark = prof_mark();
    int j = 0;
    FgState S{};
    if (prog) {   // the previous cycle has been synchronised: no kernel writes the slot now
      progress_set(&prog->fg_j, -1);
      progress_set(&prog->fg_done, 0);
    }
    // iteration j's launches: the pass, its column sums, the Gram-Schmidt sweeps
    auto iteration = [&](int jj) {
      const int Gw = (jj == 0) ? Gf + d.Gh : d.Gs;
      if (AP)   // the x part of v_j times W, before the pass
        hipLaunchKernelGGL(k_fg_zx, dim3((unsigned)ls_cdiv(n, 16)), dim3(1024), 0, lst, W, n, F, m, jj, w.xin);
      fg_pass(jj, Gw, prof_events(kProfFgPass));
      // the panels once, v_j read and written, w written, v_x (or W v_x) read, t written
      prof_commit(kProfFgPass, (double)m * n * sizeof(TB) + 24.0 * m + 8.0 * n + (double)n * sizeof(TC));
      hipLaunchKernelGGL(k_fg_col<TC>, dim3((unsigned)ncb), dim3(1024), 0, lst, m, n, tpart, d.G, F, jj,
                         AP ? w.tbuf : nullptr);
      if (AP)   // w_x = W^T t
        hipLaunchKernelGGL(k_fg_wt, dim3((unsigned)ncb), dim3(1024), 0, lst, W, m, n, w.tbuf, F, jj);
      prof_begin(kProfCgs, lst);
      gram_schmidt(jj, 0);
      // V(:, 0:j) read twice, q_j and w read twice, v_j and u_{j+1} written
      prof_end(kProfCgs, lst, 2.0 * 8.0 * (jj + 2) * (double)(m + n) + 2.0 * 8.0 * (double)(m + n));
    };
    if (!use_graph) {
      for (; j < d.kmax; ++j) {
        iteration(j);
        // at most `check` iterations in flight; stop queueing once converged
        if (prog) {
          const int rc = progress_wait(&prog->fg_j, &prog->fg_done, j - check + 1, st);
          if (rc == 1) break;
          if (rc == 0) continue;
          prog = nullptr;   // the slot is not updated: read the state instead from now on
          dprog = nullptr;
        }
        if ((j + 1) % check == 0) {
          LS_HIP_TRY(hipMemcpyAsync(&S, w.st, sizeof(FgState), hipMemcpyDeviceToHost, st));
          LS_HIP_TRY(hipStreamSynchronize(st));
          if (S.done) break;
        }
      }
    } else {
      // chunks of `check` iterations, captured at this call's first cycle and
      // replayed at the later ones; one chunk queued beyond the one running
      for (int c = 0; c * check < d.kmax; ++c) {
        const int j0 = c * check, j1 = std::min(d.kmax, j0 + check);
        if ((int)chunks.v.size() <= c) {
          hipGraph_t g = nullptr;
          LS_HIP_TRY(hipStreamBeginCapture(cap.s, hipStreamCaptureModeThreadLocal));
          lst = cap.s;
          for (int jj = j0; jj < j1; ++jj) iteration(jj);
          lst = st;
          LS_HIP_TRY(hipStreamEndCapture(cap.s, &g));
          hipGraphExec_t ex = nullptr;
          const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
          if (ei != hipSuccess) return LS_E_HIP;
          chunks.v.push_back(ex);
        }
        LS_HIP_TRY(hipGraphLaunch(chunks.v[c], st));
        j = j1;
        if (prog) {
          const int rc = progress_wait(&prog->fg_j, &prog->fg_done, j0 - 1, st);
          if (rc == 1) break;
          if (rc == 0) continue;
          prog = nullptr;   // the slot is not updated: read the state instead from now on
        }
        LS_HIP_TRY(hipMemcpyAsync(&S, w.st, sizeof(FgState), hipMemcpyDeviceToHost, st));
        LS_HIP_TRY(hipStreamSynchronize(st));
        if (S.done) break;
      }
    }
    // a cycle at its iteration limit: the second pass of its last vector
    // makes the last column final (no-op when already done)
    gram_schmidt(d.kmax, 1);
    hipLaunchKernelGGL(k_fg_update<TU>, dim3((unsigned)d.Gd), dim3(kThreads), 0, st, F, m, n, d.kmax, r, w.dz, w.upart,
                       with_ref ? io->r_ref : nullptr);
    hipLaunchKernelGGL(k_fg_dx<TU>, dim3((unsigned)d.Gn), dim3(kUtThreads), 0, st, W, n, w.dz, x,
                       w.upart + 4 * (size_t)d.Gd, with_ref ? io->x_ref : nullptr);
    // the state and the norm partials in one copy (each copy to pageable
    // memory costs a round trip of the host)
    const size_t up_off = (size_t)(reinterpret_cast<char*>(w.upart) - reinterpret_cast<char*>(w.st));
    LS_HIP_TRY(hipMemcpyAsync(rb.data(), w.st, rb.size(), hipMemcpyDeviceToHost, st));
    LS_HIP_TRY(hipStreamSynchronize(st));
    LS_HIP_TRY(hipGetLastError());
    std::memcpy(&S, rb.data(), sizeof(FgState));
    std::memcpy(up.data(), rb.data() + up_off, 8 * 4 * (size_t)(d.Gd + d.Gn));
    if (S.breakdown == 2) return LS_E_NONFINITE;
    // passes and sweeps of iterations 0 .. k (iteration k's stage found the
    // convergence of column k-1); later ones were queued past convergence
    prof_keep(kProfFgPass, pmark, S.k + 1);
    prof_keep(kProfCgs, pmark, S.k + 1);
    total_fg += S.k;
    double nr[4] = {0, 0, 0, 0}, nx[4] = {0, 0, 0, 0};
    for (int g = 0; g < d.Gd; ++g)
      for (int q = 0; q < 4; ++q) nr[q] += up[4 * (size_t)g + q];
    for (int g = 0; g < d.Gn; ++g)
      for (int q = 0; q < 4; ++q) nx[q] += up[4 * (size_t)(d.Gd + g) + q];
    dr_rel = sqrt(nr[0]) / (nr[1] > 0 ? sqrt(nr[1]) : 1.0);
    dx_rel = sqrt(nx[0]) / (nx[1] > 0 ? sqrt(nx[1]) : 1.0);
    if (!std::isfinite(dr_rel) || !std::isfinite(dx_rel)) return LS_E_NONFINITE;
    if (with_ref) {
      // Section 5's test: forward errors of x and r against the given solution
      err_r = sqrt(nr[2]) / (nr[3] > 0 ? sqrt(nr[3]) : 1.0);
      err_x = sqrt(nx[2]) / (nx[3] > 0 ? sqrt(nx[3]) : 1.0);
      if (err_x <= lsir_tol && err_r <= lsir_tol) {
        status = LS_OK;
        break;
      }
    } else if (dx_rel <= lsir_tol && dr_rel <= lsir_tol) {
      status = LS_OK;
      break;
    }
  }
  if (its > io->lsir_maxit) its = io->lsir_maxit;
  if (stats) {
    stats->lsir_its += its;
    stats->fgmres_its_total += total_fg;
    stats->lsir_dx_rel = dx_rel;
    stats->lsir_dr_rel = dr_rel;
    stats->err_x = err_x;
    stats->err_r = err_r;
  }
  return status;
}
}  // namespace

bool fg_apath(const ls_precs_t* pr) { return pr->u == LS_FP32 && pr->u_A == LS_FP64; }

bool lsqr_on_a(const ls_problem_t* P, const ls_precs_t* pr) { return fg_apath(pr) && P->store == LS_FP32; }

size_t fg_operand_bytes(const ls_problem_t* P, const ls_precs_t* pr) {
  return fg_apath(pr) ? b_bytes(P, P->store) : b_bytes(P, pr->u_A);
}

int form_fg_operand(const ls_problem_t* P, const double* W, const float* W32, const ls_precs_t* pr, void* out,
                    hipStream_t st) {
  if (!fg_apath(pr)) return form_b(P, W, W32, pr->u_A, out, st);
  return form_a_panels(P, out, st);
}

int form_a_panels(const ls_problem_t* P, void* out, hipStream_t st) {
  const dim3 g((unsigned)ls_cdiv(P->m, 64), (unsigned)ls_cdiv(P->n, 64));
  if (P->store == LS_FP32)
    hipLaunchKernelGGL(k_a_panels<float>, g, dim3(kThreads), 0, st, (const float*)P->A, P->lda, P->m, P->n,
                       vec_aligned(P->A, P->lda, 4) ? 1 : 0, (float*)out);
  else
    hipLaunchKernelGGL(k_a_panels<double>, g, dim3(kThreads), 0, st, (const double*)P->A, P->lda, P->m, P->n,
                       vec_aligned(P->A, P->lda, 8) ? 1 : 0, (double*)out);
  LS_HIP_TRY(hipGetLastError());
  return LS_OK;
}

size_t lsir_workspace(const ls_problem_t* P, const ls_precs_t* pr, int fgmres_maxit, int ncu) {
  // panels streamed by the pass (A's on the A-path, B's otherwise) and the
  // element of its column partials (binary64 on the A-path)
  const bool ap = fg_apath(pr);
  const size_t ta = (P->store == LS_FP64) ? 8 : 4;
  const size_t tb = ap ? ta : ((pr->u_A == LS_FP64) ? 8 : 4);
  const size_t tc = ap ? 8 : tb;
  const LsirDims d = lsir_dims(P, tb, ta, fgmres_maxit, ncu);
  return lsir_carve(nullptr, P, d, tc).bytes;
}

int lsir_device(const ls_problem_t* P, const double* W, const void* Bm, const ls_precs_t* pr, double* x, double* r,
                int r_given, const ls_iter_opts_t* io, ls_stats_t* stats, char* ws, size_t ws_bytes,
                hipStream_t st) {
  const ls_prec_t tb = pr->u_A;
  if (pr->u_L != tb || pr->u_R != tb) return LS_E_UNSUPPORTED;
  const bool dd = pr->u_r == LS_FP64X2;
  if (!dd && pr->u_r != LS_FP64) return LS_E_UNSUPPORTED;
  const bool u32 = pr->u == LS_FP32;
  if (!u32 && pr->u != LS_FP64) return LS_E_UNSUPPORTED;
  if (!u32 && tb == LS_FP32) return LS_E_ARG;   // products not coarser than u
  const int kmax = io->fgmres_maxit;
#define LS_LSIR_CALL(TA, TB_, TU, DD_, AP_) \
  return lsir_typed<TA, TB_, TU, DD_, AP_>(P, W, (const TB_*)Bm, x, r, r_given, io, stats, ws, ws_bytes, st, kmax)
  if (fg_apath(pr)) {   // binary32 working precision, binary64 products over A's panels
    if (P->store == LS_FP32) {
      if (dd) LS_LSIR_CALL(float, float, float, true, true);
      LS_LSIR_CALL(float, float, float, false, true);
    }
    if (dd) LS_LSIR_CALL(double, double, float, true, true);
    LS_LSIR_CALL(double, double, float, false, true);
  }
  if (P->store == LS_FP32) {
    if (tb == LS_FP32) {
      if (dd) LS_LSIR_CALL(float, float, float, true, false);
      LS_LSIR_CALL(float, float, float, false, false);
    }
    if (dd) LS_LSIR_CALL(float, double, double, true, false);
    LS_LSIR_CALL(float, double, double, false, false);
  } else {
    if (tb == LS_FP32) {
      if (dd) LS_LSIR_CALL(double, float, float, true, false);
      LS_LSIR_CALL(double, float, float, false, false);
    }
    if (dd) LS_LSIR_CALL(double, double, double, true, false);
    LS_LSIR_CALL(double, double, double, false, false);
  }
#undef LS_LSIR_CALL
}

}  // namespace ls
