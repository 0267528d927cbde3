// Algorithm 1 step 2: economic Householder QR of the sketch, R factor only,
// plus the explicit inverse R^-1 used to apply the preconditioner.
//
// Blocked right-looking Householder QR (compact WY, LAPACK's forward
// column-wise convention H = I - V T V^T):
//   * a panel of NB columns is factored by one 1024-thread block that keeps
//     the panel in registers (RPT rows per thread) and builds T on the fly;
//   * the trailing columns are updated as C <- C - V (T^T (V^T C)) by two
//     grid-wide kernels (partial V^T C over row chunks, then the update).
// Reflectors follow the usual choice beta = -sign(x_1) ||x||; at the end
// the rows of R are multiplied by the signs of its diagonal so diag(R) > 0.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int kQrThreads = 1024;
constexpr int kColBlock = 32;
constexpr int kRowChunk = 256;

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

template <typename T, int NB>
__device__ __forceinline__ T wave_multi_sum(T (&v)[NB], int lane, int& idx) {
  constexpr int L = Log2<NB>::value;
  int base = 0;
#pragma unroll
  for (int step = 0; step < L; ++step) {
    const int off = 32 >> step;
    const int h = NB >> (step + 1);
    const bool up = (lane & off) != 0;
    // lane choice as an exact blend (factors 1 and 0): a select here would be
    // folded into a run-time register index, which compiles to select chains
    const T fu = up ? T(1) : T(0);
    const T fl = T(1) - fu;
#pragma unroll
    for (int q = 0; q < NB / 2; ++q) {
      if (q < h) {
        const T send = v[q] * fu + v[q + h] * fl;
        const T keep = v[q + h] * fu + v[q] * fl;
        v[q] = keep + __shfl_xor(send, off, 64);
      }
    }
    if (up) base += h;
  }
  T s = v[0];
#pragma unroll
  for (int off = 32 >> L; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  idx = base;
  return s;
}

template <typename T, int RPT, int NB>
__global__ __launch_bounds__(kQrThreads) void k_qr_panel(T* __restrict__ Y, int64_t ldy, int64_t s, int64_t j0,
                                                          int nb, T* __restrict__ tau, T* __restrict__ Tm) {
  __shared__ T red[kQrThreads / 64][NB];
  __shared__ T dots[NB];
  __shared__ T bsum[kQrThreads / 64];
  __shared__ T x0s;
  __shared__ T Ts[NB][NB];   // Ts[col][row] = T(row, col)
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  constexpr int lowmask = 64 / NB - 1;

  T P[RPT][NB];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int64_t i = j0 + tid + (int64_t)kQrThreads * r;
#pragma unroll
    for (int c = 0; c < NB; ++c) P[r][c] = (i < s && c < nb) ? Y[i + (j0 + c) * ldy] : T(0);
  }

#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c < nb) {
      // ---- reflector for column c: x = rows li >= c of the column
      T ss = 0;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int li = tid + kQrThreads * r;
        if (li > c) ss += P[r][c] * P[r][c];
      }
      ss = ls_block_sum<T, kQrThreads>(ss, bsum);
      if (tid == c) x0s = P[0][c];
      __syncthreads();
      const T x0 = x0s;
      T beta, tauc, scal;
      if (ss == T(0)) {
        tauc = 0;
        beta = x0;
        scal = 0;
      } else {
        const T nrm = sqrt(x0 * x0 + ss);
        beta = (x0 >= T(0)) ? -nrm : nrm;
        tauc = (beta - x0) / beta;
        scal = T(1) / (x0 - beta);
      }
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int li = tid + kQrThreads * r;
        if (li > c) P[r][c] *= scal;
      }
      if (tid == c) P[0][c] = beta;

      // ---- dots: v_a . v_c (a < c) and v_c . y_b (b > c), rows li >= c
      T part[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) part[q] = 0;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int li = tid + kQrThreads * r;
        if (li >= c) {
          const T vc = (li == c) ? T(1) : P[r][c];
#pragma unroll
          for (int q = 0; q < NB; ++q)
            if (q != c) part[q] += P[r][q] * vc;
        }
      }
      int idx;
      const T wsum = wave_multi_sum<T, NB>(part, lane, idx);
      __syncthreads();
      if ((lane & lowmask) == 0) red[wv][idx] = wsum;
      __syncthreads();
      if (tid < NB) {
        T acc = 0;
#pragma unroll
        for (int w = 0; w < kQrThreads / 64; ++w) acc += red[w][tid];
        dots[tid] = acc;
      }
      __syncthreads();
      // ---- column c of T: T(0:c, c) = -tau_c T(0:c, 0:c) (V(:,0:c)^T v_c), T(c, c) = tau_c
      if (tid < c) {
        T acc = 0;
        for (int b = tid; b < c; ++b) acc += Ts[b][tid] * dots[b];
        Ts[c][tid] = -tauc * acc;
      }
      if (tid == c) Ts[c][c] = tauc;
      if (tid == 0) tau[j0 + c] = tauc;
      // ---- apply H_c to the later panel columns
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int li = tid + kQrThreads * r;
        if (li >= c) {
          const T vc = (li == c) ? T(1) : P[r][c];
#pragma unroll
          for (int b = c + 1; b < NB; ++b) P[r][b] -= tauc * dots[b] * vc;
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int64_t i = j0 + tid + (int64_t)kQrThreads * r;
    if (i < s) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nb) Y[i + (j0 + c) * ldy] = P[r][c];
    }
  }
  __syncthreads();
  for (int o = tid; o < NB * NB; o += kQrThreads) {
    const int a = o % NB, c = o / NB;
    Tm[o] = (a <= c && c < nb) ? Ts[c][a] : T(0);
  }
}

// V(i, a) of the current panel (unit lower trapezoidal, stored below the diagonal).
template <typename T>
__device__ __forceinline__ T panel_v(const T* Y, int64_t ldy, int64_t s, int64_t j0, int nb, int64_t i, int a) {
  if (a >= nb || i >= s) return T(0);
  const int64_t d = j0 + a;
  if (i == d) return T(1);
  if (i > d) return Y[i + d * ldy];
  return T(0);
}

// Wp[(x * nrc + y) * NB * 32 + a * 32 + c] = sum over rows of chunk y of V(i, a) C(i, c).
template <typename T, int NB>
__global__ __launch_bounds__(256) void k_qr_wpart(const T* __restrict__ Y, int64_t ldy, int64_t s, int64_t j0,
                                                  int nb, int64_t c_begin, int64_t ncols, T* __restrict__ Wp) {
  __shared__ T Vs[kRowChunk][NB + 1];
  __shared__ T Cs[kRowChunk][kColBlock + 1];
  const int t = threadIdx.x;
  const int64_t i = j0 + (int64_t)blockIdx.y * kRowChunk + t;
  const int64_t cc0 = c_begin + (int64_t)blockIdx.x * kColBlock;
#pragma unroll
  for (int a = 0; a < NB; ++a) Vs[t][a] = panel_v(Y, ldy, s, j0, nb, i, a);
  for (int c = 0; c < kColBlock; ++c)
    Cs[t][c] = (i < s && cc0 + c < ncols) ? Y[i + (cc0 + c) * ldy] : T(0);
  __syncthreads();
  const int nrc = gridDim.y;
  T* out = Wp + ((int64_t)blockIdx.x * nrc + blockIdx.y) * NB * kColBlock;
  for (int o = t; o < NB * kColBlock; o += 256) {
    const int a = o / kColBlock, c = o % kColBlock;
    T acc = 0;
    for (int r = 0; r < kRowChunk; ++r) acc += Vs[r][a] * Cs[r][c];
    out[o] = acc;
  }
}

template <typename T, int NB>
__global__ __launch_bounds__(256) void k_qr_apply(T* __restrict__ Y, int64_t ldy, int64_t s, int64_t j0, int nb,
                                                  int64_t c_begin, int64_t ncols, const T* __restrict__ Wp,
                                                  const T* __restrict__ Tm) {
  __shared__ T W[NB][kColBlock];
  __shared__ T W2[NB][kColBlock];
  const int t = threadIdx.x;
  const int nrc = gridDim.y;
  const T* in = Wp + (int64_t)blockIdx.x * nrc * NB * kColBlock;
  for (int o = t; o < NB * kColBlock; o += 256) {
    T acc = 0;
    for (int y = 0; y < nrc; ++y) acc += in[(int64_t)y * NB * kColBlock + o];
    W[o / kColBlock][o % kColBlock] = acc;
  }
  __syncthreads();
  for (int o = t; o < NB * kColBlock; o += 256) {
    const int a = o / kColBlock, c = o % kColBlock;
    T acc = 0;
    for (int b = 0; b <= a; ++b) acc += Tm[b + a * NB] * W[b][c];   // (T^T W)(a, c)
    W2[a][c] = acc;
  }
  __syncthreads();
  const int64_t i = j0 + (int64_t)blockIdx.y * kRowChunk + t;
  if (i >= s) return;
  T v[NB];
#pragma unroll
  for (int a = 0; a < NB; ++a) v[a] = panel_v(Y, ldy, s, j0, nb, i, a);
  const int64_t cc0 = c_begin + (int64_t)blockIdx.x * kColBlock;
  for (int c = 0; c < kColBlock; ++c) {
    if (cc0 + c >= ncols) break;
    T acc = 0;
#pragma unroll
    for (int a = 0; a < NB; ++a) acc += v[a] * W2[a][c];
    Y[i + (cc0 + c) * ldy] -= acc;
  }
}

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_copy_cols(const TI* __restrict__ X, int64_t ldx, TO* __restrict__ Z,
                                                   int64_t ldz, int64_t rows, int64_t cols) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i < rows && j < cols) Z[i + j * ldz] = (TO)X[i + j * ldx];
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
  if (i == j && i < check_cols && (d == 0.0 || !isfinite(d))) *flag = 1;
}

// W = R^-1, one block per column j: back substitution R w = e_j in binary64.
__global__ __launch_bounds__(256) void k_trinv(const double* __restrict__ R, int64_t ldr, int64_t n,
                                               double* __restrict__ W, int64_t ldw, int* __restrict__ flag) {
  extern __shared__ double bsh[];
  const int64_t j = blockIdx.x;
  const int t = threadIdx.x;
  for (int64_t i = t; i <= j; i += 256) bsh[i] = (i == j) ? 1.0 : 0.0;
  for (int64_t i = j + 1 + t; i < n; i += 256) W[i + j * ldw] = 0.0;
  for (int64_t k = j; k >= 0; --k) {
    __syncthreads();
    const double rkk = R[k + k * ldr];
    const double wk = bsh[k] / rkk;
    if (t == 0) {
      W[k + j * ldw] = wk;
      if (!isfinite(wk)) *flag = 1;
    }
    const double* rc = R + k * ldr;
    for (int64_t i = t; i < k; i += 256) bsh[i] -= rc[i] * wk;
  }
}

__global__ __launch_bounds__(256) void k_to_f32(const double* __restrict__ W, int64_t ldw, int64_t n,
                                                float* __restrict__ W32) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i < n && j < n) W32[i + j * n] = (float)W[i + j * ldw];
}

template <typename T, int RPT, int NB>
int qr_blocked(T* Y, int64_t ldy, int64_t s, int64_t ncols, char* ws, hipStream_t st) {
  const int64_t ncb_max = ls_cdiv(ncols, kColBlock);
  const int64_t nrc_max = ls_cdiv(s, kRowChunk);
  T* tau = reinterpret_cast<T*>(ws);
  T* Tm = reinterpret_cast<T*>(ws + ls_align256(sizeof(T) * ncols));
  T* Wp = reinterpret_cast<T*>(ws + ls_align256(sizeof(T) * ncols) + ls_align256(sizeof(T) * NB * NB));
  (void)ncb_max;
  (void)nrc_max;
  for (int64_t j0 = 0; j0 < ncols; j0 += NB) {
    const int nb = (int)((ncols - j0 < NB) ? (ncols - j0) : NB);
    hipLaunchKernelGGL((k_qr_panel<T, RPT, NB>), dim3(1), dim3(kQrThreads), 0, st, Y, ldy, s, j0, nb, tau, Tm);
    const int64_t c_begin = j0 + nb;
    if (c_begin >= ncols) break;
    const dim3 g((unsigned)ls_cdiv(ncols - c_begin, kColBlock), (unsigned)ls_cdiv(s - j0, kRowChunk));
    hipLaunchKernelGGL((k_qr_wpart<T, NB>), g, dim3(256), 0, st, Y, ldy, s, j0, nb, c_begin, ncols, Wp);
    hipLaunchKernelGGL((k_qr_apply<T, NB>), g, dim3(256), 0, st, Y, ldy, s, j0, nb, c_begin, ncols, Wp, Tm);
  }
  LS_HIP_TRY(hipGetLastError());
  return LS_OK;
}

template <typename T>
int qr_dispatch(T* Y, int64_t ldy, int64_t s, int64_t ncols, char* ws, hipStream_t st) {
  // Panel width chosen so that RPT x NB panel values stay in registers
  // (1024-thread blocks allow 128 VGPRs per lane).
  const int64_t rpt = ls_cdiv(s, kQrThreads);
  if constexpr (sizeof(T) == 4) {
    if (rpt <= 1) return qr_blocked<T, 1, 16>(Y, ldy, s, ncols, ws, st);
    if (rpt <= 2) return qr_blocked<T, 2, 16>(Y, ldy, s, ncols, ws, st);
    if (rpt <= 4) return qr_blocked<T, 4, 8>(Y, ldy, s, ncols, ws, st);
    if (rpt <= 8) return qr_blocked<T, 8, 4>(Y, ldy, s, ncols, ws, st);
  } else {
    if (rpt <= 1) return qr_blocked<T, 1, 8>(Y, ldy, s, ncols, ws, st);
    if (rpt <= 2) return qr_blocked<T, 2, 8>(Y, ldy, s, ncols, ws, st);
    if (rpt <= 4) return qr_blocked<T, 4, 4>(Y, ldy, s, ncols, ws, st);
    if (rpt <= 8) return qr_blocked<T, 8, 2>(Y, ldy, s, ncols, ws, st);
  }
  return LS_E_UNSUPPORTED;
}

}  // namespace

namespace ls {

size_t qr_workspace(int64_t s, int64_t ncols, ls_prec_t u_qr) {
  const size_t elt = (u_qr == LS_FP32) ? 4 : 8;
  size_t b = 0;
  if (u_qr == LS_FP32) b += ls_align256(elt * (size_t)s * ncols);      // binary32 working copy
  b += ls_align256(elt * ncols);                                         // tau
  b += ls_align256(elt * 16 * 16);                                       // T
  b += ls_align256(elt * (size_t)ls_cdiv(ncols, kColBlock) * ls_cdiv(s, kRowChunk) * 16 * kColBlock);
  return b;
}

int qr_run(int64_t s, int64_t ncols, ls_prec_t u_qr, double* Y, int64_t ldy, double* R, int64_t ldr, char* ws,
           size_t ws_bytes, int* d_flag, int64_t check_cols, hipStream_t st) {
  if (ws_bytes < qr_workspace(s, ncols, u_qr)) return LS_E_WORKSPACE;
  if (s > 8 * (int64_t)kQrThreads) return LS_E_UNSUPPORTED;
  const dim3 gfin((unsigned)ls_cdiv(ncols, 256), (unsigned)ncols);
  if (u_qr == LS_FP32) {
    float* Yw = reinterpret_cast<float*>(ws);
    char* rest = ws + ls_align256(4 * (size_t)s * ncols);
    hipLaunchKernelGGL((k_copy_cols<double, float>), dim3((unsigned)ls_cdiv(s, 256), (unsigned)ncols), dim3(256), 0,
                       st, Y, ldy, Yw, s, s, ncols);
    LS_TRY(qr_dispatch<float>(Yw, s, s, ncols, rest, st));
    hipLaunchKernelGGL(k_qr_finish<float>, gfin, dim3(256), 0, st, Yw, s, ncols, check_cols, R, ldr, d_flag);
  } else if (u_qr == LS_FP64) {
    LS_TRY(qr_dispatch<double>(Y, ldy, s, ncols, ws, st));
    hipLaunchKernelGGL(k_qr_finish<double>, gfin, dim3(256), 0, st, Y, ldy, ncols, check_cols, R, ldr, d_flag);
  } else {
    return LS_E_UNSUPPORTED;
  }
  LS_HIP_TRY(hipGetLastError());
  return LS_OK;
}

int trinv_run(const double* R, int64_t ldr, int64_t n, double* W, int64_t ldw, float* W32, int* d_flag,
              hipStream_t st) {
  hipLaunchKernelGGL(k_trinv, dim3((unsigned)n), dim3(256), (size_t)n * sizeof(double), st, R, ldr, n, W, ldw,
                     d_flag);
  if (W32)
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)ls_cdiv(n, 256), (unsigned)n), dim3(256), 0, st, W, ldw, n, W32);
  LS_HIP_TRY(hipGetLastError());
  return LS_OK;
}

}  // namespace ls
