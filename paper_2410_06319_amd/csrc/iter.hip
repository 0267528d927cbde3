// Algorithm 2 on gfx950: LSQR right-preconditioned with R (line 1) and
// augmented-system refinement with split-preconditioned FGMRES (lines 2-10).
//
// R^-1 is applied through the explicit upper-triangular W = R^-1 (formed once
// in binary64), so every preconditioner application is a parallel triangular
// matrix-vector product.  The products with A are HBM-bound; each iteration
// reads A once: a block of RB rows of A (all n columns) is staged in LDS and
// used for both the row products (A p) and the column products (A^T u).
// Column products are per-block partial sums reduced by a second kernel in a
// fixed order, so results are reproducible run to run.
//
// Scalars live in device memory; kernels of one iteration are enqueued back
// to back and the host only reads a convergence flag every few iterations.
#include <cmath>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace ls {
namespace {

constexpr int kThreads = 256;

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ double* align8(void* p) {
  return reinterpret_cast<double*>(((uintptr_t)p + 7) & ~(uintptr_t)7);
}

template <typename T>
__device__ __forceinline__ T block_sum256(T v, T* sh) {
  return ls_block_sum<T, kThreads>(v, sh);
}

// Stage rows [i0, i0+RB) x columns [0, n) of A into As[j * (RB+1) + r] (type T).
template <typename TA, typename T, int RB>
__device__ __forceinline__ void load_rows(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n, int64_t i0,
                                          bool vec_ok, T* __restrict__ As) {
  constexpr int LDR = RB + 1;
  constexpr int V = 16 / (int)sizeof(TA);
  static_assert(RB % V == 0, "row block must hold whole vectors");
  if (vec_ok && i0 + RB <= m) {
    constexpr int PER = RB / V;
    const int total = (int)n * PER;
    for (int idx = threadIdx.x; idx < total; idx += kThreads) {
      const int j = idx / PER;
      const int q = idx - j * PER;
      const TA* src = A + i0 + q * V + (int64_t)j * lda;
      T* dst = As + j * LDR + q * V;
      if constexpr (V == 4) {
        const float4 v = *reinterpret_cast<const float4*>(src);
        dst[0] = (T)v.x;
        dst[1] = (T)v.y;
        dst[2] = (T)v.z;
        dst[3] = (T)v.w;
      } else {
        const double2 v = *reinterpret_cast<const double2*>(src);
        dst[0] = (T)v.x;
        dst[1] = (T)v.y;
      }
    }
  } else {
    const int total = (int)n * RB;
    for (int idx = threadIdx.x; idx < total; idx += kThreads) {
      const int j = idx / RB;
      const int r = idx - j * RB;
      const int64_t i = i0 + r;
      As[j * LDR + r] = (i < m) ? (T)A[i + (int64_t)j * lda] : T(0);
    }
  }
}

// q[r] = sum_j As[j][r] * vec[j] for r < RB, via RB x (256/RB) thread layout.
template <typename T, int RB>
__device__ __forceinline__ T rows_times_vec(const T* __restrict__ As, const T* __restrict__ vec, int64_t n,
                                            T* __restrict__ red) {
  constexpr int LDR = RB + 1;
  constexpr int G1 = kThreads / RB;
  const int r = threadIdx.x % RB;
  const int g = threadIdx.x / RB;
  T acc = 0;
  for (int j = g; j < n; j += G1) acc += As[j * LDR + r] * vec[j];
  red[g * RB + r] = acc;
  __syncthreads();
  T q = 0;
  if (threadIdx.x < RB) {
#pragma unroll 4
    for (int gg = 0; gg < G1; ++gg) q += red[gg * RB + threadIdx.x];
  }
  return q;   // valid in threads < RB
}

// ================================================================== LSQR
// One pass over A:  u <- A p - coef * u  (coef = alpha_i / beta_i), partial
// ||u||^2, partial t = A^T u.  Init mode: u <- b - A x0 (p holds -x0, coef = -1,
// the old u is b) and partial ||b||^2.
template <typename TA, typename T, int RB>
__global__ __launch_bounds__(kThreads) void k_lsqr_pass(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                        int vec_ok, const T* __restrict__ p, T* __restrict__ u,
                                                        const TA* __restrict__ b, const LsqrState* __restrict__ st,
                                                        int par, int init, T* __restrict__ tpart,
                                                        double* __restrict__ nupart, double* __restrict__ nbpart) {
  if (!init && st->rec[par].done) return;
  extern __shared__ __align__(16) char smem[];
  constexpr int LDR = RB + 1;
  T* As = reinterpret_cast<T*>(smem);
  T* ps = As + n * LDR;
  T* tacc = ps + n;
  T* uu = tacc + n;
  T* red = uu + RB;
  double* dsh = align8(red + kThreads);
  const T coef = init ? T(-1) : (T)(st->rec[par].alpha / st->beta);
  for (int j = threadIdx.x; j < n; j += kThreads) {
    ps[j] = init ? -p[j] : p[j];
    tacc[j] = 0;
  }
  double nu = 0.0, nb = 0.0;
  const int64_t nrb = ls_cdiv(m, RB);
  for (int64_t rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
    const int64_t i0 = rb * RB;
    __syncthreads();
    load_rows<TA, T, RB>(A, lda, m, n, i0, vec_ok != 0, As);
    __syncthreads();
    const T q = rows_times_vec<T, RB>(As, ps, n, red);
    if (threadIdx.x < RB) {
      const int64_t i = i0 + threadIdx.x;
      T un = 0;
      if (i < m) {
        const T uo = init ? (T)b[i] : u[i];
        un = q - coef * uo;
        u[i] = un;
        if (init) nb += (double)uo * (double)uo;
      }
      uu[threadIdx.x] = un;
      nu += (double)un * (double)un;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += kThreads) {
      T acc = 0;
#pragma unroll 8
      for (int r = 0; r < RB; ++r) acc += As[j * LDR + r] * uu[r];
      tacc[j] += acc;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += kThreads) tpart[(int64_t)blockIdx.x * n + j] = tacc[j];
  nu = block_sum256(nu, dsh);
  nb = block_sum256(nb, dsh + 4);
  if (threadIdx.x == 0) {
    nupart[blockIdx.x] = nu;
    if (init) nbpart[blockIdx.x] = nb;
  }
}

// beta = sqrt(sum nupart); t[j] = (sum_g tpart[g][j]) / beta.  Block: 64 columns x 4 groups.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_lsqr_reduce(const T* __restrict__ tpart, int G, int64_t n,
                                                          const double* __restrict__ nupart,
                                                          const double* __restrict__ nbpart, LsqrState* st, int par,
                                                          int init, T* __restrict__ t) {
  if (!init && st->rec[par].done) return;
  __shared__ double dsh[8];
  __shared__ T red[4][64];
  double s = 0.0, sb = 0.0;
  for (int g = threadIdx.x; g < G; g += kThreads) {
    s += nupart[g];
    if (init) sb += nbpart[g];
  }
  s = block_sum256(s, dsh);
  sb = block_sum256(sb, dsh + 4);
  const double beta = sqrt(s);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->beta = beta;
    if (init) st->normb = sqrt(sb);
    if (!isfinite(beta)) st->flag = 1;
  }
  const int c = threadIdx.x & 63;
  const int gg = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + c;
  T acc = 0;
  if (j < n)
    for (int g = gg; g < G; g += 4) acc += tpart[(int64_t)g * n + j];
  red[gg][c] = acc;
  __syncthreads();
  if (gg == 0 && j < n) {
    const T tot = red[0][c] + red[1][c] + red[2][c] + red[3][c];
    t[j] = (beta > 0.0) ? (T)(tot / (T)beta) : T(0);
  }
}

// v <- W^T t - (beta_{i+1} / alpha_i) v   (init: v <- W^T t); partial ||v||^2.
// One wave per column j: v_j = sum_{i <= j} W[i + j ldw] t[i].
template <typename T>
__global__ __launch_bounds__(kThreads) void k_lsqr_vupdate(const T* __restrict__ W, int64_t ldw, int64_t n,
                                                           const T* __restrict__ t, T* __restrict__ v,
                                                           const LsqrState* __restrict__ st, int par, int init,
                                                           double* __restrict__ nvpart) {
  if (!init && st->rec[par].done) return;
  __shared__ double dsh[4];
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  double contrib = 0.0;
  if (j < n) {
    const T* wc = W + j * ldw;
    T acc = 0;
    for (int64_t i = lane; i <= j; i += 64) acc += wc[i] * t[i];
    acc = ls_wave_sum(acc);
    if (lane == 0) {
      T vn = acc;
      if (!init) vn -= (T)(st->beta / st->rec[par].alpha) * v[j];
      v[j] = vn;
      contrib = (double)vn * (double)vn;
    }
  }
  contrib = block_sum256(contrib, dsh);
  if (threadIdx.x == 0) nvpart[blockIdx.x] = contrib;
}

// Start of iteration `it`: alpha_it = ||v||, the plane rotation of iteration
// it-1, the stopping tests, x <- x + (phi/rho) what, then p = W v / alpha and
// what <- p - (theta/rho) what.  Reads rec[par], writes rec[par ^ 1].
// Block: 64 rows of W; its 4 waves split the columns.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_lsqr_step(const T* __restrict__ W, int64_t ldw, int64_t n,
                                                        const T* __restrict__ v, const double* __restrict__ nvpart,
                                                        int Gv, LsqrState* st, int par, int it, int final_step,
                                                        double tol, int maxit, T* __restrict__ p,
                                                        T* __restrict__ what, double* __restrict__ x) {
  __shared__ double dsh[4];
  __shared__ T red[4][64];
  const LsqrRec R = st->rec[par];
  if (R.done) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st->rec[par ^ 1] = R;
    return;
  }
  double s = 0.0;
  for (int g = threadIdx.x; g < Gv; g += kThreads) s += nvpart[g];
  s = block_sum256(s, dsh);
  const double alpha = sqrt(s);
  const double beta = st->beta;
  LsqrRec N = R;
  double xcoef = 0.0, wcoef = 0.0;
  int stop = 0;
  if (it == 1) {
    N.rhobar = alpha;
    N.phibar = beta;
    N.normB2 = 0.0;
    N.normr = beta;
    if (beta == 0.0) stop = 4;
  } else {
    N.normB2 = R.normB2 + R.alpha * R.alpha + beta * beta;
    const double rho = hypot(R.rhobar, beta);
    const double c = R.rhobar / rho;
    const double sn = beta / rho;
    const double theta = sn * alpha;
    N.rhobar = -c * alpha;
    const double phi = c * R.phibar;
    N.phibar = sn * R.phibar;
    xcoef = phi / rho;
    wcoef = theta / rho;
    N.normr = N.phibar;
    N.normar = N.phibar * alpha * fabs(c);
    N.normB = sqrt(N.normB2);
    N.its = it - 1;
    if (N.normr <= tol * st->normb) stop = 1;
    else if (N.normar <= tol * N.normB * N.normr) stop = 2;
    else if (beta == 0.0 || alpha == 0.0) stop = 4;
    else if (final_step || it - 1 >= maxit) stop = 3;
    if (!isfinite(xcoef) || !isfinite(wcoef)) {
      stop = 5;
      xcoef = 0.0;
    }
  }
  N.alpha = alpha;
  N.phi_over_rho = xcoef;
  N.theta_over_rho = wcoef;
  const bool done = stop != 0;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * 64 + lane;
  T acc = 0;
  if (!done && r < n) {
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    for (int64_t j = r0 + wv; j < n; j += 4) acc += W[r + j * ldw] * v[j];
  }
  red[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && r < n) {
    if (it > 1) x[r] = (double)((T)x[r] + (T)xcoef * what[r]);
    if (!done) {
      const T pr = (red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane]) / (T)alpha;
      p[r] = pr;
      what[r] = (it == 1) ? pr : pr - (T)wcoef * what[r];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    N.done = done ? 1 : 0;
    N.stop = stop;
    if (stop == 5) st->flag = 1;
    st->rec[par ^ 1] = N;
  }
}

template <typename TO>
__global__ __launch_bounds__(kThreads) void k_cast_vec(const double* __restrict__ a, TO* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) b[i] = (TO)a[i];
}

__global__ void k_zero_bytes(char* p, size_t nbytes) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < nbytes; i += (size_t)gridDim.x * kThreads) p[i] = 0;
}

// ================================================================== refinement
// r = b - A x in precision T (Algorithm 2 line 2).
template <typename TA, typename T>
__global__ __launch_bounds__(kThreads) void k_resid_u(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                      const TA* __restrict__ b, const double* __restrict__ x,
                                                      double* __restrict__ r) {
  extern __shared__ __align__(16) char smem[];
  T* xs = reinterpret_cast<T*>(smem);
  for (int j = threadIdx.x; j < n; j += kThreads) xs[j] = (T)x[j];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= m) return;
  T acc = 0;
  for (int64_t j = 0; j < n; ++j) acc += (T)A[i + j * lda] * xs[j];
  r[i] = (double)((T)b[i] - acc);
}

// Line 5 in u_r: f = b - r - A x (rows, written to V[:, 0]) and partial
// t = A^T r; binary64, or double-double accumulation when DD.
template <typename TA, bool DD, int RB>
__global__ __launch_bounds__(kThreads) void k_lsir_resid(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                         int vec_ok, const TA* __restrict__ b,
                                                         const double* __restrict__ r, const double* __restrict__ x,
                                                         double* __restrict__ V, double* __restrict__ tpart_hi,
                                                         double* __restrict__ tpart_lo, double* __restrict__ fpart) {
  extern __shared__ __align__(16) char smem[];
  constexpr int LDR = RB + 1;
  constexpr int G1 = kThreads / RB;
  double* As = reinterpret_cast<double*>(smem);
  double* xs = As + n * LDR;
  double* thi = xs + n;
  double* tlo = thi + n;
  double* rr = tlo + n;
  double* rhi = rr + RB;
  double* rlo = rhi + kThreads;
  double* dsh = rlo + kThreads;
  for (int j = threadIdx.x; j < n; j += kThreads) {
    xs[j] = x[j];
    thi[j] = 0.0;
    tlo[j] = 0.0;
  }
  double fn = 0.0;
  const int64_t nrb = ls_cdiv(m, RB);
  for (int64_t rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
    const int64_t i0 = rb * RB;
    __syncthreads();
    load_rows<TA, double, RB>(A, lda, m, n, i0, vec_ok != 0, As);
    __syncthreads();
    {
      const int rw = threadIdx.x % RB;
      const int g = threadIdx.x / RB;
      ls_dd acc{0.0, 0.0};
      for (int j = g; j < n; j += G1) {
        if (DD) acc = ls_dd_fma(acc, As[j * LDR + rw], xs[j]);
        else acc.hi += As[j * LDR + rw] * xs[j];
      }
      rhi[g * RB + rw] = acc.hi;
      rlo[g * RB + rw] = acc.lo;
    }
    __syncthreads();
    if (threadIdx.x < RB) {
      const int64_t i = i0 + threadIdx.x;
      double ri = 0.0;
      if (i < m) {
        ri = r[i];
        double f;
        if (DD) {
          ls_dd q{0.0, 0.0};
          for (int gg = 0; gg < G1; ++gg) q = ls_dd_add(q, ls_dd{rhi[gg * RB + threadIdx.x], rlo[gg * RB + threadIdx.x]});
          ls_dd fb = ls_two_sum((double)b[i], -ri);
          fb = ls_dd_add(fb, ls_dd{-q.hi, -q.lo});
          f = fb.hi + fb.lo;
        } else {
          double q = 0.0;
          for (int gg = 0; gg < G1; ++gg) q += rhi[gg * RB + threadIdx.x];
          f = ((double)b[i] - ri) - q;
        }
        V[i] = f;
        fn += f * f;
      }
      rr[threadIdx.x] = ri;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += kThreads) {
      if (DD) {
        ls_dd acc{thi[j], tlo[j]};
        for (int rw = 0; rw < RB; ++rw) acc = ls_dd_fma(acc, As[j * LDR + rw], rr[rw]);
        thi[j] = acc.hi;
        tlo[j] = acc.lo;
      } else {
        double acc = 0.0;
        for (int rw = 0; rw < RB; ++rw) acc += As[j * LDR + rw] * rr[rw];
        thi[j] += acc;
      }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n; j += kThreads) {
    tpart_hi[(int64_t)blockIdx.x * n + j] = thi[j];
    tpart_lo[(int64_t)blockIdx.x * n + j] = tlo[j];
  }
  fn = block_sum256(fn, dsh);
  if (threadIdx.x == 0) fpart[blockIdx.x] = fn;
}

// g = -(sum of column partials), then h = W^T g (line 6) into V[m:, 0]; partial ||h||^2.
// Block: 4 waves, one column each; each wave first needs g[0..j]: g is formed
// by a preceding reduction into gbuf.
template <bool DD>
__global__ __launch_bounds__(kThreads) void k_lsir_g(const double* __restrict__ tpart_hi,
                                                     const double* __restrict__ tpart_lo, int G, int64_t n,
                                                     double* __restrict__ g) {
  __shared__ double rh[4][64];
  __shared__ double rl[4][64];
  const int c = threadIdx.x & 63;
  const int gg = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + c;
  ls_dd acc{0.0, 0.0};
  if (j < n)
    for (int q = gg; q < G; q += 4) {
      if (DD) acc = ls_dd_add(acc, ls_dd{tpart_hi[(int64_t)q * n + j], tpart_lo[(int64_t)q * n + j]});
      else acc.hi += tpart_hi[(int64_t)q * n + j];
    }
  rh[gg][c] = acc.hi;
  rl[gg][c] = acc.lo;
  __syncthreads();
  if (gg == 0 && j < n) {
    ls_dd t{0.0, 0.0};
    for (int q = 0; q < 4; ++q) {
      if (DD) t = ls_dd_add(t, ls_dd{rh[q][c], rl[q][c]});
      else t.hi += rh[q][c];
    }
    g[j] = -(t.hi + t.lo);
  }
}

template <bool DD>
__global__ __launch_bounds__(kThreads) void k_lsir_h(const double* __restrict__ W, int64_t ldw, int64_t n, int64_t m,
                                                     const double* __restrict__ g, double* __restrict__ V,
                                                     double* __restrict__ hpart) {
  __shared__ double dsh[4];
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  double contrib = 0.0;
  if (j < n) {
    const double* wc = W + j * ldw;
    ls_dd acc{0.0, 0.0};
    for (int64_t i = lane; i <= j; i += 64) {
      if (DD) acc = ls_dd_fma(acc, wc[i], g[i]);
      else acc.hi += wc[i] * g[i];
    }
    // wave sum of the (hi, lo) pairs
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

// ------------------------------------------------------------------ FGMRES
struct FgPtrs {
  double* V;        // (m + n) x (kmax + 1), ld ldv
  int64_t ldv;
  double* Z;        // n x kmax  (M_R^-1 applied to the x part)
  double* H;        // (kmax + 1) x kmax, ld kmax + 1
  double* cs;
  double* sn;
  double* g;
  double* hj;       // current subdiagonal norm
  FgState* st;
};

// Column j: h = ||w|| from partials (j = 0: beta = ||s||), Givens rotation for
// column j-1 and the convergence test (block 0), normalisation of V_r[:, j]
// (blocks < nrb) and z = W (V_x[:, j] / h) (remaining blocks; skipped in the
// final call).  V_x[:, j] itself is normalised by the next kernel.
template <typename TP>
__global__ __launch_bounds__(kThreads) void k_fg_a(FgPtrs F, int64_t m, int64_t n, int j, int kmax,
                                                   const TP* __restrict__ W, int64_t ldw,
                                                   const double* __restrict__ w2part, int Gw, double tol,
                                                   int final_step, int nrb) {
  __shared__ double dsh[4];
  __shared__ TP red[4][64];
  if (F.st->done) return;
  double s = 0.0;
  for (int q = threadIdx.x; q < Gw; q += kThreads) s += w2part[q];
  s = block_sum256(s, dsh);
  const double h = sqrt(s);
  const int64_t ldh = kmax + 1;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    FgState S = *F.st;
    *F.hj = h;
    if (j == 0) {
      S.beta = h;
      F.g[0] = h;
      S.relres = 1.0;
      S.k = 0;
      if (h == 0.0 || !isfinite(h)) {
        S.done = 1;
        S.breakdown = (h == 0.0) ? 0 : 2;
      }
    } else {
      const int c = j - 1;
      double* Hc = F.H + c * ldh;
      Hc[j] = h;
      for (int i = 0; i < c; ++i) {
        const double a = Hc[i], bb = Hc[i + 1];
        Hc[i] = F.cs[i] * a + F.sn[i] * bb;
        Hc[i + 1] = -F.sn[i] * a + F.cs[i] * bb;
      }
      const double d = hypot(Hc[c], Hc[c + 1]);
      const double cc = (d > 0.0) ? Hc[c] / d : 1.0;
      const double ss = (d > 0.0) ? Hc[c + 1] / d : 0.0;
      F.cs[c] = cc;
      F.sn[c] = ss;
      Hc[c] = d;
      Hc[c + 1] = 0.0;
      F.g[c + 1] = -ss * F.g[c];
      F.g[c] = cc * F.g[c];
      S.relres = fabs(F.g[c + 1]) / S.beta;
      S.k = j;
      if (!isfinite(S.relres)) {
        S.done = 1;
        S.breakdown = 2;
      } else if (S.relres <= tol || h == 0.0 || final_step || j >= kmax) {
        S.done = 1;
        if (h == 0.0) S.breakdown = 1;
      }
    }
    *F.st = S;
  }
  if (h == 0.0 || !isfinite(h) || final_step || j >= kmax) return;
  const double inv = 1.0 / h;
  double* vj = F.V + (int64_t)j * F.ldv;
  if ((int)blockIdx.x < nrb) {
    for (int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x; i < m && i < ((int64_t)blockIdx.x + 1) * 1024;
         i += kThreads)
      vj[i] *= inv;
    return;
  }
  const int bx = blockIdx.x - nrb;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t r = (int64_t)bx * 64 + lane;
  TP acc = 0;
  if (r < n) {
    const int64_t r0 = (int64_t)bx * 64;
    for (int64_t c = r0 + wv; c < n; c += 4) acc += W[r + c * ldw] * (TP)(vj[m + c] * inv);
  }
  red[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && r < n) F.Z[r + (int64_t)j * n] = (double)(red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane]);
}

// One pass over A for column j:  w_r = v_r + A z  -> V[:, j+1] (rows < m),
// partial t = A^T v_r, partial h1_r[c] = V_r[:, c] . w_r (c <= j), stored
// column-major hpart[c * G + block].  Block 0 also normalises V_x[:, j].
template <typename TA, typename TP, int RB>
__global__ __launch_bounds__(kThreads) void k_fg_pass(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                      int vec_ok, FgPtrs F, int j, TP* __restrict__ tpart,
                                                      double* __restrict__ hpart) {
  if (F.st->done) return;
  extern __shared__ __align__(16) char smem[];
  constexpr int LDR = RB + 1;
  TP* As = reinterpret_cast<TP*>(smem);
  TP* zs = As + n * LDR;
  TP* tacc = zs + n;
  TP* uu = tacc + n;
  TP* red = uu + RB;
  double* wv = align8(red + kThreads);
  double* hacc = wv + RB;     // j + 1 entries
  const double* vj = F.V + (int64_t)j * F.ldv;
  double* w = F.V + (int64_t)(j + 1) * F.ldv;
  if (blockIdx.x == 0) {
    const double inv = 1.0 / *F.hj;
    double* vx = F.V + (int64_t)j * F.ldv + m;
    for (int64_t c = threadIdx.x; c < n; c += kThreads) vx[c] *= inv;
  }
  for (int c = threadIdx.x; c < n; c += kThreads) {
    zs[c] = (TP)F.Z[c + (int64_t)j * n];
    tacc[c] = 0;
  }
  for (int c = threadIdx.x; c <= j; c += kThreads) hacc[c] = 0.0;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t nrb = ls_cdiv(m, RB);
  for (int64_t rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
    const int64_t i0 = rb * RB;
    __syncthreads();
    load_rows<TA, TP, RB>(A, lda, m, n, i0, vec_ok != 0, As);
    __syncthreads();
    const TP q = rows_times_vec<TP, RB>(As, zs, n, red);
    if (threadIdx.x < RB) {
      const int64_t i = i0 + threadIdx.x;
      TP vr = 0;
      double wr = 0.0;
      if (i < m) {
        vr = (TP)vj[i];
        wr = (double)(vr + q);
        w[i] = wr;
      }
      uu[threadIdx.x] = vr;
      wv[threadIdx.x] = wr;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += kThreads) {
      TP acc = 0;
#pragma unroll 8
      for (int rw = 0; rw < RB; ++rw) acc += As[c * LDR + rw] * uu[rw];
      tacc[c] += acc;
    }
    // h1 (r part): wave per Krylov column, lanes over the block's rows
    for (int c = wave; c <= j; c += 4) {
      double prod = 0.0;
      if (lane < RB && i0 + lane < m) prod = F.V[i0 + lane + (int64_t)c * F.ldv] * wv[lane];
      prod = ls_wave_sum(prod);
      if (lane == 0) hacc[c] += prod;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += kThreads) tpart[(int64_t)blockIdx.x * n + c] = tacc[c];
  for (int c = threadIdx.x; c <= j; c += kThreads) hpart[(int64_t)c * gridDim.x + blockIdx.x] = hacc[c];
}

// t[c] = sum_g tpart[g][c] (blocks < ncb, 64 columns each) and
// h1r[c] = sum_g hpart[c][g] (remaining blocks, one Krylov column each).
template <typename TP>
__global__ __launch_bounds__(kThreads) void k_fg_reduce(const TP* __restrict__ tpart, const double* __restrict__ hpart,
                                                        int G, int64_t n, int j, int ncb, double* __restrict__ t,
                                                        double* __restrict__ h1r, const FgState* st) {
  if (st->done) return;
  __shared__ TP red[4][64];
  __shared__ double dsh[4];
  if ((int)blockIdx.x < ncb) {
    const int c = threadIdx.x & 63;
    const int gg = threadIdx.x >> 6;
    const int64_t col = (int64_t)blockIdx.x * 64 + c;
    TP acc = 0;
    if (col < n)
      for (int q = gg; q < G; q += 4) acc += tpart[(int64_t)q * n + col];
    red[gg][c] = acc;
    __syncthreads();
    if (gg == 0 && col < n) t[col] = (double)(red[0][c] + red[1][c] + red[2][c] + red[3][c]);
    return;
  }
  const int c = blockIdx.x - ncb;
  if (c > j) return;
  double s = 0.0;
  for (int q = threadIdx.x; q < G; q += kThreads) s += hpart[(int64_t)c * G + q];
  s = block_sum256(s, dsh);
  if (threadIdx.x == 0) h1r[c] = s;
}

// w_x = W^T t (M_L^-1 on the x part) -> V[m:, j+1]; partial h1_x[c] over the
// block's 16 columns, stored column-major hxpart[c * G + block].
template <typename TP>
__global__ __launch_bounds__(1024) void k_fg_c(const TP* __restrict__ W, int64_t ldw, int64_t n, int64_t m,
                                               const double* __restrict__ t, FgPtrs F, int j,
                                               double* __restrict__ hxpart) {
  if (F.st->done) return;
  __shared__ double wx[16];
  const int lane = threadIdx.x & 63;
  const int wvi = threadIdx.x >> 6;
  const int64_t col = (int64_t)blockIdx.x * 16 + wvi;
  double* w = F.V + (int64_t)(j + 1) * F.ldv;
  double val = 0.0;
  if (col < n) {
    const TP* wc = W + col * ldw;
    TP acc = 0;
    for (int64_t i = lane; i <= col; i += 64) acc += wc[i] * (TP)t[i];
    acc = ls_wave_sum(acc);
    val = (double)acc;
    if (lane == 0) w[m + col] = val;
  }
  if (lane == 0) wx[wvi] = val;
  __syncthreads();
  for (int c = threadIdx.x; c <= j; c += 1024) {
    double s = 0.0;
    for (int q = 0; q < 16; ++q) {
      const int64_t cc = (int64_t)blockIdx.x * 16 + q;
      if (cc < n) s += F.V[m + cc + (int64_t)c * F.ldv] * wx[q];
    }
    hxpart[(int64_t)c * gridDim.x + blockIdx.x] = s;
  }
}

// Classical Gram-Schmidt sweep over rows [1024 b, 1024 (b+1)) of w = V[:, j+1]:
//   hsum[c] = h_in[c] (+ sum of x-part partials in the first sweep);
//   w <- w - V[:, 0:j+1] hsum;  partial dots V[:, c] . w (second=0) or partial ||w||^2 (second=1).
// Block 0 records hsum in column j of H (first sweep) or adds it (second sweep).
__global__ __launch_bounds__(kThreads) void k_cgs(FgPtrs F, int64_t m, int64_t n, int j, int kmax,
                                                  const double* __restrict__ h_in, const double* __restrict__ hx,
                                                  int Gx, const double* __restrict__ h2part, int G2, int second,
                                                  double* __restrict__ out_part, double* __restrict__ w2part) {
  if (F.st->done) return;
  __shared__ double hs[96];
  __shared__ double wsh[1024];
  __shared__ double dsh[4];
  const int64_t rows = m + n;
  for (int c = threadIdx.x; c <= j; c += kThreads) {
    double s = 0.0;
    if (!second) {
      s = h_in[c];
      for (int q = 0; q < Gx; ++q) s += hx[(int64_t)c * Gx + q];
    } else {
      for (int q = 0; q < G2; ++q) s += h2part[(int64_t)c * G2 + q];
    }
    hs[c] = s;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x <= j) {
    double* Hc = F.H + (int64_t)j * (kmax + 1);
    if (!second) Hc[threadIdx.x] = hs[threadIdx.x];
    else Hc[threadIdx.x] += hs[threadIdx.x];
  }
  double* w = F.V + (int64_t)(j + 1) * F.ldv;
  const int64_t base = (int64_t)blockIdx.x * 1024;
  double nrm = 0.0;
  for (int q = 0; q < 4; ++q) {
    const int li = q * kThreads + threadIdx.x;
    const int64_t i = base + li;
    double wi = 0.0;
    if (i < rows) {
      wi = w[i];
      for (int c = 0; c <= j; ++c) wi -= F.V[i + (int64_t)c * F.ldv] * hs[c];
      w[i] = wi;
      nrm += wi * wi;
    }
    wsh[li] = wi;
  }
  __syncthreads();
  if (second) {
    nrm = block_sum256(nrm, dsh);
    if (threadIdx.x == 0) w2part[blockIdx.x] = nrm;
    return;
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int c = wave; c <= j; c += 4) {
    double prod = 0.0;
    const double* vc = F.V + (int64_t)c * F.ldv;
    for (int q = 0; q < 16; ++q) {
      const int li = q * 64 + lane;
      const int64_t i = base + li;
      if (i < rows) prod += vc[i] * wsh[li];
    }
    prod = ls_wave_sum(prod);
    if (lane == 0) out_part[(int64_t)c * gridDim.x + blockIdx.x] = prod;
  }
}

// Correction of one refinement step: y = H(0:k,0:k)^-1 g(0:k) (every block),
// dr = V_r y, dx = Z y; r += dr and x += dx rounded to the working precision
// TU; partial sums of ||dr||^2, ||dx||^2, ||r||^2, ||x||^2 -> part[4 * block + q].
template <typename TU>
__global__ __launch_bounds__(kThreads) void k_fg_update(FgPtrs F, int64_t m, int64_t n, int kmax,
                                                        double* __restrict__ r, double* __restrict__ x,
                                                        double* __restrict__ part) {
  __shared__ double y[128];
  __shared__ double dsh[16];
  const int k = F.st->k;
  const int64_t ldh = kmax + 1;
  for (int i = threadIdx.x; i < k; i += kThreads) y[i] = F.g[i];
  for (int i = k - 1; i >= 0; --i) {
    __syncthreads();
    const double yi = y[i] / F.H[i + (int64_t)i * ldh];
    __syncthreads();
    if (threadIdx.x == 0) y[i] = yi;
    for (int t = threadIdx.x; t < i; t += kThreads) y[t] -= F.H[t + (int64_t)i * ldh] * yi;
  }
  __syncthreads();
  const int64_t rows = m + n;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int q = 0; q < 4; ++q) {
    const int64_t i = (int64_t)blockIdx.x * 1024 + q * kThreads + threadIdx.x;
    if (i >= rows) continue;
    double d = 0.0;
    if (i < m) {
      for (int c = 0; c < k; ++c) d += F.V[i + (int64_t)c * F.ldv] * y[c];
      const double rn = (double)((TU)r[i] + (TU)d);
      r[i] = rn;
      acc[0] += d * d;
      acc[2] += rn * rn;
    } else {
      const int64_t ix = i - m;
      for (int c = 0; c < k; ++c) d += F.Z[ix + (int64_t)c * n] * y[c];
      const double xn = (double)((TU)x[ix] + (TU)d);
      x[ix] = xn;
      acc[1] += d * d;
      acc[3] += xn * xn;
    }
  }
  for (int q = 0; q < 4; ++q) {
    const double s = block_sum256(acc[q], dsh + 4 * q);
    if (threadIdx.x == 0) part[4 * (int64_t)blockIdx.x + q] = s;
  }
}

// ------------------------------------------------------------------ host helpers
size_t device_lds_limit() {
  static size_t cached = 0;
  if (cached == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cached = prop.sharedMemPerBlock;
    if (cached == 0) cached = 64 * 1024;
  }
  return cached;
}

int pick_rb(int64_t n, size_t elt) {
  // LDS budget ~ 72 KB per block so that two blocks share a compute unit,
  // capped by what the device grants one block.
  size_t budget = 72 * 1024;
  const size_t lim = device_lds_limit();
  if (lim < budget + 1024) budget = lim - 1024;
  if ((size_t)n * 33 * elt + 4 * (size_t)n * elt + 8192 <= budget) return 32;
  if ((size_t)n * 17 * elt + 4 * (size_t)n * elt + 8192 <= budget) return 16;
  return 8;
}

bool vec_aligned(const void* A, int64_t lda, size_t elt) {
  const size_t v = 16 / elt;
  return ((uintptr_t)A % 16 == 0) && (lda % (int64_t)v == 0);
}

}  // namespace

int device_cu_count() {
  static int cached = 0;
  if (cached == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cached = prop.multiProcessorCount;
    if (cached <= 0) cached = 256;
  }
  return cached;
}

// ================================================================== LSQR driver
namespace {
struct LsqrWs {
  LsqrState* st;
  char* p;
  char* u;
  char* t;
  char* v;
  char* what;
  char* tpart;
  double* nupart;
  double* nbpart;
  double* nvpart;
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
  w.p = take(elt * P->n);
  w.u = take(elt * P->m);
  w.t = take(elt * P->n);
  w.v = take(elt * P->n);
  w.what = take(elt * P->n);
  w.tpart = take(elt * P->n * (size_t)G);
  w.nupart = reinterpret_cast<double*>(take(8 * (size_t)G));
  w.nbpart = reinterpret_cast<double*>(take(8 * (size_t)G));
  w.nvpart = reinterpret_cast<double*>(take(8 * (size_t)Gv));
  w.bytes = off;
  return w;
}

int lsqr_grid(const ls_problem_t* P, int rb, int ncu) {
  const int64_t nrb = ls_cdiv(P->m, rb);
  int64_t G = 2 * (int64_t)ncu;
  if (G > nrb) G = nrb;
  if (G < 1) G = 1;
  return (int)G;
}

template <typename TA, typename T>
int lsqr_typed(const ls_problem_t* P, const T* Wt, int64_t ldw, double* x, const ls_iter_opts_t* io,
               ls_stats_t* stats, char* ws, size_t ws_bytes, hipStream_t st) {
  const int64_t m = P->m, n = P->n;
  const int rb = pick_rb(n, sizeof(T));
  const int ncu = device_cu_count();
  const int G = lsqr_grid(P, rb, ncu);
  const int Gv = (int)ls_cdiv(n, 4);
  LsqrWs w = lsqr_carve(ws, P, sizeof(T), G, Gv);
  if (w.bytes > ws_bytes) return LS_E_WORKSPACE;
  const TA* A = static_cast<const TA*>(P->A);
  const TA* b = static_cast<const TA*>(P->b);
  T* p = reinterpret_cast<T*>(w.p);
  T* u = reinterpret_cast<T*>(w.u);
  T* t = reinterpret_cast<T*>(w.t);
  T* v = reinterpret_cast<T*>(w.v);
  T* what = reinterpret_cast<T*>(w.what);
  T* tpart = reinterpret_cast<T*>(w.tpart);
  const int vec_ok = vec_aligned(A, P->lda, sizeof(TA)) ? 1 : 0;
  const size_t lds = ((size_t)n * (rb + 1) + 2 * (size_t)n + rb + kThreads) * sizeof(T) + 8 * sizeof(double) + 16;
  if (lds > device_lds_limit()) return LS_E_UNSUPPORTED;
  const int maxit = io->lsqr_maxit;
  const double tol = io->lsqr_tol;
  const int check = io->check_every > 0 ? io->check_every : 8;

  hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(kThreads), 0, st, reinterpret_cast<char*>(w.st), sizeof(LsqrState));
  hipLaunchKernelGGL(k_cast_vec<T>, dim3((unsigned)ls_cdiv(n, kThreads)), dim3(kThreads), 0, st, x, p, n);
  auto pass = [&](int par, int init) {
    prof_begin(kProfLsqrPass, st);
    switch (rb) {
      case 32:
        hipLaunchKernelGGL((k_lsqr_pass<TA, T, 32>), dim3(G), dim3(kThreads), lds, st, A, P->lda, m, n, vec_ok, p, u,
                           b, w.st, par, init, tpart, w.nupart, w.nbpart);
        break;
      case 16:
        hipLaunchKernelGGL((k_lsqr_pass<TA, T, 16>), dim3(G), dim3(kThreads), lds, st, A, P->lda, m, n, vec_ok, p, u,
                           b, w.st, par, init, tpart, w.nupart, w.nbpart);
        break;
      default:
        hipLaunchKernelGGL((k_lsqr_pass<TA, T, 8>), dim3(G), dim3(kThreads), lds, st, A, P->lda, m, n, vec_ok, p, u,
                           b, w.st, par, init, tpart, w.nupart, w.nbpart);
        break;
    }
    // A once, u read and written, p read, t written
    prof_end(kProfLsqrPass, st, (double)m * n * sizeof(TA) + 2.0 * m * sizeof(T) + 2.0 * n * sizeof(T));
  };
  const dim3 gred((unsigned)ls_cdiv(n, 64));
  const dim3 gv((unsigned)Gv);
  const dim3 gstep((unsigned)ls_cdiv(n, 64));
  // init: u = b - A x0, beta_1, t = A^T u / beta_1, v = W^T t
  pass(1, 1);
  hipLaunchKernelGGL(k_lsqr_reduce<T>, gred, dim3(kThreads), 0, st, tpart, G, n, w.nupart, w.nbpart, w.st, 1, 1, t);
  hipLaunchKernelGGL(k_lsqr_vupdate<T>, gv, dim3(kThreads), 0, st, Wt, ldw, n, t, v, w.st, 1, 1, w.nvpart);
  int it = 1;
  int last_par_written = 0;
  LsqrRec rec{};
  bool done = false;
  for (; it <= maxit; ++it) {
    const int rd = it & 1, wr = rd ^ 1;
    hipLaunchKernelGGL(k_lsqr_step<T>, gstep, dim3(kThreads), 0, st, Wt, ldw, n, v, w.nvpart, Gv, w.st, rd, it, 0,
                       tol, maxit, p, what, x);
    last_par_written = wr;
    pass(wr, 0);
    hipLaunchKernelGGL(k_lsqr_reduce<T>, gred, dim3(kThreads), 0, st, tpart, G, n, w.nupart, w.nbpart, w.st, wr, 0, t);
    hipLaunchKernelGGL(k_lsqr_vupdate<T>, gv, dim3(kThreads), 0, st, Wt, ldw, n, t, v, w.st, wr, 0, w.nvpart);
    if (it % check == 0) {
      LS_HIP_TRY(hipMemcpyAsync(&rec, &w.st->rec[wr], sizeof(LsqrRec), hipMemcpyDeviceToHost, st));
      LS_HIP_TRY(hipStreamSynchronize(st));
      if (rec.done) {
        done = true;
        break;
      }
    }
  }
  if (!done) {
    const int rd = last_par_written;
    hipLaunchKernelGGL(k_lsqr_step<T>, gstep, dim3(kThreads), 0, st, Wt, ldw, n, v, w.nvpart, Gv, w.st, rd,
                       (it > maxit ? maxit + 1 : it + 1), 1, tol, maxit, p, what, x);
    last_par_written = rd ^ 1;
  }
  LsqrState S;
  LS_HIP_TRY(hipMemcpyAsync(&S, w.st, sizeof(LsqrState), hipMemcpyDeviceToHost, st));
  LS_HIP_TRY(hipStreamSynchronize(st));
  LS_HIP_TRY(hipGetLastError());
  rec = S.rec[last_par_written];
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
  const int rb = pick_rb(P->n, elt);
  return lsqr_carve(nullptr, P, elt, lsqr_grid(P, rb, ncu), (int)ls_cdiv(P->n, 4)).bytes;
}

int lsqr_device(const ls_problem_t* P, const double* W, const float* W32, int64_t ldw, ls_prec_t u, double* x,
                const ls_iter_opts_t* io, ls_stats_t* stats, char* ws, size_t ws_bytes, hipStream_t st) {
  if (u == LS_FP32) {
    if (!W32) return LS_E_ARG;
    if (P->store == LS_FP32) return lsqr_typed<float, float>(P, W32, P->n, x, io, stats, ws, ws_bytes, st);
    return lsqr_typed<double, float>(P, W32, P->n, x, io, stats, ws, ws_bytes, st);
  }
  if (u == LS_FP64) {
    if (P->store == LS_FP32) return lsqr_typed<float, double>(P, W, ldw, x, io, stats, ws, ws_bytes, st);
    return lsqr_typed<double, double>(P, W, ldw, x, io, stats, ws, ws_bytes, st);
  }
  return LS_E_UNSUPPORTED;
}

// ================================================================== refinement driver
namespace {
struct LsirWs {
  FgState* st;
  double* V;
  int64_t ldv;
  double* Z;
  double* H;
  double* cs;
  double* sn;
  double* g;
  double* hj;
  char* tpart;        // G x n (TP)
  double* hpart;      // (kmax+1) x G
  double* tbuf;       // n
  double* h1r;        // kmax + 1
  double* hxpart;     // (kmax+1) x Gc
  double* h2part;     // (kmax+1) x Gd
  double* w2part;     // max(G + Gh, Gd)
  double* rt_hi;      // G x n
  double* rt_lo;      // G x n
  double* gvec;       // n
  double* upart;      // 4 x Gd
  size_t bytes;
};

LsirWs lsir_carve(char* ws, const ls_problem_t* P, int kmax, int G, int Gc, int Gd, int Gh) {
  LsirWs w{};
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = ws ? ws + off : nullptr;
    off += ls_align256(b);
    return q;
  };
  const int64_t m = P->m, n = P->n;
  w.ldv = m + n;
  w.st = reinterpret_cast<FgState*>(take(sizeof(FgState)));
  w.V = reinterpret_cast<double*>(take(8 * (size_t)w.ldv * (kmax + 1)));
  w.Z = reinterpret_cast<double*>(take(8 * (size_t)n * kmax));
  w.H = reinterpret_cast<double*>(take(8 * (size_t)(kmax + 1) * kmax));
  w.cs = reinterpret_cast<double*>(take(8 * (size_t)kmax));
  w.sn = reinterpret_cast<double*>(take(8 * (size_t)kmax));
  w.g = reinterpret_cast<double*>(take(8 * (size_t)(kmax + 1)));
  w.hj = reinterpret_cast<double*>(take(8));
  w.tpart = take(8 * (size_t)G * n);
  w.hpart = reinterpret_cast<double*>(take(8 * (size_t)(kmax + 1) * G));
  w.tbuf = reinterpret_cast<double*>(take(8 * (size_t)n));
  w.h1r = reinterpret_cast<double*>(take(8 * (size_t)(kmax + 1)));
  w.hxpart = reinterpret_cast<double*>(take(8 * (size_t)(kmax + 1) * Gc));
  w.h2part = reinterpret_cast<double*>(take(8 * (size_t)(kmax + 1) * Gd));
  const int w2n = (G + Gh > Gd) ? G + Gh : Gd;
  w.w2part = reinterpret_cast<double*>(take(8 * (size_t)w2n));
  w.rt_hi = reinterpret_cast<double*>(take(8 * (size_t)G * n));
  w.rt_lo = reinterpret_cast<double*>(take(8 * (size_t)G * n));
  w.gvec = reinterpret_cast<double*>(take(8 * (size_t)n));
  w.upart = reinterpret_cast<double*>(take(8 * 4 * (size_t)Gd));
  w.bytes = off;
  return w;
}

struct LsirDims {
  int kmax, rbp, rbr, G, Gc, Gd, Gh;
};

LsirDims lsir_dims(const ls_problem_t* P, size_t tp_elt, int fgmres_maxit, int ncu) {
  LsirDims d{};
  d.kmax = fgmres_maxit;
  d.rbp = pick_rb(P->n, tp_elt);
  d.rbr = pick_rb(P->n, 8);
  int64_t G = 2 * (int64_t)ncu;
  const int64_t nrb = ls_cdiv(P->m, d.rbr < d.rbp ? d.rbr : d.rbp);
  if (G > nrb) G = nrb;
  if (G < 1) G = 1;
  d.G = (int)G;
  d.Gc = (int)ls_cdiv(P->n, 16);
  d.Gd = (int)ls_cdiv(P->m + P->n, 1024);
  d.Gh = (int)ls_cdiv(P->n, 4);
  return d;
}

template <typename TA, typename TP, typename TU, bool DD>
int lsir_typed(const ls_problem_t* P, const double* W, const TP* Wp, int64_t ldwp, double* x, double* r,
               int r_given, const ls_iter_opts_t* io, ls_stats_t* stats, char* ws, size_t ws_bytes,
               hipStream_t st, int fg_maxit) {
  const int64_t m = P->m, n = P->n;
  const int ncu = device_cu_count();
  const LsirDims d = lsir_dims(P, sizeof(TP), fg_maxit, ncu);
  if (d.kmax > 120) return LS_E_ARG;
  LsirWs w = lsir_carve(ws, P, d.kmax, d.G, d.Gc, d.Gd, d.Gh);
  if (w.bytes > ws_bytes) return LS_E_WORKSPACE;
  FgPtrs F{w.V, w.ldv, w.Z, w.H, w.cs, w.sn, w.g, w.hj, w.st};
  const TA* A = static_cast<const TA*>(P->A);
  const TA* b = static_cast<const TA*>(P->b);
  const int vec_ok = vec_aligned(A, P->lda, sizeof(TA)) ? 1 : 0;
  TP* tpart = reinterpret_cast<TP*>(w.tpart);
  const int check = io->check_every > 0 ? io->check_every : 8;
  const double tol = io->fgmres_tol;
  const double lsir_tol = io->lsir_tol;
  const int nrb_norm = (int)ls_cdiv(m, 1024);
  const int nwb = (int)ls_cdiv(n, 64);
  const size_t lds_r = ((size_t)n * (d.rbr + 1) + 3 * (size_t)n + d.rbr + 2 * kThreads + 8) * 8;
  const size_t lds_p =
      ((size_t)n * (d.rbp + 1) + 2 * (size_t)n + d.rbp + kThreads) * sizeof(TP) + ((size_t)d.rbp + d.kmax + 2) * 8 + 16;

  if (lds_r > device_lds_limit() || lds_p > device_lds_limit()) return LS_E_UNSUPPORTED;
  if (!r_given)
    hipLaunchKernelGGL((k_resid_u<TA, TU>), dim3((unsigned)ls_cdiv(m, kThreads)), dim3(kThreads), n * sizeof(TU), st, A,
                       P->lda, m, n, b, x, r);
  int total_fg = 0, its = 0, status = LS_NOT_CONVERGED;
  double dx_rel = 0.0, dr_rel = 0.0;
  std::vector<double> up(4 * (size_t)d.Gd);
  for (its = 1; its <= io->lsir_maxit; ++its) {
    // lines 5-6: f, g, h in u_r
    prof_begin(kProfResidPass, st);
    switch (d.rbr) {
      case 32:
        hipLaunchKernelGGL((k_lsir_resid<TA, DD, 32>), dim3(d.G), dim3(kThreads), lds_r, st, A, P->lda, m, n, vec_ok, b,
                           r, x, w.V, w.rt_hi, w.rt_lo, w.w2part);
        break;
      case 16:
        hipLaunchKernelGGL((k_lsir_resid<TA, DD, 16>), dim3(d.G), dim3(kThreads), lds_r, st, A, P->lda, m, n, vec_ok, b,
                           r, x, w.V, w.rt_hi, w.rt_lo, w.w2part);
        break;
      default:
        hipLaunchKernelGGL((k_lsir_resid<TA, DD, 8>), dim3(d.G), dim3(kThreads), lds_r, st, A, P->lda, m, n, vec_ok, b,
                           r, x, w.V, w.rt_hi, w.rt_lo, w.w2part);
        break;
    }
    // A and b once, r read, f written, x read, g written
    prof_end(kProfResidPass, st, (double)m * n * sizeof(TA) + (double)m * sizeof(TA) + 16.0 * m + 16.0 * n);
    hipLaunchKernelGGL(k_lsir_g<DD>, dim3((unsigned)ls_cdiv(n, 64)), dim3(kThreads), 0, st, w.rt_hi, w.rt_lo, d.G, n,
                       w.gvec);
    hipLaunchKernelGGL(k_lsir_h<DD>, dim3((unsigned)d.Gh), dim3(kThreads), 0, st, W, n, n, m, w.gvec, w.V,
                       w.w2part + d.G);
    hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(kThreads), 0, st, reinterpret_cast<char*>(w.st), sizeof(FgState));
    // line 7: FGMRES
    int j = 0;
    FgState S{};
    for (; j < d.kmax; ++j) {
      const int Gw = (j == 0) ? d.G + d.Gh : d.Gd;
      hipLaunchKernelGGL(k_fg_a<TP>, dim3((unsigned)(nrb_norm + nwb)), dim3(kThreads), 0, st, F, m, n, j, d.kmax, Wp,
                         ldwp, w.w2part, Gw, tol, 0, nrb_norm);
      prof_begin(kProfFgPass, st);
      switch (d.rbp) {
        case 32:
          hipLaunchKernelGGL((k_fg_pass<TA, TP, 32>), dim3(d.G), dim3(kThreads), lds_p, st, A, P->lda, m, n, vec_ok, F,
                             j, tpart, w.hpart);
          break;
        case 16:
          hipLaunchKernelGGL((k_fg_pass<TA, TP, 16>), dim3(d.G), dim3(kThreads), lds_p, st, A, P->lda, m, n, vec_ok, F,
                             j, tpart, w.hpart);
          break;
        default:
          hipLaunchKernelGGL((k_fg_pass<TA, TP, 8>), dim3(d.G), dim3(kThreads), lds_p, st, A, P->lda, m, n, vec_ok, F,
                             j, tpart, w.hpart);
          break;
      }
      // A once, v_j read, w written, z read, t written, V_r(:, 0:j) for the fused dots
      prof_end(kProfFgPass, st,
               (double)m * n * sizeof(TA) + 16.0 * m + 8.0 * n + (double)n * sizeof(TP) + 8.0 * (j + 1) * m);
      const int ncb = (int)ls_cdiv(n, 64);
      hipLaunchKernelGGL(k_fg_reduce<TP>, dim3((unsigned)(ncb + j + 1)), dim3(kThreads), 0, st, tpart, w.hpart, d.G, n,
                         j, ncb, w.tbuf, w.h1r, w.st);
      hipLaunchKernelGGL(k_fg_c<TP>, dim3((unsigned)d.Gc), dim3(1024), 0, st, Wp, ldwp, n, m, w.tbuf, F, j, w.hxpart);
      prof_begin(kProfCgs, st);
      hipLaunchKernelGGL(k_cgs, dim3((unsigned)d.Gd), dim3(kThreads), 0, st, F, m, n, j, d.kmax, w.h1r, w.hxpart, d.Gc,
                         w.h2part, d.Gd, 0, w.h2part, w.w2part);
      hipLaunchKernelGGL(k_cgs, dim3((unsigned)d.Gd), dim3(kThreads), 0, st, F, m, n, j, d.kmax, w.h1r, w.hxpart, d.Gc,
                         w.h2part, d.Gd, 1, w.h2part, w.w2part);
      // two sweeps over V(:, 0:j), each reading and writing w
      prof_end(kProfCgs, st, 2.0 * 8.0 * (j + 1) * (double)(m + n) + 4.0 * 8.0 * (double)(m + n));
      if ((j + 1) % check == 0) {
        LS_HIP_TRY(hipMemcpyAsync(&S, w.st, sizeof(FgState), hipMemcpyDeviceToHost, st));
        LS_HIP_TRY(hipStreamSynchronize(st));
        if (S.done) break;
      }
    }
    // final Givens step for the last column (no-op when already done)
    hipLaunchKernelGGL(k_fg_a<TP>, dim3((unsigned)(nrb_norm + nwb)), dim3(kThreads), 0, st, F, m, n,
                       (j < d.kmax ? j + 1 : d.kmax), d.kmax, Wp, ldwp, w.w2part, d.Gd, tol, 1, nrb_norm);
    hipLaunchKernelGGL(k_fg_update<TU>, dim3((unsigned)d.Gd), dim3(kThreads), 0, st, F, m, n, d.kmax, r, x, w.upart);
    LS_HIP_TRY(hipMemcpyAsync(&S, w.st, sizeof(FgState), hipMemcpyDeviceToHost, st));
    LS_HIP_TRY(hipMemcpyAsync(up.data(), w.upart, 8 * 4 * (size_t)d.Gd, hipMemcpyDeviceToHost, st));
    LS_HIP_TRY(hipStreamSynchronize(st));
    LS_HIP_TRY(hipGetLastError());
    if (S.breakdown == 2) return LS_E_NONFINITE;
    total_fg += S.k;
    double nd[4] = {0, 0, 0, 0};
    for (int g = 0; g < d.Gd; ++g)
      for (int q = 0; q < 4; ++q) nd[q] += up[4 * (size_t)g + q];
    dr_rel = sqrt(nd[0]) / (sqrt(nd[2]) > 0 ? sqrt(nd[2]) : 1.0);
    dx_rel = sqrt(nd[1]) / (sqrt(nd[3]) > 0 ? sqrt(nd[3]) : 1.0);
    if (!std::isfinite(dr_rel) || !std::isfinite(dx_rel)) return LS_E_NONFINITE;
    if (dx_rel <= lsir_tol && dr_rel <= lsir_tol) {
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
  }
  return status;
}
}  // namespace

size_t lsir_workspace(const ls_problem_t* P, const ls_precs_t* pr, int fgmres_maxit, int ncu) {
  const size_t tp = (pr->u_A == LS_FP64) ? 8 : 4;
  const LsirDims d = lsir_dims(P, tp, fgmres_maxit, ncu);
  return lsir_carve(nullptr, P, d.kmax, d.G, d.Gc, d.Gd, d.Gh).bytes;
}

int lsir_device(const ls_problem_t* P, const double* W, const float* W32, int64_t ldw, const ls_precs_t* pr,
                double* x, double* r, int r_given, const ls_iter_opts_t* io, ls_stats_t* stats, char* ws,
                size_t ws_bytes, hipStream_t st) {
  const ls_prec_t tp = pr->u_A;
  if (pr->u_L != tp || pr->u_R != tp) return LS_E_UNSUPPORTED;
  const bool dd = pr->u_r == LS_FP64X2;
  if (!dd && pr->u_r != LS_FP64) return LS_E_UNSUPPORTED;
  const bool u32 = pr->u == LS_FP32;
  if (!u32 && pr->u != LS_FP64) return LS_E_UNSUPPORTED;
  if (u32 == false && tp == LS_FP32) return LS_E_ARG;   // products not coarser than u
  const int kmax = io->fgmres_maxit;
#define LS_LSIR_CALL(TA, TP_, TU, DD_, WP, LDWP) \
  return lsir_typed<TA, TP_, TU, DD_>(P, W, WP, LDWP, x, r, r_given, io, stats, ws, ws_bytes, st, kmax)
  if (P->store == LS_FP32) {
    if (tp == LS_FP32) {
      if (!W32) return LS_E_ARG;
      if (dd) LS_LSIR_CALL(float, float, float, true, W32, P->n);
      LS_LSIR_CALL(float, float, float, false, W32, P->n);
    }
    if (u32) {
      if (dd) LS_LSIR_CALL(float, double, float, true, W, ldw);
      LS_LSIR_CALL(float, double, float, false, W, ldw);
    }
    if (dd) LS_LSIR_CALL(float, double, double, true, W, ldw);
    LS_LSIR_CALL(float, double, double, false, W, ldw);
  } else {
    if (tp == LS_FP32) {
      if (!W32) return LS_E_ARG;
      if (dd) LS_LSIR_CALL(double, float, float, true, W32, P->n);
      LS_LSIR_CALL(double, float, float, false, W32, P->n);
    }
    if (u32) {
      if (dd) LS_LSIR_CALL(double, double, float, true, W, ldw);
      LS_LSIR_CALL(double, double, float, false, W, ldw);
    }
    if (dd) LS_LSIR_CALL(double, double, double, true, W, ldw);
    LS_LSIR_CALL(double, double, double, false, W, ldw);
  }
#undef LS_LSIR_CALL
}

}  // namespace ls
