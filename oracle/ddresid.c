/*
 * Augmented-system residuals in double-double arithmetic (oracle, test use
 * only; built on its own by oracle/build_dd.py, linked with nothing else).
 *
 * For the least-squares problem min ||b - A x|| written as the augmented
 * system [I A; A^T 0] [r; x] = [b; 0] (Section 1; the refinement of
 * Algorithm 2 computes these residuals in its precision u_r), with A (m x n,
 * column major, binary64), b (binary64) and x, r given as unevaluated sums
 * x = xh + xl, r = rh + rl of binary64 numbers:
 *
 *     f = b - r - A x      (m entries)
 *     g =   - A^T r        (n entries)
 *
 * each returned as a double-double (hi, lo).  Every product a * y of two
 * binary64 numbers is split exactly into p + e with one fused multiply-add
 * (e = fma(a, y, -p)), and every sum uses Knuth's two-sum, so each entry is
 * accurate to about 2^-104 times the sum of the magnitudes of its terms.
 * The file must be compiled without floating-point contraction
 * (-ffp-contract=off): the error-free steps rely on each product and sum
 * being rounded exactly as written.
 */
#include <math.h>
#include <stdint.h>

typedef struct {
  double hi, lo;
} dd_t;

/* s + e = a + b exactly (Knuth). */
static inline dd_t two_sum(double a, double b) {
  const double s = a + b;
  const double bv = s - a;
  const double av = s - bv;
  dd_t r = {s, (a - av) + (b - bv)};
  return r;
}

/* acc + x, x a double. */
static inline dd_t dd_add_d(dd_t acc, double x) {
  const dd_t s = two_sum(acc.hi, x);
  return two_sum(s.hi, s.lo + acc.lo);
}

/* acc + a * y with the product split exactly by a fused multiply-add. */
static inline dd_t dd_add_prod(dd_t acc, double a, double y) {
  const double p = a * y;
  const double e = fma(a, y, -p);
  const dd_t s = two_sum(acc.hi, p);
  return two_sum(s.hi, s.lo + (acc.lo + e));
}

/* acc + a * (yh + yl): the low part's product is far below the result's last
 * bits of the high part and is added in plain binary64. */
static inline dd_t dd_add_prod_dd(dd_t acc, double a, double yh, double yl) {
  acc = dd_add_prod(acc, a, yh);
  acc.lo += a * yl;
  return two_sum(acc.hi, acc.lo);
}

void ls_oracle_dd_aug_residual(int64_t m, int64_t n, const double *A, int64_t lda, const double *b,
                               const double *xh, const double *xl, const double *rh, const double *rl,
                               double *fh, double *fl, double *gh, double *gl) {
  /* f: rows split over the threads; each thread walks the columns of A over
   * its rows (contiguous in column-major storage) with one accumulator per row. */
  const int64_t rb = 2048;
#pragma omp parallel for schedule(static)
  for (int64_t i0 = 0; i0 < m; i0 += rb) {
    const int64_t i1 = (i0 + rb < m) ? i0 + rb : m;
    dd_t acc[2048];
    for (int64_t i = i0; i < i1; ++i) {
      dd_t a = {b[i], 0.0};
      a = dd_add_d(a, -rh[i]);
      a = dd_add_d(a, -rl[i]);
      acc[i - i0] = a;
    }
    for (int64_t j = 0; j < n; ++j) {
      const double *col = A + j * lda;
      const double yh = -xh[j], yl = -xl[j];
      for (int64_t i = i0; i < i1; ++i) acc[i - i0] = dd_add_prod_dd(acc[i - i0], col[i], yh, yl);
    }
    for (int64_t i = i0; i < i1; ++i) {
      fh[i] = acc[i - i0].hi;
      fl[i] = acc[i - i0].lo;
    }
  }
  /* g: one column of A per iteration, a double-double dot product with r. */
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t j = 0; j < n; ++j) {
    const double *col = A + j * lda;
    dd_t a = {0.0, 0.0};
    for (int64_t i = 0; i < m; ++i) a = dd_add_prod_dd(a, -col[i], rh[i], rl[i]);
    gh[j] = a.hi;
    gl[j] = a.lo;
  }
}

/* x + y for double-double vectors given as hi/lo arrays (in place into x). */
void ls_oracle_dd_axpy1(int64_t k, double *xh, double *xl, const double *y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < k; ++i) {
    dd_t a = {xh[i], xl[i]};
    a = dd_add_d(a, y[i]);
    xh[i] = a.hi;
    xl[i] = a.lo;
  }
}
