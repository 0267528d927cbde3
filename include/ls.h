/*
 * ls.h -- C ABI of libls: sketch-preconditioned least squares on one MI355X.
 *
 * Method: Carson and Dauzickaite, "Mixed precision sketching for
 * least-squares problems and its application in GMRES-based iterative
 * refinement".  Problem (Section 1, eq. LS_problem): min_x ||b - A x||_2 with
 * A dense, m x n, full rank, m >= n.  Algorithm 1 builds R from a sketch,
 * Algorithm 2 runs preconditioned LSQR and then refinement on the augmented
 * system [I A; A^T 0][r; x] = [b; 0] with split-preconditioned FGMRES.
 *
 * Conventions for every entry point:
 *  - Matrices are column major: element (i, j) of a matrix with leading
 *    dimension ld is at offset i + j * ld.
 *  - Pointers named as device pointers must be device memory of the current
 *    HIP device; the library never allocates or frees them.  Scratch space is
 *    the caller's workspace (size from ls_workspace_size), device memory,
 *    256-byte aligned.
 *  - `stream` is a hipStream_t (passed as void*); NULL is the default stream.
 *    All work is enqueued on it.  Entry points that iterate synchronise the
 *    stream at their convergence checks and before returning, so their
 *    outputs and statistics are valid on return.  ls_qr_r and
 *    ls_qr_r_noalloc also synchronise the stream before returning (they read
 *    back the flag that reports a zero or non-finite diagonal entry of R);
 *    ls_sketch, ls_omega and ls_philox do not synchronise.
 *  - Errors are returned as negative status codes; nothing aborts or throws
 *    across the ABI.  ls_strerror(code) gives a message.
 *  - Calls that share a workspace must not overlap in time.
 *  - What the library holds of its own, once per device until the process
 *    ends: one page of pinned, device-mapped host memory for progress
 *    reports (the iterating entry points), the quantile tables of the narrow
 *    sketch (device arrays filled at the first narrow sketch), the internal
 *    streams of the batched entry point and of graph capture (default
 *    priority), and the static scratch array of ls_qr_r_noalloc.
 */
#ifndef LS_H
#define LS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Floating-point formats (unit roundoffs in Section 5: 2^-53 double, 2^-24
 * single, 2^-11 half; bf16 2^-8, e4m3 2^-4).  LS_FP64X2 is a double-double
 * accumulation format used only for the refinement residual (u_r). */
typedef enum {
  LS_FP64 = 0,
  LS_FP32 = 1,
  LS_FP16 = 2,
  LS_BF16 = 3,
  LS_FP8E4M3 = 4,
  LS_FP64X2 = 5
} ls_prec_t;

enum {
  LS_OK = 0,
  LS_NOT_CONVERGED = 1,   /* outputs hold the last iterate (Section 5's "-" entries) */
  LS_E_ARG = -1,          /* bad size, pointer, leading dimension or precision choice */
  LS_E_WORKSPACE = -2,    /* workspace smaller than ls_workspace_size reports */
  LS_E_HIP = -3,          /* a HIP runtime call failed */
  LS_E_SINGULAR = -4,     /* zero diagonal entry in R (or R^-1 overflows): A is rank
                             deficient in u_s */
  LS_E_NONFINITE = -5,    /* NaN or Inf met: in the sketch of [A b] (a non-finite
                             diagonal entry of R, e.g. from NaN or Inf in A) or in
                             an iterate (e.g. from NaN or Inf in b) */
  LS_E_UNSUPPORTED = -6   /* combination the library does not implement */
};

/* One least-squares problem (Section 1).  A: device, m x n column major,
 * lda >= m.  b: device, length m.  Both stored in `store` (LS_FP32 or
 * LS_FP64); Section 5 stores A and b in the working precision. */
typedef struct {
  int64_t m, n;
  ls_prec_t store;
  const void *A;
  int64_t lda;
  const void *b;
} ls_problem_t;

/* Precisions of Algorithms 1 and 2 (Sections 3 and 4):
 *  u_s  sketch (Algorithm 1): LS_FP64, LS_BF16, LS_FP16 or LS_FP8E4M3
 *  u_qr QR of the sketch (Algorithm 1): LS_FP32 or LS_FP64
 *  u    working precision of LSQR, FGMRES and the stored x, r: LS_FP32 or LS_FP64
 *  u_r  refinement residuals and R^-T g (Algorithm 2): LS_FP64 or LS_FP64X2
 *  u_A, u_L, u_R  products with Atilde, M_L^-1, M_R^-1 inside FGMRES: LS_FP32 or LS_FP64,
 *       not coarser than u.  The Arnoldi process itself runs in binary64. */
typedef struct {
  ls_prec_t u_s, u_qr, u, u_r, u_A, u_L, u_R;
} ls_precs_t;

/* Sketch options (Section 2: Gaussian embedding, s = c n with small c;
 * Section 5 uses s = 4n).  Omega = S / sqrt(s); key (seed mod 2^32,
 * seed / 2^32).  u_s = LS_FP64: S[k, i] from the Philox4x32-10 block with
 * counter (i / 4, k, prob_id, 0) by Box-Muller on 23-bit uniforms.  Narrow
 * u_s: S[k, i] = the format's rounding (nearest, ties to even) of
 * Phi^-1((U + 1/2) / 2^16), U the 16-bit uniform in half i % 2 of word
 * (i % 8) / 2 of the block with counter (i / 8, k, prob_id, 2): a Gaussian
 * to 16-bit resolution, eight entries per block.
 * terms: A (and b) are represented in u_s as a sum of `terms` rounded parts
 * (1 = a plain cast; each further part adds the format's precision, so that
 * u_s = u^terms, on the same MFMA; e4m3's exponent range bounds its parts'
 * combined accuracy near 2^-17 of a column's largest entry). */
typedef struct {
  int64_t s;         /* sketch rows, s >= n + 1; 0 selects 4n */
  uint64_t seed;
  uint32_t prob_id;
  int32_t terms;     /* 1..5 for LS_BF16, LS_FP16, LS_FP8E4M3; 1 for LS_FP64 */
  int32_t col_scale; /* Section 3.2 column scaling by powers of two: 0 = on for
                        LS_FP16 and LS_FP8E4M3 (whose range is narrow), off
                        otherwise; 1 = on; -1 = off */
  int32_t zeta;      /* 0: the Gaussian embedding above.  2..32 with 4 zeta <= s:
                        the sparse sign embedding of Section 2 instead, column i
                        of Omega holding zeta entries +-1/sqrt(zeta) at distinct
                        rows; rows and signs from the Philox4x32-10 words with
                        counter (i, t, prob_id, 1), t = 0, 1, ...: word w
                        proposes row floor(w s / 2^32), negative when w is odd,
                        repeats of a row skipped.  Needs u_s = LS_FP64 and
                        terms = 1: [A b] is gathered as stored, in binary64 */
  int32_t max_terms; /* ls_solve (and the batch) only.  0: `terms` parts, fixed.
                        terms < max_terms <= 5 (LS_BF16, LS_FP16, LS_FP8E4M3):
                        Section 4's convergence condition asks for
                        kappa(A) u_s < 1.  Once R is formed, kappa_est (see
                        ls_stats_t) stands for kappa(A), and while kappa_est
                        u^terms > 1 (u the format's unit roundoff: 2^-8, 2^-11,
                        2^-4) and terms < max_terms, the sketch, R and R^-1 are
                        formed again with one more part (ls_sketch_terms_for) */
  int32_t plan;      /* launch shape of the sketch kernels: 0 = the library's
                        choice (a table tuned on the device by the package's
                        autotune module, for the shape, format and parts), k >= 1 =
                        candidate k of ls_sketch_plan_info.  Changes the
                        grouping of the binary32 partial sums, not the method */
  int32_t *col_exp;  /* optional output (device, n + 1 entries; NULL: not wanted):
                        the exponents e_j of the Section 3.2 column scaling the
                        sketch applied (0 where it scaled nothing).  Y itself is
                        always the sketch of the unscaled [A b], so R needs no
                        correction; the exponents say how far each column of
                        [A b] was shifted into the format's range */
} ls_sketch_opts_t;

/* Iteration control (Section 5): LSQR at most 2n iterations, tolerance 1e-6
 * (u single) or 1e-12 (u double); FGMRES at most 50 iterations with the same
 * tolerance; at most 30 refinement steps.  Zero fields select those defaults.
 * lsir_tol: refinement stops once ||dx|| <= lsir_tol ||x|| and
 * ||dr|| <= lsir_tol ||r|| (default 4u).
 * fallback != 0 (ls_solve and the batch only; Section 5): when the refinement
 * has not converged within lsir_maxit steps with u_A = u_L = u_R = binary32
 * and kappa(A) u_s < 1 -- kappa_est (ls_stats_t) standing for kappa(A), u_s
 * the sketch's unit roundoff (u^terms for a narrow format, 2^-53 for a
 * binary64 sketch) -- the refinement loop runs again from the LSQR solution
 * with u_A = u_L = u_R = u^2 = binary64 and the same FGMRES limit (Table 3).
 * With u = binary64 the fallback would need quad products: ls_solve returns
 * LS_E_UNSUPPORTED when it is requested. */
typedef struct {
  double lsqr_tol;
  int32_t lsqr_maxit;
  double fgmres_tol;
  int32_t fgmres_maxit;
  int32_t lsir_maxit;
  double lsir_tol;
  int32_t fallback;
  int32_t check_every;   /* LSQR / FGMRES iterations the host keeps queued ahead of
                            the last one the device has reached (default 3); the
                            device reports progress and convergence through a slot
                            of pinned host memory, which the library allocates once
                            per device (one page); without it the host synchronises
                            every check_every iterations */
  int32_t profile;       /* nonzero: time the main kernels with HIP events (see ls_stats_t) */
  int32_t inner_adapt;   /* 0: every refinement step runs FGMRES to fgmres_tol (Section 5).
                            1: from the second step on, to
                            min(1e-2, max(fgmres_tol, 0.1 lsir_tol / rho)), rho the larger
                            relative correction of x and r in the previous step: a step
                            whose correction is far below lsir_tol needs it only roughly */
  /* x_ref, r_ref: optional (both or neither): device, binary64, the solution x*
   * (length n) and residual r* = b - A x* (length m).  Given, the refinement
   * stops as in Section 5, once the forward errors ||x* - x|| / ||x*|| and
   * ||r* - r|| / ||r*|| are both at most lsir_tol, and ls_stats_t reports them
   * (err_x, err_r). */
  const double *x_ref;
  const double *r_ref;
  /* lsqr_operand: how LSQR applies the preconditioned operator A R^-1 (the
   * method is the same; the rounding differs).  1: B = A R^-1 is formed once in
   * u (an MFMA product) and each iteration streams B.  2: each iteration
   * streams A itself (stored in u) and applies R^-1 as the products W v and
   * W^T (A^T u), W = R^-1, in binary64 rounded to u, so that B is never formed
   * (m n^2 flops and one m x n operand saved); for ls_solve this needs the
   * refinement's A-path (u = binary32, u_A = binary64, A stored in binary32),
   * whose operand LSQR then shares.  0 (default): 2 where ls_solve runs that
   * A-path, else 1 (ls_lsqr_precond: 1).  (Measured on the m = 1e6, n = 1000,
   * e4m3 workload over six sketch seeds: 2 saves the 15 ms product and one
   * 4 GB operand and needed four refinement steps each time; 1 needed three
   * once and four five times, 248.6 ms against 243.2 ms on average.)
   * Unsupported combinations: LS_E_UNSUPPORTED. */
  int32_t lsqr_operand;
  /* graph: nonzero: the refinement's FGMRES iterations are captured, in chunks
   * of check_every iterations, into HIP graphs at the first refinement step of
   * a call and replayed at the later ones (the host still polls between
   * chunks and stops queueing once the device reports convergence); the
   * results are bitwise those of the launches one by one.  Ignored while
   * profile is set (per-kernel events are not captured).  0 (default): off. */
  int32_t graph;
} ls_iter_opts_t;

/* Results and timings of one call. */
typedef struct {
  int32_t status;
  int32_t lsqr_its;
  int32_t lsir_its;
  int32_t fgmres_its_total;
  int32_t fallback_used;  /* 0: no fallback run; 1: the refinement was rerun with
                             binary64 products; 2: not converged, but the fallback
                             was declined because kappa_est u_s >= 1 */
  double lsqr_normr;      /* LSQR estimate of ||b - A x0|| */
  double lsqr_normar;     /* LSQR estimate of ||(A R^-1)^T (b - A x0)|| */
  double lsqr_normB;      /* LSQR estimate of ||A R^-1||_F */
  double lsir_dx_rel;     /* last ||dx|| / ||x|| */
  double lsir_dr_rel;     /* last ||dr|| / ||r|| */
  double ms_sketch, ms_qr, ms_lsqr, ms_lsir;
  /* With profile != 0: summed device time and launch count of the main
   * kernels, by class: 0 sketch MFMA, 1 LSQR pass over A, 2 FGMRES pass
   * over A, 3 refinement residual pass over A, 4 Gram-Schmidt sweeps,
   * 5 sparse sign sketch gather. */
  double kernel_ms[6];
  int32_t kernel_launches[6];
  /* Algorithmic work of those launches: flops for class 0, bytes that the
   * operation must move to or from HBM for classes 1-5. */
  double kernel_work[6];
  int32_t sketch_terms;   /* parts of [A b] the sketch used (ls_solve) */
  int32_t sketch_plan;    /* launch shape the sketch took (ls_solve; see ls_sketch_plan_info) */
  double kappa_est;       /* ||R||_F ||R^-1||_F / sqrt(n) of the preconditioner
                             (ls_solve): kappa_2(R) / sqrt(n) <= kappa_est <=
                             sqrt(n) kappa_2(R), and kappa_2(R) is kappa(A) up to
                             the embedding's distortion (Section 2) */
  double err_x, err_r;    /* with x_ref and r_ref: the forward errors after the last
                             refinement step; -1 otherwise */
} ls_stats_t;

/* Fill the defaults described above for a problem with n columns and
 * working precision u. */
void ls_default_iter_opts(int64_t n, ls_prec_t u, ls_iter_opts_t *opts);

/* Bytes of workspace ls_solve needs for this problem and these options
 * (the individual entry points need no more than that).  Returns LS_OK or
 * LS_E_ARG. */
int ls_workspace_size(const ls_problem_t *P, const ls_sketch_opts_t *so,
                      const ls_precs_t *pr, const ls_iter_opts_t *io, size_t *bytes);

/* Algorithm 1's sketch, of [A b]: Y = Omega [A b], s x (n+1), binary64,
 * column major with leading dimension ldy >= s (device).  Column n is
 * Omega b, which Algorithm 2's sketch-and-solve start needs.  With u_s =
 * LS_BF16, LS_FP16 or LS_FP8E4M3 (OCP e4m3, largest value 448, saturating)
 * the entries of S are the format's table values above; the columns of
 * [A b] are optionally scaled by 2^e_j (e_j the
 * largest integer with max_i |[A b]_ij| 2^e_j <= the format's largest value,
 * Section 3.2) and represented as `terms` rounded parts (nearest, ties to
 * even); products run on MFMA with binary32 accumulation over chunks of rows
 * of A, the chunks are summed in binary64 and the scaling is undone, so Y is
 * the sketch of [A b] itself.  A may be stored in binary32 or binary64.
 * With u_s = LS_FP64 everything is binary64. */
int ls_sketch(const ls_problem_t *P, const ls_sketch_opts_t *so, ls_prec_t u_s,
              double *Y, int64_t ldy, void *ws, size_t ws_bytes, void *stream);

/* Algorithm 1's QR: economic Householder QR of Y (s x ncols, binary64,
 * device, left unchanged: the factorisation runs on a copy in the workspace)
 * in precision u_qr, returning only R: ncols x ncols
 * upper triangular with positive diagonal, binary64, leading dimension
 * ldr (device; the strictly lower part is set to zero).  With Y = Omega[A b]
 * and ncols = n + 1, R[0:n, 0:n] is the preconditioner and R[0:n, n] is
 * Q^T Omega b (Algorithm 2, sketch-and-solve start). */
int ls_qr_r(int64_t s, int64_t ncols, ls_prec_t u_qr, double *Y, int64_t ldy,
            double *R, int64_t ldr, void *ws, size_t ws_bytes, void *stream);

/* Bytes of workspace ls_qr_r needs for an s x ncols sketch in u_qr (the
 * working copy of Y in u_qr, the Householder scalars, two T factors and the
 * flag word).  Returns LS_OK, LS_E_ARG (bad sizes) or LS_E_UNSUPPORTED. */
int ls_qr_workspace_size(int64_t s, int64_t ncols, ls_prec_t u_qr, size_t *bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): ls_qr_r with the
 * same arguments and results, but no workspace argument.  Its scratch (the
 * working copy of Y, the Householder scalars and T factors, the flag word) is
 * a static device array of LS_NOALLOC_SCRATCH_BYTES that each GPU the library
 * runs on holds until the process ends; the call allocates nothing.  Shapes
 * whose scratch exceeds it (256 + the QR's workspace: about
 * s * ncols * (4 or 8) bytes) return LS_E_WORKSPACE without touching the
 * device.  All calls on one GPU share that GPU's array, and its contents are
 * the last call's: calls that overlap in time on one GPU (other streams or
 * host threads) race and must be serialised by the caller.  Synchronises the
 * stream before returning. */
#define LS_NOALLOC_SCRATCH_BYTES (64u << 20)
int ls_qr_r_noalloc(int64_t s, int64_t ncols, ls_prec_t u_qr, double *Y, int64_t ldy,
                    double *R, int64_t ldr, void *stream);

/* Algorithm 2's LSQR solve: LSQR on A R^-1 (right preconditioning, Paige and
 * Saunders' recurrences) in precision u, started from x (device, length n,
 * binary64 in and out; typically x^s = R^-1 Q^T Omega b).  R: device, n x n
 * upper triangular, binary64, leading dimension ldr.  Stops when
 * ||r|| <= tol ||b|| or ||B^T r|| <= tol ||B||_F,est ||r||, or after
 * lsqr_maxit iterations (then LS_NOT_CONVERGED).  stats may be NULL. */
int ls_lsqr_precond(const ls_problem_t *P, const double *R, int64_t ldr, ls_prec_t u,
                    double *x, const ls_iter_opts_t *io, ls_stats_t *stats,
                    void *ws, size_t ws_bytes, void *stream);

/* Workspace (bytes, device memory the caller owns) that ls_lsqr_precond needs
 * for P, u and io (NULL: defaults).  Host only. */
int ls_lsqr_workspace_size(const ls_problem_t *P, ls_prec_t u, const ls_iter_opts_t *io, size_t *bytes);

/* Algorithm 2's refinement loop on the augmented system with
 * split-preconditioned FGMRES (M_L^-1 = diag(I, R^-T), M_R^-1 = diag(I, R^-1)).
 * x: device, length n, binary64, in and out.  r: device, length m, binary64,
 * out (and in when r_given != 0; otherwise r = b - A x is formed first,
 * as Algorithm 2 starts the refinement).  stats may be NULL. */
int ls_lsir_gmres(const ls_problem_t *P, const double *R, int64_t ldr, const ls_precs_t *pr,
                  double *x, double *r, int r_given, const ls_iter_opts_t *io,
                  ls_stats_t *stats, void *ws, size_t ws_bytes, void *stream);

/* Workspace (bytes) that ls_lsir_gmres needs for P, pr and io (NULL: defaults).
 * Host only. */
int ls_lsir_workspace_size(const ls_problem_t *P, const ls_precs_t *pr, const ls_iter_opts_t *io,
                           size_t *bytes);

/* The whole method: sketch, R, x^s, LSQR, refinement.  x (n) and r (m):
 * device, binary64, out.  stats may be NULL. */
int ls_solve(const ls_problem_t *P, const ls_sketch_opts_t *so, const ls_precs_t *pr,
             const ls_iter_opts_t *io, double *x, double *r, ls_stats_t *stats,
             void *ws, size_t ws_bytes, void *stream);

/* A batch of independent problems (the same method for each; Section 5's
 * experiments are sets of such problems): P, so, x, r and stats are host
 * arrays of nprob entries (x[i], r[i] device pointers as in ls_solve), pr and
 * io apply to all problems (io may be NULL for the defaults; per-call
 * profiling is off).  When every problem's sketch is Gaussian in a narrow
 * format (bf16, fp16, e4m3), all of them are first computed in grouped
 * launches, one per tile width and part count over the problems' blocks (the
 * workspace then also holds every problem's sketch; the call synchronises
 * once, after `stream`'s earlier work, before queueing them).  The problems
 * are then sorted by size and distributed over nworkers (1..16, 0 = 16) host
 * threads, each with its own internal stream (default priority), progress
 * slot and slice of the workspace, so that several problems occupy the
 * device at once.  Work on `stream` before the
 * call precedes the batch and work queued on it afterwards follows it.  Each
 * problem's result is bitwise the one ls_solve gives on its own.  Returns the
 * first error of any problem, else LS_NOT_CONVERGED if any problem did not
 * converge, else LS_OK; stats[i].status holds each problem's status. */
int ls_workspace_size_batched(int nprob, const ls_problem_t *P, const ls_sketch_opts_t *so,
                              const ls_precs_t *pr, const ls_iter_opts_t *io, int nworkers,
                              size_t *bytes);
int ls_solve_batched(int nprob, const ls_problem_t *P, const ls_sketch_opts_t *so,
                     const ls_precs_t *pr, const ls_iter_opts_t *io, double *const *x,
                     double *const *r, ls_stats_t *stats, int nworkers, void *ws,
                     size_t ws_bytes, void *stream);

/* The sketch operator itself, for checks and small problems: S[k, i] for
 * k < s, i < m as defined under ls_sketch_opts_t, as the sketch in format fmt
 * (LS_FP64, LS_BF16, LS_FP16 or LS_FP8E4M3) uses it, unscaled
 * (Omega = S / sqrt(s)).  The first call for a narrow format on a device (here
 * or in a sketch) fills that device's quantile tables and synchronises.
 * S: device, binary64, s x m column major, lds >= s.  Does not synchronise. */
int ls_omega(uint64_t seed, uint32_t prob_id, int64_t s, int64_t m, ls_prec_t fmt,
             double *S, int64_t lds, void *stream);

/* Raw Philox4x32-10 blocks for counters (c0 + t, c1, c2, c3), t < count,
 * key (k0, k1): out (device, uint32, 4 * count words, block t at 4t).
 * Does not synchronise. */
int ls_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
              int64_t count, uint32_t *out, void *stream);

/* The number of parts ls_solve sketches with next, given the estimate
 * kappa_est of kappa(A) from an R formed with `terms` parts: terms + 1 when
 * u_s is LS_BF16, LS_FP16 or LS_FP8E4M3, terms < max_terms and
 * kappa_est u^terms > 1 (u = 2^-8, 2^-11, 2^-4: Section 4's condition
 * kappa(A) u_s < 1 with u_s = u^terms, the accuracy of a terms-part
 * representation); otherwise terms.  Host only. */
int ls_sketch_terms_for(double kappa_est, ls_prec_t u_s, int32_t terms, int32_t max_terms);

/* Launch shape candidate `plan` (1-based) of the sketch in format u_s:
 * columns of [A b] per block (0: the narrowest of 128, 256 and 512 that holds
 * n + 1; binary64 blocks hold 128) and the blocks the K-splits aim at, in
 * quarters of the device's compute units.  Returns LS_E_ARG past the last
 * candidate (the count is the first plan that fails).  Host only. */
int ls_sketch_plan_info(ls_prec_t u_s, int32_t plan, int32_t *tile_cols, int32_t *quarter_cus);

/* Rows of [A b] that each binary32 partial sum of the narrow-format sketch
 * covers (the K-split length, the same for every split but possibly the last)
 * for this problem, these options and u_s; the partial sums are then added in
 * binary64.  For the binary64 sketch the split of its binary64 sums; 0 for
 * the sparse sign embedding (an exact-order binary64 gather).  Lets a caller
 * bound the sketch's rounding error.  Host only; returns LS_OK or an argument
 * error. */
int ls_sketch_split_rows(const ls_problem_t *P, const ls_sketch_opts_t *so, ls_prec_t u_s, int64_t *rows);

/* Static text for a status code. */
const char *ls_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* LS_H */
