// C ABI of libls: argument checking, workspace carving and the stage drivers.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace {

using namespace ls;

bool prec_is(ls_prec_t p, ls_prec_t a, ls_prec_t b) { return p == a || p == b; }

int check_problem(const ls_problem_t* P) {
  if (!P || !P->A || !P->b) return LS_E_ARG;
  if (P->n < 1 || P->m < P->n || P->lda < P->m) return LS_E_ARG;
  if (!prec_is(P->store, LS_FP32, LS_FP64)) return LS_E_ARG;
  if (P->n > 2048 || P->m > ((int64_t)1 << 31) - 4096) return LS_E_UNSUPPORTED;
  return LS_OK;
}

int64_t sketch_rows(const ls_problem_t* P, const ls_sketch_opts_t* so) {
  return (so && so->s > 0) ? so->s : 4 * P->n;
}

int check_sketch(const ls_problem_t* P, const ls_sketch_opts_t* so, ls_prec_t u_s) {
  if (!so) return LS_E_ARG;
  const int64_t s = sketch_rows(P, so);
  if (s < P->n + 1) return LS_E_ARG;
  if (s > 8192) return LS_E_UNSUPPORTED;
  if (so->zeta != 0) {   // sparse sign embedding: binary64 gather of the stored data
    if (u_s != LS_FP64 || so->terms > 1 || so->max_terms > 1) return LS_E_ARG;
    return sparse_check(P->m, so->zeta, s);
  }
  if (so->plan < 0 || (so->zeta == 0 && so->plan > sketch_plan_count(u_s))) return LS_E_ARG;
  if (u_s == LS_BF16 || u_s == LS_FP16 || u_s == LS_FP8E4M3) {
    if (so->terms < 1 || so->terms > kMaxSketchTerms) return LS_E_ARG;
    if (so->max_terms != 0 && (so->max_terms < so->terms || so->max_terms > kMaxSketchTerms)) return LS_E_ARG;
  } else if (u_s == LS_FP64) {
    if (so->terms > 1 || so->max_terms > 1) return LS_E_ARG;
  } else {
    return LS_E_UNSUPPORTED;
  }
  return LS_OK;
}

ls_iter_opts_t fill_opts(const ls_iter_opts_t* io, int64_t n, ls_prec_t u) {
  ls_iter_opts_t d;
  ls_default_iter_opts(n, u, &d);
  if (!io) return d;
  ls_iter_opts_t o = *io;
  if (o.lsqr_tol <= 0) o.lsqr_tol = d.lsqr_tol;
  if (o.lsqr_maxit <= 0) o.lsqr_maxit = d.lsqr_maxit;
  if (o.fgmres_tol <= 0) o.fgmres_tol = d.fgmres_tol;
  if (o.fgmres_maxit <= 0) o.fgmres_maxit = d.fgmres_maxit;
  if (o.lsir_maxit <= 0) o.lsir_maxit = d.lsir_maxit;
  if (o.lsir_tol <= 0) o.lsir_tol = d.lsir_tol;
  if (o.check_every <= 0) o.check_every = d.check_every;
  return o;
}

int check_precs(const ls_precs_t* pr) {
  if (!pr) return LS_E_ARG;
  if (!prec_is(pr->u, LS_FP32, LS_FP64)) return LS_E_UNSUPPORTED;
  if (!prec_is(pr->u_qr, LS_FP32, LS_FP64)) return LS_E_UNSUPPORTED;
  if (!prec_is(pr->u_r, LS_FP64, LS_FP64X2)) return LS_E_UNSUPPORTED;
  const ls_prec_t ps[3] = {pr->u_A, pr->u_L, pr->u_R};
  for (ls_prec_t p : ps) {
    if (!prec_is(p, LS_FP32, LS_FP64)) return LS_E_UNSUPPORTED;
    if (pr->u == LS_FP64 && p == LS_FP32) return LS_E_ARG;   // not coarser than u
  }
  if (pr->u_A != pr->u_L || pr->u_A != pr->u_R) return LS_E_UNSUPPORTED;
  return LS_OK;
}

}  // namespace

// Status of the flag word the QR and R^-1 kernels set (bit 1: a non-finite
// diagonal entry of R, bit 0: a zero one, or an overflow in R^-1).
int ls::qr_flag_status(int flag) {
  if (flag & 2) return LS_E_NONFINITE;
  if (flag & 1) return LS_E_SINGULAR;
  return LS_OK;
}

namespace {

// x = W c with W upper triangular n x n (ld n): x^s = R^-1 (Q^T Omega b).
__global__ __launch_bounds__(kUtThreads) void k_trmv_f64(const double* __restrict__ W, int64_t n,
                                                         const double* __restrict__ c, double* __restrict__ x) {
  __shared__ double red[32 * 33];
  const double v = ls_utmv_row(W, n, n, [&](int64_t j) { return c[j]; }, red);
  const int64_t row = (int64_t)blockIdx.x * 32 + threadIdx.x;
  if (threadIdx.x < 32 && row < n) x[row] = v;
}

struct Inv {
  double* W;
  float* W32;
  int* flag;
  double* fro;   // 2n: squared column norms of R^-1 and R
  size_t bytes;
};

Inv inv_carve(char* ws, int64_t n) {
  Inv v{};
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = ws ? ws + off : nullptr;
    off += ls_align256(b);
    return q;
  };
  v.W = reinterpret_cast<double*>(take(16 * (size_t)n * n));   // R^-1, then its transpose
  v.W32 = reinterpret_cast<float*>(take(4 * (size_t)n * n));
  v.flag = reinterpret_cast<int*>(take(256));
  v.fro = reinterpret_cast<double*>(take(16 * (size_t)n));
  v.bytes = off;
  return v;
}

size_t iter_bytes(const ls_problem_t* P, const ls_precs_t* pr, const ls_iter_opts_t* io) {
  const int ncu = device_cu_count();
  size_t a = lsqr_workspace(P, pr->u, ncu);
  ls_precs_t p64 = *pr;
  p64.u_A = p64.u_L = p64.u_R = LS_FP64;
  size_t b = lsir_workspace(P, pr, io->fgmres_maxit, ncu);
  size_t c = lsir_workspace(P, &p64, io->fgmres_maxit, ncu);
  size_t m = a > b ? a : b;
  return m > c ? m : c;
}

// Unit roundoff of the sketch: u^terms for a terms-part narrow sketch
// (u = 2^-8 bf16, 2^-11 fp16, 2^-4 e4m3), binary64 otherwise (the binary64
// Gaussian sketch and the sparse sign embedding).
double sketch_unit_roundoff(ls_prec_t u_s, int32_t terms) {
  double u;
  if (u_s == LS_BF16) u = 0x1p-8;
  else if (u_s == LS_FP16) u = 0x1p-11;
  else if (u_s == LS_FP8E4M3) u = 0x1p-4;
  else return 0x1p-53;
  return std::pow(u, (double)(terms < 1 ? 1 : terms));
}

// A second FGMRES operand besides LSQR's B is needed when FGMRES takes
// binary64 products while LSQR works in binary32 (u_A = FP64 with u = FP32,
// or the binary64 fallback): A's panel copy for the A-path.
bool second_b(const ls_precs_t* pr, const ls_iter_opts_t* io) {
  if (pr->u != LS_FP32) return false;
  return pr->u_A == LS_FP64 || io->fallback != 0;
}
ls_precs_t with_binary64_products(const ls_precs_t* pr) {
  ls_precs_t p = *pr;
  p.u_A = p.u_L = p.u_R = LS_FP64;
  return p;
}

// ls_solve's LSQR operand (ls_iter_opts_t.lsqr_operand): over A's panels (the
// refinement's A-path operand, shared) or over B = A R^-1.
int solve_lsqr_on_a(const ls_problem_t* P, const ls_precs_t* pr, const ls_iter_opts_t* io, bool* on_a) {
  switch (io->lsqr_operand) {
    case 0: *on_a = lsqr_on_a(P, pr); return LS_OK;   // A's panels where the refinement streams them
    case 1: *on_a = false; return LS_OK;
    case 2:
      if (!lsqr_on_a(P, pr)) return LS_E_UNSUPPORTED;
      *on_a = true;
      return LS_OK;
    default: return LS_E_ARG;
  }
}

// Make R^-1 available: W (binary64) and its binary32 copy.
int make_inverse(const double* R, int64_t ldr, int64_t n, const Inv& v, hipStream_t st) {
  LS_HIP_TRY(hipMemsetAsync(v.flag, 0, sizeof(int), st));
  LS_TRY(trinv_run(R, ldr, n, v.W, n, v.W32, v.flag, st));
  int flag = 0;
  LS_HIP_TRY(hipMemcpyAsync(&flag, v.flag, sizeof(int), hipMemcpyDeviceToHost, st));
  LS_HIP_TRY(hipStreamSynchronize(st));
  return qr_flag_status(flag);
}

struct Timer {
  hipEvent_t e[5];
  bool ok = false;
  Timer() {
    ok = true;
    for (auto& x : e)
      if (hipEventCreate(&x) != hipSuccess) ok = false;
  }
  ~Timer() {
    for (auto& x : e) (void)hipEventDestroy(x);
  }
  void mark(int i, hipStream_t st) {
    if (ok) (void)hipEventRecord(e[i], st);
  }
  double ms(int a, int b) {
    float t = 0.f;
    if (!ok || hipEventElapsedTime(&t, e[a], e[b]) != hipSuccess) return 0.0;
    return (double)t;
  }
};

}  // namespace

namespace {
// ------------------------------------------------------------------ batches
// Internal streams for the workers of a batch, created once per device at
// the default priority.
constexpr int kMaxWorkers = 16;
struct WorkerStreams {
  std::mutex mu;
  hipStream_t st[kMaxWorkers] = {};
  int made = 0;
};
WorkerStreams& worker_streams(int dev) {
  static WorkerStreams pools[64];
  return pools[(dev >= 0 && dev < 64) ? dev : 0];
}
int worker_stream(int dev, int k, hipStream_t* out) {
  WorkerStreams& w = worker_streams(dev);
  std::lock_guard<std::mutex> g(w.mu);
  while (w.made <= k) {
    LS_HIP_TRY(hipStreamCreateWithFlags(&w.st[w.made], hipStreamNonBlocking));
    ++w.made;
  }
  *out = w.st[k];
  return LS_OK;
}

int clamp_workers(int nworkers, int nprob) {
  int k = (nworkers > 0) ? nworkers : kMaxWorkers;   // the default: measured fastest on the 256-problem batch
  if (k > kMaxWorkers) k = kMaxWorkers;
  if (k > nprob) k = nprob;
  return k < 1 ? 1 : k;
}

int solve_impl(const ls_problem_t* P, const ls_sketch_opts_t* so, const ls_precs_t* pr, const ls_iter_opts_t* io_in,
               double* x, double* r, ls_stats_t* stats, void* ws, size_t ws_bytes, void* stream, const double* Y0);

// A batch whose sketches are all Gaussian in a narrow format computes them up
// front in grouped launches (one per tile width and part count); its
// workspace then also holds the work list, every problem's sketch Y and its
// sketch workspace after the workers' slices.
bool batch_grouped(int nprob, const ls_sketch_opts_t* so, ls_prec_t u_s) {
  for (int i = 0; i < nprob; ++i)
    if (!sketch_groupable(&so[i], u_s)) return false;
  return true;
}
struct BatchSketch {
  size_t items = 0;                 // offset of the work list from the region's start
  std::vector<size_t> y, w;         // offsets of Y_i and of sketch workspace i
  size_t bytes = 0;
};
BatchSketch batch_sketch_layout(int nprob, const ls_problem_t* P, const ls_sketch_opts_t* so, ls_prec_t u_s) {
  BatchSketch b;
  b.y.resize((size_t)nprob);
  b.w.resize((size_t)nprob);
  size_t off = sketch_grouped_items_bytes(nprob);
  for (int i = 0; i < nprob; ++i) {
    const int64_t s = sketch_rows(&P[i], &so[i]);
    b.y[i] = off;
    off += ls_align256(8 * (size_t)s * (size_t)(P[i].n + 1));
    b.w[i] = off;
    off += ls_align256(sketch_grouped_bytes(&P[i], &so[i], u_s, s));
  }
  b.bytes = off;
  return b;
}

// Largest single-problem workspace of the batch.
int batch_slice_bytes(int nprob, const ls_problem_t* P, const ls_sketch_opts_t* so, const ls_precs_t* pr,
                      const ls_iter_opts_t* io, size_t* out) {
  size_t mx = 0;
  for (int i = 0; i < nprob; ++i) {
    size_t b = 0;
    LS_TRY(ls_workspace_size(&P[i], &so[i], pr, io, &b));
    mx = std::max(mx, b);
  }
  *out = ls_align256(mx);
  return LS_OK;
}
}  // namespace

extern "C" {

void ls_default_iter_opts(int64_t n, ls_prec_t u, ls_iter_opts_t* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  const bool dbl = (u == LS_FP64);
  o->lsqr_tol = dbl ? 1e-12 : 1e-6;
  o->lsqr_maxit = (int32_t)(2 * n);
  o->fgmres_tol = dbl ? 1e-12 : 1e-6;
  o->fgmres_maxit = 50;
  o->lsir_maxit = 30;
  o->lsir_tol = 4.0 * (dbl ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24));
  o->fallback = 0;
  o->check_every = 3;
  o->profile = 0;
}

const char* ls_strerror(int s) {
  switch (s) {
    case LS_OK: return "success";
    case LS_NOT_CONVERGED: return "iteration limit reached before the stopping test held";
    case LS_E_ARG: return "invalid argument";
    case LS_E_WORKSPACE: return "workspace too small";
    case LS_E_HIP: return "HIP runtime error";
    case LS_E_SINGULAR: return "R has a zero or non-finite diagonal entry (rank-deficient sketch)";
    case LS_E_NONFINITE: return "non-finite value in an iterate";
    case LS_E_UNSUPPORTED: return "combination not supported by the library";
    default: return "unknown status";
  }
}

int ls_sketch_plan_info(ls_prec_t u_s, int32_t plan, int32_t* tile_cols, int32_t* quarter_cus) {
  if (!tile_cols || !quarter_cus) return LS_E_ARG;
  int bn = 0, q = 0;
  LS_TRY(sketch_plan_shape(u_s, plan, &bn, &q));
  *tile_cols = (u_s == LS_FP64) ? 128 : bn;
  *quarter_cus = q;
  return LS_OK;
}

int ls_sketch_split_rows(const ls_problem_t* P, const ls_sketch_opts_t* so, ls_prec_t u_s, int64_t* rows) {
  if (!rows) return LS_E_ARG;
  LS_TRY(check_problem(P));
  LS_TRY(check_sketch(P, so, u_s));
  const SketchPlan sp = sketch_plan(P, so, sketch_rows(P, so), u_s);
  *rows = (sp.zeta > 0) ? 0 : sp.kchunk;
  return LS_OK;
}

int ls_sketch_terms_for(double kappa_est, ls_prec_t u_s, int32_t terms, int32_t max_terms) {
  double u;
  if (u_s == LS_BF16) u = 0x1p-8;
  else if (u_s == LS_FP16) u = 0x1p-11;
  else if (u_s == LS_FP8E4M3) u = 0x1p-4;
  else return terms;
  if (terms < 1 || terms >= max_terms) return terms;
  const double us = std::pow(u, (double)terms);   // a terms-part representation
  return (kappa_est * us > 1.0 || !std::isfinite(kappa_est)) ? terms + 1 : terms;
}

int ls_workspace_size(const ls_problem_t* P, const ls_sketch_opts_t* so, const ls_precs_t* pr,
                      const ls_iter_opts_t* io_in, size_t* bytes) {
  if (!bytes) return LS_E_ARG;
  LS_TRY(check_problem(P));
  LS_TRY(check_precs(pr));
  LS_TRY(check_sketch(P, so, pr->u_s));
  const ls_iter_opts_t io = fill_opts(io_in, P->n, pr->u);
  const int64_t n = P->n, s = sketch_rows(P, so);
  const ls_precs_t p64 = with_binary64_products(pr);
  bool on_a = false;
  LS_TRY(solve_lsqr_on_a(P, pr, &io, &on_a));
  // the sketch with the most room over the parts the solve may use (each
  // count of parts may take its own tuned launch shape)
  size_t sk_bytes = 0;
  for (int t = so->terms; t <= std::max(so->terms, so->max_terms); ++t) {
    ls_sketch_opts_t so_t = *so;
    so_t.terms = t;
    const SketchPlan sp = sketch_plan(P, &so_t, s, pr->u_s);
    sk_bytes = std::max(sk_bytes, sp.operand_bytes + sp.partial_bytes + sp.exp_bytes);
  }
  size_t fixed = ls_align256(8 * (size_t)s * (n + 1))          // Y
                 + ls_align256(8 * (size_t)(n + 1) * (n + 1))    // R_aug
                 + inv_carve(nullptr, n).bytes                   // R^-1
                 + ls_align256(8 * (size_t)(P->m + n))           // saved x0 for the fallback
                 + (on_a ? 0 : b_bytes(P, pr->u))                // B = A R^-1 for LSQR
                 + (second_b(pr, &io) ? fg_operand_bytes(P, &p64) : 0);   // A's panels for binary64 FGMRES
  size_t scratch = sk_bytes;
  const size_t q = qr_workspace(s, n + 1, pr->u_qr);
  if (q > scratch) scratch = q;
  const size_t it = iter_bytes(P, pr, &io);
  if (it > scratch) scratch = it;
  *bytes = fixed + scratch;
  return LS_OK;
}

int ls_sketch(const ls_problem_t* P, const ls_sketch_opts_t* so, ls_prec_t u_s, double* Y, int64_t ldy, void* ws,
              size_t ws_bytes, void* stream) {
  LS_TRY(check_problem(P));
  LS_TRY(check_sketch(P, so, u_s));
  const int64_t s = sketch_rows(P, so);
  if (!Y || ldy < s) return LS_E_ARG;
  const SketchPlan sp = sketch_plan(P, so, s, u_s);
  if (!ws || ws_bytes < sp.operand_bytes + sp.partial_bytes + sp.exp_bytes) return LS_E_WORKSPACE;
  prof_reset(false);
  return sketch_run(P, so, u_s, sp, s, Y, ldy, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
}

int ls_qr_r(int64_t s, int64_t ncols, ls_prec_t u_qr, double* Y, int64_t ldy, double* R, int64_t ldr, void* ws,
            size_t ws_bytes, void* stream) {
  if (!Y || !R || ncols < 1 || s < ncols || ldy < s || ldr < ncols) return LS_E_ARG;
  if (!prec_is(u_qr, LS_FP32, LS_FP64)) return LS_E_UNSUPPORTED;
  const size_t need = qr_workspace(s, ncols, u_qr) + 256;
  if (!ws || ws_bytes < need) return LS_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  int* flag = reinterpret_cast<int*>(w);
  LS_HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), st));
  LS_TRY(qr_run(s, ncols, u_qr, Y, ldy, R, ldr, w + 256, ws_bytes - 256, flag, ncols, st));
  int h = 0;
  LS_HIP_TRY(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  LS_HIP_TRY(hipStreamSynchronize(st));
  return qr_flag_status(h);
}

int ls_qr_workspace_size(int64_t s, int64_t ncols, ls_prec_t u_qr, size_t* bytes) {
  if (!bytes || ncols < 1 || s < ncols) return LS_E_ARG;
  if (!prec_is(u_qr, LS_FP32, LS_FP64)) return LS_E_UNSUPPORTED;
  *bytes = qr_workspace(s, ncols, u_qr) + 256;
  return LS_OK;
}

int ls_lsqr_workspace_size(const ls_problem_t* P, ls_prec_t u, const ls_iter_opts_t* io_in, size_t* bytes) {
  if (!bytes) return LS_E_ARG;
  LS_TRY(check_problem(P));
  if (!prec_is(u, LS_FP32, LS_FP64)) return LS_E_UNSUPPORTED;
  const ls_iter_opts_t io = fill_opts(io_in, P->n, u);
  if (io.lsqr_operand < 0 || io.lsqr_operand > 2) return LS_E_ARG;
  if (io.lsqr_operand == 2 && P->store != u) return LS_E_UNSUPPORTED;   // A's panels need A stored in u
  // R^-1, then B or A's panels (the same size when A is stored in u), then LSQR's vectors
  *bytes = inv_carve(nullptr, P->n).bytes + b_bytes(P, u) + lsqr_workspace(P, u, device_cu_count());
  return LS_OK;
}

int ls_lsqr_precond(const ls_problem_t* P, const double* R, int64_t ldr, ls_prec_t u, double* x,
                    const ls_iter_opts_t* io_in, ls_stats_t* stats, void* ws, size_t ws_bytes, void* stream) {
  LS_TRY(check_problem(P));
  if (!R || !x || ldr < P->n) return LS_E_ARG;
  size_t need = 0;
  LS_TRY(ls_lsqr_workspace_size(P, u, io_in, &need));
  if (!ws || ws_bytes < need) return LS_E_WORKSPACE;
  const ls_iter_opts_t io = fill_opts(io_in, P->n, u);
  const bool on_a = (io.lsqr_operand == 2);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  const Inv inv = inv_carve(base, P->n);
  const size_t bb = b_bytes(P, u);
  LS_TRY(make_inverse(R, ldr, P->n, inv, st));
  void* Bm = base + inv.bytes;
  if (on_a) {
    LS_TRY(form_a_panels(P, Bm, st));
  } else {
    LS_TRY(form_b(P, inv.W, inv.W32, u, Bm, st));
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->err_x = stats->err_r = -1.0;
  }
  prof_reset(io.profile != 0);
  const int rc = lsqr_device(P, R, ldr, inv.W, Bm, on_a ? 1 : 0, u, x, &io, stats, base + inv.bytes + bb,
                             ws_bytes - inv.bytes - bb, st);
  if (stats) {
    stats->status = rc;
    if (io.profile && hipStreamSynchronize(st) == hipSuccess) prof_collect(stats);
  }
  prof_reset(false);
  return rc;
}

int ls_lsir_workspace_size(const ls_problem_t* P, const ls_precs_t* pr, const ls_iter_opts_t* io_in,
                           size_t* bytes) {
  if (!bytes) return LS_E_ARG;
  LS_TRY(check_problem(P));
  LS_TRY(check_precs(pr));
  const ls_iter_opts_t io = fill_opts(io_in, P->n, pr->u);
  if (io.fgmres_maxit > 95) return LS_E_ARG;
  // R^-1, the FGMRES operand, then the refinement's vectors
  *bytes = inv_carve(nullptr, P->n).bytes + fg_operand_bytes(P, pr) +
           lsir_workspace(P, pr, io.fgmres_maxit, device_cu_count());
  return LS_OK;
}

int ls_lsir_gmres(const ls_problem_t* P, const double* R, int64_t ldr, const ls_precs_t* pr, double* x, double* r,
                  int r_given, const ls_iter_opts_t* io_in, ls_stats_t* stats, void* ws, size_t ws_bytes,
                  void* stream) {
  LS_TRY(check_problem(P));
  if (!R || !x || !r || ldr < P->n) return LS_E_ARG;
  size_t need = 0;
  LS_TRY(ls_lsir_workspace_size(P, pr, io_in, &need));
  if (!ws || ws_bytes < need) return LS_E_WORKSPACE;
  const ls_iter_opts_t io = fill_opts(io_in, P->n, pr->u);
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  const Inv inv = inv_carve(base, P->n);
  const size_t bb = fg_operand_bytes(P, pr);
  LS_TRY(make_inverse(R, ldr, P->n, inv, st));
  void* Bm = base + inv.bytes;
  LS_TRY(form_fg_operand(P, inv.W, inv.W32, pr, Bm, st));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->err_x = stats->err_r = -1.0;
  }
  prof_reset(io.profile != 0);
  const int rc = lsir_device(P, inv.W, Bm, pr, x, r, r_given, &io, stats, base + inv.bytes + bb,
                             ws_bytes - inv.bytes - bb, st);
  if (stats) {
    stats->status = rc;
    if (io.profile && hipStreamSynchronize(st) == hipSuccess) prof_collect(stats);
  }
  prof_reset(false);
  return rc;
}

int ls_solve(const ls_problem_t* P, const ls_sketch_opts_t* so, const ls_precs_t* pr, const ls_iter_opts_t* io_in,
             double* x, double* r, ls_stats_t* stats, void* ws, size_t ws_bytes, void* stream) {
  return solve_impl(P, so, pr, io_in, x, r, stats, ws, ws_bytes, stream, nullptr);
}

}  // extern "C"

namespace {
// ls_solve, with the first sketch Y0 (s x (n+1), leading dimension s) given
// when the batch has computed it in a grouped launch (null: sketched here).
int solve_impl(const ls_problem_t* P, const ls_sketch_opts_t* so, const ls_precs_t* pr, const ls_iter_opts_t* io_in,
               double* x, double* r, ls_stats_t* stats, void* ws, size_t ws_bytes, void* stream, const double* Y0) {
  LS_TRY(check_problem(P));
  LS_TRY(check_precs(pr));
  LS_TRY(check_sketch(P, so, pr->u_s));
  if (!x || !r) return LS_E_ARG;
  size_t need = 0;
  LS_TRY(ls_workspace_size(P, so, pr, io_in, &need));
  if (!ws || ws_bytes < need) return LS_E_WORKSPACE;
  const ls_iter_opts_t io = fill_opts(io_in, P->n, pr->u);
  if (io.fgmres_maxit > 95) return LS_E_ARG;
  // the fallback raises the products to u^2: quad for u = binary64, not implemented
  if (io.fallback && pr->u == LS_FP64) return LS_E_UNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t m = P->m, n = P->n, s = sketch_rows(P, so);
  ls_stats_t local;
  ls_stats_t* S = stats ? stats : &local;
  std::memset(S, 0, sizeof(*S));
  S->err_x = S->err_r = -1.0;

  char* base = static_cast<char*>(ws);
  size_t off = 0;
  double* Y = reinterpret_cast<double*>(base + off);
  off += ls_align256(8 * (size_t)s * (n + 1));
  double* Raug = reinterpret_cast<double*>(base + off);
  off += ls_align256(8 * (size_t)(n + 1) * (n + 1));
  const Inv inv = inv_carve(base + off, n);
  off += inv.bytes;
  double* saved = reinterpret_cast<double*>(base + off);
  off += ls_align256(8 * (size_t)(m + n));
  bool on_a = false;
  LS_TRY(solve_lsqr_on_a(P, pr, &io, &on_a));
  void* B1 = base + off;                       // B in the working precision u (unless LSQR runs over A)
  off += on_a ? 0 : b_bytes(P, pr->u);
  const ls_precs_t p64 = with_binary64_products(pr);
  void* B2 = nullptr;                          // A's panels for binary64 FGMRES when needed
  if (second_b(pr, &io)) {
    B2 = base + off;
    off += fg_operand_bytes(P, &p64);
  }
  char* scratch = base + off;
  const size_t scratch_bytes = ws_bytes - off;

  prof_reset(io.profile != 0);
  Timer tm;
  ls_sketch_opts_t so_t = *so;   // the parts of the current sketch
  std::vector<double> fro(2 * (size_t)n);
  std::vector<char> rb((size_t)(reinterpret_cast<char*>(inv.fro) - reinterpret_cast<char*>(inv.flag)) +
                       16 * (size_t)n);
  double ms_sk = 0.0, ms_qr = 0.0;
  bool first = true;
  for (;;) {
    tm.mark(0, st);
    // Algorithm 1: the sketch (the first one given by a grouped batch launch)
    const SketchPlan sp = sketch_plan(P, &so_t, s, pr->u_s);
    const double* Yc = Y;
    if (first && Y0) Yc = Y0;
    else LS_TRY(sketch_run(P, &so_t, pr->u_s, sp, s, Y, s, scratch, st));
    first = false;
    tm.mark(1, st);
    // Algorithm 1: the QR, then x^s = R^-1 (Q^T Omega b)
    LS_HIP_TRY(hipMemsetAsync(inv.flag, 0, sizeof(int), st));
    LS_TRY(qr_run(s, n + 1, pr->u_qr, Yc, s, Raug, n + 1, scratch, scratch_bytes, inv.flag, n, st));
    LS_TRY(trinv_run(Raug, n + 1, n, inv.W, n, inv.W32, inv.flag, st, inv.fro));
    hipLaunchKernelGGL(k_trmv_f64, dim3((unsigned)ls_cdiv(n, 32)), dim3(kUtThreads), 0, st, inv.W, n,
                       Raug + n * (n + 1), x);
    // the flag and the norms in one copy (they are adjacent in the workspace)
    const size_t fro_off = (size_t)(reinterpret_cast<char*>(inv.fro) - reinterpret_cast<char*>(inv.flag));
    LS_HIP_TRY(hipMemcpyAsync(rb.data(), inv.flag, rb.size(), hipMemcpyDeviceToHost, st));
    tm.mark(2, st);
    LS_HIP_TRY(hipStreamSynchronize(st));
    int flag = 0;
    std::memcpy(&flag, rb.data(), sizeof(int));
    std::memcpy(fro.data(), rb.data() + fro_off, 16 * (size_t)n);
    if (flag) {
      S->status = qr_flag_status(flag);
      return S->status;
    }
    double w2 = 0.0, r2 = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      w2 += fro[2 * (size_t)j];
      r2 += fro[2 * (size_t)j + 1];
    }
    S->kappa_est = std::sqrt(w2) * std::sqrt(r2) / std::sqrt((double)n);
    S->sketch_terms = so_t.terms;
    S->sketch_plan = sp.plan;
    ms_sk += tm.ms(0, 1);
    ms_qr += tm.ms(1, 2);
    const int next = ls_sketch_terms_for(S->kappa_est, pr->u_s, so_t.terms, so->max_terms);
    if (next == so_t.terms) break;
    so_t.terms = next;   // Section 4: kappa(A) u_s < 1 not met with this many parts
  }
  // Algorithm 2's LSQR solve on the preconditioned operator A R^-1: over
  // B = A R^-1 formed once, or over A's panels (the refinement's operand)
  // with R^-1 applied around each pass
  if (on_a) {
    LS_TRY(form_fg_operand(P, inv.W, inv.W32, pr, B2, st));
  } else {
    LS_TRY(form_b(P, inv.W, inv.W32, pr->u, B1, st));
  }
  int rc = lsqr_device(P, Raug, n + 1, inv.W, on_a ? B2 : B1, on_a ? 1 : 0, pr->u, x, &io, S, scratch,
                       scratch_bytes, st);
  tm.mark(3, st);
  if (rc < 0) {
    S->status = rc;
    return rc;
  }
  // Algorithm 2's refinement loop
  if (io.fallback) {
    LS_HIP_TRY(hipMemcpyAsync(saved, x, 8 * (size_t)n, hipMemcpyDeviceToDevice, st));
  }
  void* Bfg = B1;
  bool have_b2 = false;
  if (pr->u_A != pr->u) {   // u = binary32, u_A = binary64: the A-path
    if (!on_a) LS_TRY(form_fg_operand(P, inv.W, inv.W32, pr, B2, st));
    Bfg = B2;
    have_b2 = true;
  }
  rc = lsir_device(P, inv.W, Bfg, pr, x, r, 0, &io, S, scratch, scratch_bytes, st);
  if (rc == LS_NOT_CONVERGED && io.fallback && pr->u_A == LS_FP32) {
    // Section 5: when the refinement has not converged within its limit and
    // kappa(A) < 1/u_s (kappa_est standing for kappa(A)), raise u_A, u_L and u_R
    // to u^2 (binary64 for u = binary32; the FGMRES limit stays, as in Table 3)
    // and run the refinement loop again from the LSQR solution.
    if (S->kappa_est * sketch_unit_roundoff(pr->u_s, so_t.terms) < 1.0) {
      LS_HIP_TRY(hipMemcpyAsync(x, saved, 8 * (size_t)n, hipMemcpyDeviceToDevice, st));
      S->fallback_used = 1;
      if (!have_b2) LS_TRY(form_fg_operand(P, inv.W, inv.W32, &p64, B2, st));
      rc = lsir_device(P, inv.W, B2, &p64, x, r, 0, &io, S, scratch, scratch_bytes, st);
    } else {
      S->fallback_used = 2;   // declined: outside the condition of Section 4
    }
  }
  tm.mark(4, st);
  LS_HIP_TRY(hipStreamSynchronize(st));
  S->ms_sketch = ms_sk;
  S->ms_qr = ms_qr;
  S->ms_lsqr = tm.ms(2, 3);
  S->ms_lsir = tm.ms(3, 4);
  if (io.profile) prof_collect(S);
  prof_reset(false);
  S->status = rc;
  return rc;
}
}  // namespace

extern "C" {

int ls_omega(uint64_t seed, uint32_t prob_id, int64_t s, int64_t m, ls_prec_t fmt, double* S, int64_t lds,
             void* stream) {
  if (!S || s < 1 || m < 1 || lds < s || s > 65535) return LS_E_ARG;
  if (!(fmt == LS_FP64 || fmt == LS_BF16 || fmt == LS_FP16 || fmt == LS_FP8E4M3)) return LS_E_UNSUPPORTED;
  return omega_run(seed, prob_id, s, m, fmt, S, lds, static_cast<hipStream_t>(stream));
}

int ls_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1, int64_t count,
              uint32_t* out, void* stream) {
  if (!out || count < 0) return LS_E_ARG;
  if (count == 0) return LS_OK;
  return philox_run(c0, c1, c2, c3, k0, k1, count, out, static_cast<hipStream_t>(stream));
}

int ls_workspace_size_batched(int nprob, const ls_problem_t* P, const ls_sketch_opts_t* so, const ls_precs_t* pr,
                              const ls_iter_opts_t* io, int nworkers, size_t* bytes) {
  if (nprob < 1 || !P || !so || !pr || !bytes) return LS_E_ARG;
  size_t slice = 0;
  LS_TRY(batch_slice_bytes(nprob, P, so, pr, io, &slice));
  *bytes = slice * (size_t)clamp_workers(nworkers, nprob);
  if (batch_grouped(nprob, so, pr->u_s)) *bytes += batch_sketch_layout(nprob, P, so, pr->u_s).bytes;
  return LS_OK;
}

int ls_solve_batched(int nprob, const ls_problem_t* P, const ls_sketch_opts_t* so, const ls_precs_t* pr,
                     const ls_iter_opts_t* io_in, double* const* x, double* const* r, ls_stats_t* stats,
                     int nworkers, void* ws, size_t ws_bytes, void* stream) {
  if (nprob < 1 || !P || !so || !pr || !x || !r || !ws) return LS_E_ARG;
  for (int i = 0; i < nprob; ++i) {
    LS_TRY(check_problem(&P[i]));
    LS_TRY(check_sketch(&P[i], &so[i], pr->u_s));
    if (!x[i] || !r[i]) return LS_E_ARG;
  }
  LS_TRY(check_precs(pr));
  ls_iter_opts_t io;
  if (io_in) {
    io = *io_in;
  } else {
    std::memset(&io, 0, sizeof(io));
  }
  io.profile = 0;
  const int K = clamp_workers(nworkers, nprob);
  size_t slice = 0;
  LS_TRY(batch_slice_bytes(nprob, P, so, pr, io_in ? &io : nullptr, &slice));
  const bool grouped = batch_grouped(nprob, so, pr->u_s);
  BatchSketch bs;
  if (grouped) bs = batch_sketch_layout(nprob, P, so, pr->u_s);
  if (ws_bytes < slice * (size_t)K + bs.bytes) return LS_E_WORKSPACE;
  int dev = 0;
  LS_HIP_TRY(hipGetDevice(&dev));
  hipStream_t caller = static_cast<hipStream_t>(stream);
  hipStream_t wst[kMaxWorkers];
  for (int k = 0; k < K; ++k) LS_TRY(worker_stream(dev, k, &wst[k]));

  // work lists: largest problems first, each to the worker with the least work so far
  std::vector<int> order(nprob);
  for (int i = 0; i < nprob; ++i) order[i] = i;
  auto work = [&](int i) { return (double)P[i].m * (double)P[i].n * (double)(P[i].n + 8); };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
  std::vector<std::vector<int>> lists(K);
  std::vector<double> load(K, 0.0);
  for (int i : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    lists[k].push_back(i);
    load[k] += work(i);
  }

  // the workers start after the caller's earlier work (and the grouped
  // sketches, queued on the first worker's stream) and the caller's stream
  // continues after all of them
  hipEvent_t start;
  LS_HIP_TRY(hipEventCreateWithFlags(&start, hipEventDisableTiming));
  LS_HIP_TRY(hipEventRecord(start, caller));
  std::vector<const double*> Y0((size_t)nprob, nullptr);
  if (grouped) {
    char* region = static_cast<char*>(ws) + slice * (size_t)K;
    std::vector<double*> Yg((size_t)nprob);
    std::vector<char*> Wg((size_t)nprob);
    std::vector<int64_t> sg((size_t)nprob);
    for (int i = 0; i < nprob; ++i) {
      Yg[i] = reinterpret_cast<double*>(region + bs.y[i]);
      Wg[i] = region + bs.w[i];
      sg[i] = sketch_rows(&P[i], &so[i]);
      Y0[i] = Yg[i];
    }
    int rc_sk = (hipStreamWaitEvent(wst[0], start, 0) == hipSuccess) ? LS_OK : LS_E_HIP;
    if (rc_sk == LS_OK)
      rc_sk = sketch_grouped(nprob, P, so, pr->u_s, sg.data(), Yg.data(), Wg.data(), region + bs.items, wst[0]);
    if (rc_sk == LS_OK && hipEventRecord(start, wst[0]) != hipSuccess) rc_sk = LS_E_HIP;
    if (rc_sk != LS_OK) {
      (void)hipEventDestroy(start);
      return rc_sk;
    }
  }
  std::vector<int> status(nprob, LS_OK);
  std::vector<ls_stats_t> local(stats ? 0 : nprob);
  std::atomic<int> hip_err{0};
  std::vector<std::thread> th;
  for (int k = 0; k < K; ++k) {
    th.emplace_back([&, k]() {
      if (hipSetDevice(dev) != hipSuccess || hipStreamWaitEvent(wst[k], start, 0) != hipSuccess) {
        hip_err = 1;
        for (int i : lists[k]) status[i] = LS_E_HIP;
        return;
      }
      char* slice_ws = static_cast<char*>(ws) + slice * (size_t)k;
      for (int i : lists[k]) {
        ls_stats_t* S = stats ? &stats[i] : &local[i];
        status[i] = solve_impl(&P[i], &so[i], pr, io_in ? &io : nullptr, x[i], r[i], S, slice_ws, slice, wst[k],
                               Y0[i]);
      }
    });
  }
  for (auto& t : th) t.join();
  std::vector<hipEvent_t> done(K);
  int rc_ev = LS_OK;
  for (int k = 0; k < K; ++k) {
    if (hipEventCreateWithFlags(&done[k], hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(done[k], wst[k]) != hipSuccess || hipStreamWaitEvent(caller, done[k], 0) != hipSuccess)
      rc_ev = LS_E_HIP;
  }
  for (int k = 0; k < K; ++k) (void)hipEventDestroy(done[k]);
  (void)hipEventDestroy(start);
  if (hip_err || rc_ev != LS_OK) return LS_E_HIP;
  int rc = LS_OK;
  for (int i = 0; i < nprob; ++i) {
    if (status[i] < 0) return status[i];
    if (status[i] != LS_OK) rc = status[i];
  }
  return rc;
}

}  // extern "C"
