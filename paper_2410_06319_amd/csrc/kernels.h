// Internal interfaces between the host drivers and the kernel files of libls.
#pragma once

#include <hip/hip_ext.h>

#include "common.h"

namespace ls {

// ------------------------------------------------------------------ sketch
// Parts a narrow-format sketch may split [A b] into.
constexpr int kMaxSketchTerms = 5;

struct SketchPlan {
  int64_t ncols;          // n + 1
  int64_t s_pad;          // s rounded up to the rows of S per block
  int64_t n_pad;          // n + 1 rounded up to the column tile
  int64_t m_pad;          // rows of the packed operand (kchunk * nsplit)
  int64_t kchunk;         // rows of A per K-split
  int64_t nsplit;         // number of K-splits (partial sums combined in binary64)
  int nb;                 // binary64 path: 16-column MFMA blocks per wave
  int kstep;              // rows of A per MFMA step
  int terms;
  int64_t bn;             // narrow formats: columns per block
  int64_t ns, nn;         // narrow formats: row tiles of S (128 rows), column tiles
  int64_t nkb;            // narrow formats: K-blocks of 32 rows in the packed operand
  int64_t kb_per_split;   // narrow formats: K-blocks per split
  int ebytes;             // bytes per operand element
  size_t exp_bytes;       // column exponents (narrow formats)
  size_t operand_bytes;   // packed [A b]
  size_t partial_bytes;   // per-split partial sketches (followed by the exponents)
  int zeta;               // sparse sign embedding: nonzeros per column of Omega (0: Gaussian)
  int plan;               // launch shape taken (1-based; see sketch_plan_shape)
};

SketchPlan sketch_plan(const ls_problem_t* P, const ls_sketch_opts_t* so, int64_t s, ls_prec_t u_s);
int sketch_plan_count(ls_prec_t u_s);
int sketch_plan_shape(ls_prec_t u_s, int plan, int* bn, int* quarter_cus);
// Sparse sign embedding (Section 2): argument check, workspace, run.
int sparse_check(int64_t m, int zeta, int64_t s);
size_t sparse_workspace(int64_t m, int64_t n, int zeta, int64_t s, size_t ta_bytes);
int sparse_run(const ls_problem_t* P, const ls_sketch_opts_t* so, int64_t s, double* Y, int64_t ldy, char* ws,
               hipStream_t st);
// Whether the sketch scales the columns of [A b] by powers of two (Section 3.2).
bool sketch_colscale(ls_prec_t u_s, int32_t col_scale);
int sketch_run(const ls_problem_t* P, const ls_sketch_opts_t* so, ls_prec_t u_s, const SketchPlan& p,
               int64_t s, double* Y, int64_t ldy, char* ws, hipStream_t st);
// Grouped Gaussian sketches of a batch (narrow formats): problem i's Y[i]
// (s[i] x (n_i + 1), leading dimension s[i]) from its own sketch workspace
// ws[i] (sketch_grouped_bytes), one launch per tile width and part count over
// the problems' blocks, each result the one sketch_run gives; items_dev holds
// the work list (sketch_grouped_items_bytes).  Synchronises st once, before
// queueing the launches.
bool sketch_groupable(const ls_sketch_opts_t* so, ls_prec_t u_s);
size_t sketch_grouped_bytes(const ls_problem_t* P, const ls_sketch_opts_t* so, ls_prec_t u_s, int64_t s);
size_t sketch_grouped_items_bytes(int nprob);
int sketch_grouped(int nprob, const ls_problem_t* P, const ls_sketch_opts_t* so, ls_prec_t u_s, const int64_t* s,
                   double* const* Y, char* const* ws, void* items_dev, hipStream_t st);
int omega_run(uint64_t seed, uint32_t prob, int64_t s, int64_t m, ls_prec_t fmt, double* S, int64_t lds,
              hipStream_t st);
int philox_run(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1, int64_t count,
               uint32_t* out, hipStream_t st);

// ------------------------------------------------------------------ QR and R^-1
size_t qr_workspace(int64_t s, int64_t ncols, ls_prec_t u_qr);
// check_cols: leading diagonal entries of R tested for zero / non-finite values.
int qr_run(int64_t s, int64_t ncols, ls_prec_t u_qr, const double* Y, int64_t ldy, double* R, int64_t ldr,
           char* ws, size_t ws_bytes, int* d_flag, int64_t check_cols, hipStream_t st);
// LS_OK, LS_E_SINGULAR or LS_E_NONFINITE from the flag word of qr_run / trinv_run.
int qr_flag_status(int flag);
// W = R^-1 (n x n upper, binary64, ldw) and, if W32 != NULL, its binary32 copy (ld n).
// With fro != NULL: fro[2j] = ||W[:, j]||^2, fro[2j+1] = ||R[:, j]||^2 (2n doubles).
// W^T is written right after W (W + ldw n, ld n): W needs 2 ldw n entries.
int trinv_run(const double* R, int64_t ldr, int64_t n, double* W, int64_t ldw, float* W32, int* d_flag,
              hipStream_t st, double* fro = nullptr);

// ------------------------------------------------------------------ iterations
struct FgState {
  double beta;                 // ||s||
  double relres;
  int32_t k;                   // Arnoldi columns in the solution
  int32_t done;
  int32_t breakdown;
  int32_t pad;
  double tol;                  // the cycle's tolerance (set at its start)
};

// B = A W with W = R^-1 (binary64 n x n, ld n; W32 its binary32 copy), in precision tb.
int form_b(const ls_problem_t* P, const double* W, const float* W32, ls_prec_t tb, void* Bout, hipStream_t st);
size_t b_bytes(const ls_problem_t* P, ls_prec_t tb);

// W below is R^-1 (n x n binary64, ld n) followed by its transpose, as
// trinv_run writes it.
// LSQR on B = A R^-1 from x (in/out): R (ldr) maps x0 to z0 = R x0, W maps z back.
// Bm is B in the panel layout, or with apply_w A's panels in precision u
// (form_fg_operand's A-path copy), W then being applied around each pass.
int lsqr_device(const ls_problem_t* P, const double* R, int64_t ldr, const double* W, const void* Bm, int apply_w,
                ls_prec_t u, double* x, const ls_iter_opts_t* io, ls_stats_t* stats, char* ws, size_t ws_bytes,
                hipStream_t st);
// LSQR can run over A's panels (no B) when the refinement uses them and A is
// stored in the working precision (ls_iter_opts_t.lsqr_operand = 2).
bool lsqr_on_a(const ls_problem_t* P, const ls_precs_t* pr);
size_t lsqr_workspace(const ls_problem_t* P, ls_prec_t u, int ncu);

// The operand of the refinement's FGMRES pass.  B-path: B = A W in u_A.
// A-path (u = binary32 with u_A = binary64): A itself in its storage
// precision, in B's panel layout, with the products in binary64 and W = R^-1
// applied on either side (no binary64 copy of B).
bool fg_apath(const ls_precs_t* pr);
size_t fg_operand_bytes(const ls_problem_t* P, const ls_precs_t* pr);
int form_fg_operand(const ls_problem_t* P, const double* W, const float* W32, const ls_precs_t* pr, void* out,
                    hipStream_t st);
// A in its storage precision, in B's panel layout (b_bytes(P, P->store) bytes).
int form_a_panels(const ls_problem_t* P, void* out, hipStream_t st);

// Refinement with FGMRES on [I B; B^T 0]; Bm from form_fg_operand.
int lsir_device(const ls_problem_t* P, const double* W, const void* Bm, const ls_precs_t* pr, double* x, double* r,
                int r_given, const ls_iter_opts_t* io, ls_stats_t* stats, char* ws, size_t ws_bytes,
                hipStream_t st);
size_t lsir_workspace(const ls_problem_t* P, const ls_precs_t* pr, int fgmres_maxit, int ncu);

int device_cu_count();
int device_lds_bytes();   // LDS available to one block

}  // namespace ls

namespace ls {
// Optional per-kernel timing with HIP events (enabled per call through
// ls_iter_opts_t.profile).  The record is per host thread.
enum ProfClass { kProfSketch = 0, kProfLsqrPass = 1, kProfFgPass = 2, kProfResidPass = 3, kProfCgs = 4, kProfSparse = 5 };
constexpr int kProfClasses = 6;
void prof_reset(bool on);
void prof_begin(int cls, hipStream_t st);
void prof_end(int cls, hipStream_t st, double work);   // work: algorithmic flops or bytes
// Single-kernel classes: the event pair that the class's next launch carries
// (hipExtLaunchKernelGGL stamps it with the kernel's own start and end; both
// null when profiling is off), then prof_commit files that launch.
struct ProfEv {
  hipEvent_t a = nullptr, b = nullptr;
};
ProfEv prof_events(int cls);
void prof_commit(int cls, double work);
// Launches queued beyond convergence return at once: after a loop, keep only
// the first `keep` records of class cls filed since position `from`.
size_t prof_mark();
void prof_keep(int cls, size_t from, int keep);
void prof_collect(ls_stats_t* stats);   // after the stream has been synchronised
}  // namespace ls
