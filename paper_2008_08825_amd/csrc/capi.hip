// C ABI entry points: argument checks, workspace plan and the sequence of
// phases of Alg. 3 (CHOL+SVD) on one stream.
//
//   form      M1 = A + B, M2 = A - B (lower triangles, padded to np = 64k)
//   chol      L1 L1^H = M1, L2 L2^H = M2            (Alg. 3 steps 1-2)
//   W         W = L2^H L1 = (L1^H L2)^H             (step 3's matrix, transposed)
//   jacobi    one-sided block Jacobi: W U = V Lambda (step 3)
//   finalize  Ws = W_out diag(column norms)^-3/2 = V Lambda^-1/2
//   back      V2 = L2 Ws = L2 V Lambda^-1/2          (step 5)
//             T = L1^H V2; lambda_k = ||T_k|| / ||Ws_k|| (Rayleigh quotient)
//             V1 = L1 T Lambda^-1 = M1 V2 Lambda^-1 = L1 U Lambda^-1/2
//                                                    (step 4 via Lemma SVDScalarFactors)
//   assemble  X = [(V1 + V2)/2; (V2 - V1)/2], ascending lambda (step 6)
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/bse.h"
#include "common.hpp"
#include "internal.hpp"

using namespace bse;

namespace {

constexpr int kErrHip = -1000;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int pad64(int n) { return ((n + 63) / 64) * 64; }

struct Plan {
  int n = 0, np = 0;
  size_t off_m1 = 0, off_m2 = 0, off_w = 0, off_y = 0;
  size_t off_linv = 0, off_sigma = 0, off_perm = 0, off_invlam = 0, off_status = 0;
  size_t off_bnorm = 0, off_anorm = 0, off_lamu = 0, off_scl = 0;
  size_t off_jac = 0;
  size_t total = 0;
};

bool opts_valid(const bse_opts_t& o) {
  if (o.route != BSE_ROUTE_SVD) return false;
  if (o.precision != BSE_PREC_FP64) return false;
  if (o.max_sweeps < 0 || o.refine_steps < 0 || !(o.jacobi_tol >= 0.0)) return false;
  if (!(o.uplo == 0 || o.uplo == 'L' || o.uplo == 'U' || o.uplo == 'l' || o.uplo == 'u')) return false;
  for (int i = 0; i < 6; ++i)
    if (o.reserved[i] != 0) return false;
  return true;
}

Plan make_plan(int n) {
  Plan p;
  p.n = n;
  p.np = pad64(n > 0 ? n : 1);
  const size_t mat = (size_t)p.np * p.np * sizeof(double2);
  size_t o = 0;
  p.off_m1 = o; o = align256(o + mat);
  p.off_m2 = o; o = align256(o + mat);
  p.off_w = o; o = align256(o + mat);
  p.off_y = o; o = align256(o + mat);
  p.off_linv = o; o = align256(o + 64 * 64 * sizeof(double2));
  p.off_sigma = o; o = align256(o + (size_t)p.np * sizeof(double));
  p.off_perm = o; o = align256(o + (size_t)p.np * sizeof(int));
  p.off_invlam = o; o = align256(o + (size_t)p.np * sizeof(double));
  p.off_bnorm = o; o = align256(o + (size_t)p.np * sizeof(double));
  p.off_anorm = o; o = align256(o + (size_t)p.np * sizeof(double));
  p.off_lamu = o; o = align256(o + (size_t)p.np * sizeof(double));
  p.off_scl = o; o = align256(o + (size_t)p.np * sizeof(double));
  p.off_status = o; o = align256(o + 64);
  p.off_jac = o; o = align256(o + jacobi_work_bytes(p.np, sizeof(double)));
  p.total = o + 256;  // slack for aligning the caller's base pointer
  return p;
}

inline int hip_status(hipError_t e) { return kErrHip - (int)e; }

#define BSE_TRY(expr)                          \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return hip_status(e_); \
  } while (0)

struct Timer {
  bool on;
  hipStream_t s;
  hipEvent_t ev[9];
  int k = 0;
  Timer(bool enable, hipStream_t st) : on(enable), s(st) {
    if (on)
      for (int i = 0; i < 9; ++i) (void)hipEventCreate(&ev[i]);
  }
  void mark() {
    if (on && k < 9) (void)hipEventRecord(ev[k++], s);
  }
  void fill(bse_info_t* info) {
    if (!on || !info) return;
    (void)hipEventSynchronize(ev[k - 1]);
    for (int i = 0; i + 1 < k && i < 8; ++i) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
      info->ms_phase[i] = ms;
    }
    float tot = 0.f;
    (void)hipEventElapsedTime(&tot, ev[0], ev[k - 1]);
    info->ms_phase[7] = tot;
  }
  ~Timer() {
    if (on)
      for (int i = 0; i < 9; ++i) (void)hipEventDestroy(ev[i]);
  }
};

}  // namespace

extern "C" {

void bse_default_opts(bse_opts_t* opts) {
  if (!opts) return;
  memset(opts, 0, sizeof(*opts));
  opts->route = BSE_ROUTE_SVD;
  opts->precision = BSE_PREC_FP64;
  opts->uplo = 'L';
}

size_t bse_workspace_bytes(int n, const bse_opts_t* opts) {
  bse_opts_t o;
  bse_default_opts(&o);
  if (opts) o = *opts;
  if (n < 0 || n > 46000 || !opts_valid(o)) return 0;
  return make_plan(n).total;
}

int bse_solve_h1(int n, const void* A, int lda, const void* B, int ldb, double* lambda, void* X,
                 int ldx, void* work, size_t work_bytes, const bse_opts_t* opts, bse_info_t* info,
                 void* stream) {
  bse_opts_t o;
  bse_default_opts(&o);
  if (opts) o = *opts;
  const int want_timing = info ? info->timing : 0;
  if (info) {
    memset(info, 0, sizeof(*info));
    info->timing = want_timing;
  }
  if (n < 0 || n > 46000) return -1;
  if (n > 0 && !A) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (n > 0 && !B) return -4;
  if (ldb < (n > 1 ? n : 1)) return -5;
  if (n > 0 && !lambda) return -6;
  if (n > 0 && !X) return -7;
  if (ldx < (2 * n > 1 ? 2 * n : 1)) return -8;
  if (!opts_valid(o)) return -11;
  if (n == 0) return 0;
  const Plan p = make_plan(n);
  if (!work) return -9;
  if (work_bytes < p.total) return -10;

  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(work) + 255) & ~(uintptr_t)255);
  const int np = p.np;
  const long ld = np;
  double2* M1 = reinterpret_cast<double2*>(base + p.off_m1);
  double2* M2 = reinterpret_cast<double2*>(base + p.off_m2);
  double2* W = reinterpret_cast<double2*>(base + p.off_w);
  double2* Y = reinterpret_cast<double2*>(base + p.off_y);
  double2* linv = reinterpret_cast<double2*>(base + p.off_linv);
  double* sigma = reinterpret_cast<double*>(base + p.off_sigma);
  int* perm = reinterpret_cast<int*>(base + p.off_perm);
  double* invlam = reinterpret_cast<double*>(base + p.off_invlam);
  double* bnorm = reinterpret_cast<double*>(base + p.off_bnorm);
  double* anorm = reinterpret_cast<double*>(base + p.off_anorm);
  double* lamu = reinterpret_cast<double*>(base + p.off_lamu);
  double* scl = reinterpret_cast<double*>(base + p.off_scl);
  int* status = reinterpret_cast<int*>(base + p.off_status);
  JacobiWork jw;
  jacobi_carve(np, sizeof(double), base + p.off_jac, jw);

  const int upper = (o.uplo == 'U' || o.uplo == 'u');
  const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 30;
  const double tol = o.jacobi_tol > 0.0 ? o.jacobi_tol : (double)(n > 64 ? n : 64) * 2.220446049250313e-16;

  Timer tm(want_timing != 0, s);
  tm.mark();
  const int big = 0x7fffffff;
  BSE_TRY(hipMemcpyAsync(status, &big, sizeof(int), hipMemcpyHostToDevice, s));
  BSE_TRY(form_m12(n, np, static_cast<const double2*>(A), lda, static_cast<const double2*>(B), ldb,
                   upper, M1, M2, ld, s));
  tm.mark();
  BSE_TRY(cholesky_z(np, n, M1, ld, linv, status, 0, s));
  BSE_TRY(cholesky_z(np, n, M2, ld, linv, status, n, s));
  int st = 0;
  BSE_TRY(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
  BSE_TRY(hipStreamSynchronize(s));
  if (st != big) {
    if (info) { info->status = st; info->fail_index = st > n ? st - n : st; }
    return st;
  }
  tm.mark();
  {
    GemmDesc g;  // W = L2^H L1, zero outside the leading n x n block
    g.M = np; g.N = np; g.K = np;
    g.A = M2; g.lda = ld; g.opA = 1; g.triA = 1;
    g.B = M1; g.ldb = ld; g.opB = 0; g.triB = 1;
    g.C = W; g.ldc = ld; g.mask = n;
    BSE_TRY(gemm_z(g, s));
  }
  tm.mark();
  JacobiResult jr;
  BSE_TRY(jacobi_z(np, W, ld, jw, tol, max_sweeps, jr, s, want_timing >= 2));
  tm.mark();
  // Ws = W sigma^-3/2 in place; bnorm = ||Ws_k||
  BSE_TRY(scale_singular_cols_z(n, np, W, ld, sigma, bnorm, s));
  tm.mark();
  {
    // V2 = L2 Ws  (to Y)
    GemmDesc g;
    g.M = np; g.N = np; g.K = np;
    g.A = M2; g.lda = ld; g.opA = 0; g.triA = 1;
    g.B = W; g.ldb = ld; g.opB = 0;
    g.C = Y; g.ldc = ld;
    BSE_TRY(gemm_z(g, s));
    // T = L1^H V2  (to W)
    GemmDesc h;
    h.M = np; h.N = np; h.K = np;
    h.A = M1; h.lda = ld; h.opA = 1; h.triA = 1;
    h.B = Y; h.ldb = ld; h.opB = 0;
    h.C = W; h.ldc = ld;
    BSE_TRY(gemm_z(h, s));
    // Rayleigh-quotient eigenvalues, scales and the ascending order
    BSE_TRY(rq_lambda_z(n, np, W, ld, bnorm, anorm, lamu, invlam, scl, perm, lambda,
                        o.want_negative, s));
    // V1 = L1 T Lambda^-1  (to M2: L2 is no longer needed)
    GemmDesc v;
    v.M = np; v.N = np; v.K = np;
    v.A = M1; v.lda = ld; v.opA = 0; v.triA = 1;
    v.B = W; v.ldb = ld; v.opB = 0;
    v.C = M2; v.ldc = ld; v.colscale = invlam;
    BSE_TRY(gemm_z(v, s));
  }
  BSE_TRY(assemble_z(n, M2, Y, ld, perm, scl, static_cast<double2*>(X), ldx, o.want_negative, s));
  tm.mark();
  BSE_TRY(hipStreamSynchronize(s));
  int ret = jr.converged ? 0 : 2 * n + 1;
  if (info) {
    info->status = ret;
    info->sweeps = jr.sweeps;
    info->rotations = jr.rotations;
    info->max_off = jr.max_off;
    info->pair_checks = jr.pair_checks;
    for (int i = 0; i < 3; ++i) {
      info->kernel_ms[i] = jr.kernel_ms[i];
      info->kernel_launches[i] = jr.kernel_launches[i];
    }
    tm.fill(info);
  }
  return ret;
}

size_t bse_batched_workspace_bytes(int batch, const int* n, const bse_opts_t* opts) {
  if (batch < 0 || (batch > 0 && !n)) return 0;
  size_t mx = 0;
  for (int i = 0; i < batch; ++i) {
    const size_t b = bse_workspace_bytes(n[i], opts);
    if (n[i] < 0 || (n[i] > 0 && b == 0)) return 0;
    if (b > mx) mx = b;
  }
  return mx;
}

int bse_solve_batched(int batch, const int* n, const void* const* A, const int* lda,
                      const void* const* B, const int* ldb, double* const* lambda, void* const* X,
                      const int* ldx, void* work, size_t work_bytes, const bse_opts_t* opts,
                      bse_info_t* info, void* stream) {
  if (batch < 0) return -1;
  if (batch > 0 && !n) return -2;
  if (batch > 0 && (!A || !lda)) return -3;
  if (batch > 0 && (!B || !ldb)) return -5;
  if (batch > 0 && !lambda) return -7;
  if (batch > 0 && (!X || !ldx)) return -8;
  const size_t need = bse_batched_workspace_bytes(batch, n, opts);
  if (batch > 0 && need == 0) return -2;
  if (batch > 0 && !work) return -10;
  if (work_bytes < need) return -11;
  int first = 0;
  for (int i = 0; i < batch; ++i) {
    bse_info_t* inf = info ? &info[i] : nullptr;
    const int st = bse_solve_h1(n[i], A[i], lda[i], B[i], ldb[i], lambda[i], X[i], ldx[i], work,
                                work_bytes, opts, inf, stream);
    if (st <= kErrHip) return st;
    if (st != 0 && first == 0) first = st;
  }
  return first;
}

size_t bse_backward_workspace_bytes(int n) { return n >= 0 ? 256 : 0; }

int bse_backward(int n, const void* X, int ldx, const double* w, void* gA, int ldga, void* gB,
                 int ldgb, void* work, size_t work_bytes, void* stream) {
  if (n < 0) return -1;
  if (n > 0 && !X) return -2;
  if (ldx < (2 * n > 1 ? 2 * n : 1)) return -3;
  if (n > 0 && !w) return -4;
  if (n > 0 && !gA) return -5;
  if (ldga < (n > 1 ? n : 1)) return -6;
  if (n > 0 && !gB) return -7;
  if (ldgb < (n > 1 ? n : 1)) return -8;
  (void)work;
  (void)work_bytes;
  if (n == 0) return 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const double2* Xa = static_cast<const double2*>(X);
  const double2* Xb = Xa + n;
  // G_A = a diag(w) a^H + b diag(w) b^H ;  G_B = a diag(w) b^H + b diag(w) a^H
  const double2* lhs[2] = {Xa, Xb};
  const double2* rhsA[2] = {Xa, Xb};
  const double2* rhsB[2] = {Xb, Xa};
  for (int t = 0; t < 2; ++t) {
    GemmDesc g;
    g.M = n; g.N = n; g.K = n;
    g.A = lhs[t]; g.lda = ldx; g.opA = 0;
    g.B = rhsA[t]; g.ldb = ldx; g.opB = 1;
    g.kscale = w;
    g.C = gA; g.ldc = ldga;
    g.beta_re = t == 0 ? 0.0 : 1.0;
    BSE_TRY(gemm_z(g, s));
    GemmDesc h = g;
    h.B = rhsB[t];
    h.C = gB; h.ldc = ldgb;
    BSE_TRY(gemm_z(h, s));
  }
  BSE_TRY(hipStreamSynchronize(s));
  return 0;
}

const char* bse_status_string(int status, int n) {
  if (status == 0) return "success";
  if (status <= kErrHip) return "HIP runtime error";
  if (status < 0) return "invalid argument";
  if (status <= n) return "A + B is not positive definite";
  if (status <= 2 * n) return "A - B is not positive definite";
  if (status == 2 * n + 1) return "Jacobi iteration did not converge";
  if (status == 2 * n + 2) return "refinement did not reach its tolerance";
  return "unknown status";
}

}  // extern "C"
