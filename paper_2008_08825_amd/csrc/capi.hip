// C ABI entry points: argument checks, workspace plans and the sequence of
// phases on one stream.
//
// FP64 form, Alg. 3 (CHOL+SVD):
//   form      M1 = A + B, M2 = A - B (lower triangles, padded to np = 64k)
//   chol      L1 L1^H = M1, L2 L2^H = M2            (Alg. 3 steps 1-2)
//   W         W = L2^H L1 = (L1^H L2)^H             (step 3's matrix, transposed)
//   jacobi    one-sided block Jacobi: W U = V Lambda (step 3)
//   finalize  Ws = W_out diag(column norms)^-3/2 = V Lambda^-1/2
//   back      V2 = L2 Ws = L2 V Lambda^-1/2          (step 5)
//             T = L1^H V2; lambda_k = ||T_k|| / ||Ws_k|| (Rayleigh quotient)
//             V1 = L2^-H Ws sigma = L1 U Lambda^-1/2 (step 4: L1 U = L2^-H W_out,
//                                                    one block triangular solve)
//   assemble  X = [(V1 + V2)/2; (V2 - V1)/2], ascending lambda (step 6)
// Mixed form: the same steps with complex64 data on FP32 MFMA (Cholesky
// diagonal blocks factored in FP64), then (V1, V2) widened to FP64 and
// refined against the FP64 M1, M2 (refine.hip), eigenvalues from FP64
// Rayleigh quotients.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/bse.h"
#include "common.hpp"
#include "internal.hpp"
#include "plan.hpp"

using namespace bse;

namespace {

void fill_info(bse_info_t* info, int ret, const JacobiResult& jr) {
  if (!info) return;
  info->status = ret;
  info->sweeps = jr.sweeps;
  info->rotations = jr.rotations;
  info->max_off = jr.max_off;
  info->pair_checks = jr.pair_checks;
  info->cross_pair_checks = jr.cross_pair_checks;
  info->inner_rotations = jr.inner_rotations;
  for (int i = 0; i < 3; ++i) {
    info->kernel_ms[i] = jr.kernel_ms[i];
    info->kernel_launches[i] = jr.kernel_launches[i];
  }
}


// Shared front end: form M1, M2 (lower, FP64) into the plan's M1/M2 regions.
int form_and_check_args(int n, const void* A, int lda, const void* B, int ldb, int upper, char* base,
                        const Plan& p, hipStream_t s) {
  double2* M1 = reinterpret_cast<double2*>(base + p.off_m1);
  double2* M2 = reinterpret_cast<double2*>(base + p.off_m2);
  BSE_TRY(form_m12(n, p.np, static_cast<const double2*>(A), lda, static_cast<const double2*>(B), ldb,
                   upper, M1, M2, p.np, s));
  return 0;
}

int read_status(int* status, int n, bse_info_t* info, hipStream_t s) {
  const int big = 0x7fffffff;
  int st = 0;
  BSE_TRY(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
  BSE_TRY(hipStreamSynchronize(s));
  if (st != big) {
    if (info) {
      info->status = st;
      info->fail_index = st > n ? st - n : st;
    }
    return st;
  }
  return 0;
}

// Alg. 3 steps 4-6 from the orthogonalised columns Z = W_out (in Zb, FP64):
//   Zb <- Ws = Z sigma^-3/2, Y <- V2 = L2 Ws, T <- L1^H V2 (Rayleigh
//   quotients, sort), T <- V1 = L2^-H Ws (Zb is overwritten by the solve),
//   X <- final setup with V1 scaled by 1 / ||Ws_k||^2.
// L1 and L2 are read only.
int back_transform_z(int n, int np, const double2* L1, const double2* L2, double2* Zb, double2* Y,
                     double2* T, double2* inv, char* base, const Plan& p, double* lambda, void* X,
                     int ldx, int want_negative, int values_only, hipStream_t s) {
  const long ld = np;
  double* sigma = reinterpret_cast<double*>(base + p.off_sigma);
  int* perm = reinterpret_cast<int*>(base + p.off_perm);
  double* invlam = reinterpret_cast<double*>(base + p.off_invlam);
  double* bnorm = reinterpret_cast<double*>(base + p.off_bnorm);
  double* anorm = reinterpret_cast<double*>(base + p.off_anorm);
  double* lamu = reinterpret_cast<double*>(base + p.off_lamu);
  double* scl = reinterpret_cast<double*>(base + p.off_scl);
  BSE_TRY(scale_singular_cols_z(n, np, Zb, ld, sigma, bnorm, s));  // Ws = Z sigma^-3/2
  BSE_TRY(gemm_z(tri_gemm(np, ld, L2, 0, Zb, 0, 0, Y), s));       // V2 = L2 Ws
  BSE_TRY(gemm_z(tri_gemm(np, ld, L1, 1, Y, 0, 0, T), s));        // T = L1^H V2
  BSE_TRY(rq_lambda_z(n, np, T, ld, bnorm, anorm, lamu, invlam, scl, perm, lambda, want_negative, s));
  if (values_only) return 0;
  BSE_TRY(trsm_lh_z(np, L2, ld, Zb, T, inv, s));                    // V1 = L2^-H Ws (unscaled)
  BSE_TRY(assemble_z(n, T, Y, ld, perm, nullptr, static_cast<double2*>(X), ldx, want_negative, s,
                     scl));
  return 0;
}

int solve_fp64(int n, const void* A, int lda, const void* B, int ldb, double* lambda, void* X,
               int ldx, char* base, const Plan& p, const bse_opts_t& o, bse_info_t* info,
               int want_timing, hipStream_t s) {
  const int np = p.np;
  const long ld = np;
  double2* M1 = reinterpret_cast<double2*>(base + p.off_m1);
  double2* M2 = reinterpret_cast<double2*>(base + p.off_m2);
  double2* W = reinterpret_cast<double2*>(base + p.off_w);
  double2* Y = reinterpret_cast<double2*>(base + p.off_y);
  double2* T = reinterpret_cast<double2*>(base + p.off_t);
  double2* inv = reinterpret_cast<double2*>(base + p.off_inv);
  double2* linv = reinterpret_cast<double2*>(base + p.off_linv);
  int* status = reinterpret_cast<int*>(base + p.off_status);
  JacobiWork jw;
  jacobi_carve(np, sizeof(double), base + p.off_jac, jw, p.kc, p.rrows);
  const int upper = (o.uplo == 'U' || o.uplo == 'u');
  const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 30;
  const double tol = o.jacobi_tol > 0.0 ? o.jacobi_tol : default_tol64(n);

  Timer tm(want_timing != 0, s);
  const int slots[8] = {0, 1, 2, 3, 5, -1, -1, -1};
  tm.mark();
  const int big = 0x7fffffff;
  BSE_TRY(hipMemcpyAsync(status, &big, sizeof(int), hipMemcpyHostToDevice, s));
  if (int e = form_and_check_args(n, A, lda, B, ldb, upper, base, p, s)) return e;
  tm.mark();
  BSE_TRY(cholesky_pair_z(np, n, M1, M2, ld, linv, status, s, p.side));
  if (int st = read_status(status, n, info, s)) return st;
  tm.mark();
  {
    GemmDesc g = tri_gemm(np, ld, M2, 1, M1, 0, 1, W);  // W = L2^H L1
    g.mask = n;                                         // zero outside the leading n x n block
    BSE_TRY(gemm_z(g, s));
  }
  tm.mark();
  JacobiResult jr;
  BSE_TRY(jacobi_z(np, W, ld, jw, tol, max_sweeps, jr, s, kernel_time_stride(want_timing)));
  tm.mark();
  if (int e = back_transform_z(n, np, M1, M2, W, Y, T, inv, base, p, lambda, X, ldx,
                               o.want_negative, o.values_only, s))
    return e;
  tm.mark();
  BSE_TRY(hipStreamSynchronize(s));
  const int ret = jr.converged ? 0 : 2 * n + 1;
  fill_info(info, ret, jr);
  tm.fill(info, slots);
  return ret;
}

// Tamm-Dancoff approximation (B = 0; Sec. 4, Table 3): H1 = diag(A, -A), so
// the positive eigenpairs are A u = lambda u with eigenvectors [u; 0] (u^H u
// = 1 gives the Sigma-normalisation) and the negative ones [0; u] with
// -lambda (Lemma ComputeNegEvecs).  A is Hermitian positive definite (A + B
// and A - B are), so the one-sided Jacobi on A itself leaves columns z_k =
// lambda_k u_k: A J = U Lambda.  Eigenvalues are the Rayleigh quotients
// z^H A z / z^H z (second order in the vector error), vectors z / ||z||.
int solve_tda(int n, const void* A, int lda, double* lambda, void* X, int ldx, char* base,
              const Plan& p, const bse_opts_t& o, bse_info_t* info, int want_timing, hipStream_t s) {
  const int np = p.np;
  const long ld = np;
  double2* M1 = reinterpret_cast<double2*>(base + p.off_m1);
  double2* M2 = reinterpret_cast<double2*>(base + p.off_m2);
  double2* W = reinterpret_cast<double2*>(base + p.off_w);
  double2* Y = reinterpret_cast<double2*>(base + p.off_y);
  int* perm = reinterpret_cast<int*>(base + p.off_perm);
  double* lamu = reinterpret_cast<double*>(base + p.off_lamu);
  double* scl = reinterpret_cast<double*>(base + p.off_scl);
  JacobiWork jw;
  jacobi_carve(np, sizeof(double), base + p.off_jac, jw, p.kc, p.rrows);
  const int upper = (o.uplo == 'U' || o.uplo == 'u');
  const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 30;
  const double tol = o.jacobi_tol > 0.0 ? o.jacobi_tol : default_tol64(n);

  Timer tm(want_timing != 0, s);
  const int slots[8] = {0, 3, 5, -1, -1, -1, -1, -1};
  tm.mark();
  // M1 = A (full Hermitian, identity beyond n), W = copy; the padded columns
  // are unit vectors orthogonal to the rest, so the sweeps leave them alone
  BSE_TRY(form_m12(n, np, static_cast<const double2*>(A), lda, nullptr, 0, upper, M1, M2, ld, s));
  BSE_TRY(mirror_upper_z(np, M1, ld, s));
  BSE_TRY(hipMemcpyAsync(W, M1, (size_t)np * np * sizeof(double2), hipMemcpyDeviceToDevice, s));
  tm.mark();
  JacobiResult jr;
  BSE_TRY(jacobi_z(np, W, ld, jw, tol, max_sweeps, jr, s, kernel_time_stride(want_timing)));
  tm.mark();
  {
    GemmDesc g;  // Y = A Z
    g.M = n; g.N = n; g.K = n;
    g.A = M1; g.lda = ld; g.opA = 0;
    g.B = W; g.ldb = ld; g.opB = 0;
    g.C = Y; g.ldc = ld;
    BSE_TRY(gemm_z(g, s));
  }
  BSE_TRY(rq_pairs_z(n, ld, W, W, Y, Y, lamu, scl, s));  // z^H A z / z^H z, 1 / ||z||
  BSE_TRY(sort_lambda(n, lamu, perm, lambda, o.want_negative, s));
  // final setup with V1 = V2 = z / ||z||: X = [u; 0] (and [0; u])
  if (!o.values_only)
    BSE_TRY(assemble_z(n, W, W, ld, perm, scl, static_cast<double2*>(X), ldx, o.want_negative, s));
  tm.mark();
  BSE_TRY(hipStreamSynchronize(s));
  const int ret = jr.converged ? 0 : 2 * n + 1;
  fill_info(info, ret, jr);
  tm.fill(info, slots);
  return ret;
}

// Alg. 1 (SQRT, Sec. 3.1).  M1 = A + B and M2 = A - B in full; the one-sided
// Jacobi on the Hermitian positive definite M2 leaves columns z_k = d_k v_k
// (M2 = V_C D_C V_C^H, d the column norms), so the principal square root and
// its inverse are Hermitian products with the columns scaled along k:
//   S = Z diag(d^-3/2) Z^H = V_C D_C^1/2 V_C^H,   S^-1 = Z diag(d^-5/2) Z^H;
// M = S M1 S (two GEMMs), the one-sided Jacobi on M leaves y_k = d_k v_k with
// d = lambda^2, and V1 = S^-1 V_M Lambda^1/2 = S^-1 Y diag(d^-3/4),
// V2 = S V_M Lambda^-1/2 = S Y diag(d^-5/4).
int solve_sqrt(int n, const void* A, int lda, const void* B, int ldb, double* lambda, void* X,
               int ldx, char* base, const Plan& p, const bse_opts_t& o, bse_info_t* info,
               int want_timing, hipStream_t s) {
  const int np = p.np;
  const long ld = np;
  double2* M1 = reinterpret_cast<double2*>(base + p.off_m1);
  double2* M2 = reinterpret_cast<double2*>(base + p.off_m2);
  double2* Sb = reinterpret_cast<double2*>(base + p.off_w);
  double2* Si = reinterpret_cast<double2*>(base + p.off_y);
  double2* T = reinterpret_cast<double2*>(base + p.off_t);
  int* perm = reinterpret_cast<int*>(base + p.off_perm);
  double* dC = reinterpret_cast<double*>(base + p.off_sigma);
  double* dM = reinterpret_cast<double*>(base + p.off_bnorm);
  double* ks = reinterpret_cast<double*>(base + p.off_anorm);
  double* kis = reinterpret_cast<double*>(base + p.off_invlam);
  double* c1 = reinterpret_cast<double*>(base + p.off_scl);
  double* c2 = reinterpret_cast<double*>(base + p.off_ritz);
  double* lamu = reinterpret_cast<double*>(base + p.off_lamu);
  JacobiWork jw;
  jacobi_carve(np, sizeof(double), base + p.off_jac, jw, p.kc, p.rrows);
  const int upper = (o.uplo == 'U' || o.uplo == 'u');
  const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 30;
  const double tol = o.jacobi_tol > 0.0 ? o.jacobi_tol : default_tol64(n);
  auto full = [&](const double2* a, int opA, const double2* b, int opB, double2* c,
                  const double* kscale, const double* colscale) {
    GemmDesc g;
    g.M = np; g.N = np; g.K = np;
    g.A = a; g.lda = ld; g.opA = opA;
    g.B = b; g.ldb = ld; g.opB = opB;
    g.C = c; g.ldc = ld;
    g.kscale = kscale;
    g.colscale = colscale;
    return gemm_z(g, s);
  };

  Timer tm(want_timing != 0, s);
  const int slots[8] = {0, 3, 3, 5, -1, -1, -1, -1};
  tm.mark();
  BSE_TRY(form_m12(n, np, static_cast<const double2*>(A), lda, static_cast<const double2*>(B), ldb,
                   upper, M1, M2, ld, s));
  BSE_TRY(mirror_upper_z(np, M1, ld, s));
  BSE_TRY(mirror_upper_z(np, M2, ld, s));
  tm.mark();
  JacobiResult j1, j2;
  BSE_TRY(jacobi_z(np, M2, ld, jw, tol, max_sweeps, j1, s, kernel_time_stride(want_timing)));  // Z = V_C D_C
  BSE_TRY(colnorm_z(np, M2, ld, dC, s));
  BSE_TRY(sqrt_scales(n, np, dC, dC, ks, kis, c1, c2, lamu, s));  // ks, kis (c1, c2 redone below)
  BSE_TRY(full(M2, 0, M2, 1, Sb, ks, nullptr));   // S = Z diag(d^-3/2) Z^H
  BSE_TRY(full(M2, 0, M2, 1, Si, kis, nullptr));  // S^-1 = Z diag(d^-5/2) Z^H
  BSE_TRY(full(M1, 0, Sb, 0, T, nullptr, nullptr));  // T = M1 S
  BSE_TRY(full(Sb, 0, T, 0, M1, nullptr, nullptr));  // M = S M1 S
  tm.mark();
  BSE_TRY(jacobi_z(np, M1, ld, jw, tol, max_sweeps, j2, s, kernel_time_stride(want_timing)));  // Y = V_M D
  BSE_TRY(colnorm_z(np, M1, ld, dM, s));
  BSE_TRY(sqrt_scales(n, np, dC, dM, ks, kis, c1, c2, lamu, s));
  BSE_TRY(sort_lambda(n, lamu, perm, lambda, o.want_negative, s));
  tm.mark();
  if (!o.values_only) {
    BSE_TRY(full(Si, 0, M1, 0, M2, nullptr, c1));  // V1 = S^-1 Y d^-3/4
    BSE_TRY(full(Sb, 0, M1, 0, T, nullptr, c2));   // V2 = S Y d^-5/4
    BSE_TRY(assemble_z(n, M2, T, ld, perm, nullptr, static_cast<double2*>(X), ldx, o.want_negative, s));
  }
  tm.mark();
  BSE_TRY(hipStreamSynchronize(s));
  const int ret = j1.converged && j2.converged ? 0 : 2 * n + 1;
  JacobiResult both = j2;
  both.sweeps = j1.sweeps + j2.sweeps;
  both.rotations = j1.rotations + j2.rotations;
  both.pair_checks = j1.pair_checks + j2.pair_checks;
  both.cross_pair_checks = j1.cross_pair_checks + j2.cross_pair_checks;
  both.inner_rotations = j1.inner_rotations + j2.inner_rotations;
  for (int i = 0; i < 3; ++i) {
    both.kernel_ms[i] += j1.kernel_ms[i];
    both.kernel_launches[i] += j1.kernel_launches[i];
  }
  fill_info(info, ret, both);
  tm.fill(info, slots);
  return ret;
}

// Alg. 2 (CHOL): L L^H = A - B; M = L^H (A + B) L; M V_M = V_M D by the same
// one-sided Jacobi (M is Hermitian positive definite, so its columns after the
// iteration are q_k d_k); Lambda = D^1/2; V1 = L^-H V_M Lambda^1/2 (blocked
// triangular solve), V2 = L V_M Lambda^-1/2; X = [(V1 + V2)/2; (V2 - V1)/2].
int solve_alg2(int n, const void* A, int lda, const void* B, int ldb, double* lambda, void* X,
               int ldx, char* base, const Plan& p, const bse_opts_t& o, bse_info_t* info,
               int want_timing, hipStream_t s) {
  const int np = p.np;
  const long ld = np;
  double2* M1 = reinterpret_cast<double2*>(base + p.off_m1);
  double2* M2 = reinterpret_cast<double2*>(base + p.off_m2);
  double2* W = reinterpret_cast<double2*>(base + p.off_w);
  double2* Y = reinterpret_cast<double2*>(base + p.off_y);
  double2* Z = reinterpret_cast<double2*>(base + p.off_z);
  double2* inv = reinterpret_cast<double2*>(base + p.off_inv);
  double2* linv = reinterpret_cast<double2*>(base + p.off_linv);
  double* d = reinterpret_cast<double*>(base + p.off_sigma);
  int* perm = reinterpret_cast<int*>(base + p.off_perm);
  double* lamu = reinterpret_cast<double*>(base + p.off_lamu);
  double* fx = reinterpret_cast<double*>(base + p.off_anorm);
  double* fy = reinterpret_cast<double*>(base + p.off_bnorm);
  int* status = reinterpret_cast<int*>(base + p.off_status);
  JacobiWork jw;
  jacobi_carve(np, sizeof(double), base + p.off_jac, jw, p.kc, p.rrows);
  const int upper = (o.uplo == 'U' || o.uplo == 'u');
  const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 30;
  const double tol = o.jacobi_tol > 0.0 ? o.jacobi_tol : default_tol64(n);

  Timer tm(want_timing != 0, s);
  const int slots[8] = {0, 1, 2, 3, 4, 5, -1, -1};
  tm.mark();
  const int big = 0x7fffffff;
  BSE_TRY(hipMemcpyAsync(status, &big, sizeof(int), hipMemcpyHostToDevice, s));
  if (int e = form_and_check_args(n, A, lda, B, ldb, upper, base, p, s)) return e;
  // A + B is not factored by Alg. 2; a factorisation of a copy checks its definiteness.
  BSE_TRY(hipMemcpyAsync(Z, M1, (size_t)np * np * sizeof(double2), hipMemcpyDeviceToDevice, s));
  BSE_TRY(mirror_upper_z(np, M1, ld, s));
  tm.mark();
  BSE_TRY(cholesky_pair_z(np, n, Z, M2, ld, linv, status, s, p.side));
  if (int st = read_status(status, n, info, s)) return st;
  tm.mark();
  {
    GemmDesc t;  // T = (A + B) L
    t.M = np; t.N = np; t.K = np;
    t.A = M1; t.lda = ld; t.opA = 0;
    t.B = M2; t.ldb = ld; t.opB = 0; t.triB = 1;
    t.C = W; t.ldc = ld;
    BSE_TRY(gemm_z(t, s));
    GemmDesc m = tri_gemm(np, ld, M2, 1, W, 0, 0, Y);  // M = L^H T
    m.mask = n;
    BSE_TRY(gemm_z(m, s));
  }
  tm.mark();
  JacobiResult jr;
  BSE_TRY(jacobi_z(np, Y, ld, jw, tol, max_sweeps, jr, s, kernel_time_stride(want_timing)));
  tm.mark();
  BSE_TRY(colnorm_z(np, Y, ld, d, s));
  BSE_TRY(alg2_lambda_z(n, d, lamu, perm, lambda, o.want_negative, fx, fy, s));
  if (o.values_only) {
    tm.mark();
    BSE_TRY(hipStreamSynchronize(s));
    const int ret = jr.converged ? 0 : 2 * n + 1;
    fill_info(info, ret, jr);
    tm.fill(info, slots);
    return ret;
  }
  BSE_TRY(gather_scale_z(n, np, Y, ld, perm, fx, M1, s));  // V_M Lambda^1/2 (sorted)
  BSE_TRY(gather_scale_z(n, np, Y, ld, perm, fy, W, s));   // V_M Lambda^-1/2
  tm.mark();
  BSE_TRY(gemm_z(tri_gemm(np, ld, M2, 0, W, 0, 0, Y), s));  // V2 = L V_M Lambda^-1/2
  BSE_TRY(trsm_lh_z(np, M2, ld, M1, W, inv, s));            // V1 = L^-H V_M Lambda^1/2
  BSE_TRY(assemble_z(n, W, Y, ld, nullptr, nullptr, static_cast<double2*>(X), ldx, o.want_negative, s));
  tm.mark();
  BSE_TRY(hipStreamSynchronize(s));
  const int ret = jr.converged ? 0 : 2 * n + 1;
  fill_info(info, ret, jr);
  tm.fill(info, slots);
  return ret;
}

// The mixed form re-solves in FP64 when its complex64 stage cannot carry the
// problem (a complex64 Cholesky factor fails, or the FP64 refinement does not
// reach its tolerance from the complex64 pairs), as mixed-precision
// iterative-refinement solvers fall back to the working precision when the
// refinement does not converge.  The FP64 plan fits in the mixed plan's
// workspace (5 against 10 n x n buffers).
}  // namespace

namespace bse {
int solve_fp64_fallback(int n, const void* A, int lda, const void* B, int ldb, double* lambda,
                        void* X, int ldx, char* base, const Plan& p, const bse_opts_t& o,
                        bse_info_t* info, hipStream_t s) {
  bse_opts_t o64 = o;
  o64.precision = BSE_PREC_FP64;
  o64.jacobi_tol = 0.0;
  o64.max_sweeps = 0;
  Plan p64 = make_plan(n, o64);
  p64.side = p.side;
  if (p64.total > p.total) return 2 * n + 2;
  const int timing = info ? info->timing : 0;
  if (info) {
    memset(info, 0, sizeof(*info));
    info->timing = timing;
  }
  const int ret = solve_fp64(n, A, lda, B, ldb, lambda, X, ldx, base, p64, o64, info, timing, s);
  if (info) info->fallback = 2;
  return ret;
}
}  // namespace bse

namespace {

int solve_mixed(int n, const void* A, int lda, const void* B, int ldb, double* lambda, void* X,
                int ldx, char* base, const Plan& p, const bse_opts_t& o, bse_info_t* info,
                int want_timing, hipStream_t s) {
  const int np = p.np;
  const long ld = np;
  const size_t half = (size_t)np * np * sizeof(float2);
  double2* M1 = reinterpret_cast<double2*>(base + p.off_m1);
  double2* M2 = reinterpret_cast<double2*>(base + p.off_m2);
  double2* X1 = reinterpret_cast<double2*>(base + p.off_x1);
  double2* X2 = reinterpret_cast<double2*>(base + p.off_x2);
  float2* L1c = reinterpret_cast<float2*>(base + p.off_lc);
  float2* L2c = reinterpret_cast<float2*>(base + p.off_lc + half);
  float2* Wc = reinterpret_cast<float2*>(base + p.off_wc);
  float2* Yc = reinterpret_cast<float2*>(base + p.off_wc + half);
  float2* linv = reinterpret_cast<float2*>(base + p.off_linv);
  double* sigma = reinterpret_cast<double*>(base + p.off_sigma);
  int* perm = reinterpret_cast<int*>(base + p.off_perm);
  double* invlam = reinterpret_cast<double*>(base + p.off_invlam);
  double* bnorm = reinterpret_cast<double*>(base + p.off_bnorm);
  double* anorm = reinterpret_cast<double*>(base + p.off_anorm);
  double* lamu = reinterpret_cast<double*>(base + p.off_lamu);
  double* scl = reinterpret_cast<double*>(base + p.off_scl);
  int* status = reinterpret_cast<int*>(base + p.off_status);
  JacobiWork jw;
  jacobi_carve(np, sizeof(float), base + p.off_jac, jw, p.kc, p.rrows);
  RefineWork rw;
  rw.Q = reinterpret_cast<double2*>(base + p.off_q);
  rw.F = reinterpret_cast<double2*>(base + p.off_f);
  rw.P1 = reinterpret_cast<double2*>(base + p.off_p1);
  rw.P2 = reinterpret_cast<double2*>(base + p.off_p2);
  rw.Ex = reinterpret_cast<double2*>(base + p.off_lc);
  rw.Ey = reinterpret_cast<double2*>(base + p.off_wc);
  rw.ritz = reinterpret_cast<double*>(base + p.off_ritz);
  rw.maxcorr = reinterpret_cast<double*>(base + p.off_small);
  rw.Cb0 = reinterpret_cast<double2*>(base + p.off_cb0);
  rw.arena = base + p.off_arena;
  rw.arena_cap = refine_arena_bytes(np);
  rw.perm = perm;
  rw.windows = kWindowPasses;
  rw.low_update = 1;
  const int upper = (o.uplo == 'U' || o.uplo == 'u');
  const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : 20;
  const int steps = o.refine_steps > 0 ? o.refine_steps : 8;
  const double eps32 = 1.1920928955078125e-07;
  const double tol = o.jacobi_tol > 0.0 ? o.jacobi_tol : 4.0 * sqrt((double)(n > 64 ? n : 64)) * eps32;

  Timer tm(want_timing != 0, s);
  const int slots[8] = {0, 1, 2, 3, 4, 5, 6, -1};
  tm.mark();
  const int big = 0x7fffffff;
  BSE_TRY(hipMemcpyAsync(status, &big, sizeof(int), hipMemcpyHostToDevice, s));
  if (int e = form_and_check_args(n, A, lda, B, ldb, upper, base, p, s)) return e;
  BSE_TRY(lower_to_c64(np, M1, ld, L1c, s));
  BSE_TRY(lower_to_c64(np, M2, ld, L2c, s));
  tm.mark();
  BSE_TRY(cholesky_pair_c(np, n, L1c, L2c, ld, linv, status, s, p.side));
  {
    int st = 0;
    BSE_TRY(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
    BSE_TRY(hipStreamSynchronize(s));
    // A complex64 factor failed: kappa(A +- B) eps32 is near 1 (or the input
    // is not definite, which the FP64 factorisation then reports).
    if (st != big) return solve_fp64_fallback(n, A, lda, B, ldb, lambda, X, ldx, base, p, o, info, s);
  }
  tm.mark();
  {
    GemmDesc g = tri_gemm(np, ld, L2c, 1, L1c, 0, 1, Wc);  // W = L2^H L1 (complex64)
    g.mask = n;
    BSE_TRY(gemm_c(g, s));
  }
  tm.mark();
  JacobiResult jr;
  // the refinement's window Rayleigh-Ritz resolves what the last sweeps would
  // (neighbour mixing), so the complex64 iteration ends, like the polish's,
  // once a sweep rotates fewer than 1/32 of its pairs, with the same inner
  // stopping rule
  BSE_TRY(jacobi_c(np, Wc, ld, jw, tol, 1.0e-5, max_sweeps, jr, s, kernel_time_stride(want_timing), 1.0,
                   1.0 / 32));
  tm.mark();
  BSE_TRY(scale_singular_cols_c(n, np, Wc, ld, sigma, bnorm, s));
  tm.mark();
  // Alg. 3 steps 4-5 in complex64 as in the FP64 form: V2 = L2 Ws, T = L1^H V2
  // (Rayleigh quotients), V1 = L2^-H Ws / ||Ws||^2 by a block triangular solve
  // (backward stable: the x, y of each pair stay balanced to the complex64
  // rounding, which the refinement's coupling to the negative half needs)
  float2* Tc = reinterpret_cast<float2*>(base + p.off_q);
  float2* invc = reinterpret_cast<float2*>(base + p.off_f);
  BSE_TRY(gemm_c(tri_gemm(np, ld, L2c, 0, Wc, 0, 0, Yc), s));  // V2 = L2 Ws
  BSE_TRY(gemm_c(tri_gemm(np, ld, L1c, 1, Yc, 0, 0, Tc), s));  // T = L1^H V2
  BSE_TRY(colnorm_c(np, Tc, ld, anorm, s));
  BSE_TRY(lambda_from_norms(n, np, anorm, bnorm, lamu, invlam, scl, s, 1));
  BSE_TRY(trsm_lh_c(np, L2c, ld, Wc, L1c, invc, s));            // V1 = L2^-H Ws (L1 is done)
  BSE_TRY(c64_to_c128(np, L1c, ld, X1, ld, scl, s));  // x = V1 / ||Ws||^2 (FP64)
  BSE_TRY(c64_to_c128(np, Yc, ld, X2, ld, nullptr, s));  // y = V2
  tm.mark();
  // FP64 Cholesky factors of M1, M2 (in place; the strict upper parts stay
  // zero) for the refinement's products
  BSE_TRY(cholesky_pair_z(np, n, M1, M2, ld, reinterpret_cast<double2*>(linv), status, s, p.side));
  {
    int st = 0;
    BSE_TRY(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
    BSE_TRY(hipStreamSynchronize(s));
    if (st != big) return solve_fp64_fallback(n, A, lda, B, ldb, lambda, X, ldx, base, p, o, info, s);
  }
  double2* x = X1;
  double2* y = X2;
  double maxcorr = 0.0;
  int steps_done = 0;
  double hist[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int win_steps = 0;
  BSE_TRY(refine_z(n, ld, M1, M2, &x, &y, rw, steps, kRefineStop, lamu, scl, &maxcorr, &steps_done, s, hist,
                   &win_steps));
  BSE_TRY(sort_lambda(n, lamu, perm, lambda, o.want_negative, s));
  if (!o.values_only)
    BSE_TRY(assemble_z(n, x, y, ld, perm, scl, static_cast<double2*>(X), ldx, o.want_negative, s));
  tm.mark();
  BSE_TRY(hipStreamSynchronize(s));
  // the complex64 iteration may end early (stop fraction); the refinement decides
  int ret = jr.sweeps > 0 ? 0 : 2 * n + 1;
  // a last correction above 1e-4 leaves errors above 1e-8 in the vectors
  if (ret == 0 && !(maxcorr <= 1.0e-4)) ret = 2 * n + 2;
  if (ret != 0) return solve_fp64_fallback(n, A, lda, B, ldb, lambda, X, ldx, base, p, o, info, s);
  fill_info(info, ret, jr);
  if (info) {
    info->refine_delta = maxcorr;
    info->refine_steps_done = steps_done;
    info->refine_window_steps = win_steps;
    for (int i = 0; i < 8; ++i) info->refine_corr[i] = hist[i];
  }
  tm.fill(info, slots);
  return ret;
}

// Mixed form with an FP64 Jacobi polish (BSE_PREC_MIXED_POLISH).
//   1. M1, M2, their FP64 Cholesky factors and W = L2^H L1 in FP64.
//   2. One-sided Jacobi on a complex64 copy of W (FP32 MFMA) to the FP32
//      tolerance, or until a sweep rotates fewer than 1/32 of its pairs:
//      Z = W32 V32 with V32 the product of the applied rotations.
//   3. V' = W^-1 Z = L1^-1 (L2^-H Z) by two FP64 block triangular solves;
//      V' is unitary up to the complex64 rounding of the iteration.
//   4. Cholesky QR in FP64: V'^H V' = L_G L_G^H and V = V' L_G^-H is unitary
//      to FP64 rounding, so W V = Z L_G^-H has exactly the singular values
//      of W and nearly orthogonal columns.
//   5. FP64 Jacobi sweeps on W V, which start in the quadratically convergent
//      regime, until no pair exceeds the FP64 tolerance; then the FP64
//      form's finalisation (Rayleigh quotients, back-transform, assembly).
int solve_polish(int n, const void* A, int lda, const void* B, int ldb, double* lambda, void* X,
                 int ldx, char* base, const Plan& p, const bse_opts_t& o, bse_info_t* info,
                 int want_timing, hipStream_t s) {
  const int np = p.np;
  const long ld = np;
  double2* M1 = reinterpret_cast<double2*>(base + p.off_m1);
  double2* M2 = reinterpret_cast<double2*>(base + p.off_m2);
  double2* W = reinterpret_cast<double2*>(base + p.off_w);
  double2* Y = reinterpret_cast<double2*>(base + p.off_y);
  double2* X1 = reinterpret_cast<double2*>(base + p.off_x1);
  double2* X2 = reinterpret_cast<double2*>(base + p.off_x2);
  float2* Wc = reinterpret_cast<float2*>(base + p.off_x1);
  double2* inv = reinterpret_cast<double2*>(base + p.off_inv);
  double2* linv = reinterpret_cast<double2*>(base + p.off_linv);
  int* status = reinterpret_cast<int*>(base + p.off_status);
  JacobiWork jw32, jw64;
  jacobi_carve(np, sizeof(float), base + p.off_jac, jw32, p.kc, p.rrows);
  jacobi_carve(np, sizeof(double), base + p.off_jac, jw64, p.kc, p.rrows);
  const int upper = (o.uplo == 'U' || o.uplo == 'u');
  const double nn = (double)(n > 64 ? n : 64);
  const double eps32 = 1.1920928955078125e-07;
  const int max32 = o.max_sweeps > 0 ? o.max_sweeps : 20;
  const double tol32 = 4.0 * sqrt(nn) * eps32;
  const double tol64 = o.jacobi_tol > 0.0 ? o.jacobi_tol : default_tol64(n);

  Timer tm(want_timing != 0, s);
  const int slots[8] = {0, 1, 2, 3, 6, 4, 5, -1};
  tm.mark();
  const int big = 0x7fffffff;
  BSE_TRY(hipMemcpyAsync(status, &big, sizeof(int), hipMemcpyHostToDevice, s));
  if (int e = form_and_check_args(n, A, lda, B, ldb, upper, base, p, s)) return e;
  tm.mark();
  BSE_TRY(cholesky_pair_z(np, n, M1, M2, ld, linv, status, s, p.side));
  if (int st = read_status(status, n, info, s)) return st;
  tm.mark();
  {
    GemmDesc g = tri_gemm(np, ld, M2, 1, M1, 0, 1, W);  // W = L2^H L1
    g.mask = n;
    BSE_TRY(gemm_z(g, s));
    BSE_TRY(z_to_c64(np, W, ld, Wc, s));
  }
  tm.mark();
  JacobiResult j32;
  // The complex64 iteration only prepares the FP64 sweeps: it ends once a
  // sweep rotates fewer than 1/32 of its pairs, when the rest is rounding.
  BSE_TRY(jacobi_c(np, Wc, ld, jw32, tol32, 1.0e-5, max32, j32, s, kernel_time_stride(want_timing), 1.0, 1.0 / 32));
  tm.mark();
  // Z = W32 V32 in FP64 (Y); V' = L1^-1 L2^-H Z (W)
  BSE_TRY(c64_to_c128(np, Wc, ld, Y, ld, nullptr, s));
  BSE_TRY(hipMemcpyAsync(W, Y, (size_t)np * np * sizeof(double2), hipMemcpyDeviceToDevice, s));
  BSE_TRY(trsm_lh_z(np, M2, ld, W, X1, inv, s));    // X1 = L2^-H Z   (W is overwritten)
  BSE_TRY(trsm_ln_z(np, M1, ld, X1, W, inv, s));    // W  = L1^-1 X1 = V'
  {
    GemmDesc g;  // G = V'^H V' (lower tiles)
    g.M = np; g.N = np; g.K = np;
    g.A = W; g.lda = ld; g.opA = 1;
    g.B = W; g.ldb = ld; g.opB = 0;
    g.C = X2; g.ldc = ld;
    g.lowerC = 1;
    BSE_TRY(gemm_z(g, s));
  }
  BSE_TRY(tri_pad_z(n, np, X2, ld, 0, s));
  BSE_TRY(cholesky_z(np, n, X2, ld, linv, status, 0, s));  // G = L_G L_G^H
  int gst = 0;
  BSE_TRY(hipMemcpyAsync(&gst, status, sizeof(int), hipMemcpyDeviceToHost, s));
  BSE_TRY(hipStreamSynchronize(s));
  JacobiResult j64;
  double2* Zb = X1;  // the columns the FP64 sweeps orthogonalise
  int fallback = 0;
  // BSE_TEST_POLISH_FALLBACK set: take the failure branch below (test hook)
  if (getenv("BSE_TEST_POLISH_FALLBACK") != nullptr) gst = 1;
  if (gst == big) {
    BSE_TRY(trsm_rh_z(np, X2, ld, Y, X1, inv, s));  // W V = Z L_G^-H -> X1 (Y is overwritten)
    const double first = fmin(kInnerStopCap, fmax(1.0e-10, fmin(j32.max_off, tol32)));
    BSE_TRY(jacobi_z(np, X1, ld, jw64, tol64, 30, j64, s, kernel_time_stride(want_timing), first));
  } else {
    // V'^H V' is not numerically positive definite: the complex64 iteration
    // lost the rotation (kappa(W) eps32 near 1).  The FP64 sweeps then run
    // on W itself, as in the FP64 form.
    fallback = 1;
    BSE_TRY(hipMemcpyAsync(status, &big, sizeof(int), hipMemcpyHostToDevice, s));
    GemmDesc g = tri_gemm(np, ld, M2, 1, M1, 0, 1, W);  // W = L2^H L1
    g.mask = n;
    BSE_TRY(gemm_z(g, s));
    Zb = W;
    BSE_TRY(jacobi_z(np, W, ld, jw64, tol64, 30, j64, s, kernel_time_stride(want_timing)));
  }
  tm.mark();
  tm.mark();
  // Alg. 3 steps 4-6; T and V1 in X2 (the factor of G is no longer needed)
  if (int e = back_transform_z(n, np, M1, M2, Zb, Y, X2, inv, base, p, lambda, X, ldx,
                               o.want_negative, o.values_only, s))
    return e;
  tm.mark();
  BSE_TRY(hipStreamSynchronize(s));
  const int ret = (j32.sweeps > 0 && j64.converged) ? 0 : 2 * n + 1;
  fill_info(info, ret, j32);
  if (info) {
    info->fallback = fallback;
    info->polish_sweeps = j64.sweeps;
    info->polish_rotations = j64.rotations;
    info->polish_pair_checks = j64.pair_checks;
    info->polish_cross_pair_checks = j64.cross_pair_checks;
    info->polish_max_off = j64.max_off;
    info->polish_inner_rotations = j64.inner_rotations;
    for (int i = 0; i < 3; ++i) {
      info->polish_kernel_ms[i] = j64.kernel_ms[i];
      info->polish_kernel_launches[i] = j64.kernel_launches[i];
    }
  }
  tm.fill(info, slots);
  return ret;
}

}  // namespace

namespace bse {
// opts.checks: measure the returned pairs (positive half) on the device.
int run_checks(int n, const void* A, int lda, const void* B, int ldb, const double* lambda,
               const void* X, int ldx, char* base, const Plan& p, const bse_opts_t& o,
               bse_info_t* info, hipStream_t s) {
  double2* bufs[5];
  check_buffers(p, base, bufs);
  double out[2] = {0.0, 0.0};
  const int upper = (o.uplo == 'U' || o.uplo == 'u');
  BSE_TRY(check_pairs_z(n, p.np, static_cast<const double2*>(A), lda, static_cast<const double2*>(B),
                        ldb, upper, lambda, static_cast<const double2*>(X), ldx, bufs,
                        reinterpret_cast<double*>(base + p.off_check), out, s));
  if (info) {
    info->sigma_orth_fro = out[0];
    info->max_rel_resid = out[1];
  }
  return 0;
}

int check_h1_args(int n, const void* A, int lda, const void* B, int ldb, const double* lambda,
                  const void* X, int ldx, const bse_opts_t& o) {
  if (n < 0 || n > 46000) return -1;
  if (n > 0 && !A) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (!opts_valid(o)) return -11;
  const int tda = o.route == BSE_ROUTE_TDA;
  if (n > 0 && !B && !tda) return -4;
  if (!tda && ldb < (n > 1 ? n : 1)) return -5;
  if (n > 0 && !lambda) return -6;
  if (n > 0 && !X && !o.values_only) return -7;
  if (!o.values_only && ldx < (2 * n > 1 ? 2 * n : 1)) return -8;
  return 0;
}

// bse_solve_h1 and its variant without allocation (noalloc != 0: the second
// Cholesky factorisation on `stream` too, no timing events).
int solve_h1_impl(int n, const void* A, int lda, const void* B, int ldb, double* lambda, void* X,
                  int ldx, void* work, size_t work_bytes, const bse_opts_t* opts, bse_info_t* info,
                  void* stream, int noalloc) {
  bse_opts_t o;
  bse_default_opts(&o);
  if (opts) o = *opts;
  const int want_timing = info && !noalloc ? info->timing : 0;
  if (info) {
    memset(info, 0, sizeof(*info));
    info->timing = want_timing;
  }
  if (int e = check_h1_args(n, A, lda, B, ldb, lambda, X, ldx, o)) return e;
  if (n == 0) return 0;
  Plan p = make_plan(n, o);
  if (noalloc) p.side = 0;
  if (!work) return -9;
  if (work_bytes < p.total) return -10;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(work) + 255) & ~(uintptr_t)255);
  int ret;
  if (p.tda) ret = solve_tda(n, A, lda, lambda, X, ldx, base, p, o, info, want_timing, s);
  else if (p.sqrt_route) ret = solve_sqrt(n, A, lda, B, ldb, lambda, X, ldx, base, p, o, info, want_timing, s);
  else if (p.alg2) ret = solve_alg2(n, A, lda, B, ldb, lambda, X, ldx, base, p, o, info, want_timing, s);
  else if (p.mixed) ret = solve_mixed(n, A, lda, B, ldb, lambda, X, ldx, base, p, o, info, want_timing, s);
  else if (p.polish) ret = solve_polish(n, A, lda, B, ldb, lambda, X, ldx, base, p, o, info, want_timing, s);
  else ret = solve_fp64(n, A, lda, B, ldb, lambda, X, ldx, base, p, o, info, want_timing, s);
  if (ret == 0 && o.checks) {
    if (int e = run_checks(n, A, lda, B, ldb, lambda, X, ldx, base, p, o, info, s)) return e;
  }
  return ret;
}

}  // namespace bse

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
  return make_plan(n, o).total;
}

int bse_solve_h1(int n, const void* A, int lda, const void* B, int ldb, double* lambda, void* X,
                 int ldx, void* work, size_t work_bytes, const bse_opts_t* opts, bse_info_t* info,
                 void* stream) {
  return bse::solve_h1_impl(n, A, lda, B, ldb, lambda, X, ldx, work, work_bytes, opts, info, stream, 0);
}

size_t bse_batched_workspace_bytes(int batch, const int* n, const bse_opts_t* opts) {
  if (batch < 0 || (batch > 0 && !n)) return 0;
  bse_opts_t o;
  bse_default_opts(&o);
  if (opts) o = *opts;
  if (!opts_valid(o)) return 0;
  for (int i = 0; i < batch; ++i)
    if (n[i] < 0 || n[i] > 46000) return 0;
  return batched_workspace(batch, n, o);
}

int bse_solve_batched(int batch, const int* n, const void* const* A, const int* lda,
                      const void* const* B, const int* ldb, double* const* lambda, void* const* X,
                      const int* ldx, void* work, size_t work_bytes, const bse_opts_t* opts,
                      bse_info_t* info, void* stream) {
  if (batch < 0) return -1;
  if (batch > 0 && !n) return -2;
  if (batch > 0 && (!A || !lda)) return -3;
  bse_opts_t o;
  bse_default_opts(&o);
  if (opts) o = *opts;
  if (!opts_valid(o)) return -12;
  if (batch > 0 && (!B || !ldb) && o.route != BSE_ROUTE_TDA) return -5;
  if (batch > 0 && !lambda) return -7;
  if (batch > 0 && (!X || !ldx) && !o.values_only) return -8;
  const int tda = o.route == BSE_ROUTE_TDA;
  for (int i = 0; i < batch; ++i) {
    if (n[i] < 0 || n[i] > 46000) return -2;
    if (n[i] == 0) continue;
    if (!A[i] || lda[i] < n[i]) return -3;
    if (!tda && (!B[i] || ldb[i] < n[i])) return -5;
    if (!lambda[i]) return -7;
    if (!o.values_only && (!X[i] || ldx[i] < 2 * n[i])) return -8;
  }
  if (batch == 0) return 0;
  const size_t need = bse_batched_workspace_bytes(batch, n, &o);
  if (need == 0) return -2;
  if (batch > 0 && !work) return -10;
  if (work_bytes < need) return -11;
  const int want_timing = info ? info[0].timing : 0;
  if (info)
    for (int i = 0; i < batch; ++i) {
      memset(&info[i], 0, sizeof(info[i]));
      info[i].timing = want_timing;
    }
  hipStream_t s = static_cast<hipStream_t>(stream);
  return solve_batched_grouped(batch, n, A, lda, B, ldb, lambda, X, ldx, work, o, info, want_timing, s);
}

size_t bse_backward_workspace_bytes(int n) { return n >= 0 && n <= 46000 ? adjoint_work_bytes(n) : 0; }

int bse_backward(int n, const void* X, int ldx, const double* w, void* gA, int ldga, void* gB,
                 int ldgb, void* work, size_t work_bytes, void* stream) {
  if (n < 0 || n > 46000) return -1;
  if (n > 0 && !X) return -2;
  if (ldx < (2 * n > 1 ? 2 * n : 1)) return -3;
  if (n > 0 && !w) return -4;
  if (n > 0 && !gA) return -5;
  if (ldga < (n > 1 ? n : 1)) return -6;
  if (n > 0 && !gB) return -7;
  if (ldgb < (n > 1 ? n : 1)) return -8;
  if (n == 0) return 0;
  if (!work) return -9;
  if (work_bytes < adjoint_work_bytes(n)) return -10;
  hipStream_t s = static_cast<hipStream_t>(stream);
  BSE_TRY(adjoint_z(n, static_cast<const double2*>(X), ldx, w, static_cast<double2*>(gA), ldga,
                    static_cast<double2*>(gB), ldgb, work, s));
  BSE_TRY(hipStreamSynchronize(s));
  return 0;
}

size_t bse_backward_vec_workspace_bytes(int n) {
  return n >= 0 && n <= 46000 ? adjoint_vec_work_bytes(n) : 0;
}

int bse_backward_vec(int n, const double* lambda, const void* X, int ldx, const double* g_lambda,
                     const void* G_X, int ldg, double degen_rtol, void* gA, int ldga, void* gB,
                     int ldgb, void* work, size_t work_bytes, void* stream) {
  if (n < 0 || n > 46000) return -1;
  if (n > 0 && !lambda) return -2;
  if (n > 0 && !X) return -3;
  if (ldx < (2 * n > 1 ? 2 * n : 1)) return -4;
  if (n > 0 && !g_lambda) return -5;
  if (n > 0 && !G_X) return -6;
  if (ldg < (2 * n > 1 ? 2 * n : 1)) return -7;
  if (!(degen_rtol >= 0.0 && degen_rtol < 1.0)) return -8;
  if (n > 0 && !gA) return -9;
  if (ldga < (n > 1 ? n : 1)) return -10;
  if (n > 0 && !gB) return -11;
  if (ldgb < (n > 1 ? n : 1)) return -12;
  if (n == 0) return 0;
  if (!work) return -13;
  if (work_bytes < adjoint_vec_work_bytes(n)) return -14;
  hipStream_t s = static_cast<hipStream_t>(stream);
  BSE_TRY(adjoint_vec_z(n, lambda, static_cast<const double2*>(X), ldx, g_lambda,
                        static_cast<const double2*>(G_X), ldg, degen_rtol, static_cast<double2*>(gA),
                        ldga, static_cast<double2*>(gB), ldgb, work, s));
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
