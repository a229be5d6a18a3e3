/*
 * bse.h -- C ABI of the MI355X (gfx950) solver for the Bethe-Salpeter
 * eigenproblem of form I (and of form II through it: bse_solve_h2).
 *
 * Problem (Benner & Penke, Sec. 1 Eq. Hform1; Alg. 3 Require/Ensure):
 *   H1 = [ A  B ; -B  -A ]  with  A = A^H, B = B^H  in C^{n x n}
 *   and A + B, A - B positive definite (Lemma Qtransform, part 2).
 * Output: the n positive eigenvalues lambda_1 <= ... <= lambda_n and
 *   X in C^{2n x n} with H1 X = X diag(lambda) and X^H Sigma X = I_n,
 *   Sigma = diag(I_n, -I_n) (Thm ProdEig, Eq. SigmaOrthEVecs; the
 *   normalisation of Sec. 4).  Optionally also the mirrored negative half
 *   -lambda_k with eigenvectors [0 I; I 0] x_k (Lemma ComputeNegEvecs, part 1).
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major (LAPACK convention); complex values are
 *     interleaved (re, im) pairs of IEEE doubles (complex128).
 *   - Every matrix and vector pointer is a DEVICE pointer owned by the
 *     caller.  The library never allocates or frees device memory: the
 *     caller passes a workspace of at least the size the matching
 *     *_workspace_bytes query returns.  No data is retained after return.
 *   - All device work is enqueued on `stream` (a hipStream_t; NULL = the
 *     default stream), with one exception: of the two Cholesky
 *     factorisations of Alg. 3 steps 1-2 (and of the Alg. 2 route), the
 *     second runs on a stream the library creates once per device (default
 *     priority, with two events; kept until the process ends), ordered after
 *     the work already on `stream`, and `stream` waits for it before the next
 *     step.  The calls are synchronous: they wait on `stream` to read the
 *     device status word (and, in the Jacobi phase, once per sweep for the
 *     convergence count) before returning.  Calls from several host threads
 *     may run at once on different streams.
 *   - Only the triangle selected by `uplo` ('L' or 'U') of A and B is read;
 *     the imaginary parts of their diagonals are ignored.
 *   - No C++ exception crosses the ABI.  Return codes:
 *        0            success
 *       -i            argument i (1-based) is invalid
 *        1..n         leading minor i of A + B is not positive definite
 *        n+1..2n      leading minor (i - n) of A - B is not positive definite
 *        2n+1         Jacobi iteration did not converge within max_sweeps
 *                     (outputs are written; info->max_off says how far off)
 *        2n+2         mixed precision: the last refinement correction still
 *                     exceeded 1e-4 (outputs are written)
 *       <= -1000      HIP runtime error (-1000 - hipError_t)
 */
#ifndef BSE_H
#define BSE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Route: Alg. 3 (CHOL+SVD: chol(A+B), chol(A-B), SVD of L2^H L1),
 * Alg. 2 (CHOL: chol(A-B), Hermitian eigenproblem of L^H (A+B) L), or the
 * Tamm-Dancoff approximation B = 0 (Sec. 4, Table 3: H1 = diag(A, -A), so the
 * positive eigenpairs are those of the Hermitian positive definite A with
 * eigenvectors [u; 0]; B is not read and may be NULL; one-sided Jacobi on A
 * itself, Rayleigh-quotient eigenvalues u^H A u; FP64 only). */
/* BSE_ROUTE_SQRT: Alg. 1 (Sec. 3.1), the square-root method the paper compares
 * with: S = (A - B)^1/2 from the one-sided Jacobi on A - B, M = S (A + B) S,
 * the one-sided Jacobi on M (eigenvalues lambda^2), V1 = S^-1 V_M Lambda^1/2,
 * V2 = S V_M Lambda^-1/2; FP64 only.  It squares the eigenvalues and loses
 * the accuracy Table 2 shows; provided for that comparison. */
enum { BSE_ROUTE_SVD = 0, BSE_ROUTE_EIG = 1, BSE_ROUTE_TDA = 2, BSE_ROUTE_SQRT = 3 };
/* Arithmetic:
 *   FP64          plain FP64 throughout;
 *   MIXED         complex64 bulk work (Cholesky, W, Jacobi, back-transform)
 *                 on FP32 MFMA with FP64 diagonal Cholesky blocks, then an
 *                 FP64 residual-based refinement of the eigenpairs and FP64
 *                 Rayleigh quotients;
 *   MIXED_POLISH  FP64 Cholesky factors and W (a few percent of the work),
 *                 the bulk of the one-sided Jacobi iteration in complex64 on
 *                 FP32 MFMA, then the accumulated complex64 rotation
 *                 V = W^-1 (W V) recovered by two FP64 triangular solves,
 *                 made unitary in FP64 (Cholesky QR), and FP64 Jacobi sweeps
 *                 on W V until FP64 convergence; results carry the FP64
 *                 form's accuracy.  SVD route only. */
enum { BSE_PREC_FP64 = 0, BSE_PREC_MIXED = 1, BSE_PREC_MIXED_POLISH = 2 };

typedef struct {
  int route;          /* BSE_ROUTE_*                                            */
  int precision;      /* BSE_PREC_*                                             */
  int max_sweeps;     /* Jacobi sweep limit; 0 = default (30 FP64, 20 mixed)    */
  int refine_steps;   /* mixed only: at most this many refinement steps, fewer
                         once a step's largest correction is <= 1e-6;
                         0 = default (8), at most 8                            */
  double jacobi_tol;  /* rotate a block pair while max |g_ij|/sqrt(g_ii g_jj)
                         exceeds this; 0 = default: 8 sqrt(n) eps64 for FP64
                         sweeps, 4 sqrt(n) eps32 for complex64 ones (n >= 64) */
  int want_negative;  /* nonzero: also write -lambda and [0 I; I 0] X           */
  int uplo;           /* 'L' (default when 0) or 'U'                            */
  int tile_entries;   /* rows in tile_table; 0 = built-in tile choice           */
  int checks;         /* 1: also measure the returned pairs on the device and
                         report info->sigma_orth_fro and info->max_rel_resid
                         (one n x n GEMM and two triangular products more);
                         0 = off                                              */
  const int* tile_table; /* host array of tile_entries rows {np_max, kc, rrows}
                         for the Jacobi kernels: a problem of padded order np
                         (n rounded up to 64) takes the first row with
                         np <= np_max; kc = row chunks of the Gram sum per
                         block pair (a power of two, np % (16 kc) == 0), rrows
                         = rows per rotation work group (a multiple of 64
                         dividing np).  A row that does not fit np, or no
                         row, means the built-in choice for that problem.
                         Written by the autotuner of the Python package.     */
  int values_only;    /* 1: eigenvalues only (what Sec. 4's Table 2 measures):
                         the eigenvector recovery and final setup are skipped,
                         X may be NULL and ldx is not checked; the eigenvalues
                         are the ones the full solve returns.  0 = off         */
  int reserved;       /* must be zero                                           */
} bse_opts_t;

typedef struct {
  int status;           /* same value as the return code                      */
  int sweeps;           /* Jacobi sweeps run (the last one rotates nothing)   */
  int fail_index;       /* non-HPD: 1-based leading minor, else 0             */
  int rotations;        /* block-pair rotations over all sweeps               */
  double max_off;       /* largest relative off-diagonal seen in the last sweep */
  double refine_delta;  /* mixed: largest off-diagonal entry of the last
                           refinement correction (error left ~ its square)    */
  double ms_phase[8];   /* phase times (ms): form, chol, W, jacobi, finalize,
                           back-transform, refine, total; filled if requested  */
  int timing;           /* in: 0 none; 1 fill ms_phase; 2 also time the
                           Jacobi kernels of every 8th round with HIP events
                           on `stream` (a sample: the events then cost the
                           solve no measurable time); 3 time every round     */
  int pair_checks;      /* block pairs examined over all sweeps               */
  double kernel_ms[3];  /* timing >= 2: durations of the Jacobi Gram,
                           inner-eigensolver and rotation kernels (ms) summed
                           over all launches (timing 2: the timed rounds'
                           mean duration times the number of launches)        */
  int kernel_launches[3];
  int refine_steps_done; /* mixed: refinement steps run                       */
  double inner_rotations; /* 2 x 2 rotations applied inside the block-pair
                             eigensolvers, over all sweeps                    */
  /* MIXED_POLISH: the fields above describe the complex64 iteration; these
   * the FP64 sweeps that follow it. */
  int polish_sweeps;
  int polish_rotations;
  int polish_pair_checks;
  int cross_pair_checks;  /* pair checks of the iteration above whose Gram
                             computed only the cross block (the diagonal
                             blocks tracked: sweeps far from convergence)    */
  double polish_max_off;
  double polish_inner_rotations;
  double polish_kernel_ms[3];
  int polish_kernel_launches[3];
  int polish_cross_pair_checks;  /* the same for the FP64 sweeps               */
  int fallback;         /* 0: none; 1: MIXED_POLISH found the recovered rotation
                           too far from unitary (its Cholesky QR failed,
                           kappa(W) eps32 near 1) and ran the FP64 sweeps on W
                           itself; 2: MIXED re-solved the problem in FP64 (its
                           complex64 Cholesky failed or the refinement did not
                           reach its tolerance)                               */
  double sigma_orth_fro;  /* opts.checks: ||X^H Sigma X - I||_F of the returned
                           X (the measure of Sec. 4, Fig. 2), else 0          */
  double max_rel_resid;   /* opts.checks: max_k ||H1 x_k - lambda_k x_k||_2 /
                           (lambda_n ||x_k||_2) over the returned pairs (lambda_n
                           the largest eigenvalue), else 0                    */
  double refine_corr[8];  /* MIXED: largest correction of each refinement step */
  int refine_window_steps;  /* MIXED: refinement steps that ran the Rayleigh-Ritz
                             window passes                                     */
} bse_info_t;

/* Fill `opts` with the defaults (route SVD, FP64, lower triangles). */
void bse_default_opts(bse_opts_t* opts);

/* Workspace bytes bse_solve_h1 needs for order n under `opts` (NULL = defaults).
 * Returns 0 for an invalid n or opts. */
size_t bse_workspace_bytes(int n, const bse_opts_t* opts);

/* All eigenpairs of H1 (Alg. 3 or Alg. 2; see the file header).
 *   n        order of A and B (n >= 0; n = 0 returns 0 at once)
 *   A, lda   n x n complex128, lda >= max(1, n); triangle `uplo` read
 *   B, ldb   n x n complex128, ldb >= max(1, n)
 *   lambda   n doubles (2n if want_negative: +lambda ascending, then -lambda)
 *   X, ldx   2n x n complex128 (2n x 2n if want_negative), ldx >= max(1, 2n);
 *            columns are Sigma-normalised eigenvectors in the order of lambda
 *   work     device workspace of work_bytes >= bse_workspace_bytes(n, opts)
 *   opts     NULL = defaults
 *   info     optional (may be NULL) host struct with diagnostics
 *   stream   hipStream_t
 * A and B are not modified.  Outputs are undefined on a non-HPD status. */
int bse_solve_h1(int n, const void* A, int lda, const void* B, int ldb,
                 double* lambda, void* X, int ldx,
                 void* work, size_t work_bytes,
                 const bse_opts_t* opts, bse_info_t* info, void* stream);

/* Workspace bytes bse_solve_h2 needs for order n under `opts` (NULL =
 * defaults); 0 for an invalid n (n > 23000) or opts (route TDA included). */
size_t bse_workspace_bytes_h2(int n, const bse_opts_t* opts);

/* All eigenpairs of a BSE matrix of form II (Eq. Hform2),
 *   H2 = [A B; -B^H -A^T],  A = A^H,  B = B^T (complex symmetric),
 * with the Hamiltonian [A B; conj(B) conj(A)] positive definite (Thm Form2
 * gives the structure; the paper has no algorithm for it).  The problem is
 * mapped to a real form-I problem of order 2n, A' = [Re A  -Im A; Im A  Re A],
 * B' = [Re B  Im B; Im B  -Re B], whose eigenvalues are those of H2, each
 * twice; bse_solve_h1 solves it with `opts` (route SVD, EIG or SQRT, any
 * precision allowed there) and each pair becomes one eigenpair of H2.
 *   n, A, lda, B, ldb   as bse_solve_h1 (triangle `uplo` of A and of B read;
 *                       B's other triangle is its transpose, no conjugation)
 *   lambda   n doubles (2n if want_negative: +lambda ascending, then -lambda)
 *   X, ldx   2n x n complex128 (2n x 2n if want_negative), ldx >= max(1, 2n):
 *            eigenvectors with x^H Sigma x = 1; the negative half is
 *            [0 I; I 0] conj(X) (Lemma ComputeNegEvecs, part 2)
 *   work     device workspace of work_bytes >= bse_workspace_bytes_h2(n, opts)
 * opts.checks fills info->sigma_orth_fro (||X^H Sigma X - I||_F) and
 * info->max_rel_resid (max_k ||H2 x_k - lambda_k x_k|| / (lambda_n ||x_k||)),
 * measured on the order-2n problem with the real vectors of x_k and i x_k;
 * the other info fields are those of the order-2n solve.  An eigenvalue of
 * H2 of multiplicity m (a run of eigenvalues whose gaps are at most 1e-12
 * lambda_max) gets m Sigma-orthonormal vectors of its eigenspace (a pivoted Gram-Schmidt in the Sigma inner product
 * over the run's 2m candidates; one work group per run up to m = 64, two
 * launches per vector beyond).  A final step
 * X <- X (I - (X^H Sigma X - I) / 2) makes the vectors Sigma-orthonormal to
 * rounding (the real solve fixes only Re(x^H Sigma y)).  The call reads the
 * eigenvalues back to the host to find the runs and returns after `stream`
 * has finished.  Returns 0; -1 n, -2 A, -3 lda, -4 B, -5 ldb, -6 lambda,
 * -7 X, -8 ldx, -9 work NULL, -10 work_bytes too small, -11 opts invalid or
 * route TDA; a positive status is bse_solve_h1's for the order-2n problem
 * (e.g. 1..2n: A' + B' not positive definite); <= -1000 HIP error. */
int bse_solve_h2(int n, const void* A, int lda, const void* B, int ldb,
                 double* lambda, void* X, int ldx,
                 void* work, size_t work_bytes,
                 const bse_opts_t* opts, bse_info_t* info, void* stream);

/* Workspace for bse_solve_batched over `batch` problems of orders n[0..batch). */
size_t bse_batched_workspace_bytes(int batch, const int* n, const bse_opts_t* opts);

/* `batch` independent problems in one call (same opts for all).
 *   n, lda, ldb, ldx                 host arrays of length batch
 *   A, B, lambda, X                  host arrays of device pointers
 *   info                             optional host array of `batch` entries
 * Returns 0 if every problem succeeded, else the status of the first problem
 * (in index order) that failed, with every problem's own status in info[i];
 * argument errors: -1 batch, -2 n, -3 A/lda, -5 B/ldb, -7 lambda, -8 X/ldx,
 * -10 work NULL, -11 work_bytes too small, -12 opts invalid.
 * Every route and precision: the problems are processed together; each phase
 * runs as grouped launches over the whole batch, with a table of per-problem
 * kernel arguments and a map from work groups to problems staged in `work`,
 * and the Jacobi sweeps of all problems advance together (one host readback
 * per sweep; a problem that has converged skips the remaining sweeps).  The
 * results of each problem are those bse_solve_h1 computes with the same
 * opts and tile table.
 * info[0].timing requests timing (as for bse_solve_h1); ms_phase then holds
 * the phase times of the whole batch in every entry. */
int bse_solve_batched(int batch, const int* n,
                      const void* const* A, const int* lda,
                      const void* const* B, const int* ldb,
                      double* const* lambda, void* const* X, const int* ldx,
                      void* work, size_t work_bytes,
                      const bse_opts_t* opts, bse_info_t* info, void* stream);

/* Workspace for bse_backward of order n (two n x n complex128 buffers);
 * 0 for n < 0 or n > 46000. */
size_t bse_backward_workspace_bytes(int n);

/* Gradient of a real loss L(lambda) with respect to Hermitian A and B.
 * With v_k = [a_k; b_k] the k-th column of X (X^H Sigma X = I) and
 * w_k = dL/dlambda_k (derivatives with respect to the negative half folded in
 * as -dL/d(-lambda_k)), first-order perturbation with the left eigenvector
 * v_k^H Sigma (Thm EValSym, part 3) gives
 *   G_A = sum_k w_k (a_k a_k^H + b_k b_k^H),
 *   G_B = sum_k w_k (a_k b_k^H + b_k a_k^H),
 * so that dL = Re tr(G_A^H dA) + Re tr(G_B^H dB) for Hermitian dA, dB.
 *   X, ldx     2n x n complex128 (as written by bse_solve_h1)
 *   w          n doubles (device)
 *   gA, ldga   n x n complex128 output (full Hermitian matrix)
 *   gB, ldgb   n x n complex128 output
 *   work       device workspace of work_bytes >= bse_backward_workspace_bytes(n)
 * With x = a - b and y = a + b the sums equal G_A = (P + Q)/2 and
 * G_B = (Q - P)/2 for P = x diag(w) x^H, Q = y diag(w) y^H, so the work is two
 * Hermitian rank-n products (lower tiles only), about 8 n^3 real flops.
 * Inside a cluster of equal eigenvalues the derivative of an individual
 * eigenvalue is not defined; the result is the gradient of L when w is
 * constant on each such cluster (a loss of the cluster's sum), and depends on
 * the basis chosen inside the cluster otherwise.
 * Synchronises on stream before returning.
 * Return codes as above (0, -i, <= -1000). */
int bse_backward(int n, const void* X, int ldx, const double* w,
                 void* gA, int ldga, void* gB, int ldgb,
                 void* work, size_t work_bytes, void* stream);

/* Workspace for bse_backward_vec of order n (six n x n complex128 buffers);
 * 0 for n < 0 or n > 46000. */
size_t bse_backward_vec_workspace_bytes(int n);

/* Gradient of a real loss L(lambda, X) of the eigenvalues and eigenvectors
 * (e.g. oscillator strengths |d^H x_k|^2 of an absorption spectrum, the use of
 * the eigenpairs in Sec. 1) with respect to Hermitian A and B.
 *   lambda     n doubles (device): the positive eigenvalues of the columns of X
 *   X, ldx     2n x n complex128, Sigma-normalised (X^H Sigma X = I), as
 *              written by bse_solve_h1
 *   g_lambda   n doubles (device): dL/dlambda_k
 *   G_X, ldg   2n x n complex128: dL = Re tr(G_X^H dX) for the eigenvector part
 *              (the gradient convention of PyTorch for complex tensors)
 *   degen_rtol pairs with |lambda_k - lambda_i| <= degen_rtol max|lambda| count
 *              as degenerate (0 <= degen_rtol < 1; 1e-13 is a sensible value)
 *   gA, gB     n x n complex128 outputs (full Hermitian), dL = Re tr(G_A^H dA)
 *              + Re tr(G_B^H dB)
 *   work       device workspace of work_bytes >= bse_backward_vec_workspace_bytes(n)
 * First-order perturbation of the Hermitian pencil (Sigma H1, Sigma) with all
 * 2n eigenvectors Z = [X, P X] (Lemma ComputeNegEvecs; Thm ProdEig
 * Eq. SigmaOrthEVecs; Thm EValSym part 3 for the eigenvalue terms): with
 * Y = Z^H G_X, dL = Re sum D_ik K_ik over K = Z^H d(Sigma H1) Z, where
 * D_kk = g_k, D_ik = (conj(Y_ik) - Y_ki) / (2 (lambda_k - lambda_i)) for two
 * positive-half indices (the Hermitian-part numerator stays finite inside
 * clusters: it vanishes for losses invariant under rotations within a cluster
 * and is a divided difference for spectral functions; degenerate pairs get 0),
 * and D_ik = -conj(Y_ik) / (lambda_k + lambda_i') for the negative half.
 * The phase of each eigenvector is held, so the loss should not depend on it.
 * Work: five n^3 complex GEMMs on MFMA (two on lower tiles only) and
 * elementwise passes: 5 n^3 complex multiply-adds (40 n^3 real flops in the
 * plain count, 30 n^3 executed in the three-product form).  Synchronises on stream.
 * Returns 0, -1 n, -2 lambda, -3 X, -4 ldx, -5 g_lambda, -6 G_X, -7 ldg,
 * -8 degen_rtol, -9 gA, -10 ldga, -11 gB, -12 ldgb, -13 work NULL,
 * -14 work_bytes too small, or <= -1000 (HIP runtime error). */
int bse_backward_vec(int n, const double* lambda, const void* X, int ldx, const double* g_lambda,
                     const void* G_X, int ldg, double degen_rtol, void* gA, int ldga, void* gB,
                     int ldgb, void* work, size_t work_bytes, void* stream);

/* Short text for a return code (static storage). */
const char* bse_status_string(int status, int n);

/* Size of the device array that bse_solve_h1_noalloc works in (per GPU). */
#define BSE_NOALLOC_SCRATCH_BYTES (64u << 20)

/* bse_solve_h1 for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same problem, arguments (less the workspace) and results as bse_solve_h1,
 * with these differences:
 *   - The workspace is a library-owned device array of
 *     BSE_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, set up on the first call on
 *     that GPU and held until the process ends; the call allocates no device
 *     memory, creates no stream or event, and runs everything on `stream`
 *     (both Cholesky factorisations one after the other; info->timing is
 *     ignored).  The caller still owns A, B, lambda and X.
 *   - Limit: the order n must satisfy bse_workspace_bytes(n, opts) <=
 *     BSE_NOALLOC_SCRATCH_BYTES (n <= 832 for FP64 and the Alg. 2 route,
 *     n <= 768 for MIXED_POLISH, n <= 576 for MIXED); a larger n returns -1.
 *   - Every call on a GPU shares that GPU's array: calls that overlap on one
 *     GPU (two streams or threads) race and must be serialised by the caller.
 *     The array keeps the last call's contents; nothing in it has to start at
 *     zero.
 * Return codes as bse_solve_h1: -1 n (negative or too large for the array),
 * -2 A, -3 lda, -4 B, -5 ldb, -6 lambda, -7 X, -8 ldx, -9 opts; 1..2n+2 as
 * documented above; <= -1000 HIP error. */
int bse_solve_h1_noalloc(int n, const void* A, int lda, const void* B, int ldb,
                         double* lambda, void* X, int ldx,
                         const bse_opts_t* opts, bse_info_t* info, void* stream);

/* BSE_NOALLOC_SCRATCH_BYTES, as compiled into the library. */
size_t bse_noalloc_scratch_bytes(void);

#ifdef __cplusplus
}
#endif

#endif /* BSE_H */
