// Internal launch interfaces of the HIP solver (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include <vector>

#include "common.hpp"

namespace bse {

// C[m, n] = alpha * sum_k opA(A)[m, k] * s[k] * opB(B)[k, n] * colscale[n] + beta * C[m, n]
// opA = 0: A is M x K column-major; opA = 1: A is K x M and opA(A) = A^H.
// opB = 0: B is K x N; opB = 1: B is N x K and opB(B) = B^H.
// triA / triB: the stored A / B is lower triangular (its strict upper part is
// zero), so the k-range of each output tile is cut to where both operands
// can be nonzero.  lowerC: only tiles on or below the diagonal are computed.
// mask > 0: outputs with m >= mask or n >= mask are written as zero.
struct GemmDesc {
  int M = 0, N = 0, K = 0;
  const void* A = nullptr; long lda = 0; int opA = 0; int triA = 0;
  const void* B = nullptr; long ldb = 0; int opB = 0; int triB = 0;
  void* C = nullptr; long ldc = 0;
  double alpha_re = 1.0, alpha_im = 0.0, beta_re = 0.0, beta_im = 0.0;
  const double* kscale = nullptr;    // real, length K
  const double* colscale = nullptr;  // real, length N
  int lowerC = 0;
  int mask = 0;
};

hipError_t gemm_z(const GemmDesc& d, hipStream_t s);  // complex128
hipError_t gemm_c(const GemmDesc& d, hipStream_t s);  // complex64

// Blocked Cholesky (lower) of an np x np Hermitian matrix held in its lower
// triangle, in place; np % 64 == 0.  The strict upper triangle must be zero
// on entry and stays zero.  First non-positive pivot (leading minor index,
// 1-based, < n_real) is reported as atomicMin(status, base + index).
hipError_t cholesky_z(int np, int n_real, double2* M, long ld, double2* linv,
                      int* status, int base, hipStream_t s);
// Both factors of Alg. 3 steps 1-2, M1 (status base 0) and M2 (base n_real):
// with side != 0, M2's factorisation runs on a library stream beside s
// (created once per device), ordered after the work already on s, and s waits
// for it at the end; side == 0 runs both on s, one after the other.  linv
// holds two 64 x 64 inverses (one per factor).
hipError_t cholesky_pair_z(int np, int n_real, double2* M1, double2* M2, long ld, double2* linv,
                           int* status, hipStream_t s, int side = 1);
hipError_t cholesky_pair_c(int np, int n_real, float2* M1, float2* M2, long ld, float2* linv,
                           int* status, hipStream_t s, int side = 1);

// M1 = A + B, M2 = A - B (lower triangles, zero strict upper part), padded to
// np with identity; reads the `upper` or lower triangle of A, B (B == nullptr
// reads as B = 0).
hipError_t form_m12(int n, int np, const double2* A, long lda, const double2* B,
                    long ldb, int upper, double2* M1, double2* M2, long ldm,
                    hipStream_t s);

struct JacobiWork {
  void* part = nullptr;    // partial Gram tiles
  void* R = nullptr;       // rotations, pairs x 64 x 64
  double2* track = nullptr;  // per column block: its 32 x 32 Gram (FP64)
  int* flags = nullptr;    // per pair
  int* counter = nullptr;  // rotated pairs in the current sweep
  int* inner = nullptr;    // inner Jacobi sweeps in the current sweep
  int* inner_rot = nullptr;  // inner Jacobi rotations applied in the current sweep
  double* maxoff = nullptr;
  int kc = 0;      // Gram split: row chunks per pair
  int rrows = 0;   // rows per rotation work group
};
// kc, rrows = 0: built-in choice for np (kc: enough work groups to fill the
// chip for one problem; rrows: largest of 256, 128, 64 dividing np).
size_t jacobi_work_bytes(int np, int elem_bytes, int kc = 0);
void jacobi_carve(int np, int elem_bytes, char* base, JacobiWork& w, int kc = 0, int rrows = 0);
// kc a power of two with np % (16 kc) == 0; rrows a multiple of 64 dividing np.
bool jacobi_tiles_valid(int np, int kc, int rrows);
int jacobi_default_kc(int np);
int jacobi_gram_blocks_kc(int np, int kc);
int jacobi_rot_blocks_rr(int np, int rrows);

struct JacobiResult {
  int sweeps = 0;
  int rotations = 0;
  int pair_checks = 0;
  int cross_pair_checks = 0;  // pair checks whose Gram computed only the cross block
  long inner_sweeps = 0;
  double inner_rotations = 0.0;
  double max_off = 0.0;
  int converged = 0;
  // per-kernel event timing (filled when time_stride > 0): summed durations,
  // estimated from the timed rounds when not every round is timed
  double kernel_ms[3] = {0.0, 0.0, 0.0};
  int kernel_launches[3] = {0, 0, 0};
};

// One-sided block-Jacobi on the np columns of W (np % 64 == 0), in place:
// on return the columns of W are mutually orthogonal (W_in Q = W_out, Q unitary).
// Largest inner stopping level of the pair eigensolver (early outer sweeps,
// where the other pairs disturb a pair's orthogonality far more anyway).
constexpr double kInnerStopCap = 3.0e-2;
// A sweep that follows one whose largest relative off-diagonal measure was
// above this level computes only the cross blocks of the pair Grams after its
// first round and tracks the diagonal blocks (the Gram each rotation leaves on
// its two column blocks, kept in FP64).  The tracked blocks drift from the
// data's by the rounding of the rotations, about 1e-11 (FP64) or 1e-5
// (complex64) per sweep, far below the off-diagonal level of such sweeps; the
// sweeps near convergence recompute every Gram tile.
constexpr double kTrackLevel64 = 1.0e-5;
constexpr double kTrackLevel32 = 1.0e-3;
// first_stop: inner stopping level of the first sweep (later sweeps use the
// previous sweep's largest off-diagonal measure, at most kInnerStopCap).
// time_stride: 0 no kernel timing; k > 0 HIP events around the three
// kernels of every k-th round (each sweep's rounds 0, k, 2k, ...).
hipError_t jacobi_z(int np, double2* W, long ld, const JacobiWork& w, double tol,
                    int max_sweeps, JacobiResult& res, hipStream_t s, int time_stride = 0,
                    double first_stop = kInnerStopCap);
// Event stride for the `timing` option of bse_info_t: 2 times every 8th
// round (a sample, so that the events do not slow the solve measurably), 3
// every round.
inline int kernel_time_stride(int timing) { return timing >= 3 ? 1 : timing == 2 ? 8 : 0; }
// complex64 columns; Gram partial sums, inner eigensolver and rotations as in
// jacobi_z (inner eigensolver in FP64), inner iteration ending once a sweep's
// largest relative off-diagonal entry is below inner_stop.
// inner_factor: multiple of the previous sweep's off-diagonal measure used as
// the inner stopping level (1 by default; smaller values leave the columns
// more orthogonal at the end, which the Newton refinement of the mixed form
// needs).
// stop_fraction: when positive, the iteration also ends after a sweep that
// rotated fewer than this fraction of its pair checks (the sweeps that would
// follow only chase complex64 rounding; converged stays 0 then).
hipError_t jacobi_c(int np, float2* W, long ld, const JacobiWork& w, double tol, double inner_stop,
                    int max_sweeps, JacobiResult& res, hipStream_t s, int time_stride = 0,
                    double inner_factor = 1.0, double stop_fraction = 0.0);

hipError_t cholesky_c(int np, int n_real, float2* M, long ld, float2* linv, int* status, int base,
                      hipStream_t s);
// Z = L^-H Rhs for lower-triangular L (np x np, np % 64 == 0): block back
// substitution with the inverses of the 64 x 64 diagonal blocks (inv holds
// np * 64 complex values) and MFMA GEMM updates; Rhs is overwritten.
hipError_t trsm_lh_z(int np, const double2* L, long ld, double2* Rhs, double2* Z, double2* inv,
                     hipStream_t s);
// The same in complex64 (FP32 MFMA; the diagonal-block inverses formed in FP64).
hipError_t trsm_lh_c(int np, const float2* L, long ld, float2* Rhs, float2* Z, float2* inv,
                     hipStream_t s);
// The block triangular solves take the 64-column diagonal blocks this many at a time.
constexpr int kTrsmGroup = 4;
// The GEMM steps of trsm_lh_z in their order (after the diagonal-block
// inverses), handed to `emit`: step `slot` (0 .. 2 kTrsmGroup - 1) of group `group` of
// kTrsmGroup block rows counted from the bottom.  Problems of different
// orders share (group, slot) numbers, so a batch can run every problem's step
// of one (group, slot) in one grouped launch, in the same order as a single
// solve.
struct TrsmStep { int group, slot; GemmDesc g; };
template <typename C2, class F>
void trsm_lh_for_each(int np, const C2* L, long ld, C2* Rhs, C2* Z, const C2* inv, F&& emit) {
  constexpr int B = 64;
  const int nb = np / B;
  auto diag = [&](int b) {
    const long rb = (long)b * B;
    GemmDesc g;  // Z_b = (L_bb^-1)^H Rhs_b
    g.M = B; g.N = np; g.K = B;
    g.A = inv + rb * B; g.lda = B; g.opA = 1; g.triA = 1;
    g.B = Rhs + rb; g.ldb = ld; g.opB = 0;
    g.C = Z + rb; g.ldc = ld;
    return g;
  };
  // Rhs[r0 .. r0 + rows) -= (L^H)[r0 .., c0 .. c0 + k) Z[c0 .. c0 + k); (L^H)_{r, c} = conj(L_{c, r})
  auto update = [&](long r0, int rows, long c0, int k) {
    GemmDesc u;
    u.M = rows; u.N = np; u.K = k;
    u.A = L + c0 + r0 * ld; u.lda = ld; u.opA = 1;
    u.B = Z + c0; u.ldb = ld; u.opB = 0;
    u.C = Rhs + r0; u.ldc = ld;
    u.alpha_re = -1.0; u.beta_re = 1.0;
    return u;
  };
  // back substitution with L^H: block rows i, i - 1, ...
  int group = 0;
  for (int i = nb - 1; i >= 0; i -= kTrsmGroup, ++group) {
    const int lo = i - kTrsmGroup + 1 > 0 ? i - kTrsmGroup + 1 : 0;  // first block row of the group
    for (int b = i; b >= lo; --b) {
      const int j = i - b;
      if (j > 0) emit(TrsmStep{group, 2 * j - 1, update((long)b * B, B, (long)(b + 1) * B, j * B)});
      emit(TrsmStep{group, 2 * j, diag(b)});
    }
    // Rhs_{0..lo-1} -= (L^H)_{0..lo-1, lo..i} Z_{lo..i}
    if (lo > 0) emit(TrsmStep{group, 2 * kTrsmGroup - 1, update(0, lo * B, (long)lo * B, (i - lo + 1) * B)});
  }
}
// The steps of Z = L^-1 Rhs (forward block substitution, trsm_ln_z), with the
// same (group, slot) numbering as trsm_lh_for_each (groups counted from the top).
template <class F>
void trsm_ln_for_each(int np, const double2* L, long ld, double2* Rhs, double2* Z, const double2* inv,
                      F&& emit) {
  constexpr int B = 64;
  const int nb = np / B;
  auto diag = [&](int b) {
    const long rb = (long)b * B;
    GemmDesc g;  // Z_b = L_bb^-1 Rhs_b
    g.M = B; g.N = np; g.K = B;
    g.A = inv + rb * B; g.lda = B; g.opA = 0; g.triA = 1;
    g.B = Rhs + rb; g.ldb = ld; g.opB = 0;
    g.C = Z + rb; g.ldc = ld;
    return g;
  };
  // Rhs[r0 .. r0 + rows) -= L[r0 .., c0 .. c0 + k) Z[c0 .. c0 + k)
  auto update = [&](long r0, int rows, long c0, int k) {
    GemmDesc u;
    u.M = rows; u.N = np; u.K = k;
    u.A = L + r0 + c0 * ld; u.lda = ld; u.opA = 0;
    u.B = Z + c0; u.ldb = ld; u.opB = 0;
    u.C = Rhs + r0; u.ldc = ld;
    u.alpha_re = -1.0; u.beta_re = 1.0;
    return u;
  };
  int group = 0;
  for (int i = 0; i < nb; i += kTrsmGroup, ++group) {
    const int hi = i + kTrsmGroup - 1 < nb ? i + kTrsmGroup - 1 : nb - 1;  // last block row of the group
    for (int b = i; b <= hi; ++b) {
      const int j = b - i;
      if (j > 0) emit(TrsmStep{group, 2 * j - 1, update((long)b * B, B, (long)i * B, j * B)});
      emit(TrsmStep{group, 2 * j, diag(b)});
    }
    // Rhs_{hi+1..} -= L_{hi+1.., i..hi} Z_{i..hi}
    const int rest = np - (hi + 1) * B;
    if (rest > 0)
      emit(TrsmStep{group, 2 * kTrsmGroup - 1, update((long)(hi + 1) * B, rest, (long)i * B, (hi - i + 1) * B)});
  }
}

// The steps of Z = Rhs L^-H (column blocks left to right, trsm_rh_z), numbered
// as above.
template <class F>
void trsm_rh_for_each(int np, const double2* L, long ld, double2* Rhs, double2* Z, const double2* inv,
                      F&& emit) {
  constexpr int B = 64;
  const int nb = np / B;
  auto diag = [&](int j) {
    GemmDesc g;  // Z_j = Rhs_j (L_jj^-1)^H
    g.M = np; g.N = B; g.K = B;
    g.A = Rhs + (long)j * B * ld; g.lda = ld; g.opA = 0;
    g.B = inv + (long)j * B * B; g.ldb = B; g.opB = 1; g.triB = 1;
    g.C = Z + (long)j * B * ld; g.ldc = ld;
    return g;
  };
  // Rhs_{c0 .. c0 + cols} -= Z_{j0 .. j0 + k} (L_{c0 .., j0 .. j0 + k})^H
  auto update = [&](int c0, int cols, int j0, int k) {
    GemmDesc u;
    u.M = np; u.N = cols; u.K = k;
    u.A = Z + (long)j0 * ld; u.lda = ld; u.opA = 0;
    u.B = L + c0 + (long)j0 * ld; u.ldb = ld; u.opB = 1;
    u.C = Rhs + (long)c0 * ld; u.ldc = ld;
    u.alpha_re = -1.0; u.beta_re = 1.0;
    return u;
  };
  int group = 0;
  for (int j = 0; j < nb; j += kTrsmGroup, ++group) {
    const int hi = j + kTrsmGroup - 1 < nb ? j + kTrsmGroup - 1 : nb - 1;
    for (int c = j; c <= hi; ++c) {
      const int q = c - j;
      if (q > 0) emit(TrsmStep{group, 2 * q - 1, update(c * B, B, j * B, q * B)});
      emit(TrsmStep{group, 2 * q, diag(c)});
    }
    const int rest = np - (hi + 1) * B;
    if (rest > 0) emit(TrsmStep{group, 2 * kTrsmGroup - 1, update((hi + 1) * B, rest, j * B, (hi - j + 1) * B)});
  }
}
// complex64 copy of all np x np entries.
hipError_t z_to_c64(int np, const double2* M, long ld, float2* Mc, hipStream_t s);
// identity == 0: zero the strict upper triangle of M and give rows/columns
// n..np-1 those of the identity; identity != 0: M = I (np x np).
hipError_t tri_pad_z(int n, int np, double2* M, long ld, int identity, hipStream_t s);
struct TriPadArgs { int n, np; double2* M; long ld; int identity; };
// Z = L^-1 Rhs (forward block substitution, same conventions as trsm_lh_z).
hipError_t trsm_ln_z(int np, const double2* L, long ld, double2* Rhs, double2* Z, double2* inv,
                     hipStream_t s);
// Z = Rhs L^-H (column blocks left to right, same conventions as trsm_lh_z).
hipError_t trsm_rh_z(int np, const double2* L, long ld, double2* Rhs, double2* Z, double2* inv,
                     hipStream_t s);
// M[i][j] = conj(M[j][i]) for i < j (np % 64 == 0).
hipError_t mirror_upper_z(int np, double2* M, long ld, hipStream_t s);
// complex64 copy of the lower triangle, strict upper part zero.
hipError_t lower_to_c64(int np, const double2* M, long ld, float2* Mc, hipStream_t s);

// Column norms out[j] = ||W[:, j]|| for j < np.
hipError_t colnorm_z(int np, const double2* W, long ld, double* out, hipStream_t s);

// sigma_k = ||W_k||; W_k <- W_k sigma_k^-3/2 (k < n; zero for k >= n); bnorm_k = ||W_k||.
hipError_t scale_singular_cols_z(int n, int np, double2* W, long ld, double* sigma,
                                 double* bnorm, hipStream_t s);

// Rayleigh-quotient eigenvalues lam_k = ||T_k|| / bnorm_k (unsorted), 1 / lam,
// the scale of V1 = L2^-H Ws that makes V1_k^H V2_k = 1 (scl_k = 1 / bnorm_k^2),
// the ascending order perm and the output lambda (with -lambda appended if
// want_negative).
hipError_t rq_lambda_z(int n, int np, const double2* T, long ld, const double* bnorm,
                       double* anorm, double* lam, double* invlam, double* scl, int* perm,
                       double* lambda, int want_negative, hipStream_t s);

hipError_t colnorm_c(int np, const float2* W, long ld, double* out, hipStream_t s);
hipError_t scale_singular_cols_c(int n, int np, float2* W, long ld, double* sigma, double* bnorm,
                                 hipStream_t s);
// D[:, j] = S[:, j] * colscale[j] (np x np), complex64 to complex128.
hipError_t c64_to_c128(int np, const float2* S, long lds, double2* D, long ldd,
                       const double* colscale, hipStream_t s);
// lam_k = anorm_k / bnorm_k, 1 / lam_k and s_k = (anorm_k bnorm_k)^-1/2 (k < n; zero above).
// v1scale: scl_k = 1 / bnorm_k^2 instead (the scale of V1 = L2^-H Ws).
hipError_t lambda_from_norms(int n, int np, const double* anorm, const double* bnorm, double* lam,
                             double* invlam, double* scl, hipStream_t s, int v1scale = 0);
// Ascending order of lam[0..n) and the output lambda (with -lambda if want_negative).
hipError_t sort_lambda(int n, const double* lam, int* perm, double* lambda, int want_negative,
                       hipStream_t s);

// Sigma-aware refinement of the positive eigenpairs in (x, y) coordinates
// against full Hermitian FP64 M1 = A + B, M2 = A - B (n x n leading blocks,
// leading dimension ld); x and y are updated in place (through the two work
// buffers), lam receives Rayleigh quotients and scl the Sigma-normalising
// scales of the final pair.  Runs up to max_steps steps and stops after a
// step whose largest off-diagonal correction is at most stop_corr; returns
// that correction in *max_corr (+inf if a correction or a final Rayleigh
// quotient broke down) and the steps run in *steps_done.
// Windows of the refinement's Rayleigh-Ritz passes (window.hip): for window
// boundaries shifted by `off` (0 or 32), window w covers pairs [a, a + m).
inline __host__ __device__ void window_range(int n, int off, int w, int& a, int& m) {
  if (off == 0) {
    a = w * 64;
  } else if (w == 0) {
    a = 0;
    m = off < n ? off : n;
    return;
  } else {
    a = off + (w - 1) * 64;
  }
  m = n - a < 64 ? n - a : 64;
}
// Pairs the first-order correction resolves slowly: count the (i, j), i < j
// <= i + 64, of the current products whose coupling K_ij = T11_ij - (l_i +
// l_j) G11_ij / 2 exceeds 1 / kCoupleRatio of their Ritz gap |l_j - l_i| (the
// correction's rotation angle is then above about 1 / kCoupleRatio, and within
// a cluster the pairwise rotations leave errors of the order of its square).
// Work group = 256 rows i.
constexpr double kCoupleRatio = 16.0;
// Complex64 operands of a refinement step's basis update when it is not the
// last: dst[k] = src[k] (k = 0, 1: x, y) and src[k] - I (k = 2, 3: Ex, Ey),
// n x n blocks, work group = a 64 x 64 tile of one matrix (4 ceil(n/64)^2).
struct LowArgs { int n; long ld; const double2* src[4]; float2* dst[4]; };
// dst[k] += src[k] (complex64 into complex128), k = 0, 1 (2 ceil(n/64)^2 work groups).
struct AddLowArgs { int n; long ld; const float2* src[2]; double2* dst[2]; };
struct CoupleArgs {
  int n; long ld; const double2* F; const double2* P1; const double2* P2; const double* ritz;
  int* count;
};
struct WinArgs {  // work group = window
  int n; long ld; const double2* F; const double2* P1; const double2* P2; int off;
  double2* C;       // window blocks, 64 x 64 each (column-major, ld 64)
  double* maxrot;   // optional: largest entry of C_w - I (atomic max)
};
int window_count(int n, int off);
hipError_t window_eig(const WinArgs& a, int windows, hipStream_t s);
hipError_t group_window(const void* table, const int2* map, int blocks, hipStream_t s);

// Pairs whose Ritz values differ by at most this fraction are corrected
// within their span only (first-order rotation part dropped).
constexpr double kRefineDelta = 1.0e-10;
// The refinement stops after a step whose largest first-order correction is
// at most this; the error it leaves is of the order of its square (about
// half of it measured), so the vectors are left within about 1e-12.
constexpr double kRefineStop = 1.0e-6;
// Window passes per refinement step (boundaries at 0, then shifted by 32).
constexpr int kWindowPasses = 2;
// Boundary offset of window pass p: 0, 32 (and 16, 48 for passes 2, 3).
inline int window_offset(int pass) { return (pass & 1) * 32 + ((pass >> 1) & 1) * 16; }
// A step after one whose first-order correction was at most this runs no
// windows: the rotations left inside near-degenerate groups are then of the
// order of that correction's square, well inside the first-order regime.
constexpr double kWindowStop = 1.0e-4;
struct RefineWork {
  double2 *Q = nullptr, *F = nullptr, *P1 = nullptr, *P2 = nullptr, *Ex = nullptr, *Ey = nullptr;
  double *ritz = nullptr, *dots = nullptr, *maxcorr = nullptr;
  // Rayleigh-Ritz windows (window.hip): block storage of the two passes and a
  // device arena for the grouped block GEMMs; windows == 0 turns them off
  double2* Cb0 = nullptr;  // kWindowPasses x (n / 64 + 2) blocks of 64 x 64
  char* arena = nullptr;
  size_t arena_cap = 0;
  int windows = 0;         // window passes per step once a step finds strongly coupled pairs (0: none)
  // nonzero: the basis updates of all steps but the last take complex64
  // products (Q, F, Ex and Ey must each hold ld x n complex128 values)
  int low_update = 0;
  int* perm = nullptr;  // n ints: the ascending order of the start's eigenvalues
};
// Block GEMMs of a window pass over the first n pairs (windows of offset
// `off`, blocks C_w at Cb): the congruence M <- C^H M C through Tmp (right
// products into `right`, then left products into `left`), and the basis
// change out = X C (into g).  Storage of pass p's blocks: window_blocks.
void window_congruence(int n, long ld, double2* M, double2* Tmp, const double2* Cb, int off,
                       std::vector<GemmDesc>& right, std::vector<GemmDesc>& left);
void window_right(int n, long ld, const double2* X, double2* out, const double2* Cb, int off,
                  std::vector<GemmDesc>& g);
double2* window_blocks(double2* Cb0, int n, int pass);
// Column k < n: lam_k = (x_k^H Qx_k + y_k^H Qy_k) / (2 Re x_k^H y_k) and
// scl_k = (Re x_k^H y_k)^-1/2.
hipError_t rq_pairs_z(int n, long ld, const double2* x, const double2* y, const double2* Qx,
                      const double2* Qy, double* lam, double* scl, hipStream_t s);
// L1, L2: the FP64 Cholesky factors of M1 = A + B and M2 = A - B (lower,
// zero strict upper part); corr_hist (host, optional): the largest correction
// of each step (first 8).
hipError_t refine_z(int n, long ld, const double2* L1, const double2* L2, double2** x, double2** y,
                    const RefineWork& w, int max_steps, double stop_corr, double* lam, double* scl,
                    double* max_corr, int* steps_done, hipStream_t s, double* corr_hist = nullptr,
                    int* window_steps = nullptr);

// out[:, r] = W[:, perm r] * f_r (r < n; zero for r >= n; np rows; f == nullptr: 1).
hipError_t gather_scale_z(int n, int np, const double2* W, long ld, const int* perm,
                          const double* f, double2* out, hipStream_t s);
// Alg. 2 eigenvalue bookkeeping from d = column norms of the iterated M:
// lam_k = sqrt(d_k), ascending order perm, output lambda (and -lambda),
// fy_r = 1 / (d sqrt(lam)) and fx_r = sqrt(lam) / d for sorted position r.
hipError_t alg2_lambda_z(int n, const double* d, double* lam, int* perm, double* lambda,
                         int want_negative, double* fx, double* fy, hipStream_t s);

// Scales of the SQRT route (Alg. 1): from the column norms dC of the iterated
// A - B and dM of the iterated M = S (A + B) S: ks = dC^-3/2, kis = dC^-5/2
// (S = Z ks Z^H, S^-1 = Z kis Z^H), c1 = dM^-3/4, c2 = dM^-5/4, lam = dM^1/2.
hipError_t sqrt_scales(int n, int np, const double* dC, const double* dM, double* ks, double* kis,
                       double* c1, double* c2, double* lam, hipStream_t s);

// X[:, r] = s_k [(t_k V1_k + V2_k)/2; (V2_k - t_k V1_k)/2] with k = perm[r]
// (and the mirrored negative half); perm == nullptr means k = r, scl ==
// nullptr s_k = 1, scl1 == nullptr t_k = 1 (else t_k = scl1[k]).
hipError_t assemble_z(int n, const double2* V1, const double2* V2, long ldv, const int* perm,
                      const double* scl, double2* X, long ldx, int want_negative, hipStream_t s,
                      const double* scl1 = nullptr);

// Eigenvalue adjoint: G_A = sum_k w_k (a_k a_k^H + b_k b_k^H),
// G_B = sum_k w_k (a_k b_k^H + b_k a_k^H) for X = [a; b] (2n x n, ldx), written
// as full Hermitian n x n matrices; work holds adjoint_work_bytes(n) bytes.
size_t adjoint_work_bytes(int n);
// Eigenvector adjoint: G_A, G_B for a loss with dL = sum_k g_k dlambda_k +
// Re tr(G_X^H dX) (first-order perturbation of the pencil (Sigma H1, Sigma)
// with all 2n eigenvectors); pairs with |lam_k - lam_i| <= rtol max|lam|
// count as degenerate.  work holds adjoint_vec_work_bytes(n) bytes.
size_t adjoint_vec_work_bytes(int n);
hipError_t adjoint_vec_z(int n, const double* lam, const double2* X, long ldx, const double* g,
                         const double2* GX, long ldg, double rtol, double2* gA, long ldga,
                         double2* gB, long ldgb, void* work, hipStream_t s);
hipError_t adjoint_z(int n, const double2* X, long ldx, const double* w, double2* gA, long ldga,
                     double2* gB, long ldgb, void* work, hipStream_t s);

// Measurements of returned pairs (opts.checks): with bufs five np x np
// complex128 scratch buffers and `small` check_small_bytes(n) bytes of device
// memory, out[0] = ||X^H Sigma X - I||_F and out[1] = max_k ||H1 x_k -
// lambda_k x_k|| / (lambda_max ||x_k||) (synchronises on s).
size_t check_small_bytes(int n);
hipError_t check_pairs_z(int n, int np, const double2* A, long lda, const double2* B, long ldb,
                         int upper, const double* lambda, const double2* X, long ldx,
                         double2* const bufs[5], double* small, double out[2], hipStream_t s);

// ---------------------------------------------------------------- op arguments
// Argument structs of the kernels (see the op launches in common.hpp); the
// grouped form of a phase takes a device table of these, one per problem.
struct FormArgs {
  int n, np; const double2* A; long lda; const double2* B; long ldb; int upper;
  double2* M1; double2* M2; long ldm;
};
struct MirrorArgs { int np; double2* M; long ld; };
template <typename C2> struct TriInvArgsT { const C2* L; long ld; C2* inv; };  // work group = diagonal block
typedef TriInvArgsT<double2> TriInvArgs;
struct ToC64Args { int np; const double2* M; long ld; float2* Mc; };
template <typename C2> struct Potf2Args {  // aux = first column of the panel
  C2* M; long ld; C2* linv; int* status; int base; int n_real;
};
template <typename T> struct GemmArgs {
  typedef typename cpx_t<T>::type C2;
  int M, N, K;
  const C2* A; long lda; int triA;
  const C2* B; long ldb; int triB;
  C2* C; long ldc;
  T ar, ai, br, bi;
  const double* kscale;
  const double* colscale;
  int lowerC, mask;
  int tilesM, tilesN;
};
// cross != 0: rounds after the first of a sweep compute only the cross block
// X_q^H X_p of a pair's Gram; the inner eigensolver takes the diagonal blocks
// from `track` (per column block, the 32 x 32 Gram left by the block's last
// rotation, FP64, column-major), which it writes back after every pair.
// crossp, when set, points at a per-problem device flag used instead of cross.
template <typename C2> struct GramArgs {  // aux = round
  int N; const C2* W; long ld; int rc, kc; C2* part; const int* done; int cross;
  const int* crossp;
};
template <typename C2> struct EigArgs {  // aux = round
  int N, kc; const C2* part; C2* R; int* flags; int* counter; double tol; double* maxoff;
  int max_inner; int* inner; double inner_stop2; const double* stop2p; int* inner_rot;
  const int* done; double2* track; int cross; const int* crossp;
};
template <typename C2> struct RotArgs {  // aux = round
  int N; C2* W; long ld; const C2* R; const int* flags; int rrows, chunks; const int* done;
};
template <typename C2> struct ColnormArgs { const C2* W; long ld; int np; double* out; };
template <typename C2> struct ScaleArgs { int n, np; C2* W; long ld; const double* sigma; };
// v1scale = 0: scl_k = (anorm_k bnorm_k)^-1/2 (both halves of the pair);
// v1scale = 1: scl_k = 1 / bnorm_k^2 (the scale of V1 = L2^-H Ws alone).
struct LambdaArgs {
  int n, np; const double* anorm; const double* bnorm; double* lam; double* invlam; double* scl;
  int v1scale;
};
struct RankArgs { int n; const double* key; int* perm; int desc; };
struct WriteLambdaArgs { int n; const double* lam; const int* perm; double* lambda; int want_negative; };
struct GatherArgs { int n, np; const double2* W; long ld; const int* perm; const double* f; double2* out; };
struct C64Args { int np; const float2* S; long lds; double2* D; long ldd; const double* colscale; };
// Alg. 2 bookkeeping from the column norms d of the iterated M (alg2_lambda_z)
struct Alg2Args { int n; const double* d; double* lam; const int* perm; double* fx; double* fy; };
// Alg. 1 scales from the column norms dC of the iterated A - B and dM of the iterated M (sqrt_scales)
struct SqrtScalesArgs {
  int n, np; const double* dC; const double* dM; double* ks; double* kis; double* c1; double* c2;
  double* lam;
};
struct AssembleArgs {
  int n; const double2* V1; const double2* V2; long ldv; const int* perm; const double* scl;
  double2* X; long ldx; int want_negative; const double* scl1;
};
struct RitzArgs { int n; const double2* F; const double2* P1; const double2* P2; long ld; double* ritz; };
struct BuildArgs {
  int n; const double2* F; const double2* P1; const double2* P2; long ld; const double* ritz;
  double2* Ex; double2* Ey; double delta; double* maxcorr;
  double* part;  // optional: per-tile column sums for the updated pairs' quotients (3 x T x n)
};
// Rayleigh quotients and Sigma-normalising scales of the pairs after the
// correction, from the products and the tile sums of BuildOp (work group =
// 256 columns): lam_k, scl_k as RqOp computes them for x Ex, y Ey.
struct UpdRqArgs {
  int n; long ld; const double2* F; const double2* P1; const double2* P2; const double* part;
  double* lam; double* scl; double* bad;
};
// bad (optional): set to 1 if a pair is not Sigma-positive or its quotient
// is not finite and positive.
struct RqArgs {
  int n; const double2* x; const double2* y; const double2* Qx; const double2* Qy; long ld;
  double* lam; double* scl; double* bad;
};

// Per-problem Jacobi state of a batch (device memory, 128 bytes).  The
// kernels of a problem whose `done` is set return at once; the sweep op
// closes one sweep and opens the next.
struct JacState {
  int counter, inner, inner_rot, done;
  int sweeps, rotations, converged, cross;
  long pair_checks, inner_sweeps;
  double maxoff, last_off, stop2, inner_rotations;
  long cross_pair_checks;
  double pad1[5];
};
struct SweepArgs {  // aux = sweep index
  JacState* st; int* active; int pairs_per_sweep; int max_sweeps; double inner_floor; int adaptive;
  double factor;  // inner stopping level = factor x previous sweep's largest off-diagonal
  double track_level;  // sweeps after one whose largest off-diagonal exceeded this track
  int pairs_per_round;
  double stop_fraction;  // > 0: a sweep rotating fewer than this fraction of its pairs ends the iteration
  double first_stop;     // > 0: the first sweep's inner stopping level and tracking measure (default kInnerStopCap)
};

// Work-group counts of one problem for the ops above.
int gemm_tiles(const GemmDesc& d);
int jacobi_eig_blocks(int np);
int jacobi_rounds(int np);
int jacobi_pairs(int np);

// Argument structs filled the way the single-problem launches fill them.
GemmArgs<double> gemm_args_z(const GemmDesc& d);
GemmArgs<float> gemm_args_c(const GemmDesc& d);
GramArgs<double2> gram_args_z(int np, double2* W, long ld, const JacobiWork& w, const int* done);
GramArgs<float2> gram_args_c(int np, float2* W, long ld, const JacobiWork& w, const int* done);
EigArgs<double2> eig_args_z(int np, const JacobiWork& w, double tol, const double* stop2p, const int* done);
EigArgs<float2> eig_args_c(int np, const JacobiWork& w, double tol, const double* stop2p, const int* done);
RotArgs<double2> rot_args_z(int np, double2* W, long ld, const JacobiWork& w, const int* done);
RotArgs<float2> rot_args_c(int np, float2* W, long ld, const JacobiWork& w, const int* done);

// Grouped launches: table = device array of the op's Args, map = device
// array of (table row, work group) pairs, blocks = entries of map used.
enum GroupOp {
  G_FORM, G_MIRROR, G_TOC64, G_POTF2_Z, G_POTF2_C, G_TRIINV, G_TRIINV_C, G_ZTOC, G_TRIPAD,  // chol.hip
  G_GRAM_Z, G_GRAM_C, G_EIG_Z, G_EIG_C, G_ROT_Z, G_ROT_C, G_SWEEP,      // jacobi.hip
  G_COLNORM_Z, G_COLNORM_C, G_SCALE_Z, G_SCALE_C, G_LAMBDA, G_RANK,     // finalize.hip
  G_WRITE_LAMBDA, G_C64, G_ASSEMBLE, G_GATHER, G_ALG2_LAMBDA, G_ALG2_SCALES, G_SQRT_SCALES,
  G_RITZ, G_BUILD, G_RQ, G_UPDRQ, G_COUPLE, G_LOW, G_ADDLOW,                             // refine.hip
};
hipError_t group_chol(GroupOp op, const void* table, const int2* map, int blocks, int aux, hipStream_t s);
hipError_t group_jacobi(GroupOp op, const void* table, const int2* map, int blocks, int aux, hipStream_t s);
hipError_t group_finalize(GroupOp op, const void* table, const int2* map, int blocks, int aux, hipStream_t s);
hipError_t group_refine(GroupOp op, const void* table, const int2* map, int blocks, int aux, hipStream_t s);
// prec 0: complex128, 1: complex64
hipError_t group_gemm(int prec, int opA, int opB, int ks, const void* table, const int2* map,
                      int blocks, hipStream_t s);

// Blocks per problem of the fixed-shape ops.
inline int tiles64(int np) { return (np / 64) * (np / 64); }
inline int cols_blocks(int rows, int cols) { return ((rows + 255) / 256) * cols; }

}  // namespace bse
