// Workspace plan of one problem and the helpers shared by the single and the
// batched entry points (host code only).
#pragma once

#include <math.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/bse.h"
#include "internal.hpp"

namespace bse {

constexpr int kErrHip = -1000;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int pad64(int n) { return ((n + 63) / 64) * 64; }

// Workspace layout.  U = np^2 complex128 (16 np^2 bytes).
//   FP64:  M1, M2, W, Y, T (5 U) and the diagonal-block inverses of L2
//   mixed: M1, M2 (full Hermitian FP64), X1, X2 (FP64 pair), Q, F, P1, P2
//          (refinement), L1c|L2c (complex64, 1 U), Wc|Yc (complex64, 1 U):
//          10 U; the complex64 regions hold Ex, Ey during the refinement.
struct Plan {
  int n = 0, np = 0, mixed = 0;
  size_t off_m1 = 0, off_m2 = 0, off_w = 0, off_y = 0;
  size_t off_x1 = 0, off_x2 = 0, off_q = 0, off_f = 0, off_p1 = 0, off_p2 = 0;
  size_t off_z = 0, off_inv = 0, off_t = 0;
  int alg2 = 0, tda = 0, sqrt_route = 0;
  size_t off_lc = 0, off_wc = 0;
  size_t off_linv = 0, off_sigma = 0, off_perm = 0, off_invlam = 0, off_status = 0;
  size_t off_bnorm = 0, off_anorm = 0, off_lamu = 0, off_scl = 0, off_ritz = 0, off_small = 0;
  size_t off_jac = 0;
  size_t off_check = 0;  // opts.checks: reduction buffers of the measurements
  size_t off_cb0 = 0, off_cb1 = 0, off_arena = 0;  // mixed: refinement windows
  size_t total = 0;
  int kc = 0, rrows = 0;  // Jacobi tiles (0 = built-in)
  int polish = 0;
  int side = 1;  // second Cholesky factorisation on the library's side stream
};

// Device arena of the refinement's grouped block GEMMs (a ring of tables):
// room for the largest launch, the basis update of x and y by the windows of
// one pass (2 (np / 64 + 2) block GEMMs of np x 64 or 64 x np).
inline size_t refine_arena_bytes(int np) {
  const size_t descs = 2 * (size_t)(np / 64 + 2);
  GemmDesc a, b;
  a.M = np; a.N = 64; a.K = 64;
  b.M = 64; b.N = np; b.K = 64;
  const size_t tiles = (size_t)(gemm_tiles(a) > gemm_tiles(b) ? gemm_tiles(a) : gemm_tiles(b));
  return align256(descs * sizeof(GemmArgs<double>)) + align256(descs * tiles * sizeof(int2)) + 4096;
}

inline bool opts_valid(const bse_opts_t& o) {
  if (o.route < BSE_ROUTE_SVD || o.route > BSE_ROUTE_SQRT) return false;
  if ((o.route == BSE_ROUTE_TDA || o.route == BSE_ROUTE_SQRT) && o.precision != BSE_PREC_FP64)
    return false;  // TDA and SQRT: FP64 only
  if (o.values_only != 0 && o.values_only != 1) return false;
  if (o.precision != BSE_PREC_FP64 && o.precision != BSE_PREC_MIXED &&
      o.precision != BSE_PREC_MIXED_POLISH)
    return false;
  if (o.precision == BSE_PREC_MIXED_POLISH && o.route != BSE_ROUTE_SVD) return false;
  if (o.max_sweeps < 0 || o.refine_steps < 0 || o.refine_steps > 8 || !(o.jacobi_tol >= 0.0))
    return false;
  if (o.route == BSE_ROUTE_EIG && o.precision != BSE_PREC_FP64) return false;  // Alg. 2: FP64 only
  if (!(o.uplo == 0 || o.uplo == 'L' || o.uplo == 'U' || o.uplo == 'l' || o.uplo == 'u')) return false;
  if (o.checks != 0 && o.checks != 1) return false;
  if (o.reserved != 0) return false;
  if (o.tile_entries < 0 || o.tile_entries > 4096 || (o.tile_entries > 0 && !o.tile_table)) return false;
  for (int r = 0; r < o.tile_entries; ++r) {
    const int kc = o.tile_table[3 * r + 1], rr = o.tile_table[3 * r + 2];
    if (o.tile_table[3 * r] <= 0 || kc < 1 || (kc & (kc - 1)) != 0 || rr < 64 || rr % 64 != 0)
      return false;
  }
  return true;
}

// Jacobi tiles of a problem of padded order np: the first fitting row of the
// caller's table, else 0 (built-in choice).  kc is capped at the built-in
// split, for which the workspace is sized.
inline void pick_tiles(const bse_opts_t& o, int np, int* kc, int* rrows) {
  *kc = 0;
  *rrows = 0;
  for (int r = 0; r < o.tile_entries; ++r) {
    if (np > o.tile_table[3 * r]) continue;
    const int k = o.tile_table[3 * r + 1], rr = o.tile_table[3 * r + 2];
    if (jacobi_tiles_valid(np, k, rr) && k <= jacobi_default_kc(np)) {
      *kc = k;
      *rrows = rr;
    }
    return;
  }
}

inline Plan make_plan(int n, const bse_opts_t& o) {
  Plan p;
  p.n = n;
  p.np = pad64(n > 0 ? n : 1);
  p.mixed = o.precision == BSE_PREC_MIXED;
  p.polish = o.precision == BSE_PREC_MIXED_POLISH;
  pick_tiles(o, p.np, &p.kc, &p.rrows);
  p.alg2 = o.route == BSE_ROUTE_EIG;
  p.tda = o.route == BSE_ROUTE_TDA;
  p.sqrt_route = o.route == BSE_ROUTE_SQRT;
  const size_t U = (size_t)p.np * p.np * sizeof(double2);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  p.off_m1 = take(U);
  p.off_m2 = take(U);
  if (p.alg2) {
    p.off_w = take(U);
    p.off_y = take(U);
    p.off_z = take(U);
    p.off_inv = take((size_t)p.np * 64 * sizeof(double2));
  } else if (p.polish) {
    p.off_w = take(U);
    p.off_y = take(U);
    p.off_x1 = take(U);  // complex64 W during the FP32 iteration, then solve results
    p.off_x2 = take(U);  // Gram of the recovered rotation, its factor and inverse
    p.off_inv = take((size_t)p.np * 64 * sizeof(double2));
  } else if (!p.mixed) {
    p.off_w = take(U);
    p.off_y = take(U);
    p.off_t = take(U);
    p.off_inv = take((size_t)p.np * 64 * sizeof(double2));
  } else {
    p.off_x1 = take(U);
    p.off_x2 = take(U);
    p.off_q = take(U);
    p.off_f = take(U);
    p.off_p1 = take(U);
    p.off_p2 = take(U);
    p.off_lc = take(U);  // L1c | L2c, then Ex
    p.off_wc = take(U);  // Wc | Yc, then Ey
    // Rayleigh-Ritz windows of the refinement: 64 x 64 blocks of two passes,
    // and the arena of their grouped block GEMMs
    const size_t blk = (size_t)64 * 64 * sizeof(double2);
    p.off_cb0 = take(blk * (size_t)(p.np / 64 + 2) * kWindowPasses);
    p.off_arena = take(refine_arena_bytes(p.np));
  }
  p.off_linv = take(2 * 64 * 64 * sizeof(double2));  // one diagonal-block inverse per factor
  p.off_sigma = take((size_t)p.np * sizeof(double));
  p.off_perm = take((size_t)p.np * sizeof(int));
  p.off_invlam = take((size_t)p.np * sizeof(double));
  p.off_bnorm = take((size_t)p.np * sizeof(double));
  p.off_anorm = take((size_t)p.np * sizeof(double));
  p.off_lamu = take((size_t)p.np * sizeof(double));
  p.off_scl = take((size_t)p.np * sizeof(double));
  p.off_ritz = take((size_t)p.np * sizeof(double));
  p.off_small = take(256);
  p.off_status = take(64);
  p.off_jac = take(jacobi_work_bytes(p.np, p.mixed ? sizeof(float) : sizeof(double)));
  if (o.checks) p.off_check = take(check_small_bytes(p.n > 0 ? p.n : 1));
  p.total = off + 256;  // slack for aligning the caller's base pointer
  return p;
}

// Five np x np complex128 regions of a plan, free once its solve is done
// (the measurements of opts.checks use them).
inline void check_buffers(const Plan& p, char* base, double2* bufs[5]) {
  size_t off[5] = {p.off_m1, p.off_m2, p.off_w, p.off_y, p.off_t};
  if (p.alg2) off[4] = p.off_z;
  if (p.polish) off[4] = p.off_x1;
  if (p.mixed) { off[2] = p.off_x1; off[3] = p.off_x2; off[4] = p.off_q; }
  for (int i = 0; i < 5; ++i) bufs[i] = reinterpret_cast<double2*>(base + off[i]);
}

// Default stopping level of the FP64 Jacobi sweeps: a pair is rotated while
// its largest relative off-diagonal Gram entry exceeds 8 sqrt(n) eps.  After
// the last sweep the columns' relative off-orthogonality is below it, and in
// the returned vectors it appears multiplied by sqrt(sigma_i / sigma_j) (the
// Sigma-orthogonality entry of pair (i, j) is g_ij / (sigma_i^1/2 sigma_j^3/2)
// symmetrised), so the level is as low as the Gram's rounding (a sum of n
// products, about sqrt(n) eps) allows with margin.
inline double default_tol64(int n) {
  const double nn = (double)(n > 64 ? n : 64);
  return 8.0 * sqrt(nn) * 2.220446049250313e-16;
}

inline int hip_status(hipError_t e) { return kErrHip - (int)e; }

#define BSE_TRY(expr)                            \
  do {                                           \
    hipError_t e_ = (expr);                      \
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
  // phase i of ms_phase = time between marks i and i + 1 (marks may be skipped: -1)
  void fill(bse_info_t* info, const int* slot) {
    if (!on || !info) return;
    (void)hipEventSynchronize(ev[k - 1]);
    for (int i = 0; i + 1 < k; ++i) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
      if (slot[i] >= 0 && slot[i] < 7) info->ms_phase[slot[i]] += ms;
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


// Batched SVD route (batched.hip): workspace bytes and the grouped solve.
size_t batched_workspace(int batch, const int* n, const bse_opts_t& o);
int solve_batched_grouped(int batch, const int* n, const void* const* A, const int* lda,
                          const void* const* B, const int* ldb, double* const* lambda,
                          void* const* X, const int* ldx, void* work, const bse_opts_t& o,
                          bse_info_t* info, int want_timing, hipStream_t s);

// The FP64 form of bse_solve_h1 on a mixed plan's workspace (base, p): the
// mixed form's way out when its complex64 stage cannot carry the problem.
// Sets info->fallback = 2.
int solve_fp64_fallback(int n, const void* A, int lda, const void* B, int ldb, double* lambda,
                        void* X, int ldx, char* base, const Plan& p, const bse_opts_t& o,
                        bse_info_t* info, hipStream_t s);

// Argument checks of bse_solve_h1 (return codes -1 .. -8, -11 for opts), on the host.
int check_h1_args(int n, const void* A, int lda, const void* B, int ldb, const double* lambda,
                  const void* X, int ldx, const bse_opts_t& o);

// bse_solve_h1 (noalloc = 0) and bse_solve_h1_noalloc (noalloc = 1: the
// second Cholesky factorisation on `stream`, no timing events).
int solve_h1_impl(int n, const void* A, int lda, const void* B, int ldb, double* lambda, void* X,
                  int ldx, void* work, size_t work_bytes, const bse_opts_t* opts, bse_info_t* info,
                  void* stream, int noalloc);

// opts.checks: measure the returned pairs of one problem on the device into
// info->sigma_orth_fro and info->max_rel_resid (plan p on base, solve done).
int run_checks(int n, const void* A, int lda, const void* B, int ldb, const double* lambda,
               const void* X, int ldx, char* base, const Plan& p, const bse_opts_t& o,
               bse_info_t* info, hipStream_t s);

// np x np triangular product with a lower-triangular left factor (its k range cut).
inline GemmDesc tri_gemm(int np, long ld, const void* A, int opA, const void* B, int opB, int triB,
                  void* C) {
  GemmDesc g;
  g.M = np; g.N = np; g.K = np;
  g.A = A; g.lda = ld; g.opA = opA; g.triA = 1;
  g.B = B; g.ldb = ld; g.opB = opB; g.triB = triB;
  g.C = C; g.ldc = ld;
  return g;
}

}  // namespace bse
