// Many independent BSE problems of different orders in one call.
//
// Each phase of every route (Alg. 3 in FP64, mixed and mixed_polish, Alg. 2,
// Alg. 1 and the Tamm-Dancoff case) runs as grouped launches over the whole
// batch: the host builds, per
// launch, a table of per-problem kernel arguments and a map from every flat
// work group to (problem, work group within the problem) (see the op
// launches in common.hpp), so one launch fills the chip with the work of all
// problems at once:
//   form        one launch (plus the complex64 copies and mirrors, mixed form)
//   Cholesky    three launches per 64-column panel (diagonal blocks of both
//               factors of every problem that has that panel, panel solve,
//               trailing update), Alg. 3 steps 1-2
//   W           one grouped GEMM, step 3's matrix (Alg. 2: two, for
//               M = L^H (A + B) L)
//   Jacobi      per round three launches (Gram, inner eigensolver, rotation)
//               over the problems that have that round, recorded once as a
//               HIP graph and replayed every sweep; per sweep one small
//               launch that closes each problem's sweep on the device
//               (converged problems then skip all later work) and one
//               readback of the number of problems still active
//   finalize    grouped column norms, scaling, GEMMs, Rayleigh quotients,
//               sort and the final setup of step 6
//   refinement  (mixed form) per step, over the problems whose last
//               correction was still above the stopping level: grouped GEMMs
//               for the products, per window pass one grouped launch of the
//               window eigensolvers and grouped block GEMMs, the correction
//               and the basis update;
//   polish      (mixed_polish) the rotation of the complex64 iteration
//               recovered in FP64 by grouped block triangular solves and a
//               grouped Cholesky, then grouped FP64 sweeps.
// Problems are ordered by padded order, largest first, so the problems that
// take part in a Jacobi round or a Cholesky panel form a prefix of every
// table and a launch uses a prefix of its map.
//
// Every problem's arithmetic is that of bse_solve_h1 (same kernels, same
// per-problem workspace plan), so a batch reproduces the single-problem
// results; only the Jacobi tiles (Gram row chunks, rotation rows) default to
// smaller splits, since the batch rather than one problem fills the chip.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <vector>

#include "../../include/bse.h"
#include "common.hpp"
#include "internal.hpp"
#include "plan.hpp"
#include "group.hpp"

namespace bse {
namespace {

constexpr int kBig = 0x7fffffff;

// Built-in Jacobi tiles for a problem in a batch: Gram row chunks of about
// 256 rows, rotation groups of the largest of 256 / 128 / 64 rows dividing np.
void batch_tiles(const bse_opts_t& o, int np, int* kc, int* rrows) {
  pick_tiles(o, np, kc, rrows);
  if (*kc > 0) return;
  int k = 1;
  while (np / (2 * k) >= 256 && jacobi_tiles_valid(np, 2 * k, 64) && 2 * k <= jacobi_default_kc(np)) k *= 2;
  *kc = k;
  *rrows = np % 256 == 0 ? 256 : (np % 128 == 0 ? 128 : 64);
}

// Every problem's block triangular solve steps in its own order: one grouped
// GEMM launch per (group, slot).
template <typename T>
hipError_t run_steps(Arena& ar, std::vector<TrsmStep>& steps, hipStream_t s) {
  std::stable_sort(steps.begin(), steps.end(), [](const TrsmStep& a, const TrsmStep& b) {
    return a.group != b.group ? a.group < b.group : a.slot < b.slot;
  });
  for (size_t i = 0; i < steps.size();) {
    size_t j = i;
    std::vector<GemmDesc> launch;
    while (j < steps.size() && steps[j].group == steps[i].group && steps[j].slot == steps[i].slot)
      launch.push_back(steps[j++].g);
    hipError_t e = run_gemm<T>(ar, launch, s);
    if (e != hipSuccess) return e;
    i = j;
  }
  return hipSuccess;
}

struct Prob {
  int idx = 0, n = 0, np = 0;
  const double2* A = nullptr;
  const double2* B = nullptr;
  long lda = 0, ldb = 0, ldx = 0;
  double* lambda = nullptr;
  double2* X = nullptr;
  char* base = nullptr;
  Plan p;
  int kc = 0, rrows = 0;
  int status = 0;
  // mixed refinement state
  double2 *x = nullptr, *y = nullptr, *q = nullptr, *f = nullptr;
  int rsteps = 0, rdone = 0, rbad = 0, rwin = 0, rwsteps = 0;
  // polish state: status word after the Cholesky of V'^H V', the columns the FP64 sweeps
  // orthogonalise, the first sweep's inner stopping level, and whether W was re-formed
  int gst = 0, fallback = 0;
  double2* zb = nullptr;
  double first = 0.0;
  double rcorr = 0.0;
  double rhist[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  template <class T> T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
};

// Header of the batch workspace (device): per-problem status words, Jacobi
// states and refinement corrections, and the active-problem counter.
struct Header {
  size_t off_status = 0, off_state = 0, off_corr = 0, off_active = 0, off_arena = 0, arena = 0;
  size_t total = 0;
};

size_t arena_bytes(const std::vector<int>& nps) {
  // largest single launch: table rows (at most 3 per problem) plus its map
  size_t rows = 0, blocks = 0;
  for (int np : nps) {
    const int pairs = np / 64;
    size_t b = (size_t)2 * tiles64(np);
    b = std::max(b, (size_t)4 * tiles64(np));
    b = std::max(b, (size_t)2 * cols_blocks(np, np));
    b = std::max(b, (size_t)pairs * jacobi_default_kc(np));
    b = std::max(b, (size_t)pairs * (np / 64));
    b = std::max(b, (size_t)2 * np);
    // the refinement's window launches: block GEMMs per window, two matrices at once
    const int nwin = np / 64 + 2;
    GemmDesc wd;
    wd.M = np; wd.N = 64; wd.K = 64;
    b = std::max(b, (size_t)2 * nwin * gemm_tiles(wd));
    wd.M = 64; wd.N = np;
    b = std::max(b, (size_t)2 * nwin * gemm_tiles(wd));
    blocks += 3 * b + 16;  // a phase may stage up to three maps at once (Jacobi)
    rows += std::max(4, 2 * nwin);
  }
  return align256(rows * 256) + align256(blocks * sizeof(int2)) + 4096;
}

Header make_header(int batch, const std::vector<int>& nps) {
  Header h;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  h.off_status = take((size_t)batch * sizeof(int));
  h.off_state = take((size_t)batch * sizeof(JacState));
  h.off_corr = take((size_t)3 * batch * sizeof(double));  // correction, breakdown flag, coupled pairs
  h.off_active = take(256);
  h.arena = arena_bytes(nps);
  h.off_arena = take(h.arena);
  h.total = off;
  return h;
}

}  // namespace

size_t batched_workspace(int batch, const int* n, const bse_opts_t& o) {
  std::vector<int> nps;
  size_t total = 0;
  for (int i = 0; i < batch; ++i) {
    if (n[i] <= 0) continue;
    nps.push_back(pad64(n[i]));
    total += align256(make_plan(n[i], o).total);
  }
  return make_header(batch, nps).total + total + 256;
}

// Grouped solve of the SVD route (FP64 or mixed).  Argument checks are done
// by the caller.  Returns 0 or the first failing status (index order); every
// problem's status and statistics go to info[i] if given.
int solve_batched_grouped(int batch, const int* n, const void* const* A, const int* lda,
                          const void* const* B, const int* ldb, double* const* lambda,
                          void* const* X, const int* ldx, void* work, const bse_opts_t& o,
                          bse_info_t* info, int want_timing, hipStream_t s) {
  const bool mixed = o.precision == BSE_PREC_MIXED;
  const bool polish = o.precision == BSE_PREC_MIXED_POLISH;
  const bool alg2 = o.route == BSE_ROUTE_EIG;  // Alg. 2 (FP64 only)
  const bool tda = o.route == BSE_ROUTE_TDA;   // B = 0 (FP64 only): the Hermitian eigenproblem of A
  const bool sqrt_route = o.route == BSE_ROUTE_SQRT;  // Alg. 1 (FP64 only)
  const int upper = (o.uplo == 'U' || o.uplo == 'u');
  char* wbase = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(work) + 255) & ~(uintptr_t)255);

  // ---- problems, largest padded order first
  std::vector<Prob> probs;
  std::vector<int> nps;
  for (int i = 0; i < batch; ++i) {
    if (n[i] <= 0) continue;
    Prob pr;
    pr.idx = i;
    pr.n = n[i];
    pr.np = pad64(n[i]);
    pr.A = static_cast<const double2*>(A[i]);
    pr.B = B ? static_cast<const double2*>(B[i]) : nullptr;  // TDA: B = 0, may be absent
    pr.lda = lda[i];
    pr.ldb = ldb ? ldb[i] : 0;
    pr.ldx = ldx[i];
    pr.lambda = lambda[i];
    pr.X = static_cast<double2*>(X[i]);
    pr.p = make_plan(n[i], o);
    batch_tiles(o, pr.np, &pr.kc, &pr.rrows);
    probs.push_back(pr);
    nps.push_back(pr.np);
  }
  const Header h = make_header(batch, nps);
  size_t off = h.total;
  for (Prob& pr : probs) {
    pr.base = wbase + off;
    off += align256(pr.p.total);
  }
  std::stable_sort(probs.begin(), probs.end(), [](const Prob& a, const Prob& b) { return a.np > b.np; });
  const int P = (int)probs.size();
  if (P == 0) return 0;
  int* d_status = reinterpret_cast<int*>(wbase + h.off_status);
  JacState* d_state = reinterpret_cast<JacState*>(wbase + h.off_state);
  double* d_corr = reinterpret_cast<double*>(wbase + h.off_corr);
  int* d_active = reinterpret_cast<int*>(wbase + h.off_active);
  Arena ar;
  ar.dev = wbase + h.off_arena;
  ar.cap = h.arena;
  ar.s = s;

  Timer tm(want_timing != 0, s);
  // the polished form's FP64 stage (between the complex64 Jacobi and the
  // finalize) is timed as the refinement, as in the single solve
  // (Alg. 1: both of its Jacobi iterations as the Jacobi phase)
  int slots[8] = {0, 1, 2, 3, 4, 5, 6, -1};
  if (polish) { slots[4] = 6; slots[5] = 4; slots[6] = 5; }
  if (sqrt_route) { slots[4] = 3; slots[5] = 4; slots[6] = 5; }
  tm.mark();
  // ---- header: statuses "no failure", zero Jacobi states and corrections
  {
    std::vector<int> st(batch, kBig);
    BSE_TRY(hipMemcpyAsync(d_status, st.data(), (size_t)batch * sizeof(int), hipMemcpyHostToDevice, s));
    BSE_TRY(hipStreamSynchronize(s));
    BSE_TRY(hipMemsetAsync(d_state, 0, (size_t)batch * sizeof(JacState), s));
    BSE_TRY(hipMemsetAsync(d_corr, 0, (size_t)batch * sizeof(double), s));
  }

  // ---- form M1 = A + B, M2 = A - B (lower; complex64 copies for the mixed form)
  {
    Grp<FormArgs> g;
    for (const Prob& pr : probs) {
      const FormArgs a = {pr.n, pr.np, pr.A, pr.lda, tda ? nullptr : pr.B, tda ? 0 : pr.ldb, upper,
                          pr.at<double2>(pr.p.off_m1), pr.at<double2>(pr.p.off_m2), pr.np};
      g.add(a, tiles64(pr.np));
    }
    BSE_TRY(run_op(ar, g, group_chol, G_FORM, 0, s));
    if (alg2) {
      // Alg. 2 does not factor A + B; a factorisation of a copy checks its
      // definiteness, and A + B itself is kept whole (mirrored) for T = (A + B) L
      Grp<MirrorArgs> m;
      for (const Prob& pr : probs) {
        BSE_TRY(hipMemcpyAsync(pr.base + pr.p.off_z, pr.base + pr.p.off_m1,
                               (size_t)pr.np * pr.np * sizeof(double2), hipMemcpyDeviceToDevice, s));
        m.add({pr.np, pr.at<double2>(pr.p.off_m1), pr.np}, tiles64(pr.np));
      }
      BSE_TRY(run_op(ar, m, group_chol, G_MIRROR, 0, s));
    }
    if (sqrt_route) {
      // Alg. 1 works with A + B and A - B in full
      Grp<MirrorArgs> m;
      for (const Prob& pr : probs) {
        m.add({pr.np, pr.at<double2>(pr.p.off_m1), pr.np}, tiles64(pr.np));
        m.add({pr.np, pr.at<double2>(pr.p.off_m2), pr.np}, tiles64(pr.np));
      }
      BSE_TRY(run_op(ar, m, group_chol, G_MIRROR, 0, s));
    }
    if (tda) {
      // M1 = A in full (identity beyond n) and its copy W, the Jacobi's matrix;
      // the padded columns are unit vectors orthogonal to the rest
      Grp<MirrorArgs> m;
      for (const Prob& pr : probs) m.add({pr.np, pr.at<double2>(pr.p.off_m1), pr.np}, tiles64(pr.np));
      BSE_TRY(run_op(ar, m, group_chol, G_MIRROR, 0, s));
      for (const Prob& pr : probs)
        BSE_TRY(hipMemcpyAsync(pr.base + pr.p.off_w, pr.base + pr.p.off_m1,
                               (size_t)pr.np * pr.np * sizeof(double2), hipMemcpyDeviceToDevice, s));
    }
    if (mixed) {
      // complex64 copies of the lower triangles (the FP64 M1, M2 stay lower: the
      // refinement works with their FP64 Cholesky factors)
      Grp<ToC64Args> c;
      for (const Prob& pr : probs) {
        const size_t half = (size_t)pr.np * pr.np * sizeof(float2);
        const ToC64Args c1 = {pr.np, pr.at<double2>(pr.p.off_m1), pr.np, pr.at<float2>(pr.p.off_lc)};
        const ToC64Args c2 = {pr.np, pr.at<double2>(pr.p.off_m2), pr.np, pr.at<float2>(pr.p.off_lc + half)};
        c.add(c1, tiles64(pr.np));
        c.add(c2, tiles64(pr.np));
      }
      BSE_TRY(run_op(ar, c, group_chol, G_TOC64, 0, s));
    }
  }
  tm.mark();

  // ---- blocked Cholesky, two panels at a time (as the single solve: factor
  // panel j0, update the next column block with it, factor panel j0 + 64,
  // update the rest with both, K = 128), of nf factors of every problem of
  // `list` (largest padded order first); a failure writes base + column into
  // the problem's status word
  typedef std::function<void*(const Prob&, int)> FactorFn;
  auto cholesky_phase = [&](const std::vector<Prob*>& list, int nf, const FactorFn& factor_of,
                            const std::function<int(const Prob&, int)>& base_of, bool c64) -> int {
    if (list.empty()) return 0;
    const int kmax = list[0]->np / 64;
    const size_t es = c64 ? sizeof(float2) : sizeof(double2);
    auto linv_of = [&](const Prob& pr, int f) -> void* {
      return pr.base + pr.p.off_linv + (size_t)f * 64 * 64 * es;
    };
    auto at = [&](void* M, const Prob& pr, int r, int c) -> char* {
      return static_cast<char*>(M) + ((size_t)r + (size_t)c * pr.np) * es;
    };
    // Potf2 at column j0 and the solve of the rows below it, for every problem
    // with np > j0
    auto factor_panels = [&](int j0) -> int {
      std::vector<GemmDesc> trsm;
      Grp<Potf2Args<double2>> gz;
      Grp<Potf2Args<float2>> gc;
      for (const Prob* pp : list) {
        const Prob& pr = *pp;
        if (pr.np <= j0) break;
        for (int f = 0; f < nf; ++f) {
          void* M = factor_of(pr, f);
          void* linv = linv_of(pr, f);
          if (c64) {
            const Potf2Args<float2> a = {static_cast<float2*>(M), pr.np, static_cast<float2*>(linv),
                                         d_status + pr.idx, base_of(pr, f), pr.n};
            gc.add(a, 1);
          } else {
            const Potf2Args<double2> a = {static_cast<double2*>(M), pr.np, static_cast<double2*>(linv),
                                          d_status + pr.idx, base_of(pr, f), pr.n};
            gz.add(a, 1);
          }
          const int rows = pr.np - j0 - 64;
          if (rows <= 0) continue;
          GemmDesc t;  // L21 = A21 L11^-H
          t.M = rows; t.N = 64; t.K = 64;
          t.A = at(M, pr, j0 + 64, j0); t.lda = pr.np; t.opA = 0;
          t.B = linv; t.ldb = 64; t.opB = 1; t.triB = 1;
          t.C = at(M, pr, j0 + 64, j0); t.ldc = pr.np;
          trsm.push_back(t);
        }
      }
      if (c64) {
        BSE_TRY(run_op(ar, gc, group_chol, G_POTF2_C, j0, s));
        BSE_TRY(run_gemm<float>(ar, trsm, s));
      } else {
        BSE_TRY(run_op(ar, gz, group_chol, G_POTF2_Z, j0, s));
        BSE_TRY(run_gemm<double>(ar, trsm, s));
      }
      return 0;
    };
    auto run_updates = [&](std::vector<GemmDesc>& v) -> int {
      if (c64) BSE_TRY(run_gemm<float>(ar, v, s));
      else BSE_TRY(run_gemm<double>(ar, v, s));
      return 0;
    };
    for (int k = 0; k < kmax; k += 2) {
      const int j0 = 64 * k;
      if (int e = factor_panels(j0)) return e;
      std::vector<GemmDesc> next, rest;
      for (const Prob* pp : list) {
        const Prob& pr = *pp;
        const int rows = pr.np - j0 - 64;
        if (rows <= 0) break;
        for (int f = 0; f < nf; ++f) {
          void* M = factor_of(pr, f);
          GemmDesc h;  // next column block: A[j0+64.., j0+64..j0+128] -= L21 L21[0..64]^H
          h.M = rows; h.N = 64; h.K = 64;
          h.A = at(M, pr, j0 + 64, j0); h.lda = pr.np; h.opA = 0;
          h.B = h.A; h.ldb = pr.np; h.opB = 1;
          h.C = at(M, pr, j0 + 64, j0 + 64); h.ldc = pr.np;
          h.alpha_re = -1.0; h.beta_re = 1.0;
          next.push_back(h);
          const int rem = rows - 64;
          if (rem <= 0) continue;
          GemmDesc u;  // A22 -= L[rem, j0..j0+128] L[rem, j0..j0+128]^H, lower tiles
          u.M = rem; u.N = rem; u.K = 128;
          u.A = at(M, pr, j0 + 128, j0); u.lda = pr.np; u.opA = 0;
          u.B = u.A; u.ldb = pr.np; u.opB = 1;
          u.C = at(M, pr, j0 + 128, j0 + 128); u.ldc = pr.np;
          u.alpha_re = -1.0; u.beta_re = 1.0; u.lowerC = 1;
          rest.push_back(u);
        }
      }
      if (next.empty()) continue;
      if (int e = run_updates(next)) return e;
      if (int e = factor_panels(j0 + 64)) return e;
      if (!rest.empty())
        if (int e = run_updates(rest)) return e;
    }
    return 0;
  };
  auto read_statuses = [&]() -> int {
    std::vector<int> st(batch, kBig);
    BSE_TRY(hipMemcpyAsync(st.data(), d_status, (size_t)batch * sizeof(int), hipMemcpyDeviceToHost, s));
    BSE_TRY(hipStreamSynchronize(s));
    for (Prob& pr : probs) pr.gst = st[pr.idx];
    return 0;
  };

  // ---- Cholesky factors L1 L1^H = A + B and L2 L2^H = A - B of every problem (Alg. 3 steps 1-2)
  {
    std::vector<Prob*> all;
    for (Prob& pr : probs) all.push_back(&pr);
    const FactorFn factor_of = [&](const Prob& pr, int f) -> void* {
      const size_t half = (size_t)pr.np * pr.np * sizeof(float2);
      if (alg2) return static_cast<void*>(pr.base + (f ? pr.p.off_m2 : pr.p.off_z));
      return mixed ? static_cast<void*>(pr.base + pr.p.off_lc + (f ? half : 0))
                   : static_cast<void*>(pr.base + (f ? pr.p.off_m2 : pr.p.off_m1));
    };
    if (!tda && !sqrt_route) {  // the Tamm-Dancoff case and Alg. 1 factor nothing
      if (int e = cholesky_phase(all, 2, factor_of, [](const Prob& pr, int f) { return f ? pr.n : 0; }, mixed))
        return e;
      if (int e = read_statuses()) return e;
      for (Prob& pr : probs) pr.status = pr.gst == kBig ? 0 : pr.gst;
    }
  }
  std::vector<Prob*> ok;
  for (Prob& pr : probs)
    if (pr.status == 0) ok.push_back(&pr);
  tm.mark();

  // ---- W = L2^H L1 (step 3's matrix; zero outside the leading n x n block);
  // Alg. 2: M = L^H (A + B) L with L L^H = A - B
  if (tda || sqrt_route) {
    // (TDA: W is the copy of A made with the form; Alg. 1 iterates on A - B)
  } else if (alg2) {
    std::vector<GemmDesc> tg, mg;
    for (Prob* pr : ok) {
      const int np = pr->np;
      GemmDesc t;  // T = (A + B) L
      t.M = np; t.N = np; t.K = np;
      t.A = pr->base + pr->p.off_m1; t.lda = np; t.opA = 0;
      t.B = pr->base + pr->p.off_m2; t.ldb = np; t.opB = 0; t.triB = 1;
      t.C = pr->base + pr->p.off_w; t.ldc = np;
      tg.push_back(t);
      GemmDesc m = tri_gemm(np, np, pr->base + pr->p.off_m2, 1, pr->base + pr->p.off_w, 0, 0,
                            pr->base + pr->p.off_y);  // M = L^H T
      m.mask = pr->n;
      mg.push_back(m);
    }
    BSE_TRY(run_gemm<double>(ar, tg, s));
    BSE_TRY(run_gemm<double>(ar, mg, s));
  } else {
    std::vector<GemmDesc> w;
    for (Prob* pr : ok) {
      const size_t half = (size_t)pr->np * pr->np * sizeof(float2);
      GemmDesc g = mixed ? tri_gemm(pr->np, pr->np, pr->base + pr->p.off_lc + half, 1,
                                    pr->base + pr->p.off_lc, 0, 1, pr->base + pr->p.off_wc)
                         : tri_gemm(pr->np, pr->np, pr->base + pr->p.off_m2, 1, pr->base + pr->p.off_m1,
                                    0, 1, pr->base + pr->p.off_w);
      g.mask = pr->n;
      w.push_back(g);
    }
    if (mixed) BSE_TRY(run_gemm<float>(ar, w, s));
    else BSE_TRY(run_gemm<double>(ar, w, s));
    if (polish) {
      // the polished form iterates on a complex64 copy of W (in X1)
      Grp<ToC64Args> c;
      for (Prob* pr : ok)
        c.add({pr->np, pr->at<double2>(pr->p.off_w), pr->np, pr->at<float2>(pr->p.off_x1)}, tiles64(pr->np));
      BSE_TRY(run_op(ar, c, group_chol, G_ZTOC, 0, s));
    }
  }
  tm.mark();

  // ---- one-sided block Jacobi over the problems of `list` (largest padded
  // order first), complex64 (c64) or FP64, on each problem's W_of matrix;
  // per problem tolerance tol_of and first sweep's inner level first_of
  // (0: the default); leaves every problem's sweep state in `states`
  const double eps32 = 1.1920928955078125e-07;
  std::vector<JacState> states(batch);
  auto jacobi_phase = [&](const std::vector<Prob*>& list, bool c64, int msweeps, double floor,
                          double stop_fraction, const std::function<void*(Prob*)>& W_of,
                          const std::function<double(Prob*)>& tol_of,
                          const std::function<double(Prob*)>& first_of) -> int {
    BSE_TRY(hipMemsetAsync(d_state, 0, (size_t)batch * sizeof(JacState), s));
    if (list.empty()) return 0;
    Grp<GramArgs<double2>> gz;
    Grp<GramArgs<float2>> gc;
    Grp<EigArgs<double2>> ez;
    Grp<EigArgs<float2>> ec;
    Grp<RotArgs<double2>> rz;
    Grp<RotArgs<float2>> rc;
    Grp<SweepArgs> sw;
    std::vector<int> rounds;
    for (Prob* pr : list) {
      const int np = pr->np;
      JacobiWork jw;
      jacobi_carve(np, c64 ? sizeof(float) : sizeof(double), pr->base + pr->p.off_jac, jw, pr->kc,
                   pr->rrows);
      JacState* st = d_state + pr->idx;
      jw.counter = &st->counter;
      jw.inner = &st->inner;
      jw.inner_rot = &st->inner_rot;
      jw.maxoff = &st->maxoff;
      const double tol = tol_of(pr);
      if (c64) {
        float2* W = static_cast<float2*>(W_of(pr));
        GramArgs<float2> ga = gram_args_c(np, W, np, jw, &st->done);
        EigArgs<float2> ea = eig_args_c(np, jw, tol, &st->stop2, &st->done);
        ga.crossp = ea.crossp = &st->cross;
        gc.add(ga, jacobi_gram_blocks_kc(np, jw.kc));
        ec.add(ea, jacobi_eig_blocks(np));
        rc.add(rot_args_c(np, W, np, jw, &st->done), jacobi_rot_blocks_rr(np, jw.rrows));
      } else {
        double2* W = static_cast<double2*>(W_of(pr));
        GramArgs<double2> ga = gram_args_z(np, W, np, jw, &st->done);
        EigArgs<double2> ea = eig_args_z(np, jw, tol, &st->stop2, &st->done);
        ga.crossp = ea.crossp = &st->cross;
        gz.add(ga, jacobi_gram_blocks_kc(np, jw.kc));
        ez.add(ea, jacobi_eig_blocks(np));
        rz.add(rot_args_z(np, W, np, jw, &st->done), jacobi_rot_blocks_rr(np, jw.rrows));
      }
      const SweepArgs sa = {st, d_active, jacobi_pairs(np) * jacobi_rounds(np), msweeps, floor, 1, 1.0,
                            c64 ? kTrackLevel32 : kTrackLevel64, jacobi_pairs(np), stop_fraction,
                            first_of(pr)};
      sw.add(sa, 1);
      rounds.push_back(jacobi_rounds(np));
    }
    Dev dg, de, dr, ds;
    // the four tables are read by every sweep's launches: one run of the arena
    BSE_TRY(ar.reserve(c64 ? staged_bytes(gc) + staged_bytes(ec) + staged_bytes(rc) + staged_bytes(sw)
                           : staged_bytes(gz) + staged_bytes(ez) + staged_bytes(rz) + staged_bytes(sw)));
    if (c64) {
      BSE_TRY(stage(ar, gc, dg));
      BSE_TRY(stage(ar, ec, de));
      BSE_TRY(stage(ar, rc, dr));
    } else {
      BSE_TRY(stage(ar, gz, dg));
      BSE_TRY(stage(ar, ez, de));
      BSE_TRY(stage(ar, rz, dr));
    }
    BSE_TRY(stage(ar, sw, ds));
    const int R = rounds[0];
    // rows (problems) taking part in round t: a prefix, problems sorted by np
    std::vector<int> part(R);
    for (int t = 0; t < R; ++t) {
      int c = 0;
      while (c < (int)rounds.size() && rounds[c] > t) ++c;
      part[t] = c;
    }
    // The 3R launches of a sweep are the same in every sweep (same tables,
    // prefixes and rounds; what changes lives in device memory), so they are
    // recorded once into a HIP graph and the graph is replayed per sweep.
    // Recording uses a private stream; if recording fails the launches are
    // issued directly.
    auto rounds_on = [&](hipStream_t st) -> hipError_t {
      hipError_t e = hipSuccess;
      for (int t = 0; t < R && e == hipSuccess; ++t) {
        const int c = part[t];
        if (c64) {
          e = group_jacobi(G_GRAM_C, dg.tab, dg.map, gc.prefix(c), t, st);
          if (e == hipSuccess) e = group_jacobi(G_EIG_C, de.tab, de.map, ec.prefix(c), t, st);
          if (e == hipSuccess) e = group_jacobi(G_ROT_C, dr.tab, dr.map, rc.prefix(c), t, st);
        } else {
          e = group_jacobi(G_GRAM_Z, dg.tab, dg.map, gz.prefix(c), t, st);
          if (e == hipSuccess) e = group_jacobi(G_EIG_Z, de.tab, de.map, ez.prefix(c), t, st);
          if (e == hipSuccess) e = group_jacobi(G_ROT_Z, dr.tab, dr.map, rz.prefix(c), t, st);
        }
      }
      return e;
    };
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    {
      hipStream_t cap = nullptr;
      if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess) {
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess) {
          const hipError_t e1 = rounds_on(cap);
          const hipError_t e2 = hipStreamEndCapture(cap, &graph);
          if (e1 != hipSuccess || e2 != hipSuccess ||
              hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
            exec = nullptr;
        }
        (void)hipStreamDestroy(cap);
      }
      (void)hipGetLastError();  // a failed recording leaves no error behind
    }
    hipError_t loop_err = hipSuccess;
    for (int sweep = 0;; ++sweep) {
      if ((loop_err = hipMemsetAsync(d_active, 0, sizeof(int), s)) != hipSuccess) break;
      if ((loop_err = group_jacobi(G_SWEEP, ds.tab, ds.map, ds.blocks, sweep, s)) != hipSuccess) break;
      int active = 0;
      if ((loop_err = hipMemcpyAsync(&active, d_active, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) break;
      if ((loop_err = hipStreamSynchronize(s)) != hipSuccess) break;
      if (active == 0) break;
      loop_err = exec ? hipGraphLaunch(exec, s) : rounds_on(s);
      if (loop_err != hipSuccess) break;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    BSE_TRY(loop_err);
    BSE_TRY(hipMemcpyAsync(states.data(), d_state, (size_t)batch * sizeof(JacState), hipMemcpyDeviceToHost, s));
    BSE_TRY(hipStreamSynchronize(s));
    return 0;
  };

  // Alg. 3 step 3's SVD: complex64 for the mixed forms, FP64 otherwise
  const bool c64_jacobi = mixed || polish;
  const int max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : (c64_jacobi ? 20 : 30);
  {
    auto tol_of = [&](Prob* pr) {
      const double nn = (double)(pr->n > 64 ? pr->n : 64);
      // the polished form's complex64 iteration ignores opts.jacobi_tol (its
      // FP64 sweeps take it), as the single solve
      if (polish) return 4.0 * sqrt(nn) * eps32;
      return o.jacobi_tol > 0.0 ? o.jacobi_tol : (mixed ? 4.0 * sqrt(nn) * eps32 : default_tol64(pr->n));
    };
    auto W_of = [&](Prob* pr) -> void* {
      if (sqrt_route) return pr->base + pr->p.off_m2;  // Z = V_C D_C
      return pr->base + (mixed ? pr->p.off_wc : (polish ? pr->p.off_x1 : (alg2 ? pr->p.off_y : pr->p.off_w)));
    };
    if (int e = jacobi_phase(ok, c64_jacobi, max_sweeps, c64_jacobi ? 1.0e-5 : 1.0e-10,
                             c64_jacobi ? 1.0 / 32 : 0.0, W_of, tol_of, [](Prob*) { return 0.0; }))
      return e;
  }
  tm.mark();
  // ---- mixed_polish: the rotation of the complex64 iteration recovered and
  // finished in FP64, as the single solve (Z = W32 V32 in FP64, V' = L1^-1
  // L2^-H Z, Cholesky of G = V'^H V', W V = Z L_G^-H, FP64 sweeps); a problem
  // whose G is not numerically positive definite runs its FP64 sweeps on W itself
  std::vector<JacState> states32;
  if (polish && !ok.empty()) {
    states32 = states;
    auto M1_of = [](const Prob* pr) { return pr->at<double2>(pr->p.off_m1); };
    auto M2_of = [](const Prob* pr) { return pr->at<double2>(pr->p.off_m2); };
    auto W_of = [](const Prob* pr) { return pr->at<double2>(pr->p.off_w); };
    auto Y_of = [](const Prob* pr) { return pr->at<double2>(pr->p.off_y); };
    auto X1_of = [](const Prob* pr) { return pr->at<double2>(pr->p.off_x1); };
    auto X2_of = [](const Prob* pr) { return pr->at<double2>(pr->p.off_x2); };
    auto inv_of = [](const Prob* pr) { return pr->at<double2>(pr->p.off_inv); };
    {
      Grp<C64Args> cv;
      for (Prob* pr : ok) {
        const int np = pr->np;
        const float2* Wc = pr->at<float2>(pr->p.off_x1);
        cv.add({np, Wc, np, Y_of(pr), np, nullptr}, cols_blocks(np, np));
        cv.add({np, Wc, np, W_of(pr), np, nullptr}, cols_blocks(np, np));
      }
      BSE_TRY(run_op(ar, cv, group_finalize, G_C64, 0, s));
    }
    // X1 = L2^-H Z (W overwritten), then W = L1^-1 X1 = V' (X1 overwritten)
    {
      Grp<TriInvArgs> ti;
      std::vector<TrsmStep> steps;
      for (Prob* pr : ok) {
        ti.add({M2_of(pr), pr->np, inv_of(pr)}, pr->np / 64);
        trsm_lh_for_each(pr->np, (const double2*)M2_of(pr), pr->np, W_of(pr), X1_of(pr), inv_of(pr),
                         [&](const TrsmStep& st) { steps.push_back(st); });
      }
      BSE_TRY(run_op(ar, ti, group_chol, G_TRIINV, 0, s));
      BSE_TRY(run_steps<double>(ar, steps, s));
    }
    {
      Grp<TriInvArgs> ti;
      std::vector<TrsmStep> steps;
      for (Prob* pr : ok) {
        ti.add({M1_of(pr), pr->np, inv_of(pr)}, pr->np / 64);
        trsm_ln_for_each(pr->np, M1_of(pr), pr->np, X1_of(pr), W_of(pr), inv_of(pr),
                         [&](const TrsmStep& st) { steps.push_back(st); });
      }
      BSE_TRY(run_op(ar, ti, group_chol, G_TRIINV, 0, s));
      BSE_TRY(run_steps<double>(ar, steps, s));
    }
    // G = V'^H V' (lower tiles) in X2, padded, and its Cholesky factor
    {
      std::vector<GemmDesc> g;
      Grp<TriPadArgs> tp;
      for (Prob* pr : ok) {
        const int np = pr->np;
        GemmDesc d;
        d.M = np; d.N = np; d.K = np;
        d.A = W_of(pr); d.lda = np; d.opA = 1;
        d.B = W_of(pr); d.ldb = np; d.opB = 0;
        d.C = X2_of(pr); d.ldc = np;
        d.lowerC = 1;
        g.push_back(d);
        tp.add({pr->n, np, X2_of(pr), np, 0}, tiles64(np));
      }
      BSE_TRY(run_gemm<double>(ar, g, s));
      BSE_TRY(run_op(ar, tp, group_chol, G_TRIPAD, 0, s));
    }
    if (int e = cholesky_phase(ok, 1, [&](const Prob& pr, int) -> void* { return X2_of(&pr); },
                               [](const Prob&, int) { return 0; }, false))
      return e;
    if (int e = read_statuses()) return e;
    // BSE_TEST_POLISH_FALLBACK set: every problem takes the branch of a G that
    // is not positive definite (test hook, as in the single solve)
    const bool force_fallback = getenv("BSE_TEST_POLISH_FALLBACK") != nullptr;
    {
      Grp<TriInvArgs> ti;
      std::vector<TrsmStep> steps;
      std::vector<GemmDesc> wg;
      std::vector<int> reset;
      for (Prob* pr : ok) {
        const double nn = (double)(pr->n > 64 ? pr->n : 64);
        const double tol32 = 4.0 * sqrt(nn) * eps32;
        if (pr->gst == kBig && !force_fallback) {
          // W V = Z L_G^-H -> X1 (Y overwritten)
          ti.add({X2_of(pr), pr->np, inv_of(pr)}, pr->np / 64);
          trsm_rh_for_each(pr->np, X2_of(pr), pr->np, Y_of(pr), X1_of(pr), inv_of(pr),
                           [&](const TrsmStep& st) { steps.push_back(st); });
          pr->zb = X1_of(pr);
          pr->first = fmin(kInnerStopCap, fmax(1.0e-10, fmin(states32[pr->idx].last_off, tol32)));
        } else {
          // V'^H V' is not numerically positive definite: W = L2^H L1 again
          pr->fallback = 1;
          reset.push_back(pr->idx);
          GemmDesc d = tri_gemm(pr->np, pr->np, M2_of(pr), 1, M1_of(pr), 0, 1, W_of(pr));
          d.mask = pr->n;
          wg.push_back(d);
          pr->zb = W_of(pr);
          pr->first = 0.0;
        }
      }
      for (int i : reset) BSE_TRY(hipMemcpyAsync(d_status + i, &kBig, sizeof(int), hipMemcpyHostToDevice, s));
      BSE_TRY(run_op(ar, ti, group_chol, G_TRIINV, 0, s));
      BSE_TRY(run_steps<double>(ar, steps, s));
      BSE_TRY(run_gemm<double>(ar, wg, s));
    }
    auto tol64_of = [&](Prob* pr) { return o.jacobi_tol > 0.0 ? o.jacobi_tol : default_tol64(pr->n); };
    if (int e = jacobi_phase(ok, false, 30, 1.0e-10, 0.0, [](Prob* pr) -> void* { return pr->zb; },
                             tol64_of, [](Prob* pr) { return pr->first; }))
      return e;
  }
  if (polish) tm.mark();

  // ---- Alg. 1 after the Jacobi on A - B (columns z_k = d_k v_k): the square
  // root S = Z diag(d^-3/2) Z^H and its inverse (one grouped launch), M = S (A + B) S,
  // and the Jacobi on M (as solve_sqrt)
  std::vector<JacState> states1;
  if (sqrt_route && !ok.empty()) {
    states1 = states;
    Grp<ColnormArgs<double2>> cn;
    Grp<SqrtScalesArgs> sq;
    std::vector<GemmDesc> sg, tg, mg;
    auto full = [](int np, const void* a, int opA, const void* b, int opB, void* c, const double* kscale,
                   const double* colscale) {
      GemmDesc g;
      g.M = np; g.N = np; g.K = np;
      g.A = a; g.lda = np; g.opA = opA;
      g.B = b; g.ldb = np; g.opB = opB;
      g.C = c; g.ldc = np;
      g.kscale = kscale;
      g.colscale = colscale;
      return g;
    };
    for (Prob* pr : ok) {
      const int np = pr->np;
      double2* M1 = pr->at<double2>(pr->p.off_m1);
      double2* M2 = pr->at<double2>(pr->p.off_m2);
      double2* Sb = pr->at<double2>(pr->p.off_w);
      double2* Si = pr->at<double2>(pr->p.off_y);
      double2* T = pr->at<double2>(pr->p.off_t);
      double* dC = pr->at<double>(pr->p.off_sigma);
      double* ks = pr->at<double>(pr->p.off_anorm);
      double* kis = pr->at<double>(pr->p.off_invlam);
      cn.add({M2, np, np, dC}, np);
      // ks, kis (c1, c2 redone after the second iteration)
      sq.add({pr->n, np, dC, dC, ks, kis, pr->at<double>(pr->p.off_scl), pr->at<double>(pr->p.off_ritz),
              pr->at<double>(pr->p.off_lamu)}, (np + 255) / 256);
      sg.push_back(full(np, M2, 0, M2, 1, Sb, ks, nullptr));   // S = Z diag(d^-3/2) Z^H
      sg.push_back(full(np, M2, 0, M2, 1, Si, kis, nullptr));  // S^-1 = Z diag(d^-5/2) Z^H
      tg.push_back(full(np, M1, 0, Sb, 0, T, nullptr, nullptr));  // T = M1 S
      mg.push_back(full(np, Sb, 0, T, 0, M1, nullptr, nullptr));  // M = S M1 S
    }
    BSE_TRY(run_op(ar, cn, group_finalize, G_COLNORM_Z, 0, s));
    BSE_TRY(run_op(ar, sq, group_finalize, G_SQRT_SCALES, 0, s));
    BSE_TRY(run_gemm<double>(ar, sg, s));
    BSE_TRY(run_gemm<double>(ar, tg, s));
    BSE_TRY(run_gemm<double>(ar, mg, s));
    auto tol_of = [&](Prob* pr) { return o.jacobi_tol > 0.0 ? o.jacobi_tol : default_tol64(pr->n); };
    if (int e = jacobi_phase(ok, false, max_sweeps, 1.0e-10, 0.0,
                             [](Prob* pr) -> void* { return pr->base + pr->p.off_m1; }, tol_of,
                             [](Prob*) { return 0.0; }))
      return e;
  }
  if (sqrt_route) tm.mark();

  // ---- finalize: scaled singular columns, Rayleigh quotients, back-transform
  if (!ok.empty()) {
    if (sqrt_route) {
      // Y = V_M D in M1: d = lambda^2, V1 = S^-1 Y d^-3/4, V2 = S Y d^-5/4
      Grp<ColnormArgs<double2>> cn;
      Grp<SqrtScalesArgs> sq;
      Grp<RankArgs> rk;
      Grp<WriteLambdaArgs> wl;
      Grp<AssembleArgs> as;
      std::vector<GemmDesc> vg;
      for (Prob* pr : ok) {
        const int np = pr->np;
        double2* M1 = pr->at<double2>(pr->p.off_m1);
        double2* M2 = pr->at<double2>(pr->p.off_m2);
        double2* Sb = pr->at<double2>(pr->p.off_w);
        double2* Si = pr->at<double2>(pr->p.off_y);
        double2* T = pr->at<double2>(pr->p.off_t);
        double* dC = pr->at<double>(pr->p.off_sigma);
        double* dM = pr->at<double>(pr->p.off_bnorm);
        double* c1 = pr->at<double>(pr->p.off_scl);
        double* c2 = pr->at<double>(pr->p.off_ritz);
        double* lamu = pr->at<double>(pr->p.off_lamu);
        int* perm = pr->at<int>(pr->p.off_perm);
        cn.add({M1, np, np, dM}, np);
        sq.add({pr->n, np, dC, dM, pr->at<double>(pr->p.off_anorm), pr->at<double>(pr->p.off_invlam), c1, c2,
                lamu}, (np + 255) / 256);
        rk.add({pr->n, lamu, perm, 0}, (pr->n + 255) / 256);
        wl.add({pr->n, lamu, perm, pr->lambda, o.want_negative}, (pr->n + 255) / 256);
        if (o.values_only) continue;
        GemmDesc g;
        g.M = np; g.N = np; g.K = np;
        g.A = Si; g.lda = np; g.opA = 0;
        g.B = M1; g.ldb = np; g.opB = 0;
        g.C = M2; g.ldc = np;
        g.colscale = c1;
        vg.push_back(g);  // V1 = S^-1 Y d^-3/4
        g.A = Sb; g.C = T; g.colscale = c2;
        vg.push_back(g);  // V2 = S Y d^-5/4
        as.add({pr->n, M2, T, np, perm, nullptr, pr->X, pr->ldx, o.want_negative, nullptr}, cols_blocks(pr->n, pr->n));
      }
      BSE_TRY(run_op(ar, cn, group_finalize, G_COLNORM_Z, 0, s));
      BSE_TRY(run_op(ar, sq, group_finalize, G_SQRT_SCALES, 0, s));
      BSE_TRY(run_op(ar, rk, group_finalize, G_RANK, 0, s));
      BSE_TRY(run_op(ar, wl, group_finalize, G_WRITE_LAMBDA, 0, s));
      tm.mark();
      BSE_TRY(run_gemm<double>(ar, vg, s));
      BSE_TRY(run_op(ar, as, group_finalize, G_ASSEMBLE, 0, s));
      tm.mark();
    } else if (tda) {
      // as the single solve: Y = A Z, Rayleigh quotients z^H A z / z^H z and
      // 1 / ||z||, sorted, X = [u; 0] (and [0; u]) with u = z / ||z||
      std::vector<GemmDesc> g;
      Grp<RqArgs> rq;
      Grp<RankArgs> rk;
      Grp<WriteLambdaArgs> wl;
      Grp<AssembleArgs> as;
      for (Prob* pr : ok) {
        const int np = pr->np;
        double2* M1 = pr->at<double2>(pr->p.off_m1);
        double2* W = pr->at<double2>(pr->p.off_w);
        double2* Y = pr->at<double2>(pr->p.off_y);
        int* perm = pr->at<int>(pr->p.off_perm);
        double* lamu = pr->at<double>(pr->p.off_lamu);
        double* scl = pr->at<double>(pr->p.off_scl);
        GemmDesc d;
        d.M = pr->n; d.N = pr->n; d.K = pr->n;
        d.A = M1; d.lda = np; d.opA = 0;
        d.B = W; d.ldb = np; d.opB = 0;
        d.C = Y; d.ldc = np;
        g.push_back(d);
        rq.add({pr->n, W, W, Y, Y, np, lamu, scl, nullptr}, pr->n);
        rk.add({pr->n, lamu, perm, 0}, (pr->n + 255) / 256);
        wl.add({pr->n, lamu, perm, pr->lambda, o.want_negative}, (pr->n + 255) / 256);
        if (!o.values_only)
          as.add({pr->n, W, W, np, perm, scl, pr->X, pr->ldx, o.want_negative, nullptr}, cols_blocks(pr->n, pr->n));
      }
      BSE_TRY(run_gemm<double>(ar, g, s));
      BSE_TRY(run_op(ar, rq, group_refine, G_RQ, 0, s));
      BSE_TRY(run_op(ar, rk, group_finalize, G_RANK, 0, s));
      BSE_TRY(run_op(ar, wl, group_finalize, G_WRITE_LAMBDA, 0, s));
      tm.mark();
      BSE_TRY(run_op(ar, as, group_finalize, G_ASSEMBLE, 0, s));
      tm.mark();
    } else if (alg2) {
      // Alg. 2 after its eigensolver, as the single solve: d = column norms of
      // the iterated M, lambda = sqrt(d) ascending, the sorted columns scaled
      // by Lambda^(1/2) and Lambda^(-1/2), V2 = L V_M Lambda^-1/2 and
      // V1 = L^-H V_M Lambda^1/2 by grouped block triangular solves
      Grp<ColnormArgs<double2>> cn;
      Grp<Alg2Args> al;
      Grp<RankArgs> rk;
      Grp<WriteLambdaArgs> wl;
      Grp<GatherArgs> ga;
      Grp<TriInvArgs> ti;
      Grp<AssembleArgs> as;
      std::vector<GemmDesc> v2;
      std::vector<TrsmStep> steps;
      for (Prob* pr : ok) {
        const int np = pr->np;
        double2* M1 = pr->at<double2>(pr->p.off_m1);
        double2* M2 = pr->at<double2>(pr->p.off_m2);
        double2* W = pr->at<double2>(pr->p.off_w);
        double2* Y = pr->at<double2>(pr->p.off_y);
        double2* inv = pr->at<double2>(pr->p.off_inv);
        double* d = pr->at<double>(pr->p.off_sigma);
        int* perm = pr->at<int>(pr->p.off_perm);
        double* lamu = pr->at<double>(pr->p.off_lamu);
        double* fx = pr->at<double>(pr->p.off_anorm);
        double* fy = pr->at<double>(pr->p.off_bnorm);
        cn.add({Y, np, np, d}, np);
        al.add({pr->n, d, lamu, perm, fx, fy}, (pr->n + 255) / 256);
        rk.add({pr->n, lamu, perm, 0}, (pr->n + 255) / 256);
        wl.add({pr->n, lamu, perm, pr->lambda, o.want_negative}, (pr->n + 255) / 256);
        if (o.values_only) continue;
        ga.add({pr->n, np, Y, np, perm, fx, M1}, cols_blocks(np, np));  // V_M Lambda^1/2 (sorted)
        ga.add({pr->n, np, Y, np, perm, fy, W}, cols_blocks(np, np));   // V_M Lambda^-1/2
        v2.push_back(tri_gemm(np, np, M2, 0, W, 0, 0, Y));             // V2 = L V_M Lambda^-1/2
        ti.add({M2, np, inv}, np / 64);
        trsm_lh_for_each(np, (const double2*)M2, np, M1, W, inv,
                         [&](const TrsmStep& st) { steps.push_back(st); });  // V1 = L^-H V_M Lambda^1/2
        as.add({pr->n, W, Y, np, nullptr, nullptr, pr->X, pr->ldx, o.want_negative, nullptr},
               cols_blocks(pr->n, pr->n));
      }
      BSE_TRY(run_op(ar, cn, group_finalize, G_COLNORM_Z, 0, s));
      BSE_TRY(run_op(ar, al, group_finalize, G_ALG2_LAMBDA, 0, s));
      BSE_TRY(run_op(ar, rk, group_finalize, G_RANK, 0, s));
      BSE_TRY(run_op(ar, wl, group_finalize, G_WRITE_LAMBDA, 0, s));
      BSE_TRY(run_op(ar, al, group_finalize, G_ALG2_SCALES, 0, s));
      BSE_TRY(run_op(ar, ga, group_finalize, G_GATHER, 0, s));
      tm.mark();
      BSE_TRY(run_gemm<double>(ar, v2, s));
      BSE_TRY(run_op(ar, ti, group_chol, G_TRIINV, 0, s));
      BSE_TRY(run_steps<double>(ar, steps, s));
      BSE_TRY(run_op(ar, as, group_finalize, G_ASSEMBLE, 0, s));
      tm.mark();
    } else if (mixed) {
      // Alg. 3 steps 4-5 in complex64 as in the single solve: V2 = L2 Ws,
      // T = L1^H V2 (Rayleigh quotients), V1 = L2^-H Ws / ||Ws||^2 by grouped
      // block triangular solves
      Grp<ColnormArgs<float2>> n1, n2, n3;
      Grp<ScaleArgs<float2>> sc;
      Grp<LambdaArgs> la;
      Grp<C64Args> cv;
      Grp<TriInvArgsT<float2>> ti;
      std::vector<GemmDesc> v2, t;
      std::vector<TrsmStep> steps;
      for (Prob* pr : ok) {
        const int np = pr->np;
        const size_t half = (size_t)np * np * sizeof(float2);
        float2* L1c = pr->at<float2>(pr->p.off_lc);
        float2* L2c = pr->at<float2>(pr->p.off_lc + half);
        float2* Wc = pr->at<float2>(pr->p.off_wc);
        float2* Yc = pr->at<float2>(pr->p.off_wc + half);
        float2* Tc = pr->at<float2>(pr->p.off_q);
        float2* invc = pr->at<float2>(pr->p.off_f);
        double* sigma = pr->at<double>(pr->p.off_sigma);
        double* bnorm = pr->at<double>(pr->p.off_bnorm);
        double* anorm = pr->at<double>(pr->p.off_anorm);
        double* invlam = pr->at<double>(pr->p.off_invlam);
        double* scl = pr->at<double>(pr->p.off_scl);
        n1.add({Wc, np, np, sigma}, np);
        sc.add({pr->n, np, Wc, np, sigma}, cols_blocks(np, np));
        n2.add({Wc, np, np, bnorm}, np);
        v2.push_back(tri_gemm(np, np, L2c, 0, Wc, 0, 0, Yc));  // V2 = L2 Ws
        t.push_back(tri_gemm(np, np, L1c, 1, Yc, 0, 0, Tc));   // T = L1^H V2
        n3.add({Tc, np, np, anorm}, np);
        la.add({pr->n, np, anorm, bnorm, pr->at<double>(pr->p.off_lamu), invlam, scl, 1}, (np + 255) / 256);
        ti.add({L2c, np, invc}, np / 64);
        trsm_lh_for_each(np, L2c, np, Wc, L1c, invc, [&](const TrsmStep& st) { steps.push_back(st); });
        cv.add({np, L1c, np, pr->at<double2>(pr->p.off_x1), np, scl}, cols_blocks(np, np));
        cv.add({np, Yc, np, pr->at<double2>(pr->p.off_x2), np, nullptr}, cols_blocks(np, np));
        pr->x = pr->at<double2>(pr->p.off_x1);
        pr->y = pr->at<double2>(pr->p.off_x2);
        pr->q = pr->at<double2>(pr->p.off_q);
        pr->f = pr->at<double2>(pr->p.off_f);
      }
      BSE_TRY(run_op(ar, n1, group_finalize, G_COLNORM_C, 0, s));
      BSE_TRY(run_op(ar, sc, group_finalize, G_SCALE_C, 0, s));
      BSE_TRY(run_op(ar, n2, group_finalize, G_COLNORM_C, 0, s));
      tm.mark();
      BSE_TRY(run_gemm<float>(ar, v2, s));
      BSE_TRY(run_gemm<float>(ar, t, s));
      BSE_TRY(run_op(ar, n3, group_finalize, G_COLNORM_C, 0, s));
      BSE_TRY(run_op(ar, la, group_finalize, G_LAMBDA, 0, s));
      BSE_TRY(run_op(ar, ti, group_chol, G_TRIINV_C, 0, s));
      BSE_TRY(run_steps<float>(ar, steps, s));
      BSE_TRY(run_op(ar, cv, group_finalize, G_C64, 0, s));
      tm.mark();

      // ---- FP64 Cholesky factors of M1, M2 (in place) for the refinement's
      // products, as the single solve; a problem whose factorisation fails
      // skips the refinement and is re-solved in FP64 below
      {
        std::vector<Prob*> all(ok.begin(), ok.end());
        const FactorFn fac = [](const Prob& pr, int f) -> void* {
          return pr.base + (f ? pr.p.off_m2 : pr.p.off_m1);
        };
        if (int e = cholesky_phase(all, 2, fac, [](const Prob& pr, int f) { return f ? pr.n : 0; }, false))
          return e;
        if (int e = read_statuses()) return e;
        for (Prob* pr : ok)
          if (pr->gst != kBig) {
            pr->status = pr->gst;
            pr->rdone = 1;
          }
      }

      // ---- FP64 refinement (as refine_z), each problem until its
      // first-order correction is small.  The pairs first go into the
      // ascending order of their eigenvalues, so that a window of the
      // Rayleigh-Ritz passes holds spectral neighbours.
      {
        Grp<RankArgs> rk0;
        Grp<GatherArgs> ga;
        for (Prob* pr : ok) {
          const int np = pr->np;
          int* perm = pr->at<int>(pr->p.off_perm);
          rk0.add({pr->n, pr->at<double>(pr->p.off_lamu), perm, 0}, (pr->n + 255) / 256);
          ga.add({pr->n, np, pr->x, np, perm, nullptr, pr->q}, cols_blocks(np, np));
          ga.add({pr->n, np, pr->y, np, perm, nullptr, pr->f}, cols_blocks(np, np));
        }
        BSE_TRY(run_op(ar, rk0, group_finalize, G_RANK, 0, s));
        BSE_TRY(run_op(ar, ga, group_finalize, G_GATHER, 0, s));
        for (Prob* pr : ok) {
          std::swap(pr->x, pr->q);
          std::swap(pr->y, pr->f);
        }
      }
      int* d_count = reinterpret_cast<int*>(d_corr + 2 * batch);
      const int max_steps = o.refine_steps > 0 ? o.refine_steps : 8;
      // window passes of a problem's current step, as refine_z: from the first
      // step with strongly coupled pairs on, unless the previous correction was small
      auto step_win = [](const Prob* pr) {
        return (pr->rsteps == 0 || pr->rcorr > kWindowStop) ? pr->rwin : 0;
      };
      for (int it = 0; it < max_steps; ++it) {
        std::vector<Prob*> act;
        for (Prob* pr : ok)
          if (!pr->rdone) act.push_back(pr);
        if (act.empty()) break;
        BSE_TRY(hipMemsetAsync(d_corr, 0, (size_t)2 * batch * sizeof(double), s));
        std::vector<GemmDesc> g00, g10, upd;
        Grp<MirrorArgs> mi;
        Grp<RitzArgs> rt;
        Grp<BuildArgs> bd;
        Grp<UpdRqArgs> ur;
        for (Prob* pr : act) {
          const int nn = pr->n;
          const long ld = pr->np;
          const double2* M1 = pr->at<double2>(pr->p.off_m1);
          const double2* M2 = pr->at<double2>(pr->p.off_m2);
          double2* P1 = pr->at<double2>(pr->p.off_p1);
          double2* P2 = pr->at<double2>(pr->p.off_p2);
          double2* Ex = pr->at<double2>(pr->p.off_lc);
          double2* Ey = pr->at<double2>(pr->p.off_wc);
          double* ritz = pr->at<double>(pr->p.off_ritz);
          auto nn_gemm = [&](const double2* a, int opA, const double2* b, int opB, double2* c) {
            GemmDesc d;
            d.M = nn; d.N = nn; d.K = nn;
            d.A = a; d.lda = ld; d.opA = opA;
            d.B = b; d.ldb = ld; d.opB = opB;
            d.C = c; d.ldc = ld;
            return d;
          };
          // M1, M2 hold the Cholesky factors L1, L2
          GemmDesc t2 = nn_gemm(M2, 1, pr->x, 0, pr->q);      // L2^H x
          t2.triA = 1;
          g00.push_back(t2);
          GemmDesc t1 = nn_gemm(M1, 1, pr->y, 0, Ex);         // L1^H y (Ex is free until k_build)
          t1.triA = 1;
          g00.push_back(t1);
          g10.push_back(nn_gemm(pr->x, 1, pr->y, 0, pr->f));  // F = x^H y
          GemmDesc p2 = nn_gemm(pr->q, 1, pr->q, 0, P2);      // P2 = x^H M2 x (lower tiles)
          p2.lowerC = 1;
          g10.push_back(p2);
          GemmDesc p1 = nn_gemm(Ex, 1, Ex, 0, P1);            // P1 = y^H M1 y (lower tiles)
          p1.lowerC = 1;
          g10.push_back(p1);
          mi.add({(int)ld, P2, ld}, tiles64((int)ld));
          mi.add({(int)ld, P1, ld}, tiles64((int)ld));
          rt.add({nn, pr->f, P1, P2, ld, ritz}, (nn + 255) / 256);
          const int T = (nn + 63) / 64;
          // q is free until the basis update: it takes the tile sums of the quotients
          double* part = reinterpret_cast<double*>(pr->q);
          bd.add({nn, pr->f, P1, P2, ld, ritz, Ex, Ey, kRefineDelta, d_corr + pr->idx, part}, T * T);
          ur.add({nn, ld, pr->f, P1, P2, part, pr->at<double>(pr->p.off_lamu), pr->at<double>(pr->p.off_scl),
                  d_corr + batch + pr->idx}, (nn + 255) / 256);
        }
        BSE_TRY(run_gemm<double>(ar, g00, s));
        BSE_TRY(run_gemm<double>(ar, g10, s));
        BSE_TRY(run_op(ar, mi, group_chol, G_MIRROR, 0, s));
        {
          // Rayleigh-Ritz windows for a problem from its first step whose
          // products couple a pair strongly on, as refine_z
          Grp<RitzArgs> r0;
          Grp<CoupleArgs> cp;
          for (Prob* pr : act) {
            if (pr->rwin) continue;
            const long ld = pr->np;
            double2* P1 = pr->at<double2>(pr->p.off_p1);
            double2* P2 = pr->at<double2>(pr->p.off_p2);
            double* ritz = pr->at<double>(pr->p.off_ritz);
            r0.add({pr->n, pr->f, P1, P2, ld, ritz}, (pr->n + 255) / 256);
            cp.add({pr->n, ld, pr->f, P1, P2, ritz, d_count + pr->idx}, (pr->n + 255) / 256);
          }
          if (cp.blocks() > 0) {
            BSE_TRY(hipMemsetAsync(d_count, 0, (size_t)batch * sizeof(int), s));
            BSE_TRY(run_op(ar, r0, group_refine, G_RITZ, 0, s));
            BSE_TRY(run_op(ar, cp, group_refine, G_COUPLE, 0, s));
            std::vector<int> counts(batch, 0);
            BSE_TRY(hipMemcpyAsync(counts.data(), d_count, (size_t)batch * sizeof(int), hipMemcpyDeviceToHost, s));
            BSE_TRY(hipStreamSynchronize(s));
            for (Prob* pr : act)
              if (!pr->rwin) pr->rwin = counts[pr->idx] > 0 ? kWindowPasses : 0;
          }
        }
        for (Prob* pr : act)
          if (step_win(pr) > 0) pr->rwsteps += 1;
        for (int pass = 0; pass < kWindowPasses; ++pass) {
          // Rayleigh-Ritz on windows of 64 pairs, boundaries alternately at 0 and at 32
          const int off = window_offset(pass);
          Grp<WinArgs> wn;
          std::vector<GemmDesc> right[3], left[3];
          for (Prob* pr : act) {
            if (pass >= step_win(pr)) continue;
            const long ld = pr->np;
            double2* Cb = window_blocks(pr->at<double2>(pr->p.off_cb0), pr->n, pass);
            double2* P1 = pr->at<double2>(pr->p.off_p1);
            double2* P2 = pr->at<double2>(pr->p.off_p2);
            wn.add({pr->n, ld, pr->f, P1, P2, off, Cb, nullptr}, window_count(pr->n, off));
            double2* mats[3] = {pr->f, P1, P2};
            for (int k = 0; k < 3; ++k) window_congruence(pr->n, ld, mats[k], pr->q, Cb, off, right[k], left[k]);
          }
          {
            Dev dv;
            BSE_TRY(stage(ar, wn, dv));
            BSE_TRY(group_window(dv.tab, dv.map, dv.blocks, s));
          }
          for (int k = 0; k < 3; ++k) {
            BSE_TRY(run_gemm<double>(ar, right[k], s));
            BSE_TRY(run_gemm<double>(ar, left[k], s));
          }
        }
        BSE_TRY(run_op(ar, rt, group_refine, G_RITZ, 0, s));
        BSE_TRY(run_op(ar, bd, group_refine, G_BUILD, 0, s));
        BSE_TRY(run_op(ar, ur, group_refine, G_UPDRQ, 0, s));
        // x <- x C_1 C_2 (I + E11 + E21), y <- y C_1 C_2 (I + E11 - E21)
        for (int pass = 0; pass < kWindowPasses; ++pass) {
          const int off = window_offset(pass);
          std::vector<GemmDesc> g;
          for (Prob* pr : act) {
            if (pass >= step_win(pr)) continue;
            const double2* Cb = window_blocks(pr->at<double2>(pr->p.off_cb0), pr->n, pass);
            window_right(pr->n, pr->np, pr->x, pr->q, Cb, off, g);
            window_right(pr->n, pr->np, pr->y, pr->f, Cb, off, g);
          }
          BSE_TRY(run_gemm<double>(ar, g, s));
          for (Prob* pr : act) {
            if (pass >= step_win(pr)) continue;
            std::swap(pr->x, pr->q);
            std::swap(pr->y, pr->f);
          }
        }
        // the step's corrections, known before the basis updates: as refine_z,
        // all but a problem's last step update in complex64
        std::vector<double> corr(2 * batch, 0.0);
        BSE_TRY(hipMemcpyAsync(corr.data(), d_corr, (size_t)2 * batch * sizeof(double), hipMemcpyDeviceToHost, s));
        BSE_TRY(hipStreamSynchronize(s));
        std::vector<char> low(batch, 0);
        Grp<LowArgs> lw;
        Grp<AddLowArgs> al;
        std::vector<GemmDesc> lowg;
        for (Prob* pr : act) {
          const int nn = pr->n;
          const long ld = pr->np;
          double2* Ex = pr->at<double2>(pr->p.off_lc);
          double2* Ey = pr->at<double2>(pr->p.off_wc);
          GemmDesc d;
          d.M = nn; d.N = nn; d.K = nn;
          d.lda = ld; d.opA = 0;
          d.ldb = ld; d.opB = 0;
          d.ldc = ld;
          low[pr->idx] = !(corr[pr->idx] <= kRefineStop || pr->rsteps + 1 == max_steps);
          if (low[pr->idx]) {
            // operands in q and f, products in Ex and Ey (two complex64 matrices in each)
            const int T = (nn + 63) / 64;
            const long half = ld * (long)nn;
            float2* xc = reinterpret_cast<float2*>(pr->q);
            float2* exc = reinterpret_cast<float2*>(pr->f);
            float2* px = reinterpret_cast<float2*>(Ex);
            float2* py = reinterpret_cast<float2*>(Ey);
            lw.add({nn, ld, {pr->x, pr->y, Ex, Ey}, {xc, xc + half, exc, exc + half}}, 4 * T * T);
            d.A = xc; d.B = exc; d.C = px;
            lowg.push_back(d);                               // x (Ex - I)
            d.A = xc + half; d.B = exc + half; d.C = py;
            lowg.push_back(d);                               // y (Ey - I)
            al.add({nn, ld, {px, py}, {pr->x, pr->y}}, 2 * T * T);
          } else {
            d.A = pr->x; d.B = Ex; d.C = pr->q;
            upd.push_back(d);                                // x (I + E11 + E21)
            d.A = pr->y; d.B = Ey; d.C = pr->f;
            upd.push_back(d);                                // y (I + E11 - E21)
          }
        }
        BSE_TRY(run_op(ar, lw, group_refine, G_LOW, 0, s));
        BSE_TRY(run_gemm<float>(ar, lowg, s));
        BSE_TRY(run_op(ar, al, group_refine, G_ADDLOW, 0, s));
        BSE_TRY(run_gemm<double>(ar, upd, s));
        for (Prob* pr : act) {
          if (!low[pr->idx]) {
            std::swap(pr->x, pr->q);
            std::swap(pr->y, pr->f);
          }
          if (pr->rsteps < 8) pr->rhist[pr->rsteps] = corr[pr->idx];
          pr->rsteps += 1;
          pr->rcorr = corr[pr->idx];
          pr->rbad = corr[batch + pr->idx] != 0.0;
          // the error left after a step is of the order of the square of its correction
          if (pr->rcorr <= kRefineStop) pr->rdone = 1;
        }
      }
      // sort and final setup (the last step left the quotients and scales);
      // a pair that broke down in the refinement fails the problem (it is then
      // re-solved in FP64)
      Grp<RankArgs> rk;
      Grp<WriteLambdaArgs> wl;
      Grp<AssembleArgs> as;
      for (Prob* pr : ok) {
        const int nn = pr->n;
        const long ld = pr->np;
        if (pr->rbad) pr->rcorr = __builtin_inf();
        double* lamu = pr->at<double>(pr->p.off_lamu);
        double* scl = pr->at<double>(pr->p.off_scl);
        int* perm = pr->at<int>(pr->p.off_perm);
        rk.add({nn, lamu, perm, 0}, (nn + 255) / 256);
        wl.add({nn, lamu, perm, pr->lambda, o.want_negative}, (nn + 255) / 256);
        if (!o.values_only)
          as.add({nn, pr->x, pr->y, ld, perm, scl, pr->X, pr->ldx, o.want_negative, nullptr},
                 cols_blocks(nn, nn));
      }
      BSE_TRY(run_op(ar, rk, group_finalize, G_RANK, 0, s));
      BSE_TRY(run_op(ar, wl, group_finalize, G_WRITE_LAMBDA, 0, s));
      BSE_TRY(run_op(ar, as, group_finalize, G_ASSEMBLE, 0, s));
      tm.mark();
    } else {
      // Alg. 3 steps 4-6 as in the single solve: Ws, V2 = L2 Ws, T = L1^H V2
      // (Rayleigh quotients), V1 = L2^-H Ws by grouped block triangular
      // solves, final setup.
      Grp<ColnormArgs<double2>> n1, n2, n3;
      Grp<ScaleArgs<double2>> sc;
      Grp<LambdaArgs> la;
      Grp<RankArgs> rk;
      Grp<WriteLambdaArgs> wl;
      Grp<AssembleArgs> as;
      Grp<TriInvArgs> ti;
      std::vector<GemmDesc> v2, t;
      std::vector<TrsmStep> steps;
      for (Prob* pr : ok) {
        const int np = pr->np;
        double2* M1 = pr->at<double2>(pr->p.off_m1);
        double2* M2 = pr->at<double2>(pr->p.off_m2);
        // the polished form: the columns of its FP64 sweeps, T in X2 (as back_transform_z)
        double2* W = polish ? pr->zb : pr->at<double2>(pr->p.off_w);
        double2* Y = pr->at<double2>(pr->p.off_y);
        double2* T = pr->at<double2>(polish ? pr->p.off_x2 : pr->p.off_t);
        double2* inv = pr->at<double2>(pr->p.off_inv);
        double* sigma = pr->at<double>(pr->p.off_sigma);
        double* bnorm = pr->at<double>(pr->p.off_bnorm);
        double* anorm = pr->at<double>(pr->p.off_anorm);
        double* invlam = pr->at<double>(pr->p.off_invlam);
        double* scl = pr->at<double>(pr->p.off_scl);
        double* lamu = pr->at<double>(pr->p.off_lamu);
        int* perm = pr->at<int>(pr->p.off_perm);
        n1.add({W, np, np, sigma}, np);
        sc.add({pr->n, np, W, np, sigma}, cols_blocks(np, np));
        n2.add({W, np, np, bnorm}, np);
        v2.push_back(tri_gemm(np, np, M2, 0, W, 0, 0, Y));  // V2 = L2 Ws
        t.push_back(tri_gemm(np, np, M1, 1, Y, 0, 0, T));   // T = L1^H V2
        n3.add({T, np, np, anorm}, np);
        la.add({pr->n, np, anorm, bnorm, lamu, invlam, scl, 1}, (np + 255) / 256);
        rk.add({pr->n, lamu, perm, 0}, (pr->n + 255) / 256);
        wl.add({pr->n, lamu, perm, pr->lambda, o.want_negative}, (pr->n + 255) / 256);
        if (o.values_only) continue;
        ti.add({M2, np, inv}, np / 64);
        trsm_lh_for_each(np, M2, np, W, T, inv, [&](const TrsmStep& st) { steps.push_back(st); });  // V1 = L2^-H Ws -> T
        as.add({pr->n, T, Y, np, perm, nullptr, pr->X, pr->ldx, o.want_negative, scl},
               cols_blocks(pr->n, pr->n));
      }
      BSE_TRY(run_op(ar, n1, group_finalize, G_COLNORM_Z, 0, s));
      BSE_TRY(run_op(ar, sc, group_finalize, G_SCALE_Z, 0, s));
      BSE_TRY(run_op(ar, n2, group_finalize, G_COLNORM_Z, 0, s));
      tm.mark();
      BSE_TRY(run_gemm<double>(ar, v2, s));
      BSE_TRY(run_gemm<double>(ar, t, s));
      BSE_TRY(run_op(ar, n3, group_finalize, G_COLNORM_Z, 0, s));
      BSE_TRY(run_op(ar, la, group_finalize, G_LAMBDA, 0, s));
      BSE_TRY(run_op(ar, rk, group_finalize, G_RANK, 0, s));
      BSE_TRY(run_op(ar, wl, group_finalize, G_WRITE_LAMBDA, 0, s));
      BSE_TRY(run_op(ar, ti, group_chol, G_TRIINV, 0, s));
      BSE_TRY(run_steps<double>(ar, steps, s));
      BSE_TRY(run_op(ar, as, group_finalize, G_ASSEMBLE, 0, s));
      tm.mark();
    }
  }
  BSE_TRY(hipStreamSynchronize(s));

  // ---- statuses and statistics
  int first = 0;
  std::vector<int> status(batch, 0);
  for (const Prob& pr : probs) {
    int st = pr.status;
    // the polished form: js is its complex64 iteration, jp its FP64 sweeps;
    // Alg. 1: js the iteration on A - B, jp the one on M
    const JacState& js = polish && !states32.empty() ? states32[pr.idx]
                         : (sqrt_route && !states1.empty() ? states1[pr.idx] : states[pr.idx]);
    const JacState& jp = states[pr.idx];
    // the complex64 iteration may end early (stop fraction): the refinement decides
    if (st == 0 && !(mixed ? js.sweeps > 0
                           : (polish ? js.sweeps > 0 && jp.converged
                                     : (sqrt_route ? js.converged && jp.converged : js.converged))))
      st = 2 * pr.n + 1;
    if (st == 0 && mixed && !(pr.rcorr <= 1.0e-4)) st = 2 * pr.n + 2;
    if (st != 0 && mixed) {
      // the complex64 stage could not carry this problem: re-solve it in FP64
      // on its own workspace region, as the single solve does
      bse_info_t tmp;
      memset(&tmp, 0, sizeof(tmp));
      st = solve_fp64_fallback(pr.n, pr.A, (int)pr.lda, pr.B, (int)pr.ldb, pr.lambda, pr.X,
                               (int)pr.ldx, pr.base, pr.p, o, &tmp, s);
      if (st <= kErrHip) return st;
      status[pr.idx] = st;
      if (info) {
        tmp.timing = info[pr.idx].timing;
        info[pr.idx] = tmp;
      }
      continue;
    }
    status[pr.idx] = st;
    if (info) {
      bse_info_t* inf = &info[pr.idx];
      inf->status = st;
      inf->fail_index = pr.status > 0 ? (pr.status > pr.n ? pr.status - pr.n : pr.status) : 0;
      inf->sweeps = js.sweeps;
      inf->rotations = js.rotations;
      inf->max_off = js.last_off;
      inf->pair_checks = (int)js.pair_checks;
      inf->cross_pair_checks = (int)js.cross_pair_checks;
      inf->inner_rotations = js.inner_rotations;
      if (sqrt_route) {  // both iterations together (the last one's level), as the single solve
        inf->sweeps += jp.sweeps;
        inf->rotations += jp.rotations;
        inf->max_off = jp.last_off;
        inf->pair_checks += (int)jp.pair_checks;
        inf->cross_pair_checks += (int)jp.cross_pair_checks;
        inf->inner_rotations += jp.inner_rotations;
      }
      inf->refine_delta = pr.rcorr;
      inf->refine_steps_done = pr.rsteps;
      inf->refine_window_steps = pr.rwsteps;
      for (int k = 0; k < 8; ++k) inf->refine_corr[k] = pr.rhist[k];
      if (polish && pr.status == 0) {
        inf->fallback = pr.fallback;
        inf->polish_sweeps = jp.sweeps;
        inf->polish_rotations = jp.rotations;
        inf->polish_pair_checks = (int)jp.pair_checks;
        inf->polish_cross_pair_checks = (int)jp.cross_pair_checks;
        inf->polish_max_off = jp.last_off;
        inf->polish_inner_rotations = jp.inner_rotations;
      }
    }
  }
  if (o.checks)
    for (const Prob& pr : probs) {
      if (status[pr.idx] != 0) continue;
      bse_info_t tmp;
      memset(&tmp, 0, sizeof(tmp));
      if (int e = run_checks(pr.n, pr.A, (int)pr.lda, pr.B, (int)pr.ldb, pr.lambda, pr.X, (int)pr.ldx,
                             pr.base, pr.p, o, &tmp, s))
        return e;
      if (info) {
        info[pr.idx].sigma_orth_fro = tmp.sigma_orth_fro;
        info[pr.idx].max_rel_resid = tmp.max_rel_resid;
      }
    }
  for (int i = 0; i < batch; ++i)
    if (status[i] != 0) { first = status[i]; break; }
  if (info && want_timing) {
    bse_info_t whole;
    memset(&whole, 0, sizeof(whole));
    tm.fill(&whole, slots);
    for (int i = 0; i < batch; ++i)
      for (int k = 0; k < 8; ++k) info[i].ms_phase[k] = whole.ms_phase[k];
  }
  return first;
}

}  // namespace bse
