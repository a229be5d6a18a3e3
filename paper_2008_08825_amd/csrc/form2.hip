// BSE matrices of form II (Eq. Hform2): H2 = [A B; -B^H -A^T], A Hermitian,
// B complex symmetric, the Hamiltonian Sigma H2 = [A B; conj(B) conj(A)]
// Hermitian positive definite.
//
// The paper characterises form II (Thm Form2) but gives no algorithm for it;
// it notes that real form-II matrices are treated with the idea of Alg. 3,
// and a real form-II matrix is a form-I matrix.  A complex one becomes a real
// form-I matrix of twice the order: writing A = Ar + i Ai, B = Br + i Bi and
// x = [u; v], the real vector z = [Re u; Im u; Re v; -Im v] satisfies
// H1' z = lambda z with
//   H1' = [A' B'; -B' -A'],  A' = [Ar -Ai; Ai Ar],  B' = [Br Bi; Bi -Br],
// both real symmetric (A Hermitian, B symmetric), and A' +- B' positive
// definite exactly when the Hamiltonian is (a real congruence of it).  Every
// eigenvalue of H2 appears twice in H1' (z and the image of i x), so the
// form-I solver (any route and precision) runs on (A', B') of order 2n, and
// eigenpair k of H2 is eigenvalue 2k of H1' with the complex vector of its
// eigenvector; the Sigma-normalisation carries over (z^T Sigma' z = x^H Sigma x).
// An eigenvalue of H2 of multiplicity m (numerically: a run of m eigenvalues
// whose gaps are below kClusterGap lambda_max) gives 2m equal eigenvalues of
// H1' whose 2m complex vectors span its m-dimensional eigenspace; a pivoted
// Gram-Schmidt in the Sigma inner product (positive definite on the
// eigenspaces of positive eigenvalues) picks m of them and makes them
// Sigma-orthonormal (runs of up to kClusterMax in one work group each; a
// longer run takes one grid-wide update launch and one selection launch per
// vector).
// The real solver makes its vectors orthogonal in the real inner product
// z^T Sigma' z' = Re(x^H Sigma x') only; the imaginary part pairs x with the
// image of i x', whose span the computed doubled pair matches only to the
// eigenvector accuracy (about eps / gap), so close eigenvalues leave the
// complex vectors Sigma-orthogonal only to that level.  One step
// X <- X (I - (X^H Sigma X - I) / 2) (three GEMMs, second order in the
// departure) restores Sigma-orthonormality to rounding; it mixes a vector
// only with others by amounts inverse to their gaps, so residuals stay at
// rounding level.  The negative half is written last from the final X.
#include "../../include/bse.h"
#include "common.hpp"
#include "internal.hpp"
#include "plan.hpp"

#include <math.h>
#include <string.h>

#include <vector>

namespace bse {
namespace {

// A' and B' (order 2n, both triangles, padding left to the form-I solver):
// one 64 x 64 tile of the 2n x 2n matrices per work group.
struct RealifyArgs {
  int n, upper; const double2* A; long lda; const double2* B; long ldb; double2* At; double2* Bt; long ld;
};
struct RealifyOp {
  static constexpr int NT = 256;
  typedef RealifyArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int m = 2 * a.n, T = (m + 63) / 64;
    const int i = (bx % T) * 64 + (threadIdx.x & 63), j0 = (bx / T) * 64 + (threadIdx.x >> 6);
    if (i >= m) return;
    const int bi = i >= a.n, ri = i - bi * a.n;
    for (int j = j0; j < j0 + 64 && j < m; j += 4) {
      const int bj = j >= a.n, rj = j - bj * a.n;
      // A[ri][rj] (Hermitian, real diagonal) and B[ri][rj] (symmetric) from the stored triangle
      const bool low = ri >= rj;
      const bool st = a.upper ? !low : low;  // element (ri, rj) itself is stored
      const int r = st ? ri : rj, c = st ? rj : ri;
      double2 av = a.A[r + (long)c * a.lda];
      if (!st) av.y = -av.y;
      if (ri == rj) av.y = 0.0;
      const double2 bv = a.B[r + (long)c * a.ldb];
      // A' = [Ar -Ai; Ai Ar], B' = [Br Bi; Bi -Br] (real, stored as complex128)
      const double at = bi == bj ? av.x : (bi ? av.y : -av.y);
      const double bt = bi != bj ? bv.y : (bi ? -bv.x : bv.x);
      a.At[i + (long)j * a.ld] = make_double2(at, 0.0);
      a.Bt[i + (long)j * a.ld] = make_double2(bt, 0.0);
    }
  }
};

// lambda_k = (lambda'_2k + lambda'_2k+1) / 2 and x_k from z = column 2k of
// X' (order 2n, positive half): u = z1 + i z2, v = z3 - i z4; with the
// negative half, -lambda_k.  Work group = (column k, 256 rows of x).
struct ExtractArgs {
  int n; const double* lam2; const double2* X2; long ldx2; double* lambda; double2* X; long ldx;
  int want_negative, values_only;
};
struct ExtractOp {
  static constexpr int NT = 256;
  typedef ExtractArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int n = a.n, gx = (2 * n + 255) / 256;
    const int k = bx / gx, r = (bx % gx) * 256 + threadIdx.x;
    if (k >= n) return;
    if (r == 0) {
      const double l = 0.5 * (a.lam2[2 * k] + a.lam2[2 * k + 1]);
      a.lambda[k] = l;
      if (a.want_negative) a.lambda[n + k] = -l;
    }
    if (a.values_only || r >= 2 * n) return;
    const double2* z = a.X2 + (long)(2 * k) * a.ldx2;
    const int q = r % n;
    double2 x;
    if (r < n) x = make_double2(z[q].x, z[n + q].x);              // u = Re part + i Im part
    else x = make_double2(z[2 * n + q].x, -z[3 * n + q].x);      // v = conj(w)
    a.X[r + (long)k * a.ldx] = x;
  }
};

constexpr double kClusterGap = 1.0e-12;
constexpr int kClusterMax = 64;

// Y[:, j] = complex vector of column j of X' (all 2n columns), for the runs of
// multiple eigenvalues.  Work group = (column j, 256 rows of x).
struct MapArgs { int n; const double2* X2; long ldx2; double2* Y; long ldy; };
struct MapOp {
  static constexpr int NT = 256;
  typedef MapArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int n = a.n, gx = (2 * n + 255) / 256;
    const int j = bx / gx, r = (bx % gx) * 256 + threadIdx.x;
    if (j >= 2 * n || r >= 2 * n) return;
    const double2* z = a.X2 + (long)j * a.ldx2;
    const int q = r % n;
    a.Y[r + (long)j * a.ldy] = r < n ? make_double2(z[q].x, z[n + q].x) : make_double2(z[2 * n + q].x, -z[3 * n + q].x);
  }
};

// One work group per run of m (2 <= m <= kClusterMax) eigenvalues of H2 that
// are numerically equal, starting at eigenvalue k0 (runs[w] = (k0, m)): among
// the 2m vectors Y[:, 2 k0 .. 2 k0 + 2m), m steps of pivoted Gram-Schmidt in
// the inner product <x, y> = x^H Sigma y take the candidate of largest
// remaining norm, normalise it into column k0 + t of X and remove it from the
// other candidates.
struct ClusterArgs { int n; const int2* runs; double2* Y; long ldy; double2* X; long ldx; };
struct ClusterOp {
  static constexpr int NT = 256;
  typedef ClusterArgs Args;
  static BSE_DEV void run(const Args& a, int w, int) {
    __shared__ double red[2][NT];
    __shared__ double nrm[2 * kClusterMax];
    __shared__ int alive[2 * kClusterMax];
    __shared__ int piv;
    const int n = a.n, rows = 2 * n, tid = threadIdx.x;
    const int k0 = a.runs[w].x, m = a.runs[w].y, c0 = 2 * k0, nc = 2 * m;
    for (int c = tid; c < nc; c += NT) alive[c] = 1;
    __syncthreads();
    // sum over rows r of f(r) by the whole work group, result in red[0][0]
    auto reduce2 = [&](double vr, double vi) {
      red[0][tid] = vr;
      red[1][tid] = vi;
      __syncthreads();
      for (int o = NT / 2; o > 0; o >>= 1) {
        if (tid < o) {
          red[0][tid] += red[0][tid + o];
          red[1][tid] += red[1][tid + o];
        }
        __syncthreads();
      }
    };
    for (int t = 0; t < m; ++t) {
      // Sigma-norms of the candidates left
      for (int c = 0; c < nc; ++c) {
        if (!alive[c]) continue;  // uniform: alive is in LDS, read after a barrier
        const double2* y = a.Y + (long)(c0 + c) * a.ldy;
        double sacc = 0.0;
        for (int r = tid; r < rows; r += NT) {
          const double2 v = y[r];
          const double q = v.x * v.x + v.y * v.y;
          sacc += r < n ? q : -q;
        }
        reduce2(sacc, 0.0);
        if (tid == 0) nrm[c] = red[0][0];
        __syncthreads();
      }
      if (tid == 0) {
        int best = -1;
        for (int c = 0; c < nc; ++c)
          if (alive[c] && (best < 0 || nrm[c] > nrm[best])) best = c;
        piv = best;
        alive[best] = 0;
      }
      __syncthreads();
      const int p = piv;
      const double inv = nrm[p] > 0.0 ? 1.0 / sqrt(nrm[p]) : 0.0;
      double2* q = a.Y + (long)(c0 + p) * a.ldy;
      for (int r = tid; r < rows; r += NT) {
        double2 v = q[r];
        v.x *= inv;
        v.y *= inv;
        q[r] = v;
        a.X[r + (long)(k0 + t) * a.ldx] = v;
      }
      __syncthreads();
      // remove q from the other candidates: y <- y - (q^H Sigma y) q
      for (int c = 0; c < nc; ++c) {
        if (!alive[c]) continue;
        double2* y = a.Y + (long)(c0 + c) * a.ldy;
        double cr = 0.0, ci = 0.0;
        for (int r = tid; r < rows; r += NT) {
          const double2 qv = q[r], v = y[r];
          const double sg = r < n ? 1.0 : -1.0;
          cr += sg * (qv.x * v.x + qv.y * v.y);
          ci += sg * (qv.x * v.y - qv.y * v.x);
        }
        reduce2(cr, ci);
        const double2 cf = make_double2(red[0][0], red[1][0]);
        __syncthreads();
        for (int r = tid; r < rows; r += NT) {
          const double2 qv = q[r];
          double2 v = y[r];
          v.x -= cf.x * qv.x - cf.y * qv.y;
          v.y -= cf.x * qv.y + cf.y * qv.x;
          y[r] = v;
        }
        __syncthreads();
      }
    }
  }
};

// The same selection for a run longer than kClusterMax, spread over the
// chip: per step, PivUpdOp (one work group per candidate) removes the last
// chosen vector q from every live candidate and recomputes its Sigma-norm
// (first = 1: only the norms), and PivSelOp (one work group) takes the live
// candidate of largest norm, normalises it into Y (the next q) and into
// column k0 + t of X.  nrm / alive / piv live in the workspace.
struct PivArgs {
  int n; double2* Y; long ldy; int c0, nc; double* nrm; int* alive; int* piv; double2* X; long ldx;
  int col, first;
};
BSE_DEV void wg_sum2(double (&red)[2][256], double& vr, double& vi) {
  const int tid = threadIdx.x;
  red[0][tid] = vr;
  red[1][tid] = vi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      red[0][tid] += red[0][tid + o];
      red[1][tid] += red[1][tid + o];
    }
    __syncthreads();
  }
  vr = red[0][0];
  vi = red[1][0];
  __syncthreads();
}
struct PivUpdOp {
  static constexpr int NT = 256;
  typedef PivArgs Args;
  static BSE_DEV void run(const Args& a, int c, int) {
    __shared__ double red[2][NT];
    const int n = a.n, rows = 2 * n, tid = threadIdx.x;
    if (c >= a.nc) return;
    if (a.first) {
      if (tid == 0) a.alive[c] = 1;
    } else if (!a.alive[c]) {
      return;  // uniform: one value per work group
    }
    double2* y = a.Y + (long)(a.c0 + c) * a.ldy;
    double cr = 0.0, ci = 0.0;
    if (!a.first) {
      const double2* q = a.Y + (long)(a.c0 + a.piv[0]) * a.ldy;
      for (int r = tid; r < rows; r += NT) {
        const double2 qv = q[r], v = y[r];
        const double sg = r < n ? 1.0 : -1.0;
        cr += sg * (qv.x * v.x + qv.y * v.y);
        ci += sg * (qv.x * v.y - qv.y * v.x);
      }
      wg_sum2(red, cr, ci);
    }
    double s = 0.0, s_im = 0.0;
    for (int r = tid; r < rows; r += NT) {
      double2 v = y[r];
      if (!a.first) {
        const double2 qv = a.Y[(long)(a.c0 + a.piv[0]) * a.ldy + r];
        v.x -= cr * qv.x - ci * qv.y;
        v.y -= cr * qv.y + ci * qv.x;
        y[r] = v;
      }
      const double w = v.x * v.x + v.y * v.y;
      s += r < n ? w : -w;
    }
    wg_sum2(red, s, s_im);
    if (tid == 0) a.nrm[c] = s;
  }
};
struct PivSelOp {
  static constexpr int NT = 256;
  typedef PivArgs Args;
  static BSE_DEV void run(const Args& a, int, int) {
    __shared__ double bv[NT];
    __shared__ int bi[NT];
    const int tid = threadIdx.x, rows = 2 * a.n;
    double best = -1.0e300;
    int arg = -1;
    for (int c = tid; c < a.nc; c += NT)
      if (a.alive[c] && a.nrm[c] > best) {
        best = a.nrm[c];
        arg = c;
      }
    bv[tid] = best;
    bi[tid] = arg;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
      if (tid < o && (bv[tid + o] > bv[tid] || (bv[tid + o] == bv[tid] && bi[tid + o] >= 0 &&
                                                 (bi[tid] < 0 || bi[tid + o] < bi[tid])))) {
        bv[tid] = bv[tid + o];
        bi[tid] = bi[tid + o];
      }
      __syncthreads();
    }
    const int p = bi[0];
    if (p < 0) return;  // no live candidate (cannot happen for nc = 2 m, m steps)
    const double inv = bv[0] > 0.0 ? 1.0 / sqrt(bv[0]) : 0.0;
    double2* q = a.Y + (long)(a.c0 + p) * a.ldy;
    for (int r = tid; r < rows; r += NT) {
      double2 v = q[r];
      v.x *= inv;
      v.y *= inv;
      q[r] = v;
      a.X[r + (long)a.col * a.ldx] = v;
    }
    if (tid == 0) {
      a.piv[0] = p;
      a.alive[p] = 0;
    }
  }
};

// E <- E - I (E is n x n, column-major with leading dimension n).
struct DiagArgs { int n; double2* E; };
struct DiagOp {
  static constexpr int NT = 256;
  typedef DiagArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int j = bx * NT + threadIdx.x;
    if (j < a.n) a.E[j + (long)j * a.n].x -= 1.0;
  }
};

// Negative half (Lemma ComputeNegEvecs, part 2): column n + k of X is
// [0 I; I 0] conj(x_k), row r of x_k going to row r +- n, conjugated.
// Work group = (column k, 256 rows).
struct NegArgs { int n; double2* X; long ldx; };
struct NegOp {
  static constexpr int NT = 256;
  typedef NegArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int n = a.n, gx = (2 * n + 255) / 256;
    const int k = bx / gx, r = (bx % gx) * 256 + threadIdx.x;
    if (k >= n || r >= 2 * n) return;
    const double2 v = a.X[r + (long)k * a.ldx];
    const int rn = r < n ? r + n : r - n;
    a.X[rn + (long)(n + k) * a.ldx] = make_double2(v.x, -v.y);
  }
};

// opts.checks: the real vectors of the order-2n problem for the measurement,
// Z[:, 2k] = z(x_k) and Z[:, 2k + 1] = z(i x_k), z(x) = [Re u; Im u; Re v;
// -Im v] for x = [u; v] (complex128 storage, zero imaginary parts), and
// their eigenvalues lam2[2k] = lam2[2k + 1] = lambda_k.  Work group =
// (column k, 256 rows of x).
struct ZArgs { int n; const double2* X; long ldx; const double* lambda; double2* Z; long ldz; double* lam2; };
struct ZOp {
  static constexpr int NT = 256;
  typedef ZArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int n = a.n, gx = (2 * n + 255) / 256;
    const int k = bx / gx, r = (bx % gx) * 256 + threadIdx.x;
    if (k >= n || r >= 2 * n) return;
    if (r == 0) a.lam2[2 * k] = a.lam2[2 * k + 1] = a.lambda[k];
    const double2 x = a.X[r + (long)k * a.ldx];
    double2* z0 = a.Z + (long)(2 * k) * a.ldz;
    double2* z1 = z0 + a.ldz;
    // x -> (Re, Im) rows of u (r < n) or (Re, -Im) rows of v; i x = (-Im x, Re x)
    const int q = r < n ? r : r + n;  // row of the real part: u at 0.., v at 2n..
    const double s = r < n ? 1.0 : -1.0;
    z0[q] = make_double2(x.x, 0.0);
    z0[q + n] = make_double2(s * x.y, 0.0);
    z1[q] = make_double2(-x.y, 0.0);
    z1[q + n] = make_double2(s * x.x, 0.0);
  }
};

struct H2Layout {
  size_t off_at = 0, off_bt = 0, off_lam = 0, off_x = 0, off_runs = 0, off_inner = 0;
};

H2Layout h2_layout(int n, const bse_opts_t& o) {
  H2Layout L;
  const size_t m = (size_t)2 * n;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t at = off;
    off = align256(off + b);
    return at;
  };
  L.off_at = take(m * m * sizeof(double2));
  L.off_bt = take(m * m * sizeof(double2));
  L.off_lam = take(m * sizeof(double));
  L.off_x = take(o.values_only ? 0 : 2 * m * m * sizeof(double2));
  L.off_runs = take((size_t)(n + 1) * sizeof(int2));
  L.off_inner = take(0);
  return L;
}

// Options of the order-2n solve; `ws` keeps opts.checks for the workspace
// plan (its measurement buffers serve the form-II measurement afterwards).
bse_opts_t inner_opts(const bse_opts_t& o, bool ws = false) {
  bse_opts_t io = o;
  io.uplo = 'L';
  io.want_negative = 0;
  io.checks = ws ? o.checks : 0;
  return io;
}

}  // namespace
}  // namespace bse

extern "C" {

size_t bse_workspace_bytes_h2(int n, const bse_opts_t* opts) {
  bse_opts_t o;
  bse_default_opts(&o);
  if (opts) o = *opts;
  if (n < 0 || n > 23000 || !bse::opts_valid(o) || o.route == BSE_ROUTE_TDA) return 0;
  const bse::H2Layout L = bse::h2_layout(n, o);
  const bse_opts_t io = bse::inner_opts(o, true);
  const size_t inner = bse_workspace_bytes(2 * n, &io);
  if (inner == 0) return 0;
  return L.off_inner + inner + 256;
}

int bse_solve_h2(int n, const void* A, int lda, const void* B, int ldb, double* lambda, void* X,
                 int ldx, void* work, size_t work_bytes, const bse_opts_t* opts, bse_info_t* info,
                 void* stream) {
  bse_opts_t o;
  bse_default_opts(&o);
  if (opts) o = *opts;
  if (n < 0 || n > 23000) return -1;
  if (n > 0 && !A) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (n > 0 && !B) return -4;
  if (ldb < (n > 1 ? n : 1)) return -5;
  if (n > 0 && !lambda) return -6;
  if (n > 0 && !X && !o.values_only) return -7;
  if (!o.values_only && ldx < (2 * n > 1 ? 2 * n : 1)) return -8;
  if (!bse::opts_valid(o) || o.route == BSE_ROUTE_TDA) return -11;
  if (n == 0) return 0;
  const size_t need = bse_workspace_bytes_h2(n, &o);
  if (!work) return -9;
  if (work_bytes < need) return -10;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(work) + 255) & ~(uintptr_t)255);
  const bse::H2Layout L = bse::h2_layout(n, o);
  const int m = 2 * n;
  double2* At = reinterpret_cast<double2*>(base + L.off_at);
  double2* Bt = reinterpret_cast<double2*>(base + L.off_bt);
  double* lam2 = reinterpret_cast<double*>(base + L.off_lam);
  double2* X2 = o.values_only ? nullptr : reinterpret_cast<double2*>(base + L.off_x);
  const int upper = (o.uplo == 'U' || o.uplo == 'u');
  const bse::RealifyArgs ra = {n, upper, static_cast<const double2*>(A), lda, static_cast<const double2*>(B),
                               ldb, At, Bt, m};
  const int T = (m + 63) / 64;
  hipError_t e = launch_one<bse::RealifyOp>(ra, T * T, 0, s);
  if (e != hipSuccess) return bse::hip_status(e);
  const bse_opts_t io = bse::inner_opts(o);
  const int st = bse_solve_h1(m, At, m, Bt, m, lam2, X2, m > 0 ? 2 * m : 1, base + L.off_inner,
                              work_bytes - (size_t)(base - static_cast<char*>(work)) - L.off_inner, &io,
                              info, stream);
  if (st != 0) return st;
  const bse::ExtractArgs ea = {n, lam2, X2, 2 * m, lambda, static_cast<double2*>(X), ldx, o.want_negative,
                               o.values_only};
  e = launch_one<bse::ExtractOp>(ea, n * ((2 * n + 255) / 256), 0, s);
  if (e != hipSuccess) return bse::hip_status(e);
  std::vector<int2> runs;  // lives until the final synchronisation (copied from)
  std::vector<int2> long_runs;
  if (!o.values_only && n > 1) {
    // runs of numerically equal eigenvalues of H2 (pairs k, k + 1 joined when
    // the gap between copies 2k + 1 and 2k + 2 is below kClusterGap lambda_max)
    std::vector<double> l2(m);
    e = hipMemcpyAsync(l2.data(), lam2, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bse::hip_status(e);
    const double tol = bse::kClusterGap * fabs(l2[m - 1]);
    for (int k = 0; k < n;) {
      int e1 = k + 1;
      while (e1 < n && l2[2 * e1] - l2[2 * e1 - 1] <= tol) ++e1;
      if (e1 - k >= 2 && e1 - k <= bse::kClusterMax) runs.push_back(make_int2(k, e1 - k));
      if (e1 - k > bse::kClusterMax) long_runs.push_back(make_int2(k, e1 - k));
      k = e1;
    }
    if (!runs.empty() || !long_runs.empty()) {
      const bse::MapArgs ma = {n, X2, 2 * m, At, m};  // A' is free: Y in its place (2n x 2n)
      e = launch_one<bse::MapOp>(ma, m * ((2 * n + 255) / 256), 0, s);
      if (e != hipSuccess) return bse::hip_status(e);
    }
    if (!runs.empty()) {
      int2* d_runs = reinterpret_cast<int2*>(base + L.off_runs);
      e = hipMemcpyAsync(d_runs, runs.data(), runs.size() * sizeof(int2), hipMemcpyHostToDevice, s);
      const bse::ClusterArgs ca = {n, d_runs, At, m, static_cast<double2*>(X), ldx};
      if (e == hipSuccess) e = launch_one<bse::ClusterOp>(ca, (int)runs.size(), 0, s);
      if (e != hipSuccess) return bse::hip_status(e);
    }
    // longer runs: norms, live flags and the pivot in B's place (2n + 2n + 1 words)
    double* nrm = reinterpret_cast<double*>(Bt);
    int* alive = reinterpret_cast<int*>(nrm + m);
    int* piv = alive + m;
    for (const int2& r : long_runs) {
      bse::PivArgs pa = {n, At, m, 2 * r.x, 2 * r.y, nrm, alive, piv, static_cast<double2*>(X), ldx, r.x, 1};
      e = launch_one<bse::PivUpdOp>(pa, pa.nc, 0, s);
      for (int t = 0; t < r.y && e == hipSuccess; ++t) {
        pa.col = r.x + t;
        e = launch_one<bse::PivSelOp>(pa, 1, 0, s);
        pa.first = 0;
        if (e == hipSuccess && t + 1 < r.y) e = launch_one<bse::PivUpdOp>(pa, pa.nc, 0, s);
      }
      if (e != hipSuccess) return bse::hip_status(e);
    }
  }
  if (!o.values_only) {
    // X <- X - X E / 2 with E = X^H Sigma X - I: Xc = copy of X in A's place
    // (2n x n), E in B's place (n x n), both free once the solve is done
    double2* Xp = static_cast<double2*>(X);
    double2* Xc = At;
    double2* E = Bt;
    e = hipMemcpy2DAsync(Xc, (size_t)m * sizeof(double2), Xp, (size_t)ldx * sizeof(double2),
                         (size_t)m * sizeof(double2), n, hipMemcpyDeviceToDevice, s);
    bse::GemmDesc g;
    g.M = n; g.N = n; g.K = n;
    g.A = Xc; g.lda = m; g.opA = 1;
    g.B = Xc; g.ldb = m; g.opB = 0;
    g.C = E; g.ldc = n;
    if (e == hipSuccess) e = bse::gemm_z(g, s);  // u^H u
    g.A = Xc + n; g.B = Xc + n;
    g.alpha_re = -1.0; g.beta_re = 1.0;
    if (e == hipSuccess) e = bse::gemm_z(g, s);  // - v^H v
    const bse::DiagArgs da = {n, E};
    if (e == hipSuccess) e = launch_one<bse::DiagOp>(da, (n + 255) / 256, 0, s);
    bse::GemmDesc h;
    h.M = m; h.N = n; h.K = n;
    h.A = Xc; h.lda = m; h.opA = 0;
    h.B = E; h.ldb = n; h.opB = 0;
    h.C = Xp; h.ldc = ldx;
    h.alpha_re = -0.5; h.beta_re = 1.0;
    if (e == hipSuccess) e = bse::gemm_z(h, s);
    const bse::NegArgs na = {n, Xp, ldx};
    if (e == hipSuccess && o.want_negative) e = launch_one<bse::NegOp>(na, n * ((2 * n + 255) / 256), 0, s);
    if (e != hipSuccess) return bse::hip_status(e);
  }
  if (o.checks && !o.values_only) {
    // measure on the order-2n problem: (A', B') formed again, Z = [z(x_k),
    // z(i x_k)] in X's place; the real Sigma'-Gram of Z is a real form of
    // X^H Sigma X (Frobenius norm sqrt(2) times), the residuals are those of
    // the x_k; the form-I measurement's buffers are in the order-2n workspace
    e = launch_one<bse::RealifyOp>(ra, T * T, 0, s);
    const bse::ZArgs za = {n, static_cast<const double2*>(X), ldx, lambda, X2, 2 * m, lam2};
    if (e == hipSuccess) e = launch_one<bse::ZOp>(za, n * ((2 * n + 255) / 256), 0, s);
    if (e != hipSuccess) return bse::hip_status(e);
    const bse_opts_t iw = bse::inner_opts(o, true);
    const bse::Plan P = bse::make_plan(m, iw);
    bse_info_t ci;
    memset(&ci, 0, sizeof(ci));
    const int cst = bse::run_checks(m, At, m, Bt, m, lam2, X2, 2 * m, base + L.off_inner, P, iw, &ci, s);
    if (cst != 0) return cst;
    if (info) {
      info->sigma_orth_fro = ci.sigma_orth_fro / sqrt(2.0);
      info->max_rel_resid = ci.max_rel_resid;
    }
  }
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return bse::hip_status(e);
  return 0;
}

}  // extern "C"
