// Measurements of returned eigenpairs (opts.checks): Sigma-orthogonality and
// the largest relative residual, from the caller's A, B and the returned X.
//
// With X = [a; b] (columns Sigma-normalised eigenvectors of H1) and the (x, y)
// coordinates of the proof of Thm ProdEig, V1 = a - b and V2 = a + b:
//   X^H Sigma X = a^H a - b^H b = (V1^H V2 + V2^H V1) / 2,
//   H1 x_k - lambda_k x_k = 1/2 [r2 + r1; r2 - r1],  r1 = M1 V2_k - lambda_k V1_k,
//                                                   r2 = M2 V1_k - lambda_k V2_k,
// so ||H1 x_k - lambda_k x_k||^2 = (||r1||^2 + ||r2||^2) / 2 and
// ||x_k||^2 = (||V1_k||^2 + ||V2_k||^2) / 2, with M1 = A + B, M2 = A - B
// (Lemma Qtransform).  Work: three n x n complex products (M1 V2, M2 V1,
// V1^H V2) and column and tile reductions in a fixed order (deterministic).
#include "common.hpp"
#include "internal.hpp"

namespace bse {
namespace {

// V1 = a - b, V2 = a + b (np x np, zero outside the leading n x n block);
// work group = (column, 256 rows).
struct SplitArgs { int n, np; const double2* X; long ldx; double2* V1; double2* V2; };
struct SplitOp {
  static constexpr int NT = 256;
  typedef SplitArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int gx = (a.np + 255) / 256;
    const int k = bx / gx;
    const int i = (bx % gx) * 256 + threadIdx.x;
    if (i >= a.np) return;
    double2 v1 = make_double2(0.0, 0.0), v2 = v1;
    if (i < a.n && k < a.n) {
      const double2 top = a.X[i + (long)k * a.ldx];
      const double2 bot = a.X[a.n + i + (long)k * a.ldx];
      v1 = csub(top, bot);
      v2 = cadd(top, bot);
    }
    a.V1[i + (long)k * a.np] = v1;
    a.V2[i + (long)k * a.np] = v2;
  }
};

// acc[k] (+)= ||R_k - lambda_k V_k||^2 over the first n rows; with vn set,
// also vn[k] = ||V1_k||^2 + ||V2_k||^2.  Work group = column.
struct ColResArgs {
  int n; long ld; const double2* R; const double2* V; const double* lambda; double* acc; int add;
  const double2* V1; const double2* V2; double* vn;
};
struct ColResOp {
  static constexpr int NT = 256;
  typedef ColResArgs Args;
  static BSE_DEV void run(const Args& a, int k, int) {
    __shared__ double red[2][256];
    const int tid = threadIdx.x;
    const double lam = a.lambda[k];
    double r = 0.0, v = 0.0;
    for (int i = tid; i < a.n; i += 256) {
      const long e = i + (long)k * a.ld;
      const double2 d = csub(a.R[e], cscale(a.V[e], lam));
      r += cabs2(d);
      if (a.vn) v += cabs2(a.V1[e]) + cabs2(a.V2[e]);
    }
    red[0][tid] = r;
    red[1][tid] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) {
        red[0][tid] += red[0][tid + h];
        red[1][tid] += red[1][tid + h];
      }
      __syncthreads();
    }
    if (tid == 0) {
      a.acc[k] = a.add ? a.acc[k] + red[0][0] : red[0][0];
      if (a.vn) a.vn[k] = red[1][0];
    }
  }
};

// part[t] = sum over the 64 x 64 tile t of |(F_ij + conj(F_ji)) / 2 - delta_ij|^2.
struct OrthArgs { int n; long ld; const double2* F; double* part; };
struct OrthOp {
  static constexpr int NT = 256;
  typedef OrthArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    __shared__ double red[256];
    const int T = (a.n + 63) / 64;
    const int ti = bx % T, tj = bx / T;
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int e = tid; e < 64 * 64; e += 256) {
      const int i = ti * 64 + (e & 63), j = tj * 64 + (e >> 6);
      if (i >= a.n || j >= a.n) continue;
      const double2 fij = a.F[i + (long)j * a.ld];
      const double2 fji = a.F[j + (long)i * a.ld];
      double re = 0.5 * (fij.x + fji.x) - (i == j ? 1.0 : 0.0);
      double im = 0.5 * (fij.y - fji.y);
      s += re * re + im * im;
    }
    red[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) a.part[bx] = red[0];
  }
};

// out[0] = sqrt(sum of part[0..tiles)), out[1] = max_k sqrt(res[k] / vn[k]) / lambda_max.
struct FinishArgs {
  int n, tiles; const double* part; const double* res; const double* vn; const double* lambda;
  double* out;
};
struct FinishOp {
  static constexpr int NT = 256;
  typedef FinishArgs Args;
  static BSE_DEV void run(const Args& a, int, int) {
    __shared__ double red[2][256];
    const int tid = threadIdx.x;
    double s = 0.0, m = 0.0, lmax = 0.0;
    for (int t = tid; t < a.tiles; t += 256) s += a.part[t];
    for (int k = tid; k < a.n; k += 256) {
      lmax = fmax(lmax, fabs(a.lambda[k]));
      const double r = a.vn[k] > 0.0 ? sqrt(a.res[k] / a.vn[k]) : 0.0;
      m = fmax(m, r);
    }
    red[0][tid] = s;
    red[1][tid] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) {
        red[0][tid] += red[0][tid + h];
        red[1][tid] = fmax(red[1][tid], red[1][tid + h]);
      }
      __syncthreads();
    }
    // lambda_max: the largest |lambda| over the whole block
    __shared__ double lm[256];
    lm[tid] = lmax;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) lm[tid] = fmax(lm[tid], lm[tid + h]);
      __syncthreads();
    }
    if (tid == 0) {
      a.out[0] = sqrt(red[0][0]);
      a.out[1] = lm[0] > 0.0 ? red[1][0] / lm[0] : 0.0;
    }
  }
};

GemmDesc full_nn(int n, long ld, const double2* A, int opA, const double2* B, double2* C) {
  GemmDesc g;
  g.M = n; g.N = n; g.K = n;
  g.A = A; g.lda = ld; g.opA = opA;
  g.B = B; g.ldb = ld; g.opB = 0;
  g.C = C; g.ldc = ld;
  return g;
}

}  // namespace

size_t check_small_bytes(int n) {
  const int T = (n + 63) / 64;
  return (size_t)(2 * n + T * T + 2) * sizeof(double);
}

hipError_t check_pairs_z(int n, int np, const double2* A, long lda, const double2* B, long ldb,
                         int upper, const double* lambda, const double2* X, long ldx,
                         double2* const bufs[5], double* small, double out[2], hipStream_t s) {
  double2* M1 = bufs[0];
  double2* M2 = bufs[1];
  double2* V1 = bufs[2];
  double2* V2 = bufs[3];
  double2* R = bufs[4];
  const long ld = np;
  const int T = (n + 63) / 64;
  double* res = small;
  double* vn = small + n;
  double* part = small + 2 * n;
  double* dout = part + T * T;
  hipError_t e = form_m12(n, np, A, lda, B, ldb, upper, M1, M2, ld, s);
  if (e == hipSuccess) e = mirror_upper_z(np, M1, ld, s);
  if (e == hipSuccess) e = mirror_upper_z(np, M2, ld, s);
  const SplitArgs sa = {n, np, X, ldx, V1, V2};
  if (e == hipSuccess) e = launch_one<SplitOp>(sa, cols_blocks(np, np), 0, s);
  if (e == hipSuccess) e = gemm_z(full_nn(n, ld, M1, 0, V2, R), s);  // M1 V2
  const ColResArgs c1 = {n, ld, R, V1, lambda, res, 0, V1, V2, vn};
  if (e == hipSuccess) e = launch_one<ColResOp>(c1, n, 0, s);
  if (e == hipSuccess) e = gemm_z(full_nn(n, ld, M2, 0, V1, R), s);  // M2 V1
  const ColResArgs c2 = {n, ld, R, V2, lambda, res, 1, nullptr, nullptr, nullptr};
  if (e == hipSuccess) e = launch_one<ColResOp>(c2, n, 0, s);
  if (e == hipSuccess) e = gemm_z(full_nn(n, ld, V1, 1, V2, R), s);  // F = V1^H V2
  const OrthArgs oa = {n, ld, R, part};
  if (e == hipSuccess) e = launch_one<OrthOp>(oa, T * T, 0, s);
  const FinishArgs fa = {n, T * T, part, res, vn, lambda, dout};
  if (e == hipSuccess) e = launch_one<FinishOp>(fa, 1, 0, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

}  // namespace bse
