// Adjoint of the eigenvalues with respect to A and B (Thm EValSym, part 3).
//
// For a real loss L(lambda) with w_k = dL/dlambda_k and Sigma-normalised
// right eigenvectors v_k = [a_k; b_k] of H1, the left eigenvector is
// v_k^H Sigma, so dlambda_k = v_k^H Sigma dH1 v_k with
// Sigma dH1 = [dA dB; dB dA], which gives
//   G_A = sum_k w_k (a_k a_k^H + b_k b_k^H),
//   G_B = sum_k w_k (a_k b_k^H + b_k a_k^H).
// In the coordinates x = a - b, y = a + b (x_k = V1_k, y_k = V2_k of Alg. 3)
// the two sums become
//   G_A = (P + Q) / 2,  G_B = (Q - P) / 2,
//   P = x diag(w) x^H,  Q = y diag(w) y^H,
// two Hermitian rank-n products: only their lower tiles are computed (MFMA
// GEMM with the weights applied along k), then one pass forms G_A, G_B and
// mirrors them to full Hermitian matrices.
#include "common.hpp"
#include "internal.hpp"

namespace bse {
namespace {

// x[:, k] = a_k - b_k, y[:, k] = a_k + b_k from X = [a; b] (2n x n, ldx).
__global__ __launch_bounds__(256) void k_form_xy(int n, const double2* __restrict__ X, long ldx,
                                                 double2* __restrict__ x, double2* __restrict__ y,
                                                 long ld) {
  const long total = (long)n * n;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long)gridDim.x * 256) {
    const int i = (int)(e % n), k = (int)(e / n);
    const double2 a = X[i + (long)k * ldx], b = X[i + n + (long)k * ldx];
    double2 u, v;
    u.x = a.x - b.x; u.y = a.y - b.y;
    v.x = a.x + b.x; v.y = a.y + b.y;
    x[i + (long)k * ld] = u;
    y[i + (long)k * ld] = v;
  }
}

// P (in gA) and Q (in gB) hold valid lower triangles; write
// G_A = (P + Q)/2, G_B = (Q - P)/2 on and below the diagonal and their
// conjugates above it.  Each lower entry is read and written by one thread,
// each strict-upper entry only written, so the pass is race free in place.
__global__ __launch_bounds__(256) void k_combine(int n, double2* __restrict__ gA, long lda,
                                                 double2* __restrict__ gB, long ldb) {
  const int j = blockIdx.y;
  for (int i = j + (int)(blockIdx.x * 256 + threadIdx.x); i < n; i += gridDim.x * 256) {
    const double2 p = gA[i + (long)j * lda], q = gB[i + (long)j * ldb];
    double2 ga, gb;
    ga.x = 0.5 * (p.x + q.x); ga.y = 0.5 * (p.y + q.y);
    gb.x = 0.5 * (q.x - p.x); gb.y = 0.5 * (q.y - p.y);
    if (i == j) { ga.y = 0.0; gb.y = 0.0; }
    gA[i + (long)j * lda] = ga;
    gB[i + (long)j * ldb] = gb;
    if (i != j) {
      ga.y = -ga.y; gb.y = -gb.y;
      gA[j + (long)i * lda] = ga;
      gB[j + (long)i * ldb] = gb;
    }
  }
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t adjoint_work_bytes(int n) {
  const size_t m = (size_t)(n > 0 ? n : 1);
  return 2 * align256(m * m * sizeof(double2)) + 256;
}

hipError_t adjoint_z(int n, const double2* X, long ldx, const double* w, double2* gA, long ldga,
                     double2* gB, long ldgb, void* work, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(work) + 255) & ~(uintptr_t)255);
  double2* x = reinterpret_cast<double2*>(base);
  double2* y = reinterpret_cast<double2*>(base + align256((size_t)n * n * sizeof(double2)));
  const long total = (long)n * n;
  const int blocks = (int)((total + 255) / 256 < 8192 ? (total + 255) / 256 : 8192);
  k_form_xy<<<blocks, 256, 0, s>>>(n, X, ldx, x, y, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  GemmDesc g;  // P = x diag(w) x^H, lower tiles
  g.M = n; g.N = n; g.K = n;
  g.A = x; g.lda = n; g.opA = 0;
  g.B = x; g.ldb = n; g.opB = 1;
  g.kscale = w;
  g.lowerC = 1;
  g.C = gA; g.ldc = ldga;
  e = gemm_z(g, s);
  if (e != hipSuccess) return e;
  g.A = y; g.B = y;  // Q = y diag(w) y^H
  g.C = gB; g.ldc = ldgb;
  e = gemm_z(g, s);
  if (e != hipSuccess) return e;
  dim3 grid((n + 255) / 256, n);
  k_combine<<<grid, 256, 0, s>>>(n, gA, ldga, gB, ldgb);
  return hipGetLastError();
}

}  // namespace bse
