// Adjoints with respect to A and B: of the eigenvalues (Thm EValSym, part 3)
// and, further down, of the eigenvectors (adjoint_vec_z).
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

// out[0] = max_k |lam_k| (one work group).
__global__ __launch_bounds__(256) void k_absmax(int n, const double* __restrict__ lam,
                                                double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) m = fmax(m, fabs(lam[k]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// The coefficient matrices of the eigenvector adjoint.  With Y+ = u^H g_u and
// Y- = v^H g_v (u = a + b, v = a - b and likewise for G_X), the blocks of
// Y = Z^H G_X are Yt = (Y+ + Y-)/2 (positive half) and Yb = (Y+ - Y-)/2
// (negative half), and
//   Dt(i, k) = g_k (i = k),
//            = (conj(Yt_ik) - Yt_ki) / (2 (lam_k - lam_i))   (0 if degenerate),
//   Db(i, k) = -(conj(Yb_ik) + Yb_ki) / (2 (lam_i + lam_k))  (Hermitian part),
//   S+[k, i] = Dt(i, k) + Db(i, k),  S-[k, i] = Dt(i, k) - Db(i, k),
// both Hermitian.  Work group = 32 x 32 output tile (rows k, columns i); the
// transposed entries (i, k) of Y+ and Y- come through LDS.
__global__ __launch_bounds__(256) void k_adjoint_coef(int n, const double* __restrict__ lam,
                                                      const double* __restrict__ g,
                                                      const double2* __restrict__ Yp,
                                                      const double2* __restrict__ Ym,
                                                      const double* __restrict__ lmax, double rtol,
                                                      double2* __restrict__ Sp,
                                                      double2* __restrict__ Sm) {
  __shared__ double2 tp[32][33], tm[32][33];
  const int k0 = blockIdx.x * 32, i0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // ty = 0..7
  // tile (rows i0.., columns k0..) of Y+ and Y-: tp[c][r] = Y(i0 + r, k0 + c)
  for (int c = ty; c < 32; c += 8) {
    const int i = i0 + tx, k = k0 + c;
    const bool in = i < n && k < n;
    const long o = i + (long)k * n;
    tp[c][tx] = in ? Yp[o] : make_double2(0.0, 0.0);
    tm[c][tx] = in ? Ym[o] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const double tol = rtol * lmax[0];
  for (int c = ty; c < 32; c += 8) {
    const int k = k0 + tx, i = i0 + c;  // output S[k, i]
    if (k >= n || i >= n) continue;
    const long o = k + (long)i * n;
    const double2 ypd = Yp[o], ymd = Ym[o];        // Y(k, i)
    const double2 ypt = tp[tx][c], ymt = tm[tx][c];  // Y(i, k)
    const double2 yt_ki = cscale(cadd(ypd, ymd), 0.5), yb_ki = cscale(csub(ypd, ymd), 0.5);
    const double2 yt_ik = cscale(cadd(ypt, ymt), 0.5), yb_ik = cscale(csub(ypt, ymt), 0.5);
    const double li = lam[i], lk = lam[k];
    double2 dt = make_double2(0.0, 0.0);
    if (i == k) {
      dt = make_double2(g[k], 0.0);
    } else if (fabs(lk - li) > tol) {
      dt = cscale(csub(cconj(yt_ik), yt_ki), 0.5 / (lk - li));
    }
    const double2 db = cscale(cadd(cconj(yb_ik), yb_ki), -0.5 / (li + lk));
    Sp[o] = cadd(dt, db);
    Sm[o] = csub(dt, db);
  }
}

GemmDesc full_gemm(int n, const double2* A, int opA, const double2* B, int opB, double2* C, long ldc) {
  GemmDesc g;
  g.M = n; g.N = n; g.K = n;
  g.A = A; g.lda = n; g.opA = opA;
  g.B = B; g.ldb = n; g.opB = opB;
  g.C = C; g.ldc = ldc;
  return g;
}

}  // namespace

size_t adjoint_vec_work_bytes(int n) {
  const size_t m = (size_t)(n > 0 ? n : 1);
  return 6 * align256(m * m * sizeof(double2)) + 512;
}

// Eigenvector adjoint (the oracle's grad_from_eigvecs in (u, v) coordinates):
// with M = X D^T Z^H, G_A = herm(M11 + M22) = (u S+ u^H + v S- v^H) / 2 and
// G_B = herm(M12 + M21) = (u S+ u^H - v S- v^H) / 2, since
// M11 + M22 = a Q1 + b Q2, M12 + M21 = a Q2 + b Q1 with Q1 +- Q2 = (Dt +- Db)^T (a +- b)^H,
// and the Hermitian part of u S u^H is u herm(S) u^H.  Five n^3 complex GEMMs
// (two of them on lower tiles only).
hipError_t adjoint_vec_z(int n, const double* lam, const double2* X, long ldx, const double* g,
                         const double2* GX, long ldg, double rtol, double2* gA, long ldga,
                         double2* gB, long ldgb, void* work, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(work) + 255) & ~(uintptr_t)255);
  const size_t U = align256((size_t)n * n * sizeof(double2));
  double2* u = reinterpret_cast<double2*>(base);
  double2* v = reinterpret_cast<double2*>(base + U);
  double2* gu = reinterpret_cast<double2*>(base + 2 * U);  // then S+
  double2* gv = reinterpret_cast<double2*>(base + 3 * U);  // then S-
  double2* Yp = reinterpret_cast<double2*>(base + 4 * U);  // then u S+
  double2* Ym = reinterpret_cast<double2*>(base + 5 * U);  // then v S-
  double* lmax = reinterpret_cast<double*>(base + 6 * U);
  const long total = (long)n * n;
  const int blocks = (int)((total + 255) / 256 < 8192 ? (total + 255) / 256 : 8192);
  k_form_xy<<<blocks, 256, 0, s>>>(n, X, ldx, v, u, n);     // v = a - b, u = a + b
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_form_xy<<<blocks, 256, 0, s>>>(n, GX, ldg, gv, gu, n);  // likewise for G_X
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_absmax<<<1, 256, 0, s>>>(n, lam, lmax);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = gemm_z(full_gemm(n, u, 1, gu, 0, Yp, n), s)) != hipSuccess) return e;  // Y+ = u^H g_u
  if ((e = gemm_z(full_gemm(n, v, 1, gv, 0, Ym, n), s)) != hipSuccess) return e;  // Y- = v^H g_v
  dim3 grid((n + 31) / 32, (n + 31) / 32);
  k_adjoint_coef<<<grid, 256, 0, s>>>(n, lam, g, Yp, Ym, lmax, rtol, gu, gv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = gemm_z(full_gemm(n, u, 0, gu, 0, Yp, n), s)) != hipSuccess) return e;  // u S+
  if ((e = gemm_z(full_gemm(n, v, 0, gv, 0, Ym, n), s)) != hipSuccess) return e;  // v S-
  GemmDesc q = full_gemm(n, Yp, 0, u, 1, gB, ldgb);  // Q = u S+ u^H (lower tiles)
  q.lowerC = 1;
  if ((e = gemm_z(q, s)) != hipSuccess) return e;
  GemmDesc p = full_gemm(n, Ym, 0, v, 1, gA, ldga);  // P = v S- v^H (lower tiles)
  p.lowerC = 1;
  if ((e = gemm_z(p, s)) != hipSuccess) return e;
  dim3 grid2((n + 255) / 256, n);
  k_combine<<<grid2, 256, 0, s>>>(n, gA, ldga, gB, ldgb);  // G_A = (P + Q)/2, G_B = (Q - P)/2
  return hipGetLastError();
}

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
