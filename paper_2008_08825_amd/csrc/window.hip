// Rayleigh-Ritz on windows of consecutive eigenpairs, inside the FP64
// refinement of the mixed form.
//
// The complex64 one-sided Jacobi stops at a relative off-orthogonality of
// about 4 sqrt(n) eps32; between spectral neighbours, whose relative gap
// shrinks with n, that leaves the pairs mixed at angles of order
// off / relgap (0.2 - 0.5 at n = 8192).  A first-order correction cannot
// undo angles that large in one step, so the refinement solves, before its
// first-order step, the projected problem exactly on windows of 64
// consecutive pairs (the pairs sorted by eigenvalue), twice, with the window
// boundaries shifted by 32 the second time.
//
// With the pairs (x, y) of the positive half and the n x n products
// F = x^H y, P2 = x^H M2 x, P1 = y^H M1 y, the Sigma-Gram and Hcal-Gram of the
// positive half are G = (F + F^H)/2 and T = (P2 + P1)/2 (from Q^H Sigma Q and
// Q^H Hcal Q, Lemma Qtransform).  On a window w the pencil T_ww c = l G_ww c
// (G_ww Hermitian positive definite) gives C_w with C_w^H G_ww C_w = I and
// C_w^H T_ww C_w diagonal (ascending); rotating the window's pairs by C_w
// Sigma-orthonormalises them and decouples them inside the window.  The
// products follow by congruence, F <- C^H F C, P1 <- C^H P1 C,
// P2 <- C^H P2 C with C = blockdiag(C_w), as block GEMMs (O(n^2 64) work, no
// new n^3 product), and the rotations are folded into the refinement's
// correction matrices.
//
// Window solver (one work group per window, FP64 in LDS): Cholesky
// G_ww = L L^H, X = L^-1, S = X T_ww X^H, Q = X^H; cyclic two-sided Jacobi on
// S (circle ordering, 32 disjoint rotations per step) with the rotations
// applied to the columns of Q, so Q ends as C_w = L^-H J; columns sorted by
// the eigenvalues S_ii.  A window of m < 64 pairs is padded with G = I and
// T = distinct values far above the spectrum, which stay uncoupled.
#include "common.hpp"
#include "internal.hpp"
#include "lds_la.hpp"

namespace bse {
namespace {

constexpr int WN = 64;

// circle ordering on 64 indices: pair m of step s, i < j
BSE_DEV void wcircle(int s, int m, int& i, int& j) {
  const int a = m, b = WN - 1 - m;
  i = (a == 0) ? 0 : ((a - 1 + s) % (WN - 1)) + 1;
  j = ((b - 1 + s) % (WN - 1)) + 1;
  if (i > j) { const int t = i; i = j; j = t; }
}

struct WinEigOp {
  static constexpr int NT = 256;
  typedef WinArgs Args;
  static BSE_DEV void run(const Args& a, int w, int aux);
};

BSE_DEV void WinEigOp::run(const WinArgs& p, int w, int) {
  __shared__ double Sr[WN][WN + 1], Si[WN][WN + 1];
  __shared__ double Qr[WN][WN + 1], Qi[WN][WN + 1];
  __shared__ double prm[32][4];  // c, s Re u, s Im u, active
  __shared__ int pij[32][2];
  __shared__ double part[4][WN][2];
  __shared__ double dg[WN];
  __shared__ unsigned long long offbits;
  __shared__ int fail;
  const int tid = threadIdx.x;
  int a0, m;
  window_range(p.n, p.off, w, a0, m);
  const long ld = p.ld;
  double2* Cw = p.C + (long)w * WN * WN;
  if (tid == 0) fail = 0;
  // 1. G_ww (Hermitian part of F's window block; identity beyond m)
  for (int q = 0; q < 16; ++q) {
    const int r = tid & 63, c = (tid >> 6) + 4 * q;
    double gr = (r == c) ? 1.0 : 0.0, gi = 0.0;
    if (r < m && c < m) {
      const double2 f1 = p.F[(a0 + r) + (long)(a0 + c) * ld];
      const double2 f2 = p.F[(a0 + c) + (long)(a0 + r) * ld];
      gr = 0.5 * (f1.x + f2.x);
      gi = 0.5 * (f1.y - f2.y);
    }
    Sr[r][c] = gr;
    Si[r][c] = gi;
  }
  __syncthreads();
  // Cholesky with unscaled columns (step j subtracts L[i][j] conj(L[k][j]) / L[j][j]
  // from L[i][k], j < k <= i), the columns scaled by 1 / sqrt(d_j) at the end
  {
    const int i = tid & 63;
    for (int j = 0; j < WN; ++j) {
      const double d = Sr[j][j];
      if (!(d > 0.0)) {
        if (tid == 0) fail = 1;
        break;
      }
      if (i > j) {
        const double rd = 1.0 / d;
        const double lr = Sr[i][j] * rd, li = Si[i][j] * rd;
        for (int k = j + 1 + (tid >> 6); k <= i; k += 4) {
          const double kr = Sr[k][j], ki = Si[k][j];
          Sr[i][k] -= lr * kr + li * ki;
          Si[i][k] -= li * kr - lr * ki;
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (fail) {
    // G_ww not numerically positive definite: leave the window as it is
    for (int q = 0; q < 16; ++q) {
      const int r = tid & 63, c = (tid >> 6) + 4 * q;
      Cw[r + c * WN] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    }
    return;
  }
  if (tid < WN) dg[tid] = 1.0 / sqrt(Sr[tid][tid]);
  __syncthreads();
  for (int q = 0; q < 16; ++q) {
    const int r = tid & 63, c = (tid >> 6) + 4 * q;
    if (r > c) { Sr[r][c] *= dg[c]; Si[r][c] *= dg[c]; }
    else if (r == c) { Sr[r][c] *= dg[c]; Si[r][c] = 0.0; }
    else { Sr[r][c] = 0.0; Si[r][c] = 0.0; }
  }
  __syncthreads();
  tri_inverse_lds(Sr, Si, Qr, Qi, tid);  // X = L^-1 in Q
  // 2. T_ww into S (Hermitian part of (P2 + P1) / 2; distinct large values beyond m)
  for (int q = 0; q < 16; ++q) {
    const int r = tid & 63, c = (tid >> 6) + 4 * q;
    double tr = 0.0, ti = 0.0;
    if (r < m && c < m) {
      const long e1 = (a0 + r) + (long)(a0 + c) * ld, e2 = (a0 + c) + (long)(a0 + r) * ld;
      tr = 0.25 * (p.P2[e1].x + p.P1[e1].x + p.P2[e2].x + p.P1[e2].x);
      ti = 0.25 * (p.P2[e1].y + p.P1[e1].y - p.P2[e2].y - p.P1[e2].y);
    } else if (r == c) {
      tr = 1.0e30 * (1.0 + r);
    }
    Sr[r][c] = tr;
    Si[r][c] = ti;
  }
  __syncthreads();
  // 3. S <- X S (rows from the bottom: row i needs the old rows k <= i)
  {
    const int c = tid & 63, g = tid >> 6;
    for (int i = WN - 1; i >= 0; --i) {
      double sr = 0.0, si = 0.0;
      for (int k = g; k <= i; k += 4) {
        const double xr = Qr[i][k], xi = Qi[i][k], br = Sr[k][c], bi = Si[k][c];
        sr += xr * br - xi * bi;
        si += xr * bi + xi * br;
      }
      part[g][c][0] = sr;
      part[g][c][1] = si;
      __syncthreads();
      if (g == 0) {
        Sr[i][c] = part[0][c][0] + part[1][c][0] + part[2][c][0] + part[3][c][0];
        Si[i][c] = part[0][c][1] + part[1][c][1] + part[2][c][1] + part[3][c][1];
      }
      __syncthreads();
    }
    // S <- S X^H (columns from the right: column j needs the old columns k <= j)
    const int r = tid & 63;
    for (int j = WN - 1; j >= 0; --j) {
      double sr = 0.0, si = 0.0;
      for (int k = g; k <= j; k += 4) {
        const double br = Sr[r][k], bi = Si[r][k], xr = Qr[j][k], xi = -Qi[j][k];  // conj(X[j][k])
        sr += br * xr - bi * xi;
        si += br * xi + bi * xr;
      }
      part[g][r][0] = sr;
      part[g][r][1] = si;
      __syncthreads();
      if (g == 0) {
        Sr[r][j] = part[0][r][0] + part[1][r][0] + part[2][r][0] + part[3][r][0];
        Si[r][j] = part[0][r][1] + part[1][r][1] + part[2][r][1] + part[3][r][1];
      }
      __syncthreads();
    }
  }
  // 4. Q <- X^H (upper triangular); S made exactly Hermitian
  for (int e = tid; e < WN * WN; e += 256) {
    const int r = e & 63, c = e >> 6;
    if (r > c) {
      const double xr = Qr[r][c], xi = Qi[r][c];
      Qr[c][r] = xr;
      Qi[c][r] = -xi;
      Qr[r][c] = 0.0;
      Qi[r][c] = 0.0;
      const double hr = 0.5 * (Sr[r][c] + Sr[c][r]), hi = 0.5 * (Si[r][c] - Si[c][r]);
      Sr[r][c] = hr; Si[r][c] = hi;
      Sr[c][r] = hr; Si[c][r] = -hi;
    } else if (r == c) {
      Si[r][r] = 0.0;
    }
  }
  __syncthreads();
  // 5. cyclic Jacobi on S, rotations accumulated into the columns of Q
  for (int sweep = 0; sweep < 12; ++sweep) {
    if (tid == 0) offbits = 0ull;
    __syncthreads();
    for (int step = 0; step < WN - 1; ++step) {
      if (tid < 32) {
        int i, j;
        wcircle(step, tid, i, j);
        pij[tid][0] = i;
        pij[tid][1] = j;
        const double aa = Sr[i][i], dd = Sr[j][j];
        const double br = Sr[i][j], bi = Si[i][j];
        const double ab = sqrt(br * br + bi * bi);
        const double den = sqrt(fabs(aa * dd));
        double rel = den > 0.0 ? ab / den : (ab > 0.0 ? 1.0 : 0.0);
        double c = 1.0, sr = 0.0, si = 0.0, act = 0.0;
        if (rel > 1.0e-17 && ab > 0.0) {
          const double zeta = (dd - aa) / (2.0 * ab);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + t * t);
          const double sn = t * c;
          sr = sn * br / ab;  // s u, u = S_ij / |S_ij|
          si = sn * bi / ab;
          act = 1.0;
        }
        prm[tid][0] = c; prm[tid][1] = sr; prm[tid][2] = si; prm[tid][3] = act;
        atomicMax(&offbits, (unsigned long long)__double_as_longlong(rel));
      }
      __syncthreads();
      // columns i, j of S and Q:  col_i' = c col_i - conj(s u) col_j,  col_j' = (s u) col_i + c col_j
      for (int it = tid; it < 32 * WN; it += 256) {
        const int mm = it >> 6, r = it & 63;
        if (prm[mm][3] == 0.0) continue;
        const int i = pij[mm][0], j = pij[mm][1];
        const double c = prm[mm][0], ur = prm[mm][1], ui = prm[mm][2];
        double xr = Sr[r][i], xi = Si[r][i], yr = Sr[r][j], yi = Si[r][j];
        Sr[r][i] = c * xr - (ur * yr + ui * yi);
        Si[r][i] = c * xi - (ur * yi - ui * yr);
        Sr[r][j] = (ur * xr - ui * xi) + c * yr;
        Si[r][j] = (ur * xi + ui * xr) + c * yi;
        xr = Qr[r][i]; xi = Qi[r][i]; yr = Qr[r][j]; yi = Qi[r][j];
        Qr[r][i] = c * xr - (ur * yr + ui * yi);
        Qi[r][i] = c * xi - (ur * yi - ui * yr);
        Qr[r][j] = (ur * xr - ui * xi) + c * yr;
        Qi[r][j] = (ur * xi + ui * xr) + c * yi;
      }
      __syncthreads();
      // rows i, j of S:  row_i' = c row_i - (s u) row_j,  row_j' = conj(s u) row_i + c row_j
      for (int it = tid; it < 32 * WN; it += 256) {
        const int mm = it >> 6, col = it & 63;
        if (prm[mm][3] == 0.0) continue;
        const int i = pij[mm][0], j = pij[mm][1];
        const double c = prm[mm][0], ur = prm[mm][1], ui = prm[mm][2];
        const double xr = Sr[i][col], xi = Si[i][col], yr = Sr[j][col], yi = Si[j][col];
        Sr[i][col] = c * xr - (ur * yr - ui * yi);
        Si[i][col] = c * xi - (ur * yi + ui * yr);
        Sr[j][col] = (ur * xr + ui * xi) + c * yr;
        Si[j][col] = (ur * xi - ui * xr) + c * yi;
      }
      __syncthreads();
      if (tid < 32 && prm[tid][3] != 0.0) {
        const int i = pij[tid][0], j = pij[tid][1];
        Sr[i][j] = 0.0; Si[i][j] = 0.0;
        Sr[j][i] = 0.0; Si[j][i] = 0.0;
        Si[i][i] = 0.0; Si[j][j] = 0.0;
      }
      __syncthreads();
    }
    if (__longlong_as_double((long long)offbits) <= 1.0e-15) break;
  }
  // 6. columns in ascending order of the eigenvalues S_ii; largest rotation
  if (tid < WN) dg[tid] = Sr[tid][tid];
  __syncthreads();
  int rank = 0;
  if (tid < WN) {
    const double v = dg[tid];
    for (int k = 0; k < WN; ++k) rank += (dg[k] < v) || (dg[k] == v && k < tid);
  }
  __shared__ int rk[WN];
  if (tid < WN) rk[tid] = rank;
  __syncthreads();
  double mx = 0.0;
  for (int q = 0; q < 16; ++q) {
    const int r = tid & 63, c = (tid >> 6) + 4 * q;
    const int dst = rk[c];
    Cw[r + dst * WN] = make_double2(Qr[r][c], Qi[r][c]);
    if (r < m && dst < m) {
      const double er = Qr[r][c] - (r == dst ? 1.0 : 0.0), ei = Qi[r][c];
      mx = fmax(mx, sqrt(er * er + ei * ei));
    }
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if ((tid & 63) == 0 && p.maxrot) atomic_max_nonneg(p.maxrot, mx);
}

}  // namespace

int window_count(int n, int off) {
  if (n <= 0) return 0;
  if (off == 0) return (n + WN - 1) / WN;
  if (n <= off) return 1;
  return 1 + (n - off + WN - 1) / WN;
}

hipError_t window_eig(const WinArgs& a, int windows, hipStream_t s) {
  return launch_one<WinEigOp>(a, windows, 0, s);
}

hipError_t group_window(const void* table, const int2* map, int blocks, hipStream_t s) {
  return launch_grp<WinEigOp>(table, map, blocks, 0, s);
}

}  // namespace bse
