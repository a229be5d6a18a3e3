// FP64 refinement of the positive eigenpairs of H1 (the mixed-precision form).
//
// Work in the (x, y) coordinates of the proof of Thm ProdEig: an eigenvector
// is v = Q [x; y], Q = 1/2 [I I; -I I], with M1 y = lambda x, M2 x = lambda y,
// and its mirror for -lambda is [0 I; I 0] v = Q [-x; y] (Lemma
// ComputeNegEvecs).  With Z = [V, PV], Sigma-orthogonality and the
// eigen-equation of the pencil (Hcal, Sigma), Hcal = Sigma H1 = [A B; B A],
// read Z^H Sigma Z = S = diag(I, -I) and Z^H Hcal Z = diag(Lambda, Lambda).
// Since Q^H Sigma Q = 1/2 [0 I; I 0] and Q^H Hcal Q = 1/2 diag(M2, M1)
// (Lemma Qtransform), all of Z^H Sigma Z and Z^H Hcal Z follows from three
// n x n products F = x^H y, P2 = x^H M2 x, P1 = y^H M1 y (the latter two as
// Grams of L2^H x and L1^H y with the FP64 Cholesky factors M = L L^H of
// Alg. 3 steps 1-2: a triangular product and half a Gram each):
//   G11 = (F + F^H)/2,   G21 = (F^H - F)/2,
//   T11 = (P2 + P1)/2,   T21 = (P1 - P2)/2.
// A first-order correction Z <- Z (I + S E) that restores both conditions
// (the linearised equations E^H S + S E = S - G and, off the diagonal,
// T + E^H S L + L S E = diagonal) gives, with R = S - G and Ritz values
// l_i = T11_ii / G11_ii,
//   E11_ii = R11_ii / 2,
//   E11_ij = (T11_ij + l_j R11_ij) / (l_j - l_i)   (i != j; its rotation
//            part is taken with the exact 2 x 2 Jacobi angle, see k_build),
//   E21_ij = (T21_ij + l_j R21_ij) / (l_j + l_i),
// and the positive half updates as x <- x (I + E11 + E21),
// y <- y (I + E11 - E21).  This is the Newton-type refinement for symmetric
// eigenproblems written with GEMMs, here for the Sigma-Hermitian pencil.
// The eigenvalues are then the Rayleigh quotients
//   lambda_k = (x_k^H M2 x_k + y_k^H M1 y_k) / (2 Re x_k^H y_k),
// and each pair is scaled by (Re x_k^H y_k)^-1/2 so that v_k^H Sigma v_k = 1.
// The three quotient terms of the updated pairs follow from the step's
// products and its correction to third order in the correction (BuildOp), so
// the last step needs no further products with M1 and M2.
#include "common.hpp"
#include "group.hpp"
#include "internal.hpp"

#include <stdio.h>
#include <stdlib.h>

namespace bse {
namespace {

struct RitzOp {
  static constexpr int NT = 256;
  typedef RitzArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int aux) {
    const int i = bx * 256 + threadIdx.x;
    if (i >= a.n) return;
    const long d = i + (long)i * a.ld;
    a.ritz[i] = 0.5 * (a.P2[d].x + a.P1[d].x) / a.F[d].x;
  }
};

// Correction matrices Ex = I + E11 + E21 and Ey = I + E11 - E21; a 64 x 64
// tile per workgroup, the transposed tile of F staged through LDS.
struct BuildOp {
  static constexpr int NT = 256;
  typedef BuildArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int aux);
};

// max(m, v), with a NaN v counted as +inf (fmax would drop it), so that a
// correction that has broken down reads as one that has not converged.
BSE_DEV double max_or_inf(double m, double v) {
  if (v != v) return __longlong_as_double(0x7ff0000000000000LL);
  return fmax(m, v);
}

BSE_DEV void BuildOp::run(const BuildArgs& a, int bx, int) {
  const int n = a.n;
  const double2* __restrict__ F = a.F;
  const double2* __restrict__ P1 = a.P1;
  const double2* __restrict__ P2 = a.P2;
  const long ld = a.ld;
  const double* __restrict__ ritz = a.ritz;
  double2* __restrict__ Ex = a.Ex;
  double2* __restrict__ Ey = a.Ey;
  const double delta = a.delta;
  double* maxcorr = a.maxcorr;
  __shared__ double2 ft[64][65];
  __shared__ double red[256];
  const int T = (n + 63) / 64;
  const int tm = bx % T, tn = bx / T;
  const int m0 = tm * 64, n0 = tn * 64;
  const int tid = threadIdx.x;
  // ft[c][r] = F[n0 + c][m0 + r]  (rows of the transposed tile)
  for (int q = 0; q < 16; ++q) {
    const int r = tid & 63, c = (tid >> 6) + 4 * q;
    const int gi = n0 + r, gj = m0 + c;
    ft[r][c] = (gi < n && gj < n) ? F[gi + (long)gj * ld] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  // with part: the updated pair x Ex, y Ey has, up to terms of third order in
  // the correction (Ex = I + a, Ey = I + b, a and b small, the products
  // nearly diagonal in the current basis),
  //   Re (Ex^H F Ey)_kk  = Re F_kk + sum_i Re(conj(a_ik) F_ik + F_ki b_ik + conj(a_ik) F_ii b_ik),
  //   (Ex^H P2 Ex)_kk    = P2_kk + sum_i (2 Re(conj(a_ik) P2_ik) + |a_ik|^2 P2_ii),
  //   (Ey^H P1 Ey)_kk    = P1_kk + sum_i (2 Re(conj(b_ik) P1_ik) + |b_ik|^2 P1_ii);
  // each work group writes the sums over its 64 rows i, column by column.
  const int r = tid & 63, i = m0 + r;
  double2 fii = make_double2(0.0, 0.0), p1ii = fii, p2ii = fii;
  if (a.part && i < n) {
    const long d = i + (long)i * ld;
    fii = F[d];
    p1ii = P1[d];
    p2ii = P2[d];
  }
  double mc = 0.0;
  for (int q = 0; q < 16; ++q) {
    const int c = (tid >> 6) + 4 * q;
    const int j = n0 + c;
    double sf = 0.0, s2 = 0.0, s1 = 0.0;
    if (i < n && j < n) {
      const long o = i + (long)j * ld;
      const double2 fij = F[o];
      const double2 fji_c = cconj(ft[c][r]);  // conj(F[j][i])
      const double2 p1 = P1[o], p2 = P2[o];
      const double2 g11 = cscale(cadd(fij, fji_c), 0.5);
      const double2 g21 = cscale(csub(fji_c, fij), 0.5);
      const double2 t11 = cscale(cadd(p2, p1), 0.5);
      const double2 t21 = cscale(csub(p1, p2), 0.5);
      const double li = ritz[i], lj = ritz[j];
      double2 e11;
      if (i == j) {
        e11 = make_double2(0.5 * (1.0 - g11.x), 0.0);
      } else {
        // E11_ij = R_ij / 2 + K_ij / (l_j - l_i) with K = T + (l_i + l_j) R / 2 is the
        // first-order solution; its rotation part K / (l_j - l_i) = phase(K) / (2 zeta),
        // zeta = (l_j - l_i) / (2 |K|), is replaced by the exact 2 x 2 Jacobi tangent
        // phase(K) sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), equal to it for well
        // separated pairs and bounded by 1 for close pairs, where the first-order
        // term diverges.
        const double2 r11 = make_double2(-g11.x, -g11.y);
        const double dl = lj - li;
        const double2 K = cadd(t11, cscale(r11, 0.5 * (li + lj)));
        const double aK = sqrt(cabs2(K));
        e11 = cscale(r11, 0.5);
        if (aK > 0.0 && !(fabs(dl) <= delta * fmax(fabs(li), fabs(lj)) && aK <= delta * fabs(lj))) {
          const double zeta = dl / (2.0 * aK);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          e11 = cadd(e11, cscale(K, t / aK));
        }
        mc = max_or_inf(mc, sqrt(cabs2(e11)));
      }
      const double2 r21 = make_double2(-g21.x, -g21.y);
      const double2 e21 = cscale(cadd(t21, cscale(r21, lj)), 1.0 / (lj + li));
      mc = max_or_inf(mc, sqrt(cabs2(e21)));
      const double dd = (i == j) ? 1.0 : 0.0;
      const double2 ea = cadd(e11, e21);  // Ex - I
      const double2 eb = csub(e11, e21);  // Ey - I
      Ex[o] = make_double2(dd + ea.x, ea.y);
      Ey[o] = make_double2(dd + eb.x, eb.y);
      if (a.part) {
        const double2 fji = cconj(fji_c);
        const double2 fb = cmul(fii, eb);
        sf = (ea.x * fij.x + ea.y * fij.y) + (fji.x * eb.x - fji.y * eb.y) + (ea.x * fb.x + ea.y * fb.y);
        s2 = 2.0 * (ea.x * p2.x + ea.y * p2.y) + cabs2(ea) * p2ii.x;
        s1 = 2.0 * (eb.x * p1.x + eb.y * p1.y) + cabs2(eb) * p1ii.x;
      }
    }
    if (a.part) {  // the column's sums over the wave's 64 rows
      for (int sh = 32; sh > 0; sh >>= 1) {
        sf += __shfl_xor(sf, sh);
        s2 += __shfl_xor(s2, sh);
        s1 += __shfl_xor(s1, sh);
      }
      if (r == 0 && j < n) {
        a.part[((long)0 * T + tm) * n + j] = sf;
        a.part[((long)1 * T + tm) * n + j] = s2;
        a.part[((long)2 * T + tm) * n + j] = s1;
      }
    }
  }
  red[tid] = mc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
    __syncthreads();
  }
  if (tid == 0) atomic_max_nonneg(maxcorr, red[0]);
}

// Column k: lambda_k = (x_k^H Qx_k + y_k^H Qy_k) / (2 Re x_k^H y_k), scl_k = (Re x_k^H y_k)^-1/2.
struct RqOp {
  static constexpr int NT = 256;
  typedef RqArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int aux);
};

BSE_DEV void RqOp::run(const RqArgs& args, int bx, int) {
  const int n = args.n;
  const double2* __restrict__ x = args.x;
  const double2* __restrict__ y = args.y;
  const double2* __restrict__ Qx = args.Qx;
  const double2* __restrict__ Qy = args.Qy;
  const long ld = args.ld;
  double* __restrict__ lam = args.lam;
  double* __restrict__ scl = args.scl;
  __shared__ double ra[256], rb[256], rc[256];
  const int k = bx, tid = threadIdx.x;
  const long o = (long)k * ld;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = tid; i < n; i += 256) {
    const double2 xv = x[o + i], yv = y[o + i], qx = Qx[o + i], qy = Qy[o + i];
    a += xv.x * qx.x + xv.y * qx.y;
    b += yv.x * qy.x + yv.y * qy.y;
    c += xv.x * yv.x + xv.y * yv.y;
  }
  ra[tid] = a; rb[tid] = b; rc[tid] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) { ra[tid] += ra[tid + h]; rb[tid] += rb[tid + h]; rc[tid] += rc[tid + h]; }
    __syncthreads();
  }
  if (tid == 0) {
    const double l = (ra[0] + rb[0]) / (2.0 * rc[0]);
    lam[k] = l;
    scl[k] = 1.0 / sqrt(rc[0]);
    // a pair that is not Sigma-positive (Re x^H y <= 0) or a non-finite
    // quotient marks the refinement as failed
    if (args.bad && !(rc[0] > 0.0 && l > 0.0 && l < 1.0e308)) atomic_max_nonneg(args.bad, 1.0);
  }
}

struct UpdRqOp {
  static constexpr int NT = 256;
  typedef UpdRqArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int k = bx * 256 + threadIdx.x;
    if (k >= a.n) return;
    const int T = (a.n + 63) / 64;
    const long d = k + (long)k * a.ld;
    double f = a.F[d].x, p2 = a.P2[d].x, p1 = a.P1[d].x;
    for (int t = 0; t < T; ++t) {  // fixed order: deterministic
      f += a.part[((long)0 * T + t) * a.n + k];
      p2 += a.part[((long)1 * T + t) * a.n + k];
      p1 += a.part[((long)2 * T + t) * a.n + k];
    }
    const double l = (p2 + p1) / (2.0 * f);
    a.lam[k] = l;
    a.scl[k] = 1.0 / sqrt(f);
    if (a.bad && !(f > 0.0 && l > 0.0 && l < 1.0e308)) atomic_max_nonneg(a.bad, 1.0);
  }
};

struct CoupleOp {
  static constexpr int NT = 256;
  typedef CoupleArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int i = bx * 256 + threadIdx.x;
    if (i >= a.n) return;
    const double li = a.ritz[i];
    int cnt = 0;
    for (int d = 1; d <= 64 && i + d < a.n; ++d) {
      const int j = i + d;
      const long o = i + (long)j * a.ld, ot = j + (long)i * a.ld;
      const double lj = a.ritz[j];
      const double2 g11 = cscale(cadd(a.F[o], cconj(a.F[ot])), 0.5);
      const double2 t11 = cscale(cadd(a.P2[o], a.P1[o]), 0.5);
      const double2 K = csub(t11, cscale(g11, 0.5 * (li + lj)));
      if (kCoupleRatio * sqrt(cabs2(K)) > fabs(lj - li)) ++cnt;
    }
    if (cnt) atomicAdd(a.count, cnt);
  }
};

// Complex64 operands of a basis update that is not the refinement's last:
// x, y, Ex - I and Ey - I (their n x n blocks); a 64 x 64 tile of one of the
// four matrices per work group.
struct LowOp {
  static constexpr int NT = 256;
  typedef LowArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int T = (a.n + 63) / 64;
    const int mat = bx / (T * T), t = bx % (T * T);
    const int i = (t % T) * 64 + (threadIdx.x & 63), j0 = (t / T) * 64 + (threadIdx.x >> 6);
    if (i >= a.n) return;
    const double2* __restrict__ S = a.src[mat];
    float2* __restrict__ D = a.dst[mat];
    const double one = mat >= 2 ? 1.0 : 0.0;
    for (int j = j0; j < j0 + 64 && j < a.n; j += 4) {
      double2 v = S[i + (long)j * a.ld];
      if (i == j) v.x -= one;
      D[i + (long)j * a.ld] = make_float2((float)v.x, (float)v.y);
    }
  }
};

// x += Px and y += Py, with Px = x (Ex - I) and Py = y (Ey - I) in complex64.
struct AddLowOp {
  static constexpr int NT = 256;
  typedef AddLowArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int T = (a.n + 63) / 64;
    const int mat = bx / (T * T), t = bx % (T * T);
    const int i = (t % T) * 64 + (threadIdx.x & 63), j0 = (t / T) * 64 + (threadIdx.x >> 6);
    if (i >= a.n) return;
    const float2* __restrict__ S = a.src[mat];
    double2* __restrict__ D = a.dst[mat];
    for (int j = j0; j < j0 + 64 && j < a.n; j += 4) {
      const float2 p = S[i + (long)j * a.ld];
      double2 v = D[i + (long)j * a.ld];
      v.x += (double)p.x;
      v.y += (double)p.y;
      D[i + (long)j * a.ld] = v;
    }
  }
};

GemmDesc nn(int n, long ld, const double2* A, int opA, const double2* B, int opB, double2* C) {
  GemmDesc g;
  g.M = n; g.N = n; g.K = n;
  g.A = A; g.lda = ld; g.opA = opA;
  g.B = B; g.ldb = ld; g.opB = opB;
  g.C = C; g.ldc = ld;
  return g;
}

}  // namespace

hipError_t group_refine(GroupOp op, const void* table, const int2* map, int blocks, int aux,
                        hipStream_t s) {
  switch (op) {
    case G_RITZ: return launch_grp<RitzOp>(table, map, blocks, aux, s);
    case G_BUILD: return launch_grp<BuildOp>(table, map, blocks, aux, s);
    case G_RQ: return launch_grp<RqOp>(table, map, blocks, aux, s);
    case G_UPDRQ: return launch_grp<UpdRqOp>(table, map, blocks, aux, s);
    case G_COUPLE: return launch_grp<CoupleOp>(table, map, blocks, aux, s);
    case G_LOW: return launch_grp<LowOp>(table, map, blocks, aux, s);
    case G_ADDLOW: return launch_grp<AddLowOp>(table, map, blocks, aux, s);
    default: return hipErrorInvalidValue;
  }
}

void window_congruence(int n, long ld, double2* M, double2* Tmp, const double2* Cb, int off,
                       std::vector<GemmDesc>& right, std::vector<GemmDesc>& left) {
  const int nw = window_count(n, off);
  for (int w = 0; w < nw; ++w) {
    int a, m;
    window_range(n, off, w, a, m);
    if (m <= 0) continue;
    GemmDesc r;  // Tmp[:, a:a+m] = M[:, a:a+m] C_w
    r.M = n; r.N = m; r.K = m;
    r.A = M + (long)a * ld; r.lda = ld; r.opA = 0;
    r.B = Cb + (long)w * 64 * 64; r.ldb = 64; r.opB = 0;
    r.C = Tmp + (long)a * ld; r.ldc = ld;
    right.push_back(r);
    GemmDesc l;  // M[a:a+m, :] = C_w^H Tmp[a:a+m, :]
    l.M = m; l.N = n; l.K = m;
    l.A = Cb + (long)w * 64 * 64; l.lda = 64; l.opA = 1;
    l.B = Tmp + a; l.ldb = ld; l.opB = 0;
    l.C = M + a; l.ldc = ld;
    left.push_back(l);
  }
}

void window_right(int n, long ld, const double2* X, double2* out, const double2* Cb, int off,
                  std::vector<GemmDesc>& g) {
  const int nw = window_count(n, off);
  for (int w = 0; w < nw; ++w) {
    int a, m;
    window_range(n, off, w, a, m);
    if (m <= 0) continue;
    GemmDesc r;  // out[:, a:a+m] = X[:, a:a+m] C_w
    r.M = n; r.N = m; r.K = m;
    r.A = X + (long)a * ld; r.lda = ld; r.opA = 0;
    r.B = Cb + (long)w * 64 * 64; r.ldb = 64; r.opB = 0;
    r.C = out + (long)a * ld; r.ldc = ld;
    g.push_back(r);
  }
}

double2* window_blocks(double2* Cb0, int n, int pass) {
  return Cb0 + (size_t)pass * 64 * 64 * (n / 64 + 2);
}

namespace {

// One Rayleigh-Ritz pass on the windows of offset `off` (window.hip): the
// window blocks C_w into Cb, then the products by congruence,
// M <- C^H M C for M = F, P1, P2 (block GEMMs through Tmp).
hipError_t window_pass(int n, long ld, double2* F, double2* P1, double2* P2, double2* Tmp,
                       double2* Cb, int off, double* maxrot, Arena& ar, hipStream_t s) {
  const WinArgs wa = {n, ld, F, P1, P2, off, Cb, maxrot};
  hipError_t e = window_eig(wa, window_count(n, off), s);
  double2* mats[3] = {F, P1, P2};
  for (int k = 0; k < 3 && e == hipSuccess; ++k) {
    std::vector<GemmDesc> right, left;
    window_congruence(n, ld, mats[k], Tmp, Cb, off, right, left);
    e = run_gemm<double>(ar, right, s);
    if (e == hipSuccess) e = run_gemm<double>(ar, left, s);
  }
  return e;
}

}  // namespace

hipError_t rq_pairs_z(int n, long ld, const double2* x, const double2* y, const double2* Qx,
                      const double2* Qy, double* lam, double* scl, hipStream_t s) {
  const RqArgs qa = {n, x, y, Qx, Qy, ld, lam, scl, nullptr};
  return launch_one<RqOp>(qa, n, 0, s);
}

hipError_t refine_z(int n, long ld, const double2* L1, const double2* L2, double2** xp,
                    double2** yp, const RefineWork& w, int max_steps, double stop_corr, double* lam,
                    double* scl, double* max_corr, int* steps_done, hipStream_t s,
                    double* corr_hist, int* window_steps) {
  double2* x = *xp;
  double2* y = *yp;
  double2* Q = w.Q;
  double2* F = w.F;
  hipError_t e;
  *max_corr = 0.0;
  *steps_done = 0;
  if (window_steps) *window_steps = 0;
  Arena ar;
  ar.dev = w.arena;
  ar.cap = w.arena_cap;
  ar.s = s;
  if (w.windows) {
    // the pairs in the ascending order of the start's eigenvalues, so that a
    // window holds spectral neighbours
    if ((e = sort_lambda(n, lam, w.perm, w.ritz, 0, s)) != hipSuccess) return e;
    if ((e = gather_scale_z(n, (int)ld, x, ld, w.perm, nullptr, Q, s)) != hipSuccess) return e;
    if ((e = gather_scale_z(n, (int)ld, y, ld, w.perm, nullptr, F, s)) != hipSuccess) return e;
    double2* t = x; x = Q; Q = t;
    t = y; y = F; F = t;
  }
  int* count = reinterpret_cast<int*>(w.maxcorr + 4);
  int passes = 0;
  double bad = 0.0;
  for (int it = 0; it < max_steps; ++it) {
    e = hipMemsetAsync(w.maxcorr, 0, 3 * sizeof(double), s);
    if (e != hipSuccess) return e;
    if ((e = gemm_z(nn(n, ld, x, 1, y, 0, F), s)) != hipSuccess) return e;       // F = x^H y
    // P2 = x^H M2 x = (L2^H x)^H (L2^H x) and P1 = (L1^H y)^H (L1^H y): a
    // triangular product, then the lower tiles of a Gram (mirrored below)
    GemmDesc t2 = nn(n, ld, L2, 1, x, 0, Q);                                     // Q = L2^H x
    t2.triA = 1;
    if ((e = gemm_z(t2, s)) != hipSuccess) return e;
    GemmDesc p2 = nn(n, ld, Q, 1, Q, 0, w.P2);
    p2.lowerC = 1;
    if ((e = gemm_z(p2, s)) != hipSuccess) return e;
    GemmDesc t1 = nn(n, ld, L1, 1, y, 0, Q);                                     // Q = L1^H y
    t1.triA = 1;
    if ((e = gemm_z(t1, s)) != hipSuccess) return e;
    GemmDesc p1 = nn(n, ld, Q, 1, Q, 0, w.P1);
    p1.lowerC = 1;
    if ((e = gemm_z(p1, s)) != hipSuccess) return e;
    if ((e = mirror_upper_z((int)((n + 63) / 64 * 64), w.P2, ld, s)) != hipSuccess) return e;
    if ((e = mirror_upper_z((int)((n + 63) / 64 * 64), w.P1, ld, s)) != hipSuccess) return e;
    // Rayleigh-Ritz windows from the first step whose products couple a pair
    // strongly on (clusters); spectra without such pairs converge as fast
    // without them
    if (w.windows && !passes) {
      const RitzArgs r0 = {n, F, w.P1, w.P2, ld, w.ritz};
      if ((e = launch_one<RitzOp>(r0, (n + 255) / 256, 0, s)) != hipSuccess) return e;
      if ((e = hipMemsetAsync(count, 0, sizeof(int), s)) != hipSuccess) return e;
      const CoupleArgs ca = {n, ld, F, w.P1, w.P2, w.ritz, count};
      if ((e = launch_one<CoupleOp>(ca, (n + 255) / 256, 0, s)) != hipSuccess) return e;
      int strong = 0;
      e = hipMemcpyAsync(&strong, count, sizeof(int), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return e;
      passes = strong > 0 ? w.windows : 0;
      if (getenv("BSE_DEBUG")) fprintf(stderr, "[bse] refinement step %d: %d strongly coupled pairs\n", it + 1, strong);
    }
    const int step_passes = (it == 0 || *max_corr > kWindowStop) ? passes : 0;
    if (window_steps && step_passes > 0) ++*window_steps;
    for (int pass = 0; pass < step_passes; ++pass) {
      // Rayleigh-Ritz on windows of 64 pairs, boundaries alternately at 0 and at 32
      const int off = window_offset(pass);
      double2* Cb = window_blocks(w.Cb0, n, pass);
      if ((e = window_pass(n, ld, F, w.P1, w.P2, Q, Cb, off, w.maxcorr + 1, ar, s)) != hipSuccess) return e;
    }
    const RitzArgs ra = {n, F, w.P1, w.P2, ld, w.ritz};
    if ((e = launch_one<RitzOp>(ra, (n + 255) / 256, 0, s)) != hipSuccess) return e;
    const int T = (n + 63) / 64;
    // Q is free until the basis update: it takes the tile sums of the quotients
    double* part = reinterpret_cast<double*>(Q);
    const BuildArgs ba = {n, F, w.P1, w.P2, ld, w.ritz, w.Ex, w.Ey, kRefineDelta, w.maxcorr, part};
    if ((e = launch_one<BuildOp>(ba, T * T, 0, s)) != hipSuccess) return e;
    // quotients and scales of the pairs this step leaves (no products of M1, M2 after the last step)
    const UpdRqArgs ua = {n, ld, F, w.P1, w.P2, part, lam, scl, w.maxcorr + 2};
    if ((e = launch_one<UpdRqOp>(ua, (n + 255) / 256, 0, s)) != hipSuccess) return e;
    // the window rotations precede the first-order correction:
    // x <- x C_1 C_2 ... C_p (I + E11 + E21), y <- y C_1 ... C_p (I + E11 - E21)
    for (int pass = 0; pass < step_passes; ++pass) {
      const int off = window_offset(pass);
      const double2* Cb = window_blocks(w.Cb0, n, pass);
      std::vector<GemmDesc> g;
      window_right(n, ld, x, Q, Cb, off, g);
      window_right(n, ld, y, F, Cb, off, g);
      if ((e = run_gemm<double>(ar, g, s)) != hipSuccess) return e;
      double2* t = x; x = Q; Q = t;
      t = y; y = F; F = t;
    }
    // the step's correction, known before its basis update: its first-order
    // part (the window rotations also turn bases inside subspaces of nearly
    // equal eigenvalues, where any basis is as good, so they do not measure
    // the distance to convergence)
    double mcs[3] = {0.0, 0.0, 0.0};
    e = hipMemcpyAsync(mcs, w.maxcorr, 3 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    const double mc = mcs[0];
    const bool last = mc <= stop_corr || it + 1 == max_steps;
    if (w.low_update && !last) {
      // x <- x + x (Ex - I), y <- y + y (Ey - I) with the products in
      // complex64: their rounding error, about 1e-6 of the correction, is
      // far below the error the step leaves (the correction's square, or the
      // next correction) and is removed by the next step's FP64 products;
      // the last step's update stays FP64.  Q and F hold the operands, Ex and
      // Ey the products (two complex64 n x n matrices fit in each).
      float2* xc = reinterpret_cast<float2*>(Q);
      float2* exc = reinterpret_cast<float2*>(F);
      float2* px = reinterpret_cast<float2*>(w.Ex);
      float2* py = reinterpret_cast<float2*>(w.Ey);
      const long half = ld * (long)n;
      const LowArgs la = {n, ld, {x, y, w.Ex, w.Ey}, {xc, xc + half, exc, exc + half}};
      if ((e = launch_one<LowOp>(la, 4 * T * T, 0, s)) != hipSuccess) return e;
      GemmDesc gx = nn(n, ld, nullptr, 0, nullptr, 0, nullptr);
      GemmDesc gy = gx;
      gx.A = xc; gx.B = exc; gx.C = px;
      gy.A = xc + half; gy.B = exc + half; gy.C = py;
      if ((e = gemm_c(gx, s)) != hipSuccess) return e;
      if ((e = gemm_c(gy, s)) != hipSuccess) return e;
      const AddLowArgs aa = {n, ld, {px, py}, {x, y}};
      if ((e = launch_one<AddLowOp>(aa, 2 * T * T, 0, s)) != hipSuccess) return e;
    } else {
      if ((e = gemm_z(nn(n, ld, x, 0, w.Ex, 0, Q), s)) != hipSuccess) return e;    // x (I + E11 + E21)
      if ((e = gemm_z(nn(n, ld, y, 0, w.Ey, 0, F), s)) != hipSuccess) return e;    // y (I + E11 - E21)
      double2* t = x; x = Q; Q = t;
      t = y; y = F; F = t;
    }
    bad = mcs[2];
    *max_corr = mc;
    *steps_done = it + 1;
    if (corr_hist && it < 8) corr_hist[it] = mc;
    if (getenv("BSE_DEBUG"))
      fprintf(stderr, "[bse] refinement step %d: largest first-order correction %.3e, window rotation %.3e\n",
              it + 1, mcs[0], mcs[1]);
    // the error left after a step is of the order of the square of its correction
    if (mc <= stop_corr) break;
  }
  if (*steps_done == 0) {
    // no step ran: Rayleigh quotients and Sigma-normalising scales of the start
    // M2 x = L2 (L2^H x) and M1 y = L1 (L1^H y)
    for (int f = 0; f < 2; ++f) {
      const double2* L = f ? L1 : L2;
      GemmDesc a = nn(n, ld, L, 1, f ? y : x, 0, Q);
      a.triA = 1;
      if ((e = gemm_z(a, s)) != hipSuccess) return e;
      GemmDesc b = nn(n, ld, L, 0, Q, 0, f ? w.P1 : w.P2);
      b.triA = 1;
      if ((e = gemm_z(b, s)) != hipSuccess) return e;
    }
    if ((e = hipMemsetAsync(w.maxcorr, 0, sizeof(double), s)) != hipSuccess) return e;
    const RqArgs qa = {n, x, y, w.P2, w.P1, ld, lam, scl, w.maxcorr};
    if ((e = launch_one<RqOp>(qa, n, 0, s)) != hipSuccess) return e;
    e = hipMemcpyAsync(&bad, w.maxcorr, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
  }
  if (bad != 0.0) *max_corr = __builtin_inf();
  *xp = x;
  *yp = y;
  return hipSuccess;
}

}  // namespace bse
