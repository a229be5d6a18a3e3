// Finalisation of the SVD route and the final setup of Alg. 3.
//
// After the Jacobi iteration Z = W_out = L2^H L1 J (J the product of the
// rotations, unitary) has orthogonal columns z_k = sigma_k v_k (paper notation
// of Lemma SVDScalarFactors, where L1^H L2 = U Lambda V^H, so W = V Lambda U^H
// and U = J).  Alg. 3 step 4 takes V1 = L1 U Lambda^-1/2 and V2 = L2 V
// Lambda^-1/2.  Since L1 U = L1 J = L2^-H Z, the first needs no accumulated
// rotations:
//   Ws = Z diag(sigma)^-3/2          so that V2 = L2 Ws = L2 V Lambda^-1/2,
//   V1 = L2^-H Ws diag(sigma)        (= L2^-H Z Lambda^-1/2 = L1 U Lambda^-1/2),
// one block triangular solve with L2^H.  The solve is backward stable, so V1
// carries the error of Z and not that error times ||H|| / lambda_k, as the
// Lemma's other relation V1 = M1 V2 Lambda^-1 would.  The scale of V1_k is
// 1 / ||Ws_k||^2 (= sigma_k for the computed Ws_k), which makes V1_k^H V2_k = 1.
// Eigenvalues: y = V2_k is an eigenvector of the Hermitian-definite pencil
// (M1, M2^-1) with eigenvalue lambda_k^2, so its Rayleigh quotient
//   lambda_k^2 = (y^H M1 y) / (y^H M2^-1 y) = ||T_k||^2 / ||Ws_k||^2,  T = L1^H V2,
// is accurate to second order in the error of y; it replaces the column norm
// sigma_k, whose error grows with the number of rotations a column went
// through.  The eigenvalues are sorted ascending (stable by index) and the
// final setup (Alg. 3 step 6) writes X = [(V1 + V2)/2; (V2 - V1)/2] in that
// order; the negative half is [0 I; I 0] X with eigenvalues -lambda (Lemma
// ComputeNegEvecs).
//
// The complex64 stage of the mixed form still forms V1 = L1 T Lambda^-1 (the
// Lemma's relation M1 V2 = V1 Lambda); the FP64 refinement that follows it
// corrects the pair, and its scale s_k = (||T_k|| ||Ws_k||)^-1/2 applies to both
// halves.
#include "common.hpp"
#include "internal.hpp"

namespace bse {
namespace {

template <typename C2>
struct ColnormOp {
  static constexpr int NT = 256;
  typedef ColnormArgs<C2> Args;
  static BSE_DEV void run(const Args& a, int bx, int aux) {
    __shared__ double red[256];
    const int j = bx, tid = threadIdx.x;
    const C2* col = a.W + (long)j * a.ld;
    double s = 0.0;
    for (int i = tid; i < a.np; i += 256) {
      const double x = col[i].x, y = col[i].y;
      s += x * x + y * y;
    }
    red[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) a.out[j] = sqrt(red[0]);
  }
};

// rank_j = #{i : key_i < key_j or (key_i == key_j and i < j)}; perm[rank_j] = j,
// key = sigma (ascending) or -sigma (descending).
struct RankOp {
  static constexpr int NT = 256;
  typedef RankArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int aux) {
    __shared__ double sv[256];
    const int n = a.n;
    const double sg = a.desc ? -1.0 : 1.0;
    const int j = bx * 256 + threadIdx.x;
    const double s = j < n ? sg * a.key[j] : 0.0;
    int rank = 0;
    for (int base = 0; base < n; base += 256) {
      const int i = base + threadIdx.x;
      sv[threadIdx.x] = i < n ? sg * a.key[i] : 0.0;
      __syncthreads();
      const int lim = min(256, n - base);
      for (int q = 0; q < lim; ++q) {
        const double v = sv[q];
        rank += (v < s) || (v == s && base + q < j);
      }
      __syncthreads();
    }
    if (j < n) a.perm[rank] = j;
  }
};

// W[:, k] *= sigma_k^-3/2 for k < n, zero for k >= n; work group = (column, 256 rows).
template <typename C2>
struct ScaleOp {
  static constexpr int NT = 256;
  typedef ScaleArgs<C2> Args;
  static BSE_DEV void run(const Args& a, int bx, int aux) {
    const int gx = (a.np + 255) / 256;
    const int k = bx / gx;
    const int i = (bx % gx) * 256 + threadIdx.x;
    if (i >= a.np) return;
    double f = 0.0;
    if (k < a.n) {
      const double sg = a.sigma[k];
      f = sg > 0.0 ? 1.0 / (sg * sqrt(sg)) : 0.0;
    }
    C2 v = a.W[i + (long)k * a.ld];
    v.x = v.x * f;
    v.y = v.y * f;
    a.W[i + (long)k * a.ld] = v;
  }
};

struct C64Op {
  static constexpr int NT = 256;
  typedef C64Args Args;
  static BSE_DEV void run(const Args& a, int bx, int aux) {
    const int gx = (a.np + 255) / 256;
    const int j = bx / gx;
    const int i = (bx % gx) * 256 + threadIdx.x;
    if (i >= a.np) return;
    const float2 v = a.S[i + (long)j * a.lds];
    const double f = a.colscale ? a.colscale[j] : 1.0;
    a.D[i + (long)j * a.ldd] = make_double2(f * v.x, f * v.y);
  }
};

struct LambdaOp {
  static constexpr int NT = 256;
  typedef LambdaArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int aux) {
    const int k = bx * 256 + threadIdx.x;
    if (k >= a.np) return;
    if (k < a.n) {
      const double x = a.anorm[k], y = a.bnorm[k];
      const double l = x / y;
      a.lam[k] = l;
      a.invlam[k] = 1.0 / l;
      a.scl[k] = a.v1scale ? 1.0 / (y * y) : 1.0 / sqrt(x * y);
    } else {
      a.lam[k] = 0.0;
      a.invlam[k] = 0.0;
      a.scl[k] = 0.0;
    }
  }
};

struct WriteLambdaOp {
  static constexpr int NT = 256;
  typedef WriteLambdaArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int aux) {
    const int n = a.n;
    const int r = bx * 256 + threadIdx.x;
    if (r >= n) return;
    int j = a.perm[r];
    if (j < 0 || j >= n) j = r;  // only if a value was NaN (ranks then collide)
    a.lambda[r] = a.lam[j];
    if (a.want_negative) a.lambda[n + r] = -a.lam[j];
  }
};

// out[:, r] = W[:, perm r] * f_r; work group = (column r, 256 rows).
struct GatherOp {
  static constexpr int NT = 256;
  typedef GatherArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int gx = (a.np + 255) / 256;
    const int r = bx / gx;
    const int i = (bx % gx) * 256 + threadIdx.x;
    if (i >= a.np) return;
    double2* out = a.out + i + (long)r * a.ld;
    if (r >= a.n) { *out = make_double2(0.0, 0.0); return; }
    int k = a.perm[r];
    if (k < 0 || k >= a.n) k = r;
    const double2 w = a.W[i + (long)k * a.ld];
    *out = a.f ? cscale(w, a.f[r]) : w;
  }
};

// Alg. 2: lam_k = sqrt(d_k) (work group = 256 entries)
struct Alg2LambdaOp {
  static constexpr int NT = 256;
  typedef Alg2Args Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int k = bx * 256 + threadIdx.x;
    if (k < a.n) a.lam[k] = sqrt(a.d[k]);
  }
};

// Alg. 2: the column scales of the sorted pairs (work group = 256 entries)
struct Alg2ScalesOp {
  static constexpr int NT = 256;
  typedef Alg2Args Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int r = bx * 256 + threadIdx.x;
    if (r >= a.n) return;
    int k = a.perm[r];
    if (k < 0 || k >= a.n) k = r;
    const double dk = a.d[k], lk = sqrt(dk);
    a.fy[r] = 1.0 / (dk * sqrt(lk));  // column of V_M Lambda^-1/2 from the column q_k d_k
    a.fx[r] = sqrt(lk) / dk;          // column of V_M Lambda^1/2
  }
};

// X[:, r] = s_k [(t_k V1_k + V2_k)/2; (V2_k - t_k V1_k)/2], k = perm[r];
// work group = (column r, 256 rows).
struct AssembleOp {
  static constexpr int NT = 256;
  typedef AssembleArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int aux) {
    const int n = a.n;
    const int gx = (n + 255) / 256;
    const int r = bx / gx;
    const int i = (bx % gx) * 256 + threadIdx.x;
    if (i >= n) return;
    int k = a.perm ? a.perm[r] : r;
    if (k < 0 || k >= n) k = r;
    const double sc = a.scl ? 0.5 * a.scl[k] : 0.5;
    double2 x = a.V1[i + (long)k * a.ldv];
    if (a.scl1) x = cscale(x, a.scl1[k]);
    const double2 y = a.V2[i + (long)k * a.ldv];
    const double2 top = cscale(cadd(x, y), sc);
    const double2 bot = cscale(csub(y, x), sc);
    double2* X = a.X;
    const long ldx = a.ldx;
    X[i + (long)r * ldx] = top;
    X[n + i + (long)r * ldx] = bot;
    if (a.want_negative) {
      X[i + (long)(n + r) * ldx] = bot;
      X[n + i + (long)(n + r) * ldx] = top;
    }
  }
};

// Scales of the SQRT route (Alg. 1) from the column norms dC of the iterated
// A - B (its eigenvalues) and dM of the iterated M (the squared eigenvalues):
// S = Z diag(dC^-3/2) Z^H, S^-1 = Z diag(dC^-5/2) Z^H, V1 = S^-1 Y dM^-3/4,
// V2 = S Y dM^-5/4, lambda = dM^1/2 (k < n; padded columns of A - B are unit
// vectors with dC = 1 and keep S = I there, padded V columns are zero).
// Alg. 1 scales (sqrt_scales); work group = 256 of the np entries
struct SqrtScalesOp {
  static constexpr int NT = 256;
  typedef SqrtScalesArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int k = bx * 256 + threadIdx.x;
    if (k >= a.np) return;
    const double c = a.dC[k];
    a.ks[k] = c > 0.0 ? 1.0 / (c * sqrt(c)) : 0.0;
    a.kis[k] = c > 0.0 ? 1.0 / (c * c * sqrt(c)) : 0.0;
    if (k < a.n) {
      const double m = a.dM[k], q = sqrt(sqrt(m));  // m^1/4
      a.c1[k] = m > 0.0 ? 1.0 / (m / q) : 0.0;       // m^-3/4
      a.c2[k] = m > 0.0 ? 1.0 / (m * q) : 0.0;       // m^-5/4
      a.lam[k] = sqrt(m);
    } else {
      a.c1[k] = 0.0;
      a.c2[k] = 0.0;
      a.lam[k] = 0.0;
    }
  }
};

inline int b256(int n) { return (n + 255) / 256; }

}  // namespace

hipError_t colnorm_z(int np, const double2* W, long ld, double* out, hipStream_t s) {
  const ColnormArgs<double2> a = {W, ld, np, out};
  return launch_one<ColnormOp<double2>>(a, np, 0, s);
}

hipError_t colnorm_c(int np, const float2* W, long ld, double* out, hipStream_t s) {
  const ColnormArgs<float2> a = {W, ld, np, out};
  return launch_one<ColnormOp<float2>>(a, np, 0, s);
}

template <typename C2>
static hipError_t scale_singular_run(int n, int np, C2* W, long ld, double* sigma, double* bnorm,
                                     hipStream_t s) {
  const ColnormArgs<C2> c1 = {W, ld, np, sigma};
  const ScaleArgs<C2> sc = {n, np, W, ld, sigma};
  const ColnormArgs<C2> c2 = {W, ld, np, bnorm};
  hipError_t e = launch_one<ColnormOp<C2>>(c1, np, 0, s);
  if (e == hipSuccess) e = launch_one<ScaleOp<C2>>(sc, cols_blocks(np, np), 0, s);
  if (e == hipSuccess) e = launch_one<ColnormOp<C2>>(c2, np, 0, s);
  return e;
}

hipError_t scale_singular_cols_z(int n, int np, double2* W, long ld, double* sigma, double* bnorm,
                                 hipStream_t s) {
  return scale_singular_run<double2>(n, np, W, ld, sigma, bnorm, s);
}

hipError_t scale_singular_cols_c(int n, int np, float2* W, long ld, double* sigma, double* bnorm,
                                 hipStream_t s) {
  return scale_singular_run<float2>(n, np, W, ld, sigma, bnorm, s);
}

hipError_t c64_to_c128(int np, const float2* S, long lds, double2* D, long ldd,
                       const double* colscale, hipStream_t s) {
  const C64Args a = {np, S, lds, D, ldd, colscale};
  return launch_one<C64Op>(a, cols_blocks(np, np), 0, s);
}

hipError_t lambda_from_norms(int n, int np, const double* anorm, const double* bnorm, double* lam,
                             double* invlam, double* scl, hipStream_t s, int v1scale) {
  const LambdaArgs a = {n, np, anorm, bnorm, lam, invlam, scl, v1scale};
  return launch_one<LambdaOp>(a, b256(np), 0, s);
}

hipError_t sort_lambda(int n, const double* lam, int* perm, double* lambda, int want_negative,
                       hipStream_t s) {
  const RankArgs r = {n, lam, perm, 0};
  const WriteLambdaArgs w = {n, lam, perm, lambda, want_negative};
  hipError_t e = launch_one<RankOp>(r, b256(n), 0, s);
  if (e == hipSuccess) e = launch_one<WriteLambdaOp>(w, b256(n), 0, s);
  return e;
}

hipError_t rq_lambda_z(int n, int np, const double2* T, long ld, const double* bnorm, double* anorm,
                       double* lam, double* invlam, double* scl, int* perm, double* lambda,
                       int want_negative, hipStream_t s) {
  const LambdaArgs la = {n, np, anorm, bnorm, lam, invlam, scl, 1};
  hipError_t e = colnorm_z(np, T, ld, anorm, s);
  if (e == hipSuccess) e = launch_one<LambdaOp>(la, b256(np), 0, s);
  if (e == hipSuccess) e = sort_lambda(n, lam, perm, lambda, want_negative, s);
  return e;
}

hipError_t gather_scale_z(int n, int np, const double2* W, long ld, const int* perm,
                          const double* f, double2* out, hipStream_t s) {
  const GatherArgs a = {n, np, W, ld, perm, f, out};
  return launch_one<GatherOp>(a, cols_blocks(np, np), 0, s);
}

hipError_t alg2_lambda_z(int n, const double* d, double* lam, int* perm, double* lambda,
                         int want_negative, double* fx, double* fy, hipStream_t s) {
  const Alg2Args a = {n, d, lam, perm, fx, fy};
  hipError_t e = launch_one<Alg2LambdaOp>(a, b256(n), 0, s);
  if (e == hipSuccess) e = sort_lambda(n, lam, perm, lambda, want_negative, s);
  if (e == hipSuccess) e = launch_one<Alg2ScalesOp>(a, b256(n), 0, s);
  return e;
}

hipError_t sqrt_scales(int n, int np, const double* dC, const double* dM, double* ks, double* kis,
                       double* c1, double* c2, double* lam, hipStream_t s) {
  const SqrtScalesArgs a = {n, np, dC, dM, ks, kis, c1, c2, lam};
  return launch_one<SqrtScalesOp>(a, b256(np), 0, s);
}

hipError_t assemble_z(int n, const double2* V1, const double2* V2, long ldv, const int* perm,
                      const double* scl, double2* X, long ldx, int want_negative, hipStream_t s,
                      const double* scl1) {
  const AssembleArgs a = {n, V1, V2, ldv, perm, scl, X, ldx, want_negative, scl1};
  return launch_one<AssembleOp>(a, cols_blocks(n, n), 0, s);
}

hipError_t group_finalize(GroupOp op, const void* table, const int2* map, int blocks, int aux,
                          hipStream_t s) {
  switch (op) {
    case G_COLNORM_Z: return launch_grp<ColnormOp<double2>>(table, map, blocks, aux, s);
    case G_COLNORM_C: return launch_grp<ColnormOp<float2>>(table, map, blocks, aux, s);
    case G_SCALE_Z: return launch_grp<ScaleOp<double2>>(table, map, blocks, aux, s);
    case G_SCALE_C: return launch_grp<ScaleOp<float2>>(table, map, blocks, aux, s);
    case G_LAMBDA: return launch_grp<LambdaOp>(table, map, blocks, aux, s);
    case G_RANK: return launch_grp<RankOp>(table, map, blocks, aux, s);
    case G_WRITE_LAMBDA: return launch_grp<WriteLambdaOp>(table, map, blocks, aux, s);
    case G_C64: return launch_grp<C64Op>(table, map, blocks, aux, s);
    case G_ASSEMBLE: return launch_grp<AssembleOp>(table, map, blocks, aux, s);
    case G_GATHER: return launch_grp<GatherOp>(table, map, blocks, aux, s);
    case G_ALG2_LAMBDA: return launch_grp<Alg2LambdaOp>(table, map, blocks, aux, s);
    case G_ALG2_SCALES: return launch_grp<Alg2ScalesOp>(table, map, blocks, aux, s);
    case G_SQRT_SCALES: return launch_grp<SqrtScalesOp>(table, map, blocks, aux, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bse
