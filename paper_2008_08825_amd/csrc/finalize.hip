// Finalisation of the SVD route and the final setup of Alg. 3.
//
// After the Jacobi iteration W_out = L2^H L1 U (U the accumulated rotations)
// has orthogonal columns w_k = sigma_k v_k (paper notation of Lemma
// SVDScalarFactors, where L1^H L2 = U Lambda V^H, so W = V Lambda U^H).
//   Ws = W_out diag(sigma)^-3/2      so that V2 = L2 Ws = L2 V Lambda^-1/2,
//   T  = L1^H V2                     (= U Lambda^1/2 in exact arithmetic),
//   V1 = L1 T Lambda^-1              (= M1 V2 Lambda^-1, the Lemma's relation).
// Eigenvalues: y = V2_k is an eigenvector of the Hermitian-definite pencil
// (M1, M2^-1) with eigenvalue lambda_k^2, so its Rayleigh quotient
//   lambda_k^2 = (y^H M1 y) / (y^H M2^-1 y) = ||T_k||^2 / ||Ws_k||^2
// is accurate to second order in the error of y; it replaces the column norm
// sigma_k, whose error grows with the number of rotations a column went
// through.  Each pair (V1_k, V2_k) is scaled by s_k = (||T_k|| ||Ws_k||)^-1/2
// so that V1_k^H V2_k = 1 exactly as in the Lemma.  The eigenvalues are
// sorted ascending (stable by index) and the final setup (Alg. 3 step 6)
// writes X = [(V1 + V2)/2; (V2 - V1)/2] in that order; the negative half is
// [0 I; I 0] X with eigenvalues -lambda (Lemma ComputeNegEvecs).
#include "common.hpp"
#include "internal.hpp"

namespace bse {
namespace {

template <typename C2>
__global__ __launch_bounds__(256) void k_colnorm(const C2* __restrict__ W, long ld, int np,
                                                 double* __restrict__ sigma) {
  __shared__ double red[256];
  const int j = blockIdx.x, tid = threadIdx.x;
  const C2* col = W + (long)j * ld;
  double s = 0.0;
  for (int i = tid; i < np; i += 256) {
    const double a = col[i].x, b = col[i].y;
    s += a * a + b * b;
  }
  red[tid] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) sigma[j] = sqrt(red[0]);
}

// rank_j = #{i : key_i < key_j or (key_i == key_j and i < j)}; perm[rank_j] = j,
// key = sigma (ascending) or -sigma (descending).
__global__ __launch_bounds__(256) void k_rank(int n, const double* __restrict__ sigma,
                                              int* __restrict__ perm, int desc) {
  __shared__ double sv[256];
  const double sg = desc ? -1.0 : 1.0;
  const int j = blockIdx.x * 256 + threadIdx.x;
  const double s = j < n ? sg * sigma[j] : 0.0;
  int rank = 0;
  for (int base = 0; base < n; base += 256) {
    const int i = base + threadIdx.x;
    sv[threadIdx.x] = i < n ? sg * sigma[i] : 0.0;
    __syncthreads();
    const int lim = min(256, n - base);
    for (int q = 0; q < lim; ++q) {
      const double v = sv[q];
      rank += (v < s) || (v == s && base + q < j);
    }
    __syncthreads();
  }
  if (j < n) perm[rank] = j;
}

template <typename C2>
__global__ __launch_bounds__(256) void k_scale_cols(int n, int np, C2* __restrict__ W, long ld,
                                                    const double* __restrict__ sigma) {
  const int k = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  double f = 0.0;
  if (k < n) {
    const double sg = sigma[k];
    f = sg > 0.0 ? 1.0 / (sg * sqrt(sg)) : 0.0;
  }
  C2 v = W[i + (long)k * ld];
  v.x = v.x * f;
  v.y = v.y * f;
  W[i + (long)k * ld] = v;
}

__global__ __launch_bounds__(256) void k_c64_to_c128(int np, const float2* __restrict__ S, long lds,
                                                     double2* __restrict__ D, long ldd,
                                                     const double* __restrict__ colscale) {
  const int j = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  const float2 v = S[i + (long)j * lds];
  const double f = colscale ? colscale[j] : 1.0;
  D[i + (long)j * ldd] = make_double2(f * v.x, f * v.y);
}

__global__ __launch_bounds__(256) void k_lambda(int n, int np, const double* __restrict__ anorm,
                                                const double* __restrict__ bnorm,
                                                double* __restrict__ lam, double* __restrict__ invlam,
                                                double* __restrict__ scl) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= np) return;
  if (k < n) {
    const double a = anorm[k], b = bnorm[k];
    const double l = a / b;
    lam[k] = l;
    invlam[k] = 1.0 / l;
    scl[k] = 1.0 / sqrt(a * b);
  } else {
    lam[k] = 0.0;
    invlam[k] = 0.0;
    scl[k] = 0.0;
  }
}

__global__ __launch_bounds__(256) void k_write_lambda(int n, const double* __restrict__ lam,
                                                      const int* __restrict__ perm,
                                                      double* __restrict__ lambda, int want_negative) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  int j = perm[r];
  if (j < 0 || j >= n) j = r;  // only if a value was NaN (ranks then collide)
  lambda[r] = lam[j];
  if (want_negative) lambda[n + r] = -lam[j];
}

__global__ __launch_bounds__(256) void k_gather_scale(int n, int np, const double2* __restrict__ W,
                                                      long ld, const int* __restrict__ perm,
                                                      const double* __restrict__ f,
                                                      double2* __restrict__ out) {
  const int r = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  if (r >= n) { out[i + (long)r * ld] = make_double2(0.0, 0.0); return; }
  int k = perm[r];
  if (k < 0 || k >= n) k = r;
  out[i + (long)r * ld] = cscale(W[i + (long)k * ld], f[r]);
}

__global__ __launch_bounds__(256) void k_alg2_lambda(int n, const double* __restrict__ d,
                                                     double* __restrict__ lam) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < n) lam[k] = sqrt(d[k]);
}

__global__ __launch_bounds__(256) void k_alg2_scales(int n, const double* __restrict__ d,
                                                     const int* __restrict__ perm,
                                                     double* __restrict__ fx, double* __restrict__ fy) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  int k = perm[r];
  if (k < 0 || k >= n) k = r;
  const double dk = d[k], lk = sqrt(dk);
  fy[r] = 1.0 / (dk * sqrt(lk));  // column of V_M Lambda^-1/2 from the column q_k d_k
  fx[r] = sqrt(lk) / dk;          // column of V_M Lambda^1/2
}

__global__ __launch_bounds__(256) void k_assemble(int n, const double2* __restrict__ V1,
                                                  const double2* __restrict__ V2, long ldv,
                                                  const int* __restrict__ perm,
                                                  const double* __restrict__ scl,
                                                  double2* __restrict__ X, long ldx, int want_negative) {
  const int r = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int k = perm ? perm[r] : r;
  if (k < 0 || k >= n) k = r;
  const double sc = scl ? 0.5 * scl[k] : 0.5;
  const double2 a = V1[i + (long)k * ldv];
  const double2 b = V2[i + (long)k * ldv];
  const double2 top = cscale(cadd(a, b), sc);
  const double2 bot = cscale(csub(b, a), sc);
  X[i + (long)r * ldx] = top;
  X[n + i + (long)r * ldx] = bot;
  if (want_negative) {
    X[i + (long)(n + r) * ldx] = bot;
    X[n + i + (long)(n + r) * ldx] = top;
  }
}

}  // namespace

hipError_t colnorm_z(int np, const double2* W, long ld, double* out, hipStream_t s) {
  k_colnorm<double2><<<np, 256, 0, s>>>(W, ld, np, out);
  return hipGetLastError();
}

hipError_t colnorm_c(int np, const float2* W, long ld, double* out, hipStream_t s) {
  k_colnorm<float2><<<np, 256, 0, s>>>(W, ld, np, out);
  return hipGetLastError();
}

template <typename C2>
static hipError_t scale_singular_run(int n, int np, C2* W, long ld, double* sigma, double* bnorm,
                                     hipStream_t s) {
  k_colnorm<C2><<<np, 256, 0, s>>>(W, ld, np, sigma);
  dim3 g((np + 255) / 256, np);
  k_scale_cols<C2><<<g, 256, 0, s>>>(n, np, W, ld, sigma);
  k_colnorm<C2><<<np, 256, 0, s>>>(W, ld, np, bnorm);
  return hipGetLastError();
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
  dim3 g((np + 255) / 256, np);
  k_c64_to_c128<<<g, 256, 0, s>>>(np, S, lds, D, ldd, colscale);
  return hipGetLastError();
}

hipError_t lambda_from_norms(int n, int np, const double* anorm, const double* bnorm, double* lam,
                             double* invlam, double* scl, hipStream_t s) {
  k_lambda<<<(np + 255) / 256, 256, 0, s>>>(n, np, anorm, bnorm, lam, invlam, scl);
  return hipGetLastError();
}

hipError_t sort_lambda(int n, const double* lam, int* perm, double* lambda, int want_negative,
                       hipStream_t s) {
  k_rank<<<(n + 255) / 256, 256, 0, s>>>(n, lam, perm, 0);
  k_write_lambda<<<(n + 255) / 256, 256, 0, s>>>(n, lam, perm, lambda, want_negative);
  return hipGetLastError();
}

hipError_t rq_lambda_z(int n, int np, const double2* T, long ld, const double* bnorm, double* anorm,
                       double* lam, double* invlam, double* scl, int* perm, double* lambda,
                       int want_negative, hipStream_t s) {
  k_colnorm<double2><<<np, 256, 0, s>>>(T, ld, np, anorm);
  k_lambda<<<(np + 255) / 256, 256, 0, s>>>(n, np, anorm, bnorm, lam, invlam, scl);
  k_rank<<<(n + 255) / 256, 256, 0, s>>>(n, lam, perm, 0);
  k_write_lambda<<<(n + 255) / 256, 256, 0, s>>>(n, lam, perm, lambda, want_negative);
  return hipGetLastError();
}

hipError_t gather_scale_z(int n, int np, const double2* W, long ld, const int* perm,
                          const double* f, double2* out, hipStream_t s) {
  dim3 g((np + 255) / 256, np);
  k_gather_scale<<<g, 256, 0, s>>>(n, np, W, ld, perm, f, out);
  return hipGetLastError();
}

hipError_t alg2_lambda_z(int n, const double* d, double* lam, int* perm, double* lambda,
                         int want_negative, double* fx, double* fy, hipStream_t s) {
  k_alg2_lambda<<<(n + 255) / 256, 256, 0, s>>>(n, d, lam);
  k_rank<<<(n + 255) / 256, 256, 0, s>>>(n, lam, perm, 0);
  k_write_lambda<<<(n + 255) / 256, 256, 0, s>>>(n, lam, perm, lambda, want_negative);
  k_alg2_scales<<<(n + 255) / 256, 256, 0, s>>>(n, d, perm, fx, fy);
  return hipGetLastError();
}

hipError_t assemble_z(int n, const double2* V1, const double2* V2, long ldv, const int* perm,
                      const double* scl, double2* X, long ldx, int want_negative, hipStream_t s) {
  dim3 g((n + 255) / 256, n);
  k_assemble<<<g, 256, 0, s>>>(n, V1, V2, ldv, perm, scl, X, ldx, want_negative);
  return hipGetLastError();
}

}  // namespace bse
