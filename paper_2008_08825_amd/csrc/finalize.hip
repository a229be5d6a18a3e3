// Finalisation of the SVD route and the final setup of Alg. 3.
//
// After the Jacobi iteration W_out = L2^H L1 U (U the accumulated rotations)
// has orthogonal columns w_j = sigma_j v_j (paper notation of Lemma
// SVDScalarFactors, where L1^H L2 = U Lambda V^H, so W = V Lambda U^H):
//   lambda_j = sigma_j = ||w_j||              (ascending, stable by index)
//   Ws[:, r] = w_perm(r) sigma^-3/2 = v sigma^-1/2   so that  V2 = L2 Ws,
// and V1 follows from the Lemma's relation M1 V2 = V1 Lambda.
// The final setup (Alg. 3 step 6) is X = [(V1 + V2)/2; (V2 - V1)/2]; the
// negative half is [0 I; I 0] X with eigenvalues -lambda (Lemma ComputeNegEvecs).
#include "common.hpp"
#include "internal.hpp"

namespace bse {
namespace {

__global__ __launch_bounds__(256) void k_colnorm(const double2* __restrict__ W, long ld, int np,
                                                 double* __restrict__ sigma) {
  __shared__ double red[256];
  const int j = blockIdx.x, tid = threadIdx.x;
  const double2* col = W + (long)j * ld;
  double s = 0.0;
  for (int i = tid; i < np; i += 256) s += cabs2(col[i]);
  red[tid] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) sigma[j] = sqrt(red[0]);
}

// rank_j = #{i : sigma_i < sigma_j or (sigma_i == sigma_j and i < j)}; perm[rank_j] = j.
__global__ __launch_bounds__(256) void k_rank(int n, const double* __restrict__ sigma,
                                              int* __restrict__ perm) {
  __shared__ double sv[256];
  const int j = blockIdx.x * 256 + threadIdx.x;
  const double s = j < n ? sigma[j] : 0.0;
  int rank = 0;
  for (int base = 0; base < n; base += 256) {
    const int i = base + threadIdx.x;
    sv[threadIdx.x] = i < n ? sigma[i] : 0.0;
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

__global__ __launch_bounds__(256) void k_gather(int n, int np, const double2* __restrict__ W, long ld,
                                                const double* __restrict__ sigma,
                                                const int* __restrict__ perm, double* __restrict__ lambda,
                                                int want_negative, double* __restrict__ invlam,
                                                double2* __restrict__ Ws) {
  const int r = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) {
    if (i < np) Ws[i + (long)r * ld] = make_double2(0.0, 0.0);
    if (i == 0) invlam[r] = 0.0;
    return;
  }
  int j = perm[r];
  if (j < 0 || j >= n) j = r;  // only if sigma held NaN (ranks then collide)
  const double s = sigma[j];
  const double f = 1.0 / (s * sqrt(s));
  if (i < np) Ws[i + (long)r * ld] = cscale(W[i + (long)j * ld], f);
  if (i == 0) {
    lambda[r] = s;
    if (want_negative) lambda[n + r] = -s;
    invlam[r] = 1.0 / s;
  }
}

__global__ __launch_bounds__(256) void k_assemble(int n, const double2* __restrict__ V1,
                                                  const double2* __restrict__ V2, long ldv,
                                                  double2* __restrict__ X, long ldx, int want_negative) {
  const int r = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double2 a = V1[i + (long)r * ldv];
  const double2 b = V2[i + (long)r * ldv];
  const double2 top = cscale(cadd(a, b), 0.5);
  const double2 bot = cscale(csub(b, a), 0.5);
  X[i + (long)r * ldx] = top;
  X[n + i + (long)r * ldx] = bot;
  if (want_negative) {
    X[i + (long)(n + r) * ldx] = bot;
    X[n + i + (long)(n + r) * ldx] = top;
  }
}

}  // namespace

hipError_t finalize_sort_z(int n, int np, const double2* W, long ld, double* sigma, int* perm,
                           double* lambda, int want_negative, double* invlam, double2* Ws,
                           hipStream_t s) {
  k_colnorm<<<np, 256, 0, s>>>(W, ld, np, sigma);
  k_rank<<<(n + 255) / 256, 256, 0, s>>>(n, sigma, perm);
  dim3 g((np + 255) / 256, np);
  k_gather<<<g, 256, 0, s>>>(n, np, W, ld, sigma, perm, lambda, want_negative, invlam, Ws);
  return hipGetLastError();
}

hipError_t assemble_z(int n, const double2* V1, const double2* V2, long ldv, double2* X, long ldx,
                      int want_negative, hipStream_t s) {
  dim3 g((n + 255) / 256, n);
  k_assemble<<<g, 256, 0, s>>>(n, V1, V2, ldv, X, ldx, want_negative);
  return hipGetLastError();
}

}  // namespace bse
