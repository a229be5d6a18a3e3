// Forming M1 = A + B, M2 = A - B and their blocked Cholesky factorisations
// (Alg. 3 steps 1-2; Thm ProdEig defines M1, M2; Lemma Qtransform part 2 says
// both factorisations succeed exactly when the BSE Hamiltonian is definite).
//
// Right-looking blocked Cholesky with 64-column panels:
//   1. one workgroup factors the 64 x 64 diagonal block in LDS (FP64) and
//      also forms the inverse of that triangular block;
//   2. the panel below is L21 = A21 L11^-H, a GEMM against the inverse;
//   3. the trailing matrix takes the Hermitian rank-64 update
//      A22 -= L21 L21^H on MFMA, lower tiles only.
#include "common.hpp"
#include "internal.hpp"
#include "lds_la.hpp"

#include <climits>
#include <mutex>

namespace bse {
namespace {

constexpr int NB = 64;

// One 64 x 64 tile of M1/M2 per workgroup.  Reading the upper triangle of a
// column-major matrix means reading it transposed, so the tile goes through
// LDS to keep global reads coalesced.
struct FormOp {
  static constexpr int NT = 256;
  typedef FormArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int aux);
};

BSE_DEV void FormOp::run(const FormArgs& a, int bx, int) {
  const int n = a.n, np = a.np, upper = a.upper;
  const double2* __restrict__ A = a.A;
  const double2* __restrict__ B = a.B;
  const long lda = a.lda, ldb = a.ldb, ldm = a.ldm;
  double2* __restrict__ M1 = a.M1;
  double2* __restrict__ M2 = a.M2;
  __shared__ double2 tile[64][65];
  const int T = np / 64;
  const int tm = bx % T, tn = bx / T;
  const int m0 = tm * 64, n0 = tn * 64;
  const int tid = threadIdx.x;
  double2 va[16], vb[16];
  if (tn <= tm) {
    for (int pass = 0; pass < 2; ++pass) {
      const double2* S = pass == 0 ? A : B;
      const long lds = pass == 0 ? lda : ldb;
      double2* v = pass == 0 ? va : vb;
      if (!S) {  // B == nullptr: B = 0 (Tamm-Dancoff)
        for (int q = 0; q < 16; ++q) v[q] = make_double2(0.0, 0.0);
      } else if (upper) {
        // element (i, j) of the lower triangle is conj(S[j + i * lds])
        for (int q = 0; q < 16; ++q) {
          int cc = tid & 63, rr = (tid >> 6) + 4 * q;  // cc runs along j (contiguous)
          int i = m0 + rr, j = n0 + cc;
          double2 x = make_double2(0.0, 0.0);
          if (i < n && j < n && i >= j) x = S[j + (long)i * lds];
          tile[rr][cc] = x;
        }
        __syncthreads();
        for (int q = 0; q < 16; ++q) {
          int r = tid & 63, c = (tid >> 6) + 4 * q;
          double2 x = tile[r][c];
          v[q] = make_double2(x.x, -x.y);
        }
        __syncthreads();
      } else {
        for (int q = 0; q < 16; ++q) {
          int r = tid & 63, c = (tid >> 6) + 4 * q;
          int i = m0 + r, j = n0 + c;
          double2 x = make_double2(0.0, 0.0);
          if (i < n && j < n && i >= j) x = S[i + (long)j * lds];
          v[q] = x;
        }
      }
    }
  }
  for (int q = 0; q < 16; ++q) {
    int r = tid & 63, c = (tid >> 6) + 4 * q;
    int i = m0 + r, j = n0 + c;
    double2 o1, o2;
    if (i >= n || j >= n) {
      double d = (i == j) ? 1.0 : 0.0;
      o1 = make_double2(d, 0.0); o2 = o1;
    } else if (i < j) {
      o1 = make_double2(0.0, 0.0); o2 = o1;
    } else if (i == j) {
      o1 = make_double2(va[q].x + vb[q].x, 0.0);
      o2 = make_double2(va[q].x - vb[q].x, 0.0);
    } else {
      o1 = cadd(va[q], vb[q]);
      o2 = csub(va[q], vb[q]);
    }
    M1[i + (long)j * ldm] = o1;
    M2[i + (long)j * ldm] = o2;
  }
}

// Unblocked Cholesky of the diagonal block M[j0:j0+64, j0:j0+64] (lower) and
// the inverse of the resulting triangle, in one workgroup.  Writes L11 back
// with a zero strict upper triangle and L11^-1 (64 x 64, ld 64) to `linv`.
// C2 is the storage type (double2, or float2 in the mixed form); the block is
// factored in FP64 either way.
//
// The columns stay unscaled during the elimination (step j subtracts
// L[i][j] conj(L[k][j]) / L[j][j] from L[i][k], k > j, reading only column j,
// which the step does not write), so each step needs one barrier; the
// columns are scaled by 1 / sqrt(L[j][j]) at the end.
template <typename C2>
struct Potf2Op {
  static constexpr int NT = 256;
  typedef Potf2Args<C2> Args;
  static BSE_DEV void run(const Args& a, int bx, int j0);
};

template <typename C2>
BSE_DEV void Potf2Op<C2>::run(const Potf2Args<C2>& a, int, int j0) {
  C2* M = a.M;
  const long ld = a.ld;
  C2* __restrict__ linv = a.linv;
  int* status = a.status;
  const int base = a.base, n_real = a.n_real;
  __shared__ double Lr[NB][NB + 1], Li[NB][NB + 1];
  __shared__ double Xr[NB][NB + 1], Xi[NB][NB + 1];
  __shared__ double sc[NB];
  const int tid = threadIdx.x;
  C2* D = M + j0 + (long)j0 * ld;
  for (int q = 0; q < 16; ++q) {
    int r = tid & 63, c = (tid >> 6) + 4 * q;
    double vr = 0.0, vi = 0.0;
    if (r >= c) { const C2 v = D[r + (long)c * ld]; vr = v.x; vi = v.y; }
    Lr[r][c] = vr; Li[r][c] = vi;
  }
  __syncthreads();
  const int i = tid & 63;
  for (int j = 0; j < NB; ++j) {
    const double d = Lr[j][j];  // every thread reads the same pivot
    if (!(d > 0.0)) {
      // leave the block as is; the caller stops after reading the status
      if (tid == 0 && j0 + j < n_real) atomicMin(status, base + j0 + j + 1);
      return;
    }
    if (i > j) {
      const double rd = 1.0 / d;
      const double lr = Lr[i][j] * rd, li = Li[i][j] * rd;
      for (int k = j + 1 + (tid >> 6); k <= i; k += 4) {
        const double kr = Lr[k][j], ki = Li[k][j];
        Lr[i][k] -= lr * kr + li * ki;
        Li[i][k] -= li * kr - lr * ki;
      }
    }
    __syncthreads();
  }
  if (tid < NB) sc[tid] = 1.0 / sqrt(Lr[tid][tid]);
  __syncthreads();
  for (int q = 0; q < 16; ++q) {
    const int r = tid & 63, c = (tid >> 6) + 4 * q;
    if (r > c) { Lr[r][c] *= sc[c]; Li[r][c] *= sc[c]; }
    else if (r == c) { Lr[r][c] *= sc[c]; Li[r][c] = 0.0; }
  }
  __syncthreads();
  tri_inverse_lds(Lr, Li, Xr, Xi, tid);
  for (int q = 0; q < 16; ++q) {
    int r = tid & 63, c = (tid >> 6) + 4 * q;
    C2 l, x;
    l.x = (r >= c) ? Lr[r][c] : 0.0;
    l.y = (r >= c) ? Li[r][c] : 0.0;
    x.x = Xr[r][c];
    x.y = Xi[r][c];
    D[r + (long)c * ld] = l;
    linv[r + c * NB] = x;
  }
}

// Inverses of the 64 x 64 diagonal blocks of a lower-triangular L (one
// workgroup per block), written as lower triangles, block b at inv + b * 64 * 64;
// formed in FP64 for complex128 and complex64 storage alike.
template <typename C2>
struct TriInvOp {
  static constexpr int NT = 256;
  typedef TriInvArgsT<C2> Args;
  static BSE_DEV void run(const Args& a, int bx, int aux) {
    __shared__ double Lr[NB][NB + 1], Li[NB][NB + 1];
    __shared__ double Xr[NB][NB + 1], Xi[NB][NB + 1];
    const int tid = threadIdx.x;
    const int j0 = bx * NB;
    const C2* D = a.L + j0 + (long)j0 * a.ld;
    for (int q = 0; q < 16; ++q) {
      const int r = tid & 63, c = (tid >> 6) + 4 * q;
      double vr = 0.0, vi = 0.0;
      if (r >= c) { const C2 v = D[r + (long)c * a.ld]; vr = v.x; vi = v.y; }
      Lr[r][c] = vr; Li[r][c] = vi;
    }
    __syncthreads();
    tri_inverse_lds(Lr, Li, Xr, Xi, tid);
    C2* out = a.inv + (long)bx * NB * NB;
    for (int q = 0; q < 16; ++q) {
      const int r = tid & 63, c = (tid >> 6) + 4 * q;
      C2 x;
      x.x = Xr[r][c];
      x.y = Xi[r][c];
      out[r + c * NB] = x;
    }
  }
};

// Upper triangle of a square np x np matrix from its lower one: M[i][j] = conj(M[j][i]), i < j.
struct MirrorOp {
  static constexpr int NT = 256;
  typedef MirrorArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int aux);
};

BSE_DEV void MirrorOp::run(const MirrorArgs& a, int bx, int) {
  const int np = a.np;
  double2* M = a.M;
  const long ld = a.ld;
  __shared__ double2 tile[64][65];
  const int T = np / 64;
  const int tm = bx % T, tn = bx / T;
  if (tn < tm) return;  // target tile (tm, tn) on or above the diagonal
  const int m0 = tm * 64, n0 = tn * 64;
  const int tid = threadIdx.x;
  // source tile (tn, tm): rows n0.., cols m0..
  for (int q = 0; q < 16; ++q) {
    const int r = tid & 63, c = (tid >> 6) + 4 * q;
    tile[r][c] = M[(n0 + r) + (long)(m0 + c) * ld];
  }
  __syncthreads();
  for (int q = 0; q < 16; ++q) {
    const int r = tid & 63, c = (tid >> 6) + 4 * q;  // target (m0 + r, n0 + c)
    if (m0 + r < n0 + c) M[(m0 + r) + (long)(n0 + c) * ld] = cconj(tile[c][r]);
  }
}

// complex64 copy of the lower triangle (strict upper part zero), one 64 x 64 tile per workgroup.
struct ToC64Op {
  static constexpr int NT = 256;
  typedef ToC64Args Args;
  static BSE_DEV void run(const Args& a, int bx, int aux);
};

BSE_DEV void ToC64Op::run(const ToC64Args& a, int bx, int) {
  const int T = a.np / 64;
  const int m0 = (bx % T) * 64, n0 = (bx / T) * 64;
  const double2* __restrict__ M = a.M;
  float2* __restrict__ Mc = a.Mc;
  for (int q = 0; q < 16; ++q) {
    const int i = m0 + (threadIdx.x & 63), j = n0 + (threadIdx.x >> 6) + 4 * q;
    float2 v = make_float2(0.f, 0.f);
    if (i >= j) { const double2 x = M[i + (long)j * a.ld]; v = make_float2((float)x.x, (float)x.y); }
    Mc[i + (long)j * a.ld] = v;
  }
}

// complex64 copy of a whole np x np matrix, one 64 x 64 tile per workgroup.
struct ZToCOp {
  static constexpr int NT = 256;
  typedef ToC64Args Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int T = a.np / 64;
    const int m0 = (bx % T) * 64, n0 = (bx / T) * 64;
    for (int q = 0; q < 16; ++q) {
      const int i = m0 + (threadIdx.x & 63), j = n0 + (threadIdx.x >> 6) + 4 * q;
      const double2 x = a.M[i + (long)j * a.ld];
      a.Mc[i + (long)j * a.ld] = make_float2((float)x.x, (float)x.y);
    }
  }
};

// Lower triangle of a Hermitian n x n matrix embedded in np x np: strict
// upper part set to zero, rows and columns n..np-1 set to the identity's.
// mode 1 instead writes the np x np identity.
struct TriPadOp {
  static constexpr int NT = 256;
  typedef TriPadArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int) {
    const int T = a.np / 64;
    const int m0 = (bx % T) * 64, n0 = (bx / T) * 64;
    for (int q = 0; q < 16; ++q) {
      const int i = m0 + (threadIdx.x & 63), j = n0 + (threadIdx.x >> 6) + 4 * q;
      double2* p = a.M + i + (long)j * a.ld;
      if (a.identity || i < j || i >= a.n || j >= a.n)
        *p = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
  }
};

}  // namespace

hipError_t z_to_c64(int np, const double2* M, long ld, float2* Mc, hipStream_t s) {
  const ToC64Args a = {np, M, ld, Mc};
  return launch_one<ZToCOp>(a, tiles64(np), 0, s);
}

hipError_t tri_pad_z(int n, int np, double2* M, long ld, int identity, hipStream_t s) {
  const TriPadArgs a = {n, np, M, ld, identity};
  return launch_one<TriPadOp>(a, tiles64(np), 0, s);
}

hipError_t form_m12(int n, int np, const double2* A, long lda, const double2* B, long ldb,
                    int upper, double2* M1, double2* M2, long ldm, hipStream_t s) {
  const FormArgs a = {n, np, A, lda, B, ldb, upper, M1, M2, ldm};
  return launch_one<FormOp>(a, tiles64(np), 0, s);
}

hipError_t mirror_upper_z(int np, double2* M, long ld, hipStream_t s) {
  const MirrorArgs a = {np, M, ld};
  return launch_one<MirrorOp>(a, tiles64(np), 0, s);
}

hipError_t lower_to_c64(int np, const double2* M, long ld, float2* Mc, hipStream_t s) {
  const ToC64Args a = {np, M, ld, Mc};
  return launch_one<ToC64Op>(a, tiles64(np), 0, s);
}

// Right-looking, two 64-column panels at a time: the first panel's block is
// factored (Potf2), its rows below solved against the block's inverse, and
// only the next column block updated with it; then the second panel likewise;
// then the rest of the matrix is updated with both panels at once (K = 128),
// so the trailing matrix passes through the update half as often.
template <typename C2>
static hipError_t cholesky_run(int np, int n_real, C2* M, long ld, C2* linv, int* status,
                               int base, hipStream_t s) {
  hipError_t (*gemm)(const GemmDesc&, hipStream_t) = sizeof(C2) == 16 ? gemm_z : gemm_c;
  auto factor_panel = [&](int j0) -> hipError_t {  // Potf2, then L21 = A21 L11^-H below it
    const Potf2Args<C2> pa = {M, ld, linv, status, base, n_real};
    hipError_t e = launch_one<Potf2Op<C2>>(pa, 1, j0, s);
    if (e != hipSuccess) return e;
    const int rows = np - j0 - NB;
    if (rows <= 0) return hipSuccess;
    C2* panel = M + (j0 + NB) + (long)j0 * ld;
    GemmDesc t;  // in place: one workgroup per row tile
    t.M = rows; t.N = NB; t.K = NB;
    t.A = panel; t.lda = ld; t.opA = 0;
    t.B = linv; t.ldb = NB; t.opB = 1; t.triB = 1;
    t.C = panel; t.ldc = ld;
    return gemm(t, s);
  };
  for (int j0 = 0; j0 < np; j0 += 2 * NB) {
    hipError_t e = factor_panel(j0);
    if (e != hipSuccess) return e;
    const int rows = np - j0 - NB;
    if (rows <= 0) break;
    {
      GemmDesc h;  // next column block: A[j0+64.., j0+64..j0+128] -= L21 L21[0..64]^H
      C2* panel = M + (j0 + NB) + (long)j0 * ld;
      h.M = rows; h.N = NB; h.K = NB;
      h.A = panel; h.lda = ld; h.opA = 0;
      h.B = panel; h.ldb = ld; h.opB = 1;
      h.C = M + (j0 + NB) + (long)(j0 + NB) * ld; h.ldc = ld;
      h.alpha_re = -1.0; h.beta_re = 1.0;
      if ((e = gemm(h, s)) != hipSuccess) return e;
    }
    if ((e = factor_panel(j0 + NB)) != hipSuccess) return e;
    const int rest = rows - NB;
    if (rest <= 0) break;
    GemmDesc u;  // A22 -= L[rest, j0..j0+128] L[rest, j0..j0+128]^H, lower tiles
    C2* both = M + (j0 + 2 * NB) + (long)j0 * ld;
    u.M = rest; u.N = rest; u.K = 2 * NB;
    u.A = both; u.lda = ld; u.opA = 0;
    u.B = both; u.ldb = ld; u.opB = 1;
    u.C = M + (j0 + 2 * NB) + (long)(j0 + 2 * NB) * ld; u.ldc = ld;
    u.alpha_re = -1.0; u.beta_re = 1.0; u.lowerC = 1;
    if ((e = gemm(u, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t cholesky_z(int np, int n_real, double2* M, long ld, double2* linv, int* status,
                      int base, hipStream_t s) {
  return cholesky_run<double2>(np, n_real, M, ld, linv, status, base, s);
}

// The block triangular solves take the 64-column diagonal blocks kTrsmGroup
// at a time: a block of the group is first updated with the group's blocks
// already solved (K = 64, 128, ...), then solved against its diagonal block's
// inverse; after the group the rest of the right-hand side is updated with
// all of its blocks at once (K = 64 kTrsmGroup), so the remaining rows pass
// through the update kTrsmGroup times less often than with one block at a time.

hipError_t trsm_lh_z(int np, const double2* L, long ld, double2* Rhs, double2* Z, double2* inv,
                     hipStream_t s) {
  const int nb = np / NB;
  const TriInvArgs ti = {L, ld, inv};
  hipError_t e = launch_one<TriInvOp<double2>>(ti, nb, 0, s);
  if (e != hipSuccess) return e;
  trsm_lh_for_each(np, L, ld, Rhs, Z, inv, [&](const TrsmStep& st) {
    if (e == hipSuccess) e = gemm_z(st.g, s);
  });
  return e;
}

hipError_t trsm_lh_c(int np, const float2* L, long ld, float2* Rhs, float2* Z, float2* inv,
                     hipStream_t s) {
  const int nb = np / NB;
  const TriInvArgsT<float2> ti = {L, ld, inv};
  hipError_t e = launch_one<TriInvOp<float2>>(ti, nb, 0, s);
  if (e != hipSuccess) return e;
  trsm_lh_for_each(np, L, ld, Rhs, Z, inv, [&](const TrsmStep& st) {
    if (e == hipSuccess) e = gemm_c(st.g, s);
  });
  return e;
}

hipError_t trsm_ln_z(int np, const double2* L, long ld, double2* Rhs, double2* Z, double2* inv,
                     hipStream_t s) {
  const int nb = np / NB;
  const TriInvArgs ti = {L, ld, inv};
  hipError_t e = launch_one<TriInvOp<double2>>(ti, nb, 0, s);
  if (e != hipSuccess) return e;
  trsm_ln_for_each(np, L, ld, Rhs, Z, inv, [&](const TrsmStep& st) {
    if (e == hipSuccess) e = gemm_z(st.g, s);
  });
  return e;
}

hipError_t trsm_rh_z(int np, const double2* L, long ld, double2* Rhs, double2* Z, double2* inv,
                     hipStream_t s) {
  const int nb = np / NB;
  const TriInvArgs ti = {L, ld, inv};
  hipError_t e = launch_one<TriInvOp<double2>>(ti, nb, 0, s);
  if (e != hipSuccess) return e;
  trsm_rh_for_each(np, L, ld, Rhs, Z, inv, [&](const TrsmStep& st) {
    if (e == hipSuccess) e = gemm_z(st.g, s);
  });
  return e;
}

hipError_t cholesky_c(int np, int n_real, float2* M, long ld, float2* linv, int* status,
                      int base, hipStream_t s) {
  return cholesky_run<float2>(np, n_real, M, ld, linv, status, base, s);
}

// The two factorisations of Alg. 3 steps 1-2 are independent, and each is a
// chain of small latency-bound steps (one work group factors a diagonal
// block while the rest of the chip waits), so they run side by side: the
// second on a library stream of the device (default priority), forked from
// and joined back to the caller's stream by events.  The enqueue sequence
// holds a lock, so calls from several host threads do not mix up the events.
namespace {
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
constexpr int kMaxDevices = 64;
std::mutex g_side_mu;
SideStream g_side[kMaxDevices];
}  // namespace

template <typename C2>
static hipError_t cholesky_pair_run(int np, int n_real, C2* M1, C2* M2, long ld, C2* linv,
                                    int* status, hipStream_t s, int side) {
  int dev = 0;  // the device of the caller's stream (the current device for the null stream)
  hipError_t e = hipStreamGetDevice(s, &dev);
  if (e != hipSuccess) return e;
  if (!side || dev < 0 || dev >= kMaxDevices) {
    if ((e = cholesky_run<C2>(np, n_real, M1, ld, linv, status, 0, s)) != hipSuccess) return e;
    return cholesky_run<C2>(np, n_real, M2, ld, linv + NB * NB, status, n_real, s);
  }
  std::lock_guard<std::mutex> lock(g_side_mu);
  SideStream& sd = g_side[dev];
  if (!sd.s) {  // created on the stream's device, kept until the process ends
    int cur = 0;
    if ((e = hipGetDevice(&cur)) != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    e = hipStreamCreateWithFlags(&sd.s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sd.join, hipEventDisableTiming);
    const hipError_t er = cur != dev ? hipSetDevice(cur) : hipSuccess;
    if (e != hipSuccess) {
      sd.s = nullptr;  // try again on the next call
      return e;
    }
    if (er != hipSuccess) return er;
  }
  if ((e = hipEventRecord(sd.fork, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(sd.s, sd.fork, 0)) != hipSuccess) return e;
  const hipError_t e1 = cholesky_run<C2>(np, n_real, M1, ld, linv, status, 0, s);
  const hipError_t e2 = cholesky_run<C2>(np, n_real, M2, ld, linv + NB * NB, status, n_real, sd.s);
  // join even after a failed launch, so that s never runs ahead of the side stream
  if ((e = hipEventRecord(sd.join, sd.s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(s, sd.join, 0)) != hipSuccess) return e;
  return e1 != hipSuccess ? e1 : e2;
}

hipError_t cholesky_pair_z(int np, int n_real, double2* M1, double2* M2, long ld, double2* linv,
                           int* status, hipStream_t s, int side) {
  return cholesky_pair_run<double2>(np, n_real, M1, M2, ld, linv, status, s, side);
}

hipError_t cholesky_pair_c(int np, int n_real, float2* M1, float2* M2, long ld, float2* linv,
                           int* status, hipStream_t s, int side) {
  return cholesky_pair_run<float2>(np, n_real, M1, M2, ld, linv, status, s, side);
}

hipError_t group_chol(GroupOp op, const void* table, const int2* map, int blocks, int aux,
                      hipStream_t s) {
  switch (op) {
    case G_FORM: return launch_grp<FormOp>(table, map, blocks, aux, s);
    case G_MIRROR: return launch_grp<MirrorOp>(table, map, blocks, aux, s);
    case G_TOC64: return launch_grp<ToC64Op>(table, map, blocks, aux, s);
    case G_POTF2_Z: return launch_grp<Potf2Op<double2>>(table, map, blocks, aux, s);
    case G_POTF2_C: return launch_grp<Potf2Op<float2>>(table, map, blocks, aux, s);
    case G_TRIINV: return launch_grp<TriInvOp<double2>>(table, map, blocks, aux, s);
    case G_TRIINV_C: return launch_grp<TriInvOp<float2>>(table, map, blocks, aux, s);
    case G_ZTOC: return launch_grp<ZToCOp>(table, map, blocks, aux, s);
    case G_TRIPAD: return launch_grp<TriPadOp>(table, map, blocks, aux, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bse
