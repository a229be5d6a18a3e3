// Complex GEMM on MFMA for gfx950 (complex128 via f64 16x16x4, complex64 via
// f32 16x16x4), column-major operands with optional conjugate transposes.
//
// Used for the trailing Hermitian rank-64 update and the panel solve of the
// blocked Cholesky, the triangular products W = L2^H L1 and the eigenvector
// back-transform of Alg. 3 (Lemma SVDScalarFactors), and the adjoint sums.
//
// Tiling: a 256-thread workgroup (4 waves) owns a 64 x 64 output tile; each
// wave a 32 x 32 quadrant of 2 x 2 MFMA tiles.  K advances in steps of 16
// through LDS, where both operands sit in planar (re, im) form so each lane
// reads one real per MFMA operand; global loads for the next K step are
// issued before the MFMAs of the current one.
#include "common.hpp"
#include "internal.hpp"

namespace bse {
namespace {

constexpr int BM = 64, BN = 64, BK = 16, PAD = 4;

template <typename T, int OPA, int OPB>
struct GemmOp {
  static constexpr int NT = 256;
  typedef GemmArgs<T> Args;
  static BSE_DEV void run(const Args& p, int bx, int aux);
};

template <typename T, int OPA, int OPB>
BSE_DEV void GemmOp<T, OPA, OPB>::run(const GemmArgs<T>& p, int bx, int) {
  typedef typename cpx_t<T>::type C2;
  typedef typename Mfma<T>::acc Acc;
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tm = bx % p.tilesM, tn = bx / p.tilesM;
  if (p.lowerC && tn > tm) return;
  const int m0 = tm * BM, n0 = tn * BN;
  const C2* __restrict__ A = p.A;
  const C2* __restrict__ B = p.B;
  C2* C = p.C;

  int kbeg = 0, kend = p.K;
  if (p.triA) {
    if (OPA == 0) kend = min(kend, m0 + BM); else kbeg = max(kbeg, m0);
  }
  if (p.triB) {
    if (OPB == 0) kbeg = max(kbeg, n0); else kend = min(kend, n0 + BN);
  }
  kbeg = (kbeg / BK) * BK;

  Acc cr[2][2], ci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) { cr[i][j] = Mfma<T>::zero(); ci[i][j] = Mfma<T>::zero(); }

  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  C2 ra[4], rb[4];

  auto loadA = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int m, k;
      C2 v;
      if (OPA == 0) {
        m = tid & 63; k = (tid >> 6) + 4 * i;
        int gm = m0 + m, gk = k0 + k;
        if (gm < p.M && gk < p.K) v = A[gm + (long)gk * p.lda]; else { v.x = 0; v.y = 0; }
      } else {
        k = tid & 15; m = (tid >> 4) + 16 * (i & 3);
        int gm = m0 + m, gk = k0 + k;
        if (gm < p.M && gk < p.K) { v = A[gk + (long)gm * p.lda]; v.y = -v.y; } else { v.x = 0; v.y = 0; }
      }
      if (p.kscale) {
        int gk = k0 + k;
        T sc = gk < p.K ? (T)p.kscale[gk] : T(0);
        v.x *= sc; v.y *= sc;
      }
      ra[i] = v;
    }
  };
  auto storeA = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int m, k;
      if (OPA == 0) { m = tid & 63; k = (tid >> 6) + 4 * i; }
      else { k = tid & 15; m = (tid >> 4) + 16 * i; }
      As[0][k][m] = ra[i].x; As[1][k][m] = ra[i].y;
    }
  };
  auto loadB = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      C2 v;
      if (OPB == 0) {
        int k = tid & 15, n = (tid >> 4) + 16 * i;
        int gk = k0 + k, gn = n0 + n;
        if (gk < p.K && gn < p.N) v = B[gk + (long)gn * p.ldb]; else { v.x = 0; v.y = 0; }
      } else {
        int n = tid & 63, k = (tid >> 6) + 4 * i;
        int gk = k0 + k, gn = n0 + n;
        if (gk < p.K && gn < p.N) { v = B[gn + (long)gk * p.ldb]; v.y = -v.y; } else { v.x = 0; v.y = 0; }
      }
      rb[i] = v;
    }
  };
  auto storeB = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int n, k;
      if (OPB == 0) { k = tid & 15; n = (tid >> 4) + 16 * i; }
      else { n = tid & 63; k = (tid >> 6) + 4 * i; }
      Bs[0][k][n] = rb[i].x; Bs[1][k][n] = rb[i].y;
    }
  };

  if (kbeg < kend) { loadA(kbeg); loadB(kbeg); }
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    storeA();
    storeB();
    __syncthreads();
    if (k0 + BK < kend) { loadA(k0 + BK); loadB(k0 + BK); }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = 4 * s + (lane >> 4);
      T a_r[2], a_i[2], b_r[2], b_i[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a_r[t] = As[0][kk][wm + 16 * t + (lane & 15)];
        a_i[t] = As[1][kk][wm + 16 * t + (lane & 15)];
        b_r[t] = Bs[0][kk][wn + 16 * t + (lane & 15)];
        b_i[t] = Bs[1][kk][wn + 16 * t + (lane & 15)];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          cmac<T>(b_r[tj], b_i[tj], a_r[ti], a_i[ti], cr[ti][tj], ci[ti][tj]);
    }
  }

  // Epilogue: lane holds rows m0 + wm + 16 ti + lane % 16 of four columns.
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * ti + (lane & 15);
        const int n = n0 + wn + 16 * tj + Mfma<T>::drow(lane, r);
        if (m >= p.M || n >= p.N) continue;
        T vr = cr[ti][tj][r], vi = ci[ti][tj][r];
        T outr = p.ar * vr - p.ai * vi, outi = p.ar * vi + p.ai * vr;
        if (p.colscale) { T sc = (T)p.colscale[n]; outr *= sc; outi *= sc; }
        C2* cp = C + m + (long)n * p.ldc;
        if (p.br != T(0) || p.bi != T(0)) {
          C2 old = *cp;
          outr += p.br * old.x - p.bi * old.y;
          outi += p.br * old.y + p.bi * old.x;
        }
        if (p.mask > 0 && (m >= p.mask || n >= p.mask)) { outr = 0; outi = 0; }
        C2 o; o.x = outr; o.y = outi;
        *cp = o;
      }
}

template <typename T>
GemmArgs<T> make_args(const GemmDesc& d) {
  typedef typename cpx_t<T>::type C2;
  GemmArgs<T> p;
  p.M = d.M; p.N = d.N; p.K = d.K;
  p.A = static_cast<const C2*>(d.A); p.lda = d.lda; p.triA = d.triA;
  p.B = static_cast<const C2*>(d.B); p.ldb = d.ldb; p.triB = d.triB;
  p.C = static_cast<C2*>(d.C); p.ldc = d.ldc;
  p.ar = (T)d.alpha_re; p.ai = (T)d.alpha_im; p.br = (T)d.beta_re; p.bi = (T)d.beta_im;
  p.kscale = d.kscale;
  p.colscale = d.colscale;
  p.lowerC = d.lowerC; p.mask = d.mask;
  p.tilesM = (d.M + BM - 1) / BM;
  p.tilesN = (d.N + BN - 1) / BN;
  return p;
}

template <typename T>
hipError_t gemm_launch(const GemmDesc& d, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0) return hipSuccess;
  const GemmArgs<T> p = make_args<T>(d);
  const int blocks = p.tilesM * p.tilesN;
  if (d.opA == 0 && d.opB == 0) return launch_one<GemmOp<T, 0, 0>>(p, blocks, 0, s);
  if (d.opA == 0 && d.opB == 1) return launch_one<GemmOp<T, 0, 1>>(p, blocks, 0, s);
  if (d.opA == 1 && d.opB == 0) return launch_one<GemmOp<T, 1, 0>>(p, blocks, 0, s);
  return launch_one<GemmOp<T, 1, 1>>(p, blocks, 0, s);
}

template <typename T>
hipError_t gemm_group(int opA, int opB, const void* table, const int2* map, int blocks,
                      hipStream_t s) {
  if (opA == 0 && opB == 0) return launch_grp<GemmOp<T, 0, 0>>(table, map, blocks, 0, s);
  if (opA == 0 && opB == 1) return launch_grp<GemmOp<T, 0, 1>>(table, map, blocks, 0, s);
  if (opA == 1 && opB == 0) return launch_grp<GemmOp<T, 1, 0>>(table, map, blocks, 0, s);
  return launch_grp<GemmOp<T, 1, 1>>(table, map, blocks, 0, s);
}

}  // namespace

hipError_t gemm_z(const GemmDesc& d, hipStream_t s) { return gemm_launch<double>(d, s); }
hipError_t gemm_c(const GemmDesc& d, hipStream_t s) { return gemm_launch<float>(d, s); }

int gemm_tiles(const GemmDesc& d) {
  if (d.M <= 0 || d.N <= 0) return 0;
  return ((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN);
}
GemmArgs<double> gemm_args_z(const GemmDesc& d) { return make_args<double>(d); }
GemmArgs<float> gemm_args_c(const GemmDesc& d) { return make_args<float>(d); }

hipError_t group_gemm(int prec, int opA, int opB, const void* table, const int2* map, int blocks,
                      hipStream_t s) {
  return prec == 0 ? gemm_group<double>(opA, opB, table, map, blocks, s)
                   : gemm_group<float>(opA, opB, table, map, blocks, s);
}

}  // namespace bse
