// Complex GEMM on MFMA for gfx950 (complex128 via f64 16x16x4, complex64 via
// f32 16x16x4), column-major operands with optional conjugate transposes.
//
// Used for the trailing Hermitian rank-64 update and the panel solve of the
// blocked Cholesky, the triangular products W = L2^H L1 and the eigenvector
// back-transform of Alg. 3 (Lemma SVDScalarFactors), and the adjoint sums.
//
// Tiling: a 256-thread workgroup (4 waves) owns a 64 x 64 output tile; each
// wave a 32 x 32 quadrant of 2 x 2 MFMA tiles.  K advances in steps of 16
// through double-buffered LDS (one barrier per step), where both operands sit
// as interleaved complex values, swizzled so that the column-wise stores and
// the MFMA fragment reads (four k rows x sixteen columns) spread over all
// banks; global loads for the next K step are issued before the MFMAs of the
// current one.  Complex products take the three-product form (P1 = Re Re,
// P2 = Im Im, P3 on the sums): three real MFMAs per complex k-step instead
// of four, with an error bound of the plain form's kind (a small multiple of
// the unit roundoff times |A| |B| entrywise).
#include "common.hpp"
#include "internal.hpp"

namespace bse {
namespace {

constexpr int BM = 64, BN = 64, BK = 16;

// Work group -> output tile.  A lower-triangle output of a square tile grid
// launches only its T (T + 1) / 2 lower tiles, row by row; a product with one
// triangular operand dispatches its tiles longest k-range first (the tiles of
// one block row of op(A) share a k-range), so that the short ones fill the
// end of the launch; otherwise tile rows vary fastest.
__host__ __device__ inline bool lower_packed(int lowerC, int tilesM, int tilesN) {
  return lowerC && tilesM == tilesN;
}
template <int OPA, typename P>
BSE_DEV void tile_of(const P& p, int bx, int& tm, int& tn) {
  if (lower_packed(p.lowerC, p.tilesM, p.tilesN)) {
    int r = (int)((sqrt(8.0 * bx + 1.0) - 1.0) * 0.5);
    while ((r + 1) * (r + 2) / 2 <= bx) ++r;
    while (r * (r + 1) / 2 > bx) --r;
    tm = r;
    tn = bx - r * (r + 1) / 2;
  } else if (p.triA && !p.triB && !p.lowerC) {
    tm = bx / p.tilesN;
    tn = bx % p.tilesN;
    if (OPA == 0) tm = p.tilesM - 1 - tm;  // lower op(A): the last block rows are the longest
  } else {
    tm = bx % p.tilesM;
    tn = bx / p.tilesM;
  }
}

// LDS place of operand element (k, c) of a 16 x 64 staged tile
BSE_DEV int gemm_swz(int k, int c) { return k * 64 + (c ^ k ^ ((k & 1) << 4)); }

// KS: the product is A diag(kscale) B (only op(A) = A, op(B) = B^H is
// instantiated with it, the form the adjoint sums take).
template <typename T, int OPA, int OPB, bool KS = false>
struct GemmOp {
  static constexpr int NT = 256;
  // registers for two staged steps: complex128 two waves per SIMD; complex64
  // three (the compiler then fits op(A) = A^H in 168 registers without a
  // spill under a bound of two, while op(A) = A spills 8 bytes under three and
  // needs 174 registers, two waves, without it)
  static constexpr int MIN_WAVES = sizeof(T) == 8 ? 2 : (OPA == 1 ? 2 : 3);
  typedef GemmArgs<T> Args;
  static BSE_DEV void run(const Args& p, int bx, int aux);
};

template <typename T, int OPA, int OPB, bool KS>
BSE_DEV void GemmOp<T, OPA, OPB, KS>::run(const GemmArgs<T>& p, int bx, int) {
  typedef typename cpx_t<T>::type C2;
  typedef typename Mfma<T>::acc Acc;
  __shared__ C2 As[2][BK * BM];
  __shared__ C2 Bs[2][BK * BN];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int tm, tn;
  tile_of<OPA>(p, bx, tm, tn);
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

  // acc[ti][tj]: P1, P2, P3 of the three-product form
  Acc acc[2][2][3];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[i][j][c] = Mfma<T>::zero();

  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  // staging: element i of this thread, (k, m) of A and (k, n) of B
  //   op 0 of A / op 1 of B: 64 consecutive rows of one k per wave
  //   op 1 of A / op 0 of B: 16 consecutive k of four columns per wave
  const int a_m = OPA == 0 ? (tid & 63) : (tid >> 4), a_k = OPA == 0 ? (tid >> 6) : (tid & 15);
  const int b_n = OPB == 0 ? (tid >> 4) : (tid & 63), b_k = OPB == 0 ? (tid & 15) : (tid >> 6);
  // two register sets of staged operands: steps s + 1 and s + 2 load while
  // the MFMAs work on step s (prefetches past the last step re-read it, so
  // that every step issues the same loads and the waits stay partial)
  // Loads are unconditional (out-of-range lanes read a clamped in-range
  // element) and do nothing else, so the waits for them stay partial; the
  // masking of out-of-range elements, conjugation and k scaling happen when
  // the staged values go to LDS.
  C2 ra0[4], rb0[4], ra1[4], rb1[4];
  T ks0[4], ks1[4];
  auto load = [&](C2 (&ra)[4], C2 (&rb)[4], T (&ks)[4], int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = OPA == 0 ? a_m : a_m + 16 * i, k = OPA == 0 ? a_k + 4 * i : a_k;
      const int cm = min(m0 + m, p.M - 1), ck = min(k0 + k, p.K - 1);
      ra[i] = OPA == 0 ? A[cm + (long)ck * p.lda] : A[ck + (long)cm * p.lda];
      if constexpr (KS) ks[i] = (T)p.kscale[ck];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int n = OPB == 0 ? b_n + 16 * i : b_n, k = OPB == 0 ? b_k : b_k + 4 * i;
      const int ck = min(k0 + k, p.K - 1), cn = min(n0 + n, p.N - 1);
      rb[i] = OPB == 0 ? B[ck + (long)cn * p.ldb] : B[cn + (long)ck * p.ldb];
    }
  };
  auto store = [&](const C2 (&ra)[4], const C2 (&rb)[4], const T (&ks)[4], int k0, C2* Ab,
                   C2* Bb) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = OPA == 0 ? a_m : a_m + 16 * i, ka = OPA == 0 ? a_k + 4 * i : a_k;
      const bool oka = m0 + m < p.M && k0 + ka < p.K;
      T sa = oka ? T(1) : T(0);
      if constexpr (KS) sa *= ks[i];
      C2 va;
      va.x = ra[i].x * sa;
      va.y = OPA == 1 ? -ra[i].y * sa : ra[i].y * sa;
      Ab[gemm_swz(ka, m)] = va;
      const int n = OPB == 0 ? b_n + 16 * i : b_n, kb = OPB == 0 ? b_k : b_k + 4 * i;
      const bool okb = k0 + kb < p.K && n0 + n < p.N;
      const T sb = okb ? T(1) : T(0);
      C2 vb;
      vb.x = rb[i].x * sb;
      vb.y = OPB == 1 ? -rb[i].y * sb : rb[i].y * sb;
      Bb[gemm_swz(kb, n)] = vb;
    }
  };
  auto compute = [&](const C2* Ab, const C2* Bb) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = 4 * s + (lane >> 4);
      C2 a[2], b[2];
      T asum[2], bsum[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = Ab[gemm_swz(kk, wm + 16 * t + (lane & 15))];
        b[t] = Bb[gemm_swz(kk, wn + 16 * t + (lane & 15))];
        asum[t] = a[t].x + a[t].y;
        bsum[t] = b[t].x + b[t].y;
      }
      // MFMA A operand: the B fragment (D row = n); B operand: the A fragment (D column = m)
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) acc[ti][tj][0] = Mfma<T>::mac(b[tj].x, a[ti].x, acc[ti][tj][0]);
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) acc[ti][tj][1] = Mfma<T>::mac(b[tj].y, a[ti].y, acc[ti][tj][1]);
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) acc[ti][tj][2] = Mfma<T>::mac(bsum[tj], asum[ti], acc[ti][tj][2]);
    }
  };

  const int nsteps = kbeg < kend ? (kend - kbeg + BK - 1) / BK : 0;
  auto kstep = [&](int i) { return kbeg + BK * min(i, nsteps - 1); };
  int st = 0;
  if (nsteps > 0) {
    load(ra0, rb0, ks0, kstep(0));
    load(ra1, rb1, ks1, kstep(1));
    for (; st + 2 <= nsteps; st += 2) {
      store(ra0, rb0, ks0, kstep(st), As[0], Bs[0]);
      __syncthreads();
      load(ra0, rb0, ks0, kstep(st + 2));
      __builtin_amdgcn_sched_barrier(0);  // issue the prefetch before the MFMAs
      compute(As[0], Bs[0]);
      store(ra1, rb1, ks1, kstep(st + 1), As[1], Bs[1]);
      __syncthreads();
      load(ra1, rb1, ks1, kstep(st + 3));
      __builtin_amdgcn_sched_barrier(0);
      compute(As[1], Bs[1]);
    }
    if (st < nsteps) {  // an odd number of steps: the last one
      store(ra0, rb0, ks0, kstep(st), As[0], Bs[0]);
      __syncthreads();
      compute(As[0], Bs[0]);
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
        // (Ar + i Ai)(Br + i Bi) = P1 - P2 + i (P3 - P1 - P2)
        const T p1 = acc[ti][tj][0][r], p2 = acc[ti][tj][1][r], p3 = acc[ti][tj][2][r];
        T vr = p1 - p2, vi = p3 - p1 - p2;
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
  const int blocks = gemm_tiles(d);
  if (d.kscale) {
    if (d.opA == 0 && d.opB == 1) return launch_one<GemmOp<T, 0, 1, true>>(p, blocks, 0, s);
    return hipErrorInvalidValue;
  }
  if (d.opA == 0 && d.opB == 0) return launch_one<GemmOp<T, 0, 0>>(p, blocks, 0, s);
  if (d.opA == 0 && d.opB == 1) return launch_one<GemmOp<T, 0, 1>>(p, blocks, 0, s);
  if (d.opA == 1 && d.opB == 0) return launch_one<GemmOp<T, 1, 0>>(p, blocks, 0, s);
  return launch_one<GemmOp<T, 1, 1>>(p, blocks, 0, s);
}

template <typename T>
hipError_t gemm_group(int opA, int opB, int ks, const void* table, const int2* map, int blocks,
                      hipStream_t s) {
  if (ks) {
    if (opA == 0 && opB == 1) return launch_grp<GemmOp<T, 0, 1, true>>(table, map, blocks, 0, s);
    return hipErrorInvalidValue;
  }
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
  const int tm = (d.M + BM - 1) / BM, tn = (d.N + BN - 1) / BN;
  return lower_packed(d.lowerC, tm, tn) ? tm * (tm + 1) / 2 : tm * tn;
}
GemmArgs<double> gemm_args_z(const GemmDesc& d) { return make_args<double>(d); }
GemmArgs<float> gemm_args_c(const GemmDesc& d) { return make_args<float>(d); }

hipError_t group_gemm(int prec, int opA, int opB, int ks, const void* table, const int2* map,
                      int blocks, hipStream_t s) {
  return prec == 0 ? gemm_group<double>(opA, opB, ks, table, map, blocks, s)
                   : gemm_group<float>(opA, opB, ks, table, map, blocks, s);
}

}  // namespace bse
