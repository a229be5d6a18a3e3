// One-sided block-Jacobi SVD on MFMA (replaces the LAPACK SVD of Alg. 3 step 3).
//
// W (np x np, column-major) is split into N = np / 32 column blocks.  A sweep
// runs N - 1 rounds of the round-robin ("circle") ordering; each round pairs
// every block with one other, and the N / 2 pairs of a round are independent.
// For a pair (p, q) with X = [W_p W_q] (np x 64):
//   gram:   G = X^H X (64 x 64 Hermitian), split over row chunks on MFMA,
//           only the ten 16 x 16 tiles on or below the diagonal;
//   eig:    if max_{i != j} |G_ij| / sqrt(G_ii G_jj) > tol, the eigenvectors R
//           of G by cyclic two-sided Jacobi in LDS (FP64), with inner
//           rotations (|angle| <= pi/4) so R stays close to the identity as
//           G approaches diagonal form;
//   rotate: X <- X R on MFMA, in place.
// A sweep in which no pair exceeds tol ends the iteration.  Afterwards the
// columns of W are orthogonal: W_in Q = U Sigma with Q the product of the
// rotations, so column norms are the singular values and the normalised
// columns are the left singular vectors.
#include "common.hpp"
#include "internal.hpp"

#include <stdio.h>
#include <stdlib.h>

#include <vector>

namespace bse {
namespace {

constexpr int JB = 32;      // columns per block
constexpr int JP = 64;      // columns per pair
constexpr int NTILE = 10;   // 16 x 16 tiles on or below the diagonal of a 64 x 64 Gram
// Row padding of the inner eigensolver's 64 x 64 LDS arrays (entries of 16
// bytes).  Its step loop reads and writes 2 x 2 blocks at circle-ordering
// indices; a count of the bank cycles of those accesses over a sweep (16, 8
// or 32 lanes per LDS cycle) puts a padding of 5 entries at 1.7-2.3 times the
// conflict-free count, against 1.8-3.4 for a padding of 1.
constexpr int LPAD = 5;

__device__ __constant__ int kTileI[NTILE] = {0, 1, 1, 2, 2, 2, 3, 3, 3, 3};
__device__ __constant__ int kTileJ[NTILE] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3};

// Circle-method pairing: position 0 holds block 0, position i > 0 holds block
// ((i - 1 + t) mod (N - 1)) + 1; pair k joins positions k and N - 1 - k.
BSE_DEV void round_pair(int N, int t, int k, int& p, int& q) {
  const int a = k, b = N - 1 - k;
  p = (a == 0) ? 0 : ((a - 1 + t) % (N - 1)) + 1;
  q = ((b - 1 + t) % (N - 1)) + 1;
}

BSE_DEV int pair_col(int p, int q, int c) { return c < JB ? p * JB + c : q * JB + (c - JB); }

// ---------------------------------------------------------------- Gram tiles
// Workgroup (pair k, chunk c) accumulates the ten lower tiles of X^H X over
// the 16-row pieces c, c + kc, c + 2 kc, ... (rc rows) and writes them to
// part[(k * kc + c) * 10 + tile].
//
// Tile t of the lower triangle lies in block row gram_ti(t), block column
// gram_tj(t) (16-column blocks of the pair).  The work of a 16-row step (ten
// tiles x four k-steps) is split evenly over the four waves (one per SIMD):
// wave w takes tiles 2w and 2w + 1 whole and half the k-steps of a shared tile
// (tile 8 for waves 0, 1; tile 9 for waves 2, 3; the lower wave of each couple
// the first two k-steps).  Every wave runs its own copy of the loop with its
// tiles known at compile time, so the loop has no branches and the
// accumulators stay in place.
//
// Staging: 16 rows x 64 columns of complex values, double-buffered in LDS.
// Entry (row r, column c) sits at r * 64 + (c ^ r ^ 16 (r & 1)): the XOR
// spreads the column-wise writes (sixteen rows of one column per sixteen
// lanes) and the row-wise MFMA fragment reads (sixteen columns of four rows)
// over all banks.
template <typename T>
struct GramOp {
  static constexpr int NT = 256;
  // four workgroups per CU: 1024 of them fill the chip once.  Complex128 then
  // spills 52 bytes per lane at 128 registers; a bound of three (no spill, 153
  // registers, three workgroups per CU) makes the kernel 14 % slower.
  static constexpr int MIN_WAVES = 4;
  typedef GramArgs<typename cpx_t<T>::type> Args;
  static BSE_DEV void run(const Args& a, int bx, int t);
};

// Register stages of the Gram kernel's row loop: complex128 one 16-row step
// ahead, complex64 two (more stages measured no faster in either).
template <typename T>
constexpr int gram_stages() { return sizeof(T) == 8 ? 1 : 2; }
BSE_DEV constexpr int gram_ti(int t) { return t < 1 ? 0 : t < 3 ? 1 : t < 6 ? 2 : 3; }
BSE_DEV constexpr int gram_tj(int t) { return t - gram_ti(t) * (gram_ti(t) + 1) / 2; }

template <typename T>
struct GramLane {
  typedef typename cpx_t<T>::type C2;
  typedef typename Mfma<T>::acc Acc;
  int rd[4];  // LDS offset of row 4 s + lane / 16, column lane % 16 (block 0 or 1), per k-step s
  int bo[4];  // offset of 16-column block b for this lane's row parity
};

// Complex products on the real MFMAs in the three-product form: with
// P1 = Re Re, P2 = Im Im and P3 the product of the sums, one MFMA in four
// fewer than the plain form (Re = Re Re - Im Im, Im = Re Im + Im Re).  Its
// error bound is of the plain form's kind, a small multiple of the unit
// roundoff times |X| |R| entrywise, so the rotations keep the columnwise
// accuracy one-sided Jacobi relies on (on the n = 8192 workload the FP64
// results agree with the plain form's to 2e-15, at the same Sigma-
// orthogonality and residual).  cplx3m<T>() = false selects the plain form.
template <typename T>
constexpr bool cplx3m() { return true; }

// One 16-row step (four k-steps of four rows) of the wave's tiles on staged
// buffer X: acc[i] accumulates tile i (tiles 2 WV, 2 WV + 1 and, on odd
// k-steps, the shared tile at k-step 2 (WV & 1) + s / 2) as X_m^H X_n.  The
// MFMAs are ordered so that consecutive ones write different accumulators.
// The four tiles of the cross block X_q^H X_p (rows 32..63, columns 0..31 of
// the pair's Gram), one per wave when only the cross block is computed.
BSE_DEV constexpr int gram_cross_tile(int wv) { return wv < 2 ? 3 + wv : 4 + wv; }

template <typename T, int WV, bool CROSS>
BSE_DEV void gram_buffer(const typename cpx_t<T>::type* X, const GramLane<T>& g,
                         typename Mfma<T>::acc (&acc)[3][3]) {
  typedef typename cpx_t<T>::type C2;
  constexpr int TA = CROSS ? gram_cross_tile(WV) : 2 * WV, TB = 2 * WV + 1, TS = 8 + (WV >> 1);
  constexpr int SH = WV & 1;
  constexpr int tiles[3] = {TA, TB, TS};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int nt = CROSS ? 1 : (s & 1) ? 3 : 2;
    C2 xn[3], xm[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (i < nt) {
        // MFMA A operand: X[k][16 tj + l % 16] (n side); B operand: X[k][16 ti + l % 16] (m side)
        const int ks = i < 2 ? s : 2 * SH + (s >> 1);
        xn[i] = X[g.rd[ks] + g.bo[gram_tj(tiles[i])]];
        xm[i] = X[g.rd[ks] + g.bo[gram_ti(tiles[i])]];
      }
    }
    if constexpr (cplx3m<T>()) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
        if (i < nt) acc[i][0] = Mfma<T>::mac(xn[i].x, xm[i].x, acc[i][0]);
#pragma unroll
      for (int i = 0; i < 3; ++i)
        if (i < nt) acc[i][1] = Mfma<T>::mac(xn[i].y, xm[i].y, acc[i][1]);
#pragma unroll
      for (int i = 0; i < 3; ++i)
        if (i < nt) acc[i][2] = Mfma<T>::mac(xn[i].x + xn[i].y, xm[i].x - xm[i].y, acc[i][2]);
    } else {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        if (i < nt) {
          acc[i][0] = Mfma<T>::mac(xn[i].x, xm[i].x, acc[i][0]);
          acc[i][1] = Mfma<T>::mac(xn[i].y, xm[i].x, acc[i][1]);
        }
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        if (i < nt) {
          acc[i][0] = Mfma<T>::mac(xn[i].y, xm[i].y, acc[i][0]);
          acc[i][1] = Mfma<T>::mac(xn[i].x, -xm[i].y, acc[i][1]);
        }
      }
    }
  }
}

// Four staged values of one thread (pair columns c0, c0 + 16, c0 + 32, c0 + 48
// of one row), their sources in W and their swizzled places in LDS.
template <typename T>
struct GramStage {
  typedef T V2 __attribute__((ext_vector_type(2)));
  V2 v0, v1, v2, v3;
};

template <typename T>
struct GramSrc {
  typedef typename cpx_t<T>::type C2;
  typedef typename GramStage<T>::V2 V2;
  const V2* s0;
  const V2* s1;
  const V2* s2;
  const V2* s3;
  int w0, w1, w2, w3;
  BSE_DEV GramSrc(const C2* W, long ld, int p, int q, int c0, int lr)
      : s0(reinterpret_cast<const V2*>(W + (long)pair_col(p, q, c0) * ld)),
        s1(reinterpret_cast<const V2*>(W + (long)pair_col(p, q, c0 + 16) * ld)),
        s2(reinterpret_cast<const V2*>(W + (long)pair_col(p, q, c0 + 32) * ld)),
        s3(reinterpret_cast<const V2*>(W + (long)pair_col(p, q, c0 + 48) * ld)),
        w0(lr * JP + 16 * (0 ^ (lr & 1)) + (c0 ^ lr)),
        w1(lr * JP + 16 * (1 ^ (lr & 1)) + (c0 ^ lr)),
        w2(lr * JP + 16 * (2 ^ (lr & 1)) + (c0 ^ lr)),
        w3(lr * JP + 16 * (3 ^ (lr & 1)) + (c0 ^ lr)) {}
  BSE_DEV void load(GramStage<T>& st, int r) const {
    st.v0 = s0[r];
    st.v1 = s1[r];
    st.v2 = s2[r];
    st.v3 = s3[r];
  }
  BSE_DEV void store(const GramStage<T>& st, C2* X) const {
    V2* Xv = reinterpret_cast<V2*>(X);
    Xv[w0] = st.v0;
    Xv[w1] = st.v1;
    Xv[w2] = st.v2;
    Xv[w3] = st.v3;
  }
};

template <typename T, int WV, int NST, bool CROSS>
BSE_DEV void gram_wave(const typename GramOp<T>::Args& a, int p, int q, int k, int c,
                       typename cpx_t<T>::type* Xs) {
  typedef typename cpx_t<T>::type C2;
  typedef typename Mfma<T>::acc Acc;
  constexpr int TS = 8 + (WV >> 1), SH = WV & 1;
  const int tid = threadIdx.x, lane = tid & 63, h = lane >> 4, l15 = lane & 15;
  // The chunk's 16-row steps interleave with the other chunks': step j reads
  // rows 16 (j kc + c) .. + 15, so the kc work groups of a pair, which run
  // side by side, read neighbouring pieces of every column at the same time.
  const int kc = a.kc, nsteps = a.rc >> 4;
  auto row_of = [&](int j) { return 16 * (min(j, nsteps - 1) * kc + c); };
  GramLane<T> g;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int kk = 4 * s + h;
    g.rd[s] = kk * JP + (l15 ^ kk);
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) g.bo[b] = 16 * (b ^ (h & 1));
  // staging: thread reads rows r0 + lr of pair columns c0 + 16 i (sixteen
  // consecutive rows of a column per sixteen lanes) and stores them swizzled
  const int lr = tid & 15, c0 = tid >> 4;
  const GramSrc<T> src(a.W + lr, a.ld, p, q, c0, lr);
  Acc acc[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[i][j] = Mfma<T>::zero();
  // NST register stages in flight: steps j + 1, ..., j + NST load while the
  // MFMAs work on step j; steps alternate between two LDS buffers.
  // Prefetches past the chunk re-read its last step, so that every step
  // issues the same loads and the waits for them stay partial.
  GramStage<T> st[NST];
#pragma unroll
  for (int i = 0; i < NST; ++i) src.load(st[i], row_of(i));
  C2* X0 = Xs;
  C2* X1 = Xs + 16 * JP;
  int j0 = 0;
  for (; j0 + NST <= nsteps; j0 += NST) {
#pragma unroll
    for (int i = 0; i < NST; ++i) {
      C2* X = ((j0 + i) & 1) ? X1 : X0;
      src.store(st[i], X);
      __syncthreads();
      src.load(st[i], row_of(j0 + i + NST));
      __builtin_amdgcn_sched_barrier(0);  // issue the prefetch before the MFMA work
      gram_buffer<T, WV, CROSS>(X, g, acc);
    }
  }
#pragma unroll
  for (int i = 0; i < NST; ++i) {  // the last steps, fewer than NST
    if (j0 + i < nsteps) {
      C2* X = ((j0 + i) & 1) ? X1 : X0;
      src.store(st[i], X);
      __syncthreads();
      gram_buffer<T, WV, CROSS>(X, g, acc);
    }
  }
  // real and imaginary parts of the tiles
  Acc cr[3], ci[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if constexpr (cplx3m<T>()) {
      cr[i] = acc[i][0] + acc[i][1];
      ci[i] = acc[i][2] - acc[i][0] + acc[i][1];
    } else {
      cr[i] = acc[i][0];
      ci[i] = acc[i][1];
    }
  }
  if constexpr (CROSS) {  // one whole tile per wave
    C2* dst = a.part + ((long)(k * a.kc + c) * NTILE + gram_cross_tile(WV)) * 256;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      C2 v; v.x = cr[0][r]; v.y = ci[0][r];
      dst[l15 + 16 * Mfma<T>::drow(lane, r)] = v;
    }
    return;
  }
  // shared tile: the upper wave of each couple hands its half to the lower one
  __syncthreads();
  T* hand = reinterpret_cast<T*>(Xs) + (WV >> 1) * 512;  // 2 (re, im) x 4 registers x 64 lanes per couple
  if (SH) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      hand[r * 64 + lane] = cr[2][r];
      hand[(4 + r) * 64 + lane] = ci[2][r];
    }
  }
  __syncthreads();
  if (!SH) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      cr[2][r] += hand[r * 64 + lane];
      ci[2][r] += hand[(4 + r) * 64 + lane];
    }
  }
  // tile element (m_local, n_local) of G = X^H X is stored at m_local + 16 n_local
  C2* out = a.part + (long)(k * a.kc + c) * NTILE * 256;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (i < 2 || !SH) {
      const int tt = i < 2 ? 2 * WV + i : TS;
      C2* dst = out + tt * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ml = l15, nl = Mfma<T>::drow(lane, r);
        C2 v; v.x = cr[i][r]; v.y = ci[i][r];
        dst[ml + 16 * nl] = v;
      }
    }
  }
}

template <typename T>
BSE_DEV void GramOp<T>::run(const typename GramOp<T>::Args& a, int bx, int t) {
  typedef typename cpx_t<T>::type C2;
  if (a.done && *a.done) return;
  __shared__ C2 Xs[2 * 16 * JP];
  const int k = bx / a.kc, c = bx % a.kc;
  int p, q;
  round_pair(a.N, t, k, p, q);
  constexpr int kDeep = gram_stages<T>();
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if ((a.crossp ? *a.crossp : a.cross) && t > 0) {  // only the cross block; the diagonal blocks are tracked
    switch (wv) {
      case 0: gram_wave<T, 0, kDeep, true>(a, p, q, k, c, Xs); break;
      case 1: gram_wave<T, 1, kDeep, true>(a, p, q, k, c, Xs); break;
      case 2: gram_wave<T, 2, kDeep, true>(a, p, q, k, c, Xs); break;
      default: gram_wave<T, 3, kDeep, true>(a, p, q, k, c, Xs); break;
    }
    return;
  }
  switch (wv) {
    case 0: gram_wave<T, 0, kDeep, false>(a, p, q, k, c, Xs); break;
    case 1: gram_wave<T, 1, kDeep, false>(a, p, q, k, c, Xs); break;
    case 2: gram_wave<T, 2, kDeep, false>(a, p, q, k, c, Xs); break;
    default: gram_wave<T, 3, kDeep, false>(a, p, q, k, c, Xs); break;
  }
}

// ---------------------------------------------------------------- inner eigensolver
// Eigenvectors of the pair's 64 x 64 Gram by parallel cyclic Jacobi, in FP64.
// Each step applies 32 disjoint rotations chosen by the circle method on the
// 64 indices: every off-diagonal 2 x 2 block of G is replaced by
// J_P^H G_PQ J_Q (P < Q) and the rotated column pairs of R by R J, while the
// threads whose blocks hold the next step's pairs compute its rotation
// parameters (which also give the rotated diagonal 2 x 2 blocks), so a step
// takes one barrier.  G sits in LDS with both triangles kept current (a
// block update writes its mirror too, so that no access needs a conjugation
// test), complex values as double2 (one 16-byte LDS access per entry); R sits
// in registers and moves between lanes.  The kernel is bound
// by instruction issue and LDS latency.
constexpr int EIG_THREADS = 512;

// Whole-wave lane shifts by one: lane_down gives lane l the value of lane
// l + 1, lane_up that of lane l - 1 (the end lanes get zero).
template <int CTRL>
BSE_DEV double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
BSE_DEV double2 lane_down(double2 v) { return make_double2(dpp_f64<0x130>(v.x), dpp_f64<0x130>(v.y)); }
BSE_DEV double2 lane_up(double2 v) { return make_double2(dpp_f64<0x138>(v.x), dpp_f64<0x138>(v.y)); }

template <typename T>
struct EigOp {
  static constexpr int NT = EIG_THREADS;
  typedef EigArgs<typename cpx_t<T>::type> Args;
  static BSE_DEV void run(const Args& a, int bx, int t);
};

template <typename T>
BSE_DEV void EigOp<T>::run(const typename EigOp<T>::Args& a, int bx, int t) {
  typedef typename cpx_t<T>::type C2;
  if (a.done && *a.done) return;
  const int N = a.N, kc = a.kc, max_inner = a.max_inner;
  const C2* __restrict__ part = a.part;
  C2* __restrict__ Rout = a.R;
  int* __restrict__ flags = a.flags;
  int* counter = a.counter;
  int* inner_count = a.inner;
  int* inner_rot_count = a.inner_rot;
  double* maxoff = a.maxoff;
  const double tol = a.tol;
  const double inner_stop2 = a.stop2p ? *a.stop2p : a.inner_stop2;
  double2* track = a.track;
  const bool cross = (a.crossp ? *a.crossp : a.cross) && t > 0;
  __shared__ double2 G[JP][JP + LPAD];
  __shared__ double2 R[JP][JP + LPAD];
  __shared__ double4 prm[2][32];  // (c, Re s, Im s, unused) of rotation m, two steps
  __shared__ int pidx[2][32];     // i | j << 8 | rotate << 16
  __shared__ double red[NT / 64];
  __shared__ int nrot;
  __shared__ int sweepbig;
  const int tid = threadIdx.x;
  const int k = bx;
  int bp, bq;  // the pair's column blocks: pair columns 0..31 and 32..63
  round_pair(N, t, k, bp, bq);
  // (P, Q), P < Q, of this thread's off-diagonal 2 x 2 block of a step
  // (threads 0..495).  In the circle method the two indices of pair m of step
  // s + 1 come from pairs m - 1 and m + 1 of step s ((0, 1) for m = 0,
  // (30, 31) for m = 31): always the same 32 blocks, held by threads 0..31
  // (thread m for pair m), which compute the next step's rotations right
  // after updating their blocks.  Threads 32..495 take the other 464 blocks
  // column by column: Q - 1 of them in column Q = 2..30 (P = Q - 2 left
  // out), 29 in column 31 (P = 29, 30 left out).
  int bP = 0, bQ = 1;
  if (tid < 32) {
    bP = tid == 0 ? 0 : (tid == 31 ? 30 : tid - 1);
    bQ = tid == 0 ? 1 : (tid == 31 ? 31 : tid + 1);
  } else if (tid < 496) {
    int b = tid - 32, Q = 2;
    while (b >= (Q < 31 ? Q - 1 : 29)) {
      b -= Q < 31 ? Q - 1 : 29;
      ++Q;
    }
    bQ = Q;
    bP = (Q < 31 && b >= Q - 2) ? b + 1 : b;
  }

  // 1. G = sum of the partial tiles (lower part), mirrored to a full Hermitian
  // matrix; with `cross`, only the cross block comes from partial tiles (tiles
  // 3, 4, 6, 7) and the two diagonal blocks from the tracked block Grams.
  // Every thread sums five entries; the loads of several chunks are issued
  // before the sums (the order of the sum over chunks stays 0, 1, ...).
  {
    constexpr int PE = NTILE * 256 / NT;
    static_assert(PE * NT == NTILE * 256 && 4 * NT == 2 * JB * JB, "eig assembly split");
    bool use[PE];
    const C2* src[PE];
#pragma unroll
    for (int u = 0; u < PE; ++u) {
      const int e = tid + u * NT, tile = e >> 8, el = e & 255;
      const int m = 16 * kTileI[tile] + (el & 15), n = 16 * kTileJ[tile] + (el >> 4);
      use[u] = m >= n && !(cross && !(tile == 3 || tile == 4 || tile == 6 || tile == 7));
      src[u] = part + ((long)k * kc * NTILE + tile) * 256 + el;
    }
    double sr[PE], si[PE];
#pragma unroll
    for (int u = 0; u < PE; ++u) sr[u] = si[u] = 0.0;
#pragma unroll 4
    for (int c = 0; c < kc; ++c) {
#pragma unroll
      for (int u = 0; u < PE; ++u) {
        if (use[u]) {
          const C2 v = src[u][(long)c * NTILE * 256];
          sr[u] += (double)v.x;
          si[u] += (double)v.y;
        }
      }
    }
    double2 tv[4];
    if (cross) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = tid + u * NT, b = e >> 10, m = e & 31, n = (e >> 5) & 31;
        tv[u] = track[(long)(b ? bq : bp) * JB * JB + m + JB * n];
      }
    }
#pragma unroll
    for (int u = 0; u < PE; ++u) {
      if (!use[u]) continue;
      const int e = tid + u * NT, tile = e >> 8, el = e & 255;
      const int m = 16 * kTileI[tile] + (el & 15), n = 16 * kTileJ[tile] + (el >> 4);
      if (m == n) {
        G[m][m] = make_double2(sr[u], 0.0);
      } else {
        G[m][n] = make_double2(sr[u], si[u]);
        G[n][m] = make_double2(sr[u], -si[u]);
      }
    }
    if (cross) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = tid + u * NT, b = e >> 10, m = e & 31, n = (e >> 5) & 31;
        if (m < n) continue;
        const int mm = m + JB * b, nn = n + JB * b;
        if (m == n) {
          G[mm][mm] = make_double2(tv[u].x, 0.0);
        } else {
          G[mm][nn] = tv[u];
          G[nn][mm] = cconj(tv[u]);
        }
      }
    }
  }
  __syncthreads();
  // The diagonal blocks of G (after the pair's rotation, if any) become the
  // tracked Grams of the pair's two column blocks; G is current in its lower
  // triangle.
  auto write_track = [&]() {
    if (!track) return;
    for (int e = tid; e < 2 * JB * JB; e += NT) {
      const int b = e >> 10, m = e & 31, n = (e >> 5) & 31;
      const int mm = m + JB * b, nn = n + JB * b;
      track[(long)(b ? bq : bp) * JB * JB + m + JB * n] = mm >= nn ? G[mm][nn] : cconj(G[nn][mm]);
    }
  };

  // 2. Relative off-diagonal measure of the pair.
  double off2 = 0.0;
  for (int e = tid; e < JP * JP; e += NT) {
    const int i = e & 63, j = e >> 6;
    if (i > j) {
      const double dd = G[i][i].x * G[j][j].x;
      const double a2 = cabs2(G[i][j]);
      if (dd > 0.0) off2 = fmax(off2, a2 / dd);
      else if (a2 > 0.0) off2 = 1.0;
    }
  }
  // max over the wave by lane exchanges, then over the eight waves in LDS
  for (int o = 32; o > 0; o >>= 1) off2 = fmax(off2, __shfl_xor(off2, o));
  if ((tid & 63) == 0) red[tid >> 6] = off2;
  __syncthreads();
  double offw = red[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) offw = fmax(offw, red[w]);
  const double off = sqrt(offw);
  if (tid == 0) atomic_max_nonneg(maxoff, off);
  if (!(off > tol)) {
    write_track();
    if (tid == 0) flags[k] = 0;
    return;
  }

  // 3. Cyclic Jacobi.
  // R lives in registers, in circle-method slot order: the circle method keeps
  // index 0 in slot 0 and moves the others one slot down the ring of slots
  // 1..63 per step, and pair m always takes slots m and 63 - m.  Waves 1..7
  // hold R (wave 0 computes the rotations): wave w holds the row pairs
  // g = rg0 .. rg0 + nrg - 1 (five each for waves 1..4, four for 5..7), and
  // its lane L the entries of pair m = L % 32 in row 2 g + L / 32: top[u] in
  // slot m, bot[u] in slot 63 - m.  After the rotation the entries move to
  // the next step's slots by lane shifts.  Whole sweeps bring every index
  // back to its own slot.
  const int lane = tid & 63, mR = lane & 31, wv = tid >> 6;
  const int rg0 = wv <= 4 ? 5 * (wv - 1) : 20 + 4 * (wv - 5), nrg = wv == 0 ? 0 : (wv <= 4 ? 5 : 4);
  double2 top[5], bot[5];
#pragma unroll
  for (int u = 0; u < 5; ++u) {
    const int r = 2 * (rg0 + u) + (lane >> 5);
    top[u] = make_double2(r == mR ? 1.0 : 0.0, 0.0);
    bot[u] = make_double2(r == JP - 1 - mR ? 1.0 : 0.0, 0.0);
  }
  // A sweep whose largest relative off-diagonal entry (before its rotation)
  // was below sqrt(inner_stop2) leaves O(inner_stop2) behind (quadratic
  // convergence), so the confirming sweep that would rotate nothing is skipped.
  const double tol_in2 = 1.6e-31;  // (4e-16)^2
  const double stop2 = inner_stop2;
  int sweeps_done = 0;
  int applied = 0;  // rotations computed by this thread (threads 0..31)
  // Pair m of step s: indices i < j
  auto circle_pair = [&](int s, int m, int& i, int& j) {
    const int a = m, b = JP - 1 - m;
    i = (a == 0) ? 0 : ((a - 1 + s) % (JP - 1)) + 1;
    j = ((b - 1 + s) % (JP - 1)) + 1;
    if (i > j) { const int tmp = i; i = j; j = tmp; }
  };
  // Rotation of pair m = (i, j), i < j, that zeroes G_ij = cc given G_ii = aa
  // and G_jj = dd: writes the rotated diagonal entries and the parameters to
  // buffer buf; returns whether it rotates (the caller zeroes G_ij and G_ji) and sets
  // big when |G_ij|^2 > stop2 |G_ii G_jj|.
  auto pair_rotation = [&](int buf, int m, int i, int j, double aa, double dd, double2 cc,
                           int& big) -> int {
    const double cre = cc.x, cim = cc.y;
    const double ac2 = cre * cre + cim * cim;
    int rot = 0;
    double cs = 1.0, sr = 0.0, si = 0.0;
    const double add = fabs(aa * dd);
    big = ac2 > stop2 * add ? 1 : 0;
    if (ac2 > tol_in2 * add && ac2 > 0.0) {
      rot = 1;
      const double inv_ac = rsqrt(ac2);
      const double ac = ac2 * inv_ac;
      const double zeta = fmin(fmax(0.5 * (dd - aa) * inv_ac, -1.0e150), 1.0e150);
      // t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)): the smaller root, |angle| <= pi/4.
      // Any t gives a unitary rotation (c = (1 + t^2)^-1/2, s = t c), so t
      // needs no correctly rounded division: reciprocal plus two Newton steps.
      const double den = fabs(zeta) + sqrt(fma(zeta, zeta, 1.0));
      double rc = __builtin_amdgcn_rcp(den);
      rc = rc * fma(-den, rc, 2.0);
      rc = rc * fma(-den, rc, 2.0);
      const double tt = zeta >= 0.0 ? rc : -rc;
      cs = rsqrt(fma(tt, tt, 1.0));
      const double sn = tt * cs;
      sr = sn * cre * inv_ac;
      si = sn * cim * inv_ac;
      G[i][i] = make_double2(aa - tt * ac, 0.0);
      G[j][j] = make_double2(dd + tt * ac, 0.0);
    }
    pidx[buf][m] = i | (j << 8) | (rot << 16);
    prm[buf][m] = make_double4(cs, sr, si, 0.0);
    return rot;
  };
  // One barrier per step.  The parameters of step s sit in buffer s & 1; in
  // the step the 496 off-diagonal 2 x 2 blocks become G_PQ <- J_P^H G_PQ J_Q
  // (one per thread), threads 0..31 then compute the rotations of step s + 1
  // from their updated blocks and the rotated diagonal, and waves 1..7 apply
  // the step's rotations to R.  Wave 0 keeps, in uniform registers, whether
  // the sweep whose parameters it computes rotates anything and whether it
  // meets a large entry; the verdict (go on with another sweep) is written to
  // LDS with the sweep's last parameters and read in its last step.
  __shared__ int scont;
  if (max_inner > 0) {
    int rot_any = 0, big_any = 0;
    {
      int rb = 0, bb = 0;
      if (tid < 32) {
        int i, j;
        circle_pair(0, tid, i, j);
        rb = pair_rotation(0, tid, i, j, G[i][i].x, G[j][j].x, cconj(G[j][i]), bb);
        if (rb) {
          G[j][i] = make_double2(0.0, 0.0);
          G[i][j] = make_double2(0.0, 0.0);
          ++applied;
        }
      }
      if (tid < 64) {
        rot_any = __ballot(rb) != 0;
        big_any = __ballot(bb) != 0;
      }
    }
    __syncthreads();
    int gstep = 0;
    for (int sweep = 0;; ++sweep) {
      for (int step = 0; step < JP - 1; ++step, ++gstep) {
        const int cur = gstep & 1;
        // the next step's rotations, unless this is the last step of the last sweep
        const bool next = step < JP - 2 || scont;
        // Loads first (the pairs' parameters, the thread's G block and, for
        // threads 0..31, the next pair's diagonal entries; threads 496..511
        // read block (0, 1) and leave it), then R, whose arithmetic covers
        // their latency, then the block update.
        const int P = bP, Q = bQ;
        const int xP = pidx[cur][P], xQ = pidx[cur][Q];
        const double4 ppP = prm[cur][P], ppQ = prm[cur][Q];
        const int rP = xP >> 16, rQ = xQ >> 16;
        const int iP = xP & 255, jP = (xP >> 8) & 255, iQ = xQ & 255, jQ = (xQ >> 8) & 255;
        double2 g00 = G[iP][iQ], g01 = G[iP][jQ], g10 = G[jP][iQ], g11 = G[jP][jQ];
        const bool par = tid < 32 && next;
        int i2 = 0, j2 = 0;
        double aa2 = 0.0, dd2 = 0.0;
        if (tid < 32) {
          circle_pair(step + 1 < JP - 1 ? step + 1 : 0, tid, i2, j2);
          aa2 = G[i2][i2].x;
          dd2 = G[j2][j2].x;
        }
        if (wv > 0) {  // R <- R J_s in registers (an idle rotation has c = 1, s = 0)
          const double4 pp = prm[cur][mR];
          const int itop = mR == 0 ? 0 : ((mR - 1 + step) % (JP - 1)) + 1;
          const int ibot = ((JP - 2 - mR + step) % (JP - 1)) + 1;
          // top holds column i of the rotation and bot column j unless itop > ibot:
          // new top = c top + a bot, new bot = c bot - conj(a) top with
          // a = -conj(s), or a = s when swapped
          const double c = pp.x, si = pp.z, ar = itop < ibot ? -pp.y : pp.y;
#pragma unroll
          for (int u = 0; u < 5; ++u) {
            if (u >= nrg) break;
            const double2 t = top[u], b = bot[u];
            double2 nt, nb;
            nt.x = fma(c, t.x, fma(ar, b.x, -si * b.y));
            nt.y = fma(c, t.y, fma(ar, b.y, si * b.x));
            nb.x = fma(c, b.x, -fma(ar, t.x, si * t.y));
            nb.y = fma(c, b.y, fma(-ar, t.y, si * t.x));
            // to the next step's slots: top of pair m + 1 (bottom of pair 31
            // for m = 31, itself for m = 0); bottom of pair m - 1 (top of
            // pair 1 for m = 0)
            const double2 up = lane_down(nt), dn = lane_up(nb);
            top[u] = mR == 31 ? nb : (mR == 0 ? nt : up);
            bot[u] = mR == 0 ? up : dn;
          }
        }
        int rb = 0, bb = 0;
        if (tid < 496 && (rP | rQ | par)) {
          {  // G2 <- G2 J_Q, J = [c s; -conj(s) c]
            const double4 pp = ppQ;
            const double c = pp.x;
            const double2 sq = make_double2(pp.y, pp.z);
            const double2 sqc = cconj(sq);
            const double2 t00 = csub(cscale(g00, c), cmul(sqc, g01));
            const double2 t01 = cadd(cmul(sq, g00), cscale(g01, c));
            const double2 t10 = csub(cscale(g10, c), cmul(sqc, g11));
            const double2 t11 = cadd(cmul(sq, g10), cscale(g11, c));
            g00 = t00; g01 = t01; g10 = t10; g11 = t11;
          }
          {  // G2 <- J_P^H G2, J^H = [c -s; conj(s) c]
            const double4 pp = ppP;
            const double c = pp.x;
            const double2 sp = make_double2(pp.y, pp.z);
            const double2 spc = cconj(sp);
            const double2 t00 = csub(cscale(g00, c), cmul(sp, g10));
            const double2 t01 = csub(cscale(g01, c), cmul(sp, g11));
            const double2 t10 = cadd(cmul(spc, g00), cscale(g10, c));
            const double2 t11 = cadd(cmul(spc, g01), cscale(g11, c));
            g00 = t00; g01 = t01; g10 = t10; g11 = t11;
          }
          if (par) {
            // the next pair's entry: its row index from pair P, column index from pair Q
            const bool uP = iP == i2 || iP == j2, uQ = iQ == i2 || iQ == j2;
            const double2 v = uP ? (uQ ? g00 : g01) : (uQ ? g10 : g11);
            const double2 cc = (uP ? iP : jP) < (uQ ? iQ : jQ) ? v : cconj(v);  // G(i2, j2)
            rb = pair_rotation(cur ^ 1, tid, i2, j2, aa2, dd2, cc, bb);
            if (rb) {
              const double2 z = make_double2(0.0, 0.0);
              if (uP && uQ) g00 = z;
              else if (uP) g01 = z;
              else if (uQ) g10 = z;
              else g11 = z;
              ++applied;
            }
          }
          G[iP][iQ] = g00; G[iQ][iP] = cconj(g00);
          G[iP][jQ] = g01; G[jQ][iP] = cconj(g01);
          G[jP][iQ] = g10; G[iQ][jP] = cconj(g10);
          G[jP][jQ] = g11; G[jQ][jP] = cconj(g11);
        }
        if (tid < 64) {
          const int ra = __ballot(rb) != 0, ba = __ballot(bb) != 0;
          if (step == JP - 2) {  // first parameters of the next sweep
            rot_any = ra;
            big_any = ba;
          } else {
            rot_any |= ra;
            big_any |= ba;
          }
          if (step == JP - 3 && tid == 0) scont = sweep + 1 < max_inner && rot_any && big_any;
        }
        __syncthreads();
      }
      ++sweeps_done;
      if (!scont) break;
    }
  }
#pragma unroll
  for (int u = 0; u < 5; ++u) {
    if (u >= nrg) break;
    const int r = 2 * (rg0 + u) + (lane >> 5);
    R[r][mR] = top[u];
    R[r][JP - 1 - mR] = bot[u];
  }
  __syncthreads();
  write_track();
  if (tid == 0) atomicAdd(inner_count, sweeps_done);
  if (tid < 64) {
    int a = applied;
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
    if (tid == 0) atomicAdd(inner_rot_count, a);
  }

  // 4. R to global, row-major 64 x 64 (the rotation kernel then stages it
  // into LDS row by row, each wave's stores to consecutive banks)
  C2* dst = Rout + (long)k * JP * JP;
  for (int e = tid; e < JP * JP; e += NT) {
    const int j = e & 63, i = e >> 6;
    C2 v; v.x = (T)R[i][j].x; v.y = (T)R[i][j].y;
    dst[j + JP * i] = v;
  }
  if (tid == 0) {
    flags[k] = 1;
    atomicAdd(counter, 1);
  }
}

// ---------------------------------------------------------------- rotation
// Workgroup (pair k, row chunk): X[rows, :] <- X[rows, :] R, in place.  R goes
// to LDS once (rows padded in complex64 so that the MFMA fragment reads of
// four rows x sixteen columns take the minimum two bank cycles; a complex128
// row already fills them).  Each wave handles
// 16-row strips: it holds the strip's 16 x 64 inputs in registers (loaded as
// MFMA B operands: 16 consecutive rows of one column per 16 lanes) and runs
// the k-steps outermost with the four 16-column output tiles accumulating
// side by side, so that each input register is free after its k-step and is
// refilled at once with the wave's next strip.
template <typename T>
struct RotOp {
  static constexpr int NT = 256;
  // what the LDS for R allows; complex64 runs four waves per SIMD either way,
  // and a bound of three lets the compiler fit 126 registers without the
  // 12-byte spill that a bound of four forces (1 % faster)
  static constexpr int MIN_WAVES = sizeof(T) == 8 ? 2 : 3;
  typedef RotArgs<typename cpx_t<T>::type> Args;
  static BSE_DEV void run(const Args& a, int bx, int t);
};

template <typename T>
constexpr int rot_ld() { return sizeof(T) == 4 ? JP + 16 : JP; }

template <typename T, bool PREFETCH>
BSE_DEV void rot_strip(const typename cpx_t<T>::type* Rs, typename cpx_t<T>::type (&xf)[16],
                       typename cpx_t<T>::type* lp0, typename cpx_t<T>::type* lp1,
                       typename cpx_t<T>::type* sp0, typename cpx_t<T>::type* sp1, long ld,
                       int row0, int rnext, int lane) {
  typedef typename cpx_t<T>::type C2;
  typedef typename Mfma<T>::acc Acc;
  const int h = lane >> 4, l15 = lane & 15;
  // R is read from LDS afresh for every strip, and the lane's column pointers
  // are opaque to the compiler here, so that neither the R fragments nor
  // per-k-step addresses are hoisted out of the strip loop into registers
#if defined(__HIP_DEVICE_COMPILE__)
  __asm__ volatile("" : "+v"(lp0), "+v"(lp1), "+v"(sp0), "+v"(sp1) : : "memory");
#endif
  typedef T V2 __attribute__((ext_vector_type(2)));
  typedef __attribute__((address_space(1))) V2 GV2;  // global memory (not flat) accesses
  GV2* gl0 = (GV2*)lp0;
  GV2* gl1 = (GV2*)lp1;
  GV2* gs0 = (GV2*)sp0;
  GV2* gs1 = (GV2*)sp1;
  Acc acc[4][3];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj)
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[tj][j] = Mfma<T>::zero();
  // R fragments of k-step kk + 1 are read while the MFMAs of k-step kk run;
  // the scheduling barriers keep the compiler from hoisting further reads
  C2 r[4], rn[4];
  const typename cpx_t<T>::type* Rl = Rs + h * rot_ld<T>() + l15;
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) r[tj] = Rl[16 * tj];
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    if (kk + 1 < 16) {
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) rn[tj] = Rl[4 * (kk + 1) * rot_ld<T>() + 16 * tj];
    }
    // acc += R[kr][n] X[row][kr]
    if constexpr (cplx3m<T>()) {
      // P1 = Re R Re X, P2 = Im R Im X, P3 = (Re R + Im R)(Re X + Im X)
      const T xs = xf[kk].x + xf[kk].y;
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) acc[tj][0] = Mfma<T>::mac(r[tj].x, xf[kk].x, acc[tj][0]);
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) acc[tj][1] = Mfma<T>::mac(r[tj].y, xf[kk].y, acc[tj][1]);
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) acc[tj][2] = Mfma<T>::mac(r[tj].x + r[tj].y, xs, acc[tj][2]);
    } else {
      // first the products with Re R, then with Im R
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) {
        acc[tj][0] = Mfma<T>::mac(r[tj].x, xf[kk].x, acc[tj][0]);
        acc[tj][1] = Mfma<T>::mac(r[tj].x, xf[kk].y, acc[tj][1]);
      }
#pragma unroll
      for (int tj = 0; tj < 4; ++tj) {
        acc[tj][0] = Mfma<T>::mac(-r[tj].y, xf[kk].y, acc[tj][0]);
        acc[tj][1] = Mfma<T>::mac(r[tj].y, xf[kk].x, acc[tj][1]);
      }
    }
    if (PREFETCH) {
      const V2 v = (kk < 8 ? gl0 : gl1)[(long)(4 * (kk & 7)) * ld + rnext];
      xf[kk].x = v.x;
      xf[kk].y = v.y;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) r[tj] = rn[tj];
  }
  // D row of register rr is column 16 tj + drow(lane, rr) of the pair; the
  // store pointers hold drow(lane, 0)
  constexpr int rstep = sizeof(T) == 8 ? 4 : 1;
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) {
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      V2 v;
      if constexpr (cplx3m<T>()) {
        v.x = acc[tj][0][rr] - acc[tj][1][rr];
        v.y = acc[tj][2][rr] - acc[tj][0][rr] - acc[tj][1][rr];
      } else {
        v.x = acc[tj][0][rr];
        v.y = acc[tj][1][rr];
      }
      (tj < 2 ? gs0 : gs1)[(long)(16 * (tj & 1) + rstep * rr) * ld + row0] = v;
    }
  }
}

template <typename T>
BSE_DEV void RotOp<T>::run(const typename RotOp<T>::Args& a, int bx, int t) {
  typedef typename cpx_t<T>::type C2;
  if (a.done && *a.done) return;
  const int N = a.N, rows_per_wg = a.rrows, chunks = a.chunks;
  C2* W = a.W;
  const long ld = a.ld;
  const int* __restrict__ flags = a.flags;
  __shared__ C2 Rs[JP * rot_ld<T>()];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // pairs in descending order: the Gram launch before this one read them in
  // ascending order, so the most recently read blocks come first (and the
  // next round's ascending Gram starts with the most recently written ones),
  // which the memory-side cache may still hold
  const int k = N / 2 - 1 - bx / chunks, chunk = bx % chunks;
  if (!flags[k]) return;
  int p, q;
  round_pair(N, t, k, p, q);
  const C2* R = a.R + (long)k * JP * JP;
  for (int e = tid; e < JP * JP; e += 256) {
    const int j = e & 63, i = e >> 6;  // R[i][j], i = k index, j = n index (row-major in memory)
    Rs[i * rot_ld<T>() + j] = R[j + JP * i];
  }
  // the lane's input column of k-step kk is 4 kk + lane / 16 of the pair
  // (block p for kk < 8, block q after): lp0 / lp1 point at it for kk = 0 / 8
  // in the lane's row; sp0 / sp1 at the output column drow(lane, 0) of
  // block p / q
  const int h = lane >> 4, l15 = lane & 15;
  const int d0 = Mfma<T>::drow(lane, 0);
  C2* lp0 = W + (long)(p * JB + h) * ld + l15;
  C2* lp1 = W + (long)(q * JB + h) * ld + l15;
  C2* sp0 = W + (long)(p * JB + d0) * ld + l15;
  C2* sp1 = W + (long)(q * JB + d0) * ld + l15;
  int row0 = chunk * rows_per_wg + wave * 16;
  const int strips = rows_per_wg / 64;
  C2 xf[16];
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) xf[kk] = (kk < 8 ? lp0 : lp1)[(long)(4 * (kk & 7)) * ld + row0];
  __syncthreads();
  for (int sidx = 0; sidx + 1 < strips; ++sidx) {
    rot_strip<T, true>(Rs, xf, lp0, lp1, sp0, sp1, ld, row0, row0 + 64, lane);
    row0 += 64;
  }
  rot_strip<T, false>(Rs, xf, lp0, lp1, sp0, sp1, ld, row0, row0, lane);
}

// ---------------------------------------------------------------- batches
// One workgroup per problem of a batch, between sweeps: closes the previous
// sweep (aux > 0) and, unless the problem has converged (a sweep rotated no
// pair) or aux == max_sweeps, opens sweep aux with cleared counters and the
// inner stopping threshold of the adaptive rule used by jacobi_run.
struct SweepOp {
  static constexpr int NT = 64;
  typedef SweepArgs Args;
  static BSE_DEV void run(const Args& a, int bx, int sweep);
};

BSE_DEV void SweepOp::run(const SweepArgs& a, int, int sweep) {
  if (threadIdx.x != 0) return;
  JacState* st = a.st;
  if (st->done) return;
  double prev = -1.0;
  if (sweep > 0) {
    st->sweeps += 1;
    st->rotations += st->counter;
    st->inner_sweeps += st->inner;
    st->inner_rotations += (double)st->inner_rot;
    st->pair_checks += a.pairs_per_sweep;
    if (st->cross) st->cross_pair_checks += a.pairs_per_sweep - a.pairs_per_round;
    st->last_off = st->maxoff;
    prev = st->maxoff;
    if (st->counter == 0) {
      st->converged = 1;
      st->done = 1;
      return;
    }
    if (a.stop_fraction > 0.0 && st->counter < a.stop_fraction * a.pairs_per_sweep) {
      st->done = 1;
      return;
    }
  }
  if (sweep >= a.max_sweeps) {
    st->done = 1;
    return;
  }
  double stop = a.inner_floor;
  const double first = a.first_stop > 0.0 ? a.first_stop : kInnerStopCap;
  if (a.adaptive) stop = fmax(a.inner_floor, fmin(kInnerStopCap, prev < 0.0 ? first : a.factor * prev));
  st->stop2 = stop * stop;
  st->cross = (prev < 0.0 ? first : prev) > a.track_level ? 1 : 0;
  st->counter = 0;
  st->inner = 0;
  st->inner_rot = 0;
  st->maxoff = 0.0;
  atomicAdd(a.active, 1);
}

int gram_chunks(int np, int pairs) {
  // enough workgroups to fill the chip, rows per chunk a multiple of 16
  int kc = 1;
  const int rows16 = np / 16;
  while (pairs * kc < 1024 && kc * 2 <= rows16 && (np % (kc * 2 * 16)) == 0 && kc < 64) kc *= 2;
  return kc;
}

int rotate_rows(int np) {
  if (np % 256 == 0) return 256;
  if (np % 128 == 0) return 128;
  return 64;
}

}  // namespace

size_t jacobi_work_bytes(int np, int elem_bytes, int kc) {
  const int N = np / JB, pairs = N / 2;
  if (kc <= 0) kc = gram_chunks(np, pairs);
  size_t b = 0;
  b += (size_t)pairs * kc * NTILE * 256 * 2 * elem_bytes;  // part
  b = (b + 255) & ~(size_t)255;
  b += (size_t)pairs * JP * JP * 2 * elem_bytes;           // R
  b = (b + 255) & ~(size_t)255;
  b += (size_t)N * JB * JB * sizeof(double2);               // track
  b = (b + 255) & ~(size_t)255;
  b += (size_t)pairs * sizeof(int) + 256;                  // flags
  b += 256 + 256;                                          // counter, maxoff
  return (b + 255) & ~(size_t)255;
}

void jacobi_carve(int np, int elem_bytes, char* base, JacobiWork& w, int kc, int rrows) {
  const int N = np / JB, pairs = N / 2;
  w.kc = kc > 0 ? kc : gram_chunks(np, pairs);
  w.rrows = rrows > 0 ? rrows : rotate_rows(np);
  size_t o = 0;
  w.part = base + o;
  o += (size_t)pairs * w.kc * NTILE * 256 * 2 * elem_bytes;
  o = (o + 255) & ~(size_t)255;
  w.R = base + o;
  o += (size_t)pairs * JP * JP * 2 * elem_bytes;
  o = (o + 255) & ~(size_t)255;
  w.track = reinterpret_cast<double2*>(base + o);
  o += (size_t)N * JB * JB * sizeof(double2);
  o = (o + 255) & ~(size_t)255;
  w.flags = reinterpret_cast<int*>(base + o);
  o += (size_t)pairs * sizeof(int) + 256;
  o = (o + 255) & ~(size_t)255;
  w.counter = reinterpret_cast<int*>(base + o);
  w.inner = reinterpret_cast<int*>(base + o + 32);
  w.inner_rot = reinterpret_cast<int*>(base + o + 48);
  w.maxoff = reinterpret_cast<double*>(base + o + 64);
}

bool jacobi_tiles_valid(int np, int kc, int rrows) {
  if (kc < 1 || (kc & (kc - 1)) != 0 || np % (16 * kc) != 0) return false;
  if (rrows < 64 || rrows % 64 != 0 || np % rrows != 0) return false;
  return true;
}

int jacobi_default_kc(int np) { return gram_chunks(np, np / JB / 2); }
int jacobi_pairs(int np) { return np / JB / 2; }
int jacobi_rounds(int np) { return np / JB - 1; }
int jacobi_gram_blocks_kc(int np, int kc) { return jacobi_pairs(np) * kc; }
int jacobi_eig_blocks(int np) { return jacobi_pairs(np); }
int jacobi_rot_blocks_rr(int np, int rrows) { return jacobi_pairs(np) * (np / rrows); }

template <typename C2>
GramArgs<C2> make_gram(int np, C2* W, long ld, const JacobiWork& w, const int* done) {
  GramArgs<C2> a;
  a.N = np / JB; a.W = W; a.ld = ld; a.kc = w.kc; a.rc = np / w.kc;
  a.part = static_cast<C2*>(w.part); a.done = done; a.cross = 0; a.crossp = nullptr;
  return a;
}
template <typename C2>
EigArgs<C2> make_eig(int np, const JacobiWork& w, double tol, const double* stop2p, const int* done) {
  EigArgs<C2> a;
  a.N = np / JB; a.kc = w.kc;
  a.part = static_cast<const C2*>(w.part); a.R = static_cast<C2*>(w.R);
  a.flags = w.flags; a.counter = w.counter; a.tol = tol; a.maxoff = w.maxoff;
  a.max_inner = 30; a.inner = w.inner; a.inner_stop2 = 0.0; a.stop2p = stop2p;
  a.inner_rot = w.inner_rot; a.done = done; a.track = w.track; a.cross = 0; a.crossp = nullptr;
  return a;
}
template <typename C2>
RotArgs<C2> make_rot(int np, C2* W, long ld, const JacobiWork& w, const int* done) {
  RotArgs<C2> a;
  a.N = np / JB; a.W = W; a.ld = ld; a.R = static_cast<const C2*>(w.R); a.flags = w.flags;
  a.rrows = w.rrows; a.chunks = np / w.rrows; a.done = done;
  return a;
}

template <typename T>
static hipError_t jacobi_run(int np, typename cpx_t<T>::type* W, long ld, const JacobiWork& w,
                             double tol, double inner_stop, int max_sweeps, JacobiResult& res,
                             hipStream_t s, int time_stride, double first_stop = kInnerStopCap,
                             double inner_factor = 1.0, double stop_fraction = 0.0) {
  typedef typename cpx_t<T>::type C2;
  const int N = np / JB, pairs = N / 2;
  const int gblocks = jacobi_gram_blocks_kc(np, w.kc);
  const int rblocks = jacobi_rot_blocks_rr(np, w.rrows);
  GramArgs<C2> ga = make_gram<C2>(np, W, ld, w, nullptr);
  EigArgs<C2> ea = make_eig<C2>(np, w, tol, nullptr, nullptr);
  const double track_level = sizeof(T) == 8 ? kTrackLevel64 : kTrackLevel32;
  const RotArgs<C2> ra = make_rot<C2>(np, W, ld, w, nullptr);
  res = JacobiResult();
  hipError_t e;
  // Optional per-launch timing: an event before and after every Jacobi kernel
  // of every time_stride-th round.
  const bool time_kernels = time_stride > 0;
  std::vector<hipEvent_t> ev;
  if (time_kernels) {
    ev.resize((size_t)(N - 1) * 6);
    for (auto& x : ev) {
      e = hipEventCreate(&x);
      if (e != hipSuccess) return e;
    }
  }
  auto timed = [&](int t) { return time_kernels && t % time_stride == 0; };
  auto mark = [&](int t, size_t i) {
    if (timed(t)) (void)hipEventRecord(ev[i], s);
  };
  hipError_t ret = hipSuccess;
  const bool debug = getenv("BSE_DEBUG") != nullptr;
  // A pair's inner iteration ends after an inner sweep whose largest relative
  // off-diagonal entry was below s, which leaves about s^2 behind.  The
  // rotation of a pair need not be more exact than the orthogonality the
  // other pairs of the same outer sweep disturb it by, so s is inner_factor
  // times the previous outer sweep's largest off-diagonal measure (leaving
  // about its square), at most kInnerStopCap and down to the floor
  // inner_stop; the first sweep uses first_stop.
  double prev_off = -1.0;
  const bool adaptive = getenv("BSE_FIXED_INNER") == nullptr;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double sstop = inner_stop;
    if (adaptive)
      sstop = fmax(inner_stop, fmin(kInnerStopCap, prev_off < 0.0 ? first_stop : inner_factor * prev_off));
    ea.inner_stop2 = sstop * sstop;
    ga.cross = ea.cross = (prev_off < 0.0 ? first_stop : prev_off) > track_level ? 1 : 0;
    e = hipMemsetAsync(w.counter, 0, 128, s);
    if (e != hipSuccess) { ret = e; break; }
    for (int t = 0; t < N - 1; ++t) {
      const size_t b = (size_t)t * 6;
      mark(t, b + 0);
      e = launch_one<GramOp<T>>(ga, gblocks, t, s);
      mark(t, b + 1);
      mark(t, b + 2);
      if (e == hipSuccess) e = launch_one<EigOp<T>>(ea, pairs, t, s);
      mark(t, b + 3);
      mark(t, b + 4);
      if (e == hipSuccess) e = launch_one<RotOp<T>>(ra, rblocks, t, s);
      mark(t, b + 5);
      if (e != hipSuccess) break;
    }
    if (e != hipSuccess) { ret = e; break; }
    int cnt = 0, inner = 0, irot = 0;
    double mo = 0.0;
    e = hipMemcpyAsync(&cnt, w.counter, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&mo, w.maxoff, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&inner, w.inner, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&irot, w.inner_rot, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { ret = e; break; }
    if (time_kernels) {
      double msum[3] = {0.0, 0.0, 0.0};
      int timed_rounds = 0;
      for (int t = 0; t < N - 1; ++t) {
        if (!timed(t)) continue;
        ++timed_rounds;
        for (int kx = 0; kx < 3; ++kx) {
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, ev[(size_t)t * 6 + 2 * kx], ev[(size_t)t * 6 + 2 * kx + 1]);
          msum[kx] += ms;
        }
      }
      for (int kx = 0; kx < 3; ++kx) {
        res.kernel_ms[kx] += msum[kx] * (N - 1) / timed_rounds;
        res.kernel_launches[kx] += N - 1;
      }
    }
    if (debug)
      fprintf(stderr, "[bse] sweep %d: rotated pairs %d of %d, max off %.3e, inner sweeps %.2f per pair\n",
              sweep + 1, cnt, pairs * (N - 1), mo, cnt > 0 ? (double)inner / cnt : 0.0);
    prev_off = mo;
    res.sweeps = sweep + 1;
    res.rotations += cnt;
    res.inner_sweeps += inner;
    res.inner_rotations += irot;
    res.pair_checks += pairs * (N - 1);
    if (ga.cross) res.cross_pair_checks += pairs * (N - 2);  // all rounds but the first
    res.max_off = mo;
    if (cnt == 0) { res.converged = 1; break; }
    if (stop_fraction > 0.0 && cnt < stop_fraction * pairs * (N - 1)) break;
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  return ret;
}

hipError_t jacobi_z(int np, double2* W, long ld, const JacobiWork& w, double tol,
                    int max_sweeps, JacobiResult& res, hipStream_t s, int time_stride,
                    double first_stop) {
  return jacobi_run<double>(np, W, ld, w, tol, 1.0e-10, max_sweeps, res, s, time_stride, first_stop);
}

hipError_t jacobi_c(int np, float2* W, long ld, const JacobiWork& w, double tol, double inner_stop,
                    int max_sweeps, JacobiResult& res, hipStream_t s, int time_stride,
                    double inner_factor, double stop_fraction) {
  return jacobi_run<float>(np, W, ld, w, tol, inner_stop, max_sweeps, res, s, time_stride,
                           kInnerStopCap, inner_factor, stop_fraction);
}

GramArgs<double2> gram_args_z(int np, double2* W, long ld, const JacobiWork& w, const int* done) {
  return make_gram<double2>(np, W, ld, w, done);
}
GramArgs<float2> gram_args_c(int np, float2* W, long ld, const JacobiWork& w, const int* done) {
  return make_gram<float2>(np, W, ld, w, done);
}
EigArgs<double2> eig_args_z(int np, const JacobiWork& w, double tol, const double* stop2p,
                            const int* done) {
  return make_eig<double2>(np, w, tol, stop2p, done);
}
EigArgs<float2> eig_args_c(int np, const JacobiWork& w, double tol, const double* stop2p,
                           const int* done) {
  return make_eig<float2>(np, w, tol, stop2p, done);
}
RotArgs<double2> rot_args_z(int np, double2* W, long ld, const JacobiWork& w, const int* done) {
  return make_rot<double2>(np, W, ld, w, done);
}
RotArgs<float2> rot_args_c(int np, float2* W, long ld, const JacobiWork& w, const int* done) {
  return make_rot<float2>(np, W, ld, w, done);
}

hipError_t group_jacobi(GroupOp op, const void* table, const int2* map, int blocks, int aux,
                        hipStream_t s) {
  switch (op) {
    case G_GRAM_Z: return launch_grp<GramOp<double>>(table, map, blocks, aux, s);
    case G_GRAM_C: return launch_grp<GramOp<float>>(table, map, blocks, aux, s);
    case G_EIG_Z: return launch_grp<EigOp<double>>(table, map, blocks, aux, s);
    case G_EIG_C: return launch_grp<EigOp<float>>(table, map, blocks, aux, s);
    case G_ROT_Z: return launch_grp<RotOp<double>>(table, map, blocks, aux, s);
    case G_ROT_C: return launch_grp<RotOp<float>>(table, map, blocks, aux, s);
    case G_SWEEP: return launch_grp<SweepOp>(table, map, blocks, aux, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bse
