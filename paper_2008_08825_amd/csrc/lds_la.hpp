// Dense 64 x 64 linear algebra in LDS (FP64, complex values as separate real
// and imaginary arrays), shared by the Cholesky and the window eigensolver.
#pragma once

#include "common.hpp"

namespace bse {

constexpr int kLdsN = 64;

// Inverse X = L^-1 of the lower triangle L held in (Lr, Li) (real positive
// diagonal), 256 threads, into (Xr, Xi) with a zero strict upper triangle.
// Row elimination with one barrier per step: Y starts as I; step j subtracts
// L[i][j] Y[j][:] / L[j][j] from every row i > j (row j is final then, up to
// its division by L[j][j], which the last pass applies to every row).
BSE_DEV void tri_inverse_lds(const double (*Lr)[kLdsN + 1], const double (*Li)[kLdsN + 1],
                             double (*Xr)[kLdsN + 1], double (*Xi)[kLdsN + 1], int tid) {
  for (int q = 0; q < 16; ++q) {
    const int r = tid & 63, c = (tid >> 6) + 4 * q;
    Xr[r][c] = (r == c) ? 1.0 : 0.0;
    Xi[r][c] = 0.0;
  }
  __syncthreads();
  const int c = tid & 63, i0 = tid >> 6;
  for (int j = 0; j < kLdsN - 1; ++j) {
    if (c <= j) {
      const double rj = 1.0 / Lr[j][j];
      const double yr = Xr[j][c] * rj, yi = Xi[j][c] * rj;
      for (int i = j + 1 + i0; i < kLdsN; i += 4) {
        const double lr = Lr[i][j], li = Li[i][j];
        Xr[i][c] -= lr * yr - li * yi;
        Xi[i][c] -= lr * yi + li * yr;
      }
    }
    __syncthreads();
  }
  for (int q = 0; q < 16; ++q) {
    const int r = tid & 63, cc = (tid >> 6) + 4 * q;
    const double rr = 1.0 / Lr[r][r];
    Xr[r][cc] *= rr;
    Xi[r][cc] *= rr;
  }
  __syncthreads();
}


}  // namespace bse
