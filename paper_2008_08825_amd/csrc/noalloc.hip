// bse_solve_h1_noalloc: bse_solve_h1 for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that forbid
// allocation).  The workspace is a file-scope device array, `scratch`, of
// BSE_NOALLOC_SCRATCH_BYTES; each GPU the library runs on holds its own copy
// until the process ends.  In host code the array's name stands for a host
// shadow, not a device address, so the address of each device's copy is
// looked up once per device (with that device current) by
// hipGetSymbolAddress and kept; only that pointer reaches kernels and copies.
//
// Every call on a GPU shares that GPU's array: calls that overlap on one GPU
// (two streams, two host threads) race on it.  Nothing in it needs to start
// at zero: the solve writes every region before reading it (the status word,
// M1 and M2, the Jacobi counters cleared per sweep, the tracked Grams
// refreshed by the first round of every sweep).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/bse.h"
#include "plan.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[BSE_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDev = 64;
std::mutex g_mu;
void* g_ptr[kMaxDev] = {};

// Device address of this device's `scratch` (looked up once per device).
hipError_t scratch_ptr(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    const hipError_t er = cur != dev ? hipSetDevice(cur) : hipSuccess;
    if (e != hipSuccess) return e;
    if (er != hipSuccess) return er;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

int bse_solve_h1_noalloc(int n, const void* A, int lda, const void* B, int ldb, double* lambda,
                         void* X, int ldx, const bse_opts_t* opts, bse_info_t* info, void* stream) {
  bse_opts_t o;
  bse_default_opts(&o);
  if (opts) o = *opts;
  // argument numbers of bse_solve_h1 from 9 on are shifted by the two
  // workspace arguments this entry point does not have
  if (int e = bse::check_h1_args(n, A, lda, B, ldb, lambda, X, ldx, o)) return e == -11 ? -9 : e;
  if (n > 0 && bse_workspace_bytes(n, &o) > (size_t)BSE_NOALLOC_SCRATCH_BYTES)
    return -1;  // the workspace of order n would not fit in the scratch array
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  hipError_t e = hipStreamGetDevice(s, &dev);
  if (e != hipSuccess) return bse::hip_status(e);
  if (dev < 0 || dev >= kMaxDev) return bse::hip_status(hipErrorInvalidDevice);
  void* work = nullptr;
  if ((e = scratch_ptr(dev, &work)) != hipSuccess) return bse::hip_status(e);
  const int st = bse::solve_h1_impl(n, A, lda, B, ldb, lambda, X, ldx, work,
                                    (size_t)BSE_NOALLOC_SCRATCH_BYTES, &o, info, stream, 1);
  if (st == -11) return -9;
  return st;
}

size_t bse_noalloc_scratch_bytes(void) { return (size_t)BSE_NOALLOC_SCRATCH_BYTES; }

}  // extern "C"
