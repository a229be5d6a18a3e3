// Shared device helpers: complex arithmetic on interleaved (re, im) pairs and
// the MFMA wrappers for gfx950.
//
// There is no complex MFMA on CDNA4, so every complex contraction here issues
// four real 16x16x4 MFMAs per complex k-step:  Cr += Ar Br - Ai Bi,
// Ci += Ar Bi + Ai Br.
//
// Lane layouts of the 16x16x4 MFMAs (64-wide wavefront, lane l):
//   A operand (16 x 4):  lane holds A[l % 16][l / 16]
//   B operand (4 x 16):  lane holds B[l / 16][l % 16]
//   D (16 x 16), register r:
//     f64: D[4 r + l / 16][l % 16]
//     f32: D[4 (l / 16) + r][l % 16]
// Kernels feed the B-side fragment of a product as the MFMA "A" operand and
// the A-side fragment as the MFMA "B" operand, so that result lane l holds
// output row m0 + l % 16: sixteen consecutive lanes then write sixteen
// consecutive elements of a column-major output column.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define BSE_DEV __device__ __forceinline__

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T> struct cpx_t;
template <> struct cpx_t<double> { typedef double2 type; };
template <> struct cpx_t<float> { typedef float2 type; };

template <typename T> struct Mfma;

template <> struct Mfma<double> {
  typedef d4v acc;
  static BSE_DEV acc zero() { acc z = {0.0, 0.0, 0.0, 0.0}; return z; }
  static BSE_DEV acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of D held in register r of lane l
  static BSE_DEV int drow(int lane, int r) { return 4 * r + (lane >> 4); }
};

template <> struct Mfma<float> {
  typedef f4v acc;
  static BSE_DEV acc zero() { acc z = {0.f, 0.f, 0.f, 0.f}; return z; }
  static BSE_DEV acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static BSE_DEV int drow(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// One complex MFMA step: (cr, ci) += (ar + i ai) * (br + i bi) where the
// "a" side is the MFMA A operand (indexed by the D row) and the "b" side the
// MFMA B operand (indexed by the D column).
template <typename T>
BSE_DEV void cmac(T ar, T ai, T br, T bi, typename Mfma<T>::acc& cr,
                  typename Mfma<T>::acc& ci) {
  cr = Mfma<T>::mac(ar, br, cr);
  cr = Mfma<T>::mac(-ai, bi, cr);
  ci = Mfma<T>::mac(ar, bi, ci);
  ci = Mfma<T>::mac(ai, br, ci);
}

BSE_DEV double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
BSE_DEV double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
BSE_DEV double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
BSE_DEV double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
BSE_DEV double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
BSE_DEV double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
BSE_DEV double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// Positive doubles order like their bit patterns: a vector atomicMax on the
// 64-bit pattern gives a max-reduction over non-negative doubles.
BSE_DEV void atomic_max_nonneg(double* addr, double v) {
  if (!(v >= 0.0)) v = __longlong_as_double(0x7ff0000000000000LL);  // NaN -> +inf
  atomicMax(reinterpret_cast<unsigned long long*>(addr),
            static_cast<unsigned long long>(__double_as_longlong(v)));
}

// ---------------------------------------------------------------- launches
// Every kernel is an "op": a struct with the workgroup size NT, an argument
// struct Args and a device body run(args, wg, aux) that does the work of
// workgroup wg of one problem (aux carries a per-launch scalar such as the
// Jacobi round or the Cholesky panel).  An op launches two ways:
//   single:  k_one<Op><<<blocks>>>(args, aux), wg = blockIdx.x;
//   grouped: k_grp<Op><<<total>>>(table, map, aux), where table holds one
//            Args per problem and map[b] = (table row, wg) for every flat
//            workgroup b of the launch, so one launch covers many problems
//            of different sizes with no idle workgroups.
//
// An op may declare MIN_WAVES, the waves per SIMD its kernels must keep
// resident (the register budget follows from it); the default is 1.
template <typename Op, typename = void>
struct op_min_waves {
  static constexpr int value = 1;
};
template <typename Op>
struct op_min_waves<Op, decltype((void)Op::MIN_WAVES)> {
  static constexpr int value = Op::MIN_WAVES;
};

template <typename Op>
__global__ __launch_bounds__(Op::NT, op_min_waves<Op>::value) void k_one(typename Op::Args a, int aux) {
  Op::run(a, (int)blockIdx.x, aux);
}

template <typename Op>
__global__ __launch_bounds__(Op::NT, op_min_waves<Op>::value) void k_grp(const typename Op::Args* __restrict__ table,
                                                const int2* __restrict__ map, int aux) {
  const int2 m = map[blockIdx.x];
  Op::run(table[m.x], m.y, aux);
}

template <typename Op>
hipError_t launch_one(const typename Op::Args& a, int blocks, int aux, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  k_one<Op><<<blocks, Op::NT, 0, s>>>(a, aux);
  return hipGetLastError();
}

template <typename Op>
hipError_t launch_grp(const void* table, const int2* map, int blocks, int aux, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  k_grp<Op><<<blocks, Op::NT, 0, s>>>(static_cast<const typename Op::Args*>(table), map, aux);
  return hipGetLastError();
}
