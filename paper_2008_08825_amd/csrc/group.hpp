// Grouped launches from the host: per launch, a table of per-problem (or
// per-window) op arguments and a map from every flat work group to (table
// row, work group), staged into a device arena and read by the grouped form
// of an op (see the op launches in common.hpp).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "internal.hpp"
#include "plan.hpp"

namespace bse {

// Table staging: host-built tables are copied into a device arena just
// before the launch that reads them.  Copies and launches share one stream,
// so when the arena wraps around, every launch that read the overwritten
// bytes has already run.  The tables that launches still to come read (a
// launch's table and map, or the tables of a phase recorded once and
// replayed) are reserved together first, so that a wrap never falls between
// them and one cannot overwrite another.
struct Arena {
  char* dev = nullptr;
  size_t cap = 0, cur = 0;
  hipStream_t s = nullptr;
  std::vector<std::vector<char>> keep;  // host sources stay valid until the call returns

  // Room for `bytes` (the sum of the 256-aligned puts that follow) in one
  // contiguous run: wraps now if the run would not fit before the end.
  hipError_t reserve(size_t bytes) {
    if (bytes > cap) return hipErrorInvalidValue;
    if (cur + bytes > cap) cur = 0;
    return hipSuccess;
  }

  hipError_t put(const void* src, size_t bytes, const void** out) {
    const size_t need = align256(bytes);
    if (need > cap) return hipErrorInvalidValue;
    if (cur + need > cap) cur = 0;
    keep.emplace_back(static_cast<const char*>(src), static_cast<const char*>(src) + bytes);
    char* d = dev + cur;
    cur += need;
    *out = d;
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(d, keep.back().data(), bytes, hipMemcpyHostToDevice, s);
  }
};

template <class A>
struct Grp {
  std::vector<A> tab;
  std::vector<int2> map;
  std::vector<int> start;  // first map entry of each table row
  void add(const A& a, int blocks) {
    if (blocks <= 0) return;
    start.push_back((int)map.size());
    const int row = (int)tab.size();
    tab.push_back(a);
    for (int b = 0; b < blocks; ++b) map.push_back(make_int2(row, b));
  }
  int blocks() const { return (int)map.size(); }
  // map entries of the first `rows` table rows
  int prefix(int rows) const {
    return rows >= (int)start.size() ? (int)map.size() : start[rows];
  }
};

struct Dev {
  const void* tab = nullptr;
  const int2* map = nullptr;
  int blocks = 0;
};

// Arena bytes of a staged table and its map.
template <class A>
inline size_t staged_bytes(const Grp<A>& g) {
  if (g.blocks() == 0) return 0;
  return align256(g.tab.size() * sizeof(A)) + align256(g.map.size() * sizeof(int2));
}

template <class A>
inline hipError_t stage(Arena& ar, const Grp<A>& g, Dev& d) {
  d.blocks = g.blocks();
  if (d.blocks == 0) return hipSuccess;
  hipError_t e = ar.reserve(staged_bytes(g));  // table and map in one run
  if (e != hipSuccess) return e;
  e = ar.put(g.tab.data(), g.tab.size() * sizeof(A), &d.tab);
  const void* m = nullptr;
  if (e == hipSuccess) e = ar.put(g.map.data(), g.map.size() * sizeof(int2), &m);
  d.map = static_cast<const int2*>(m);
  return e;
}

inline GemmArgs<double> args_of(const GemmDesc& d, double*) { return gemm_args_z(d); }
inline GemmArgs<float> args_of(const GemmDesc& d, float*) { return gemm_args_c(d); }

// Stage and launch a grouped GEMM (all rows share opA, opB, and either all or
// none have a k scaling).
template <typename T>
inline hipError_t run_gemm(Arena& ar, const std::vector<GemmDesc>& descs, hipStream_t s) {
  if (descs.empty()) return hipSuccess;
  const int ks = descs[0].kscale != nullptr;
  for (const GemmDesc& d : descs)
    if ((d.kscale != nullptr) != (ks != 0) || d.opA != descs[0].opA || d.opB != descs[0].opB)
      return hipErrorInvalidValue;
  Grp<GemmArgs<T>> g;
  for (const GemmDesc& d : descs) {
    g.add(args_of(d, static_cast<T*>(nullptr)), gemm_tiles(d));
  }
  Dev dv;
  hipError_t e = stage(ar, g, dv);
  if (e != hipSuccess) return e;
  return group_gemm(sizeof(T) == 8 ? 0 : 1, descs[0].opA, descs[0].opB, ks, dv.tab, dv.map, dv.blocks, s);
}

typedef hipError_t (*GroupFn)(GroupOp, const void*, const int2*, int, int, hipStream_t);

template <class A>
inline hipError_t run_op(Arena& ar, const Grp<A>& g, GroupFn fn, GroupOp op, int aux, hipStream_t s) {
  Dev dv;
  hipError_t e = stage(ar, g, dv);
  if (e != hipSuccess) return e;
  return fn(op, dv.tab, dv.map, dv.blocks, aux, s);
}


}  // namespace bse
