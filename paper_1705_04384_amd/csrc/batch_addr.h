// Addressing of batch entries: entry e lives at ptrs[e] when a pointer table is given
// (gathered, e.g. solves at different Krylov steps sharing one launch), else at
// base + e * stride (contiguous batch).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fdg {

// Device pointers typed in the global address space.  Entry pointers come from tables or
// pointer arithmetic and are otherwise generic, for which the compiler emits flat memory
// instructions; a flat access also counts against the LDS wait counter, so every LDS wait
// in a kernel would also wait for its outstanding memory loads.  Kernels take entries as
// gat() pointers and keep them in this type.
#define FDG_GLOBAL __attribute__((address_space(1)))
template <typename T>
using gptr = FDG_GLOBAL T *;

struct CBatch {
  const double *base = nullptr;
  int64_t stride = 0;
  const double *const *ptrs = nullptr;
  __host__ __device__ inline const double *at(int64_t e) const { return ptrs ? ptrs[e] : base + e * stride; }
  __device__ inline gptr<const double> gat(int64_t e) const { return (gptr<const double>)at(e); }
};

struct MBatch {
  double *base = nullptr;
  int64_t stride = 0;
  double *const *ptrs = nullptr;
  __host__ __device__ inline double *at(int64_t e) const { return ptrs ? ptrs[e] : base + e * stride; }
  __device__ inline gptr<double> gat(int64_t e) const { return (gptr<double>)at(e); }
  __host__ __device__ inline bool valid() const { return base != nullptr || ptrs != nullptr; }
};

inline CBatch cstrided(const double *p, int64_t stride) { return CBatch{p, stride, nullptr}; }
inline MBatch mstrided(double *p, int64_t stride) { return MBatch{p, stride, nullptr}; }
inline CBatch cgather(const double *const *ptrs) { return CBatch{nullptr, 0, ptrs}; }
inline MBatch mgather(double *const *ptrs) { return MBatch{nullptr, 0, ptrs}; }
inline CBatch as_const(const MBatch &m) { return CBatch{m.base, m.stride, (const double *const *)m.ptrs}; }

// Per-entry integer (e.g. the number of basis vectors): table[e] when given, else uniform.
struct IBatch {
  int uniform = 0;
  const int32_t *table = nullptr;
  __host__ __device__ inline int at(int64_t e) const { return table ? table[e] : uniform; }
};

}  // namespace fdg
