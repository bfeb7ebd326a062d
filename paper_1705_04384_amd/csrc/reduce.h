// Deterministic reductions shared by the Krylov kernels (flexible GMRES and BiCGStab).
//
// A producer kernel runs G <= 256 blocks of kRed threads (G = reduction_blocks(N), a
// function of N only); block g owns the contiguous chunk [g*chunk, min(N, (g+1)*chunk))
// and stores one partial sum per component in a fixed order.  A consumer reduces the G
// partials itself (sum_partials: the same bits in every lane), so results never depend
// on scheduling.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fdg {

constexpr int kRed = 1024;  // threads of the reduction-producing kernels
constexpr int kRedWaves = kRed / 64;
constexpr int kMaxG = 256;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Contiguous chunk of block g; chunks are multiples of 64 elements (even, so 2-wide
// accesses stay aligned, and 512-byte aligned).
__device__ inline void chunk_of(int64_t N, int G, int g, int64_t &beg, int64_t &end) {
  int64_t chunk = (N + G - 1) / G;
  chunk = (chunk + 63) / 64 * 64;
  beg = (int64_t)g * chunk;
  if (beg > N) beg = N;
  end = beg + chunk < N ? beg + chunk : N;
}

// Fixed-order sum of the G <= 256 partials of component q (partial g of component q at
// P[g * ldp + q]), valid in every lane: lane l adds g = l, l + 64, l + 128, l + 192 in
// order, then an xor butterfly.
template <typename Ptr>
__device__ inline double sum_partials(Ptr P, int G, int ldp, int q) {
  const int lane = threadIdx.x & 63;
  double v[kMaxG / 64];
#pragma unroll
  for (int k = 0; k < kMaxG / 64; ++k) {
    const int g = lane + 64 * k;
    v[k] = g < G ? P[(int64_t)g * ldp + q] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kMaxG / 64; ++k) s += v[k];
  return wave_sum(s);
}

}  // namespace fdg
