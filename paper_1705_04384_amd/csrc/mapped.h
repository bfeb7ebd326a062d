// Matrix-free collocation operator of a mapped 3D domain (see mapped.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch_addr.h"

namespace fdg {

// Banded univariate factors of direction l: row i of F holds F[i][lo[i] + t] at
// F[i*w + t], t < w, lo non-decreasing; M values, D first derivatives, K minus second
// derivatives at the collocation points.  coef: 9 fields of N doubles (C_11, C_22, C_33,
// 2 C_12, 2 C_13, 2 C_23, g_1, g_2, g_3), shared by every batch entry.
struct MappedOp {
  const double *M[3];
  const double *D[3];
  const double *K[3];
  const int32_t *lo[3];
  int w[3];
  int step[3];  // max over i of lo[i+1] - lo[i]
  const double *coef;
  int64_t N;
};

// The kernel applies: band width <= 8, band starts growing by at most 1 per row in
// directions 1 and 2.
bool mapped_matvec_ok(int n, int64_t nbatch, const MappedOp &op);
// y = A x for nbatch entries; false (nothing launched) when mapped_matvec_ok fails.
bool launch_mapped_matvec_f64(hipStream_t s, CBatch x, MBatch y, int n, int64_t nbatch, const MappedOp &op);

}  // namespace fdg
