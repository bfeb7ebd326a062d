// Reduced-precision mode products of the fast-diagonalization apply (eq. 4.7 / 4.9).
//
// FP32: v_mfma_f32_16x16x4_f32 on FP32 factors and intermediates.
// BF16: every mode-product input (factor and tensor) is rounded to BF16 on load
// (round to nearest even), products accumulate in FP32 (v_mfma_f32_16x16x32_bf16),
// intermediates are stored as FP32.  The diagonal solve runs in FP32.  The first pass
// reads the FP64 Krylov vector and the last pass writes FP64.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "bf16_round.h"
#include "common.h"
#include "modeprod.h"

namespace fdg {

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kBlock = 256;

template <typename T>
__device__ inline float ld_f(const T *p) { return (float)*p; }

// Y[o*sO + k*sJ + c*sC] = sum_j W[k*ldw + j] X[o*sO + j*sJ + c*sC]; tile 64 x 64 per
// workgroup, 2 x 2 MFMA tiles of 16 x 16 per wave (the same lane layout as FP64:
// A[m = l%16][k-group = l/16], B[k-group = l/16][n = l%16], D[4*(l/16) + r][l%16]).
template <typename TIn, typename TOut>
__global__ __launch_bounds__(kBlock) void k_modeprod_f32(const TIn *__restrict__ X, TOut *__restrict__ Y,
                                                         const float *__restrict__ W, int ldw, int n,
                                                         int64_t ncols, int64_t sO, int64_t sJ, int64_t sC) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * 64 + (wave & 1) * 32;
  const int k0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int64_t o = blockIdx.z;
  const TIn *Xo = X + o * sO;
  TOut *Yo = Y + o * sO;
  flt4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = flt4{0.f, 0.f, 0.f, 0.f};
  const float *Wr0 = W + (size_t)(k0 + li) * ldw;
  const float *Wr1 = W + (size_t)(k0 + 16 + li) * ldw;
  const int64_t cA = c0 + li, cB = c0 + 16 + li;
  const bool okA = cA < ncols, okB = cB < ncols;
  for (int j0 = 0; j0 < n; j0 += 4) {
    const int j = j0 + lg;
    const float a0 = Wr0[j], a1 = Wr1[j];
    const bool jok = j < n;
    const float b0 = (jok && okA) ? ld_f(Xo + j * sJ + cA * sC) : 0.f;
    const float b1 = (jok && okB) ? ld_f(Xo + j * sJ + cB * sC) : 0.f;
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
  }
  for (int ti = 0; ti < 2; ++ti)
    for (int tj = 0; tj < 2; ++tj) {
      const int64_t c = c0 + 16 * tj + li;
      if (c >= ncols) continue;
      for (int r = 0; r < 4; ++r) {
        const int k = k0 + 16 * ti + 4 * lg + r;
        if (k < n) Yo[k * sJ + c * sC] = (TOut)acc[ti][tj][r];
      }
    }
}

// BF16 inputs: lane l supplies A[m = l%16][kk(l/16, t)] and B[kk(l/16, t)][n = l%16],
// t < 8, with kk(g, t) = 8 g + t inside each block of 32 contraction indices.
template <typename TIn, typename TOut>
__global__ __launch_bounds__(kBlock) void k_modeprod_bf16(const TIn *__restrict__ X, TOut *__restrict__ Y,
                                                          const __bf16 *__restrict__ W, int ldw, int n,
                                                          int64_t ncols, int64_t sO, int64_t sJ, int64_t sC) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * 64 + (wave & 1) * 32;
  const int k0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int64_t o = blockIdx.z;
  const TIn *Xo = X + o * sO;
  TOut *Yo = Y + o * sO;
  flt4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = flt4{0.f, 0.f, 0.f, 0.f};
  const __bf16 *Wr0 = W + (size_t)(k0 + li) * ldw;
  const __bf16 *Wr1 = W + (size_t)(k0 + 16 + li) * ldw;
  const int64_t cA = c0 + li, cB = c0 + 16 + li;
  const bool okA = cA < ncols, okB = cB < ncols;
  for (int j0 = 0; j0 < n; j0 += 32) {
    bf16x8 a0, a1, b0, b1;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int j = j0 + 8 * lg + t;
      const bool jok = j < n;
      a0[t] = Wr0[j];
      a1[t] = Wr1[j];
      b0[t] = to_bf16_once((jok && okA) ? Xo[j * sJ + cA * sC] : TIn(0));
      b1[t] = to_bf16_once((jok && okB) ? Xo[j * sJ + cB * sC] : TIn(0));
    }
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
  }
  for (int ti = 0; ti < 2; ++ti)
    for (int tj = 0; tj < 2; ++tj) {
      const int64_t c = c0 + 16 * tj + li;
      if (c >= ncols) continue;
      for (int r = 0; r < 4; ++r) {
        const int k = k0 + 16 * ti + 4 * lg + r;
        if (k < n) Yo[k * sJ + c * sC] = (TOut)acc[ti][tj][r];
      }
    }
}

__global__ __launch_bounds__(kBlock) void k_divide_f32(float *__restrict__ t, int d, int n, int64_t total,
                                                       const float *__restrict__ l1, const float *__restrict__ l2,
                                                       const float *__restrict__ l3) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= total) return;
  const int i1 = (int)(idx % n);
  const int i2 = (int)((idx / n) % n);
  float den = l2[i2] + l1[i1];
  if (d == 3) den = l3[(idx / ((int64_t)n * n)) % n] + den;
  t[idx] = t[idx] / den;
}

template <typename TIn, typename TOut>
void modeprod(hipStream_t s, int prec, const TIn *X, TOut *Y, const void *W, int ldw, int n, int64_t ncols,
              int64_t sO, int64_t sJ, int64_t sC, int64_t nbatch) {
  for (int64_t o0 = 0; o0 < nbatch; o0 += 65535) {
    const int64_t nb = nbatch - o0 < 65535 ? nbatch - o0 : 65535;
    dim3 grid((unsigned)((ncols + 63) / 64), (unsigned)((n + 63) / 64), (unsigned)nb);
    if (prec == FDG_PREC_FP32)
      hipLaunchKernelGGL((k_modeprod_f32<TIn, TOut>), grid, dim3(kBlock), 0, s, X + o0 * sO, Y + o0 * sO,
                         (const float *)W, ldw, n, ncols, sO, sJ, sC);
    else
      hipLaunchKernelGGL((k_modeprod_bf16<TIn, TOut>), grid, dim3(kBlock), 0, s, X + o0 * sO, Y + o0 * sO,
                         (const __bf16 *)W, ldw, n, ncols, sO, sJ, sC);
  }
}

// Strides of the mode-l product for the layout [batch][n_d]..[n_1].
struct ModeGeom {
  int64_t ncols, sO, sJ, sC, nb;
};

ModeGeom geom(int d, int n, int64_t B, int l) {
  const int64_t n2 = (int64_t)n * n;
  if (l == 0) return {B * (d == 3 ? n2 : n), 0, 1, n, 1};
  if (l == 1) return {n, n2, n, 1, B * (d == 3 ? n : 1)};
  return {n2, n2 * n, n2, 1, B};
}

}  // namespace

int fd_apply_lowp(hipStream_t s, int prec, int d, int n, int64_t B, const double *b, double *out, void *ta,
                  void *tb, const void *const *Wv, const void *const *Wu, float *const *lam, int ldw) {
  float *A = (float *)ta, *T = (float *)tb;
  const int64_t N = B * (int64_t)n * n * (d == 3 ? n : 1);
  auto g = [&](int l) { return geom(d, n, B, l); };
  ModeGeom q;
  // stage 1: (V_d x .. x V_1)^T b
  q = g(0);
  modeprod<double, float>(s, prec, b, A, Wv[0], ldw, n, q.ncols, q.sO, q.sJ, q.sC, q.nb);
  q = g(1);
  modeprod<float, float>(s, prec, A, T, Wv[1], ldw, n, q.ncols, q.sO, q.sJ, q.sC, q.nb);
  float *cur = T, *oth = A;
  if (d == 3) {
    q = g(2);
    modeprod<float, float>(s, prec, T, A, Wv[2], ldw, n, q.ncols, q.sO, q.sJ, q.sC, q.nb);
    cur = A;
    oth = T;
  }
  // stage 2: diagonal solve
  hipLaunchKernelGGL(k_divide_f32, dim3((unsigned)((N + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, cur, d, n, N,
                     lam[0], lam[1], d == 3 ? lam[2] : lam[1]);
  // stage 3: (U_d x .. x U_1), in 3D in the order of the fused passes (direction 3, then
  // 1 and 2), so that the roundings between the products fall at the same points
  if (d == 3) {
    q = g(2);
    modeprod<float, float>(s, prec, cur, oth, Wu[2], ldw, n, q.ncols, q.sO, q.sJ, q.sC, q.nb);
    q = g(0);
    modeprod<float, float>(s, prec, oth, cur, Wu[0], ldw, n, q.ncols, q.sO, q.sJ, q.sC, q.nb);
    q = g(1);
    modeprod<float, double>(s, prec, cur, out, Wu[1], ldw, n, q.ncols, q.sO, q.sJ, q.sC, q.nb);
  } else {
    q = g(0);
    modeprod<float, float>(s, prec, cur, oth, Wu[0], ldw, n, q.ncols, q.sO, q.sJ, q.sC, q.nb);
    q = g(1);
    modeprod<float, double>(s, prec, oth, out, Wu[1], ldw, n, q.ncols, q.sO, q.sJ, q.sC, q.nb);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(FDG_EHIP, "low-precision apply launch: %s", hipGetErrorString(e));
  return FDG_OK;
}

}  // namespace fdg
