// Fused FP32 fast-diagonalization solve (eq. 4.9 / 4.7) on FP32 MFMA: the three passes of
// the FP64 solve (slab: modes 1 and 2; fibre: mode 3, divide, mode 3; slab: modes 1 and 2)
// with the factors rounded once to FP32, FP32 products and accumulation, FP32
// intermediates between the passes, an FP64 input to the first pass and an FP64 output
// from the last.  The preconditioner is then inexact at the FP32 level, which flexible
// GMRES absorbs.
//
// v_mfma_f32_16x16x4_f32 lane layout (li = lane % 16, lg = lane / 16):
//   A[m = li][k = lg], B[k = lg][n = li], D[m = 4 lg + r][n = li] in register r.
// As in the FP64 passes, lane group lg supplies contraction index j0 + 4 lg + t to both
// operands of the t-th MFMA of a 16-wide k-block, so each lane reads four consecutive
// elements.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fd_apply.h"

namespace fdg {

namespace {

typedef float flt4 __attribute__((ext_vector_type(4)));

// NT: 16-column MFMA tiles per wave (16 NT columns per workgroup), a template parameter:
// 2 at large n, 1 where more workgroups are needed to fill the device
constexpr int kPad = 4;        // LDS row padding (floats)

__device__ inline flt4 mfma32(float a, float b, flt4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// Four consecutive elements p[0..3] as floats, zero where j + t >= jmax or !ok.
template <typename T>
__device__ inline void load4f(const T *p, int j, int jmax, bool ok, float (&v)[4]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) v[t] = (ok && j + t < jmax) ? (float)p[t] : 0.0f;
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// The same with one 4-wide load where the whole group is in range (VEC: p is aligned to
// 4 elements, i.e. n % 4 == 0 and 32-byte aligned rows).
template <bool VEC, typename T>
__device__ inline void load4v(const T *p, int j, int jmax, bool ok, float (&v)[4]) {
  if (VEC && ok && j + 3 < jmax) {
    if constexpr (sizeof(T) == 8) {
      const dbl4 x = *reinterpret_cast<const dbl4 *>(p);
#pragma unroll
      for (int t = 0; t < 4; ++t) v[t] = (float)x[t];
    } else {
      const flt4 x = *reinterpret_cast<const flt4 *>(p);
#pragma unroll
      for (int t = 0; t < 4; ++t) v[t] = x[t];
    }
    return;
  }
  load4f(p, j, jmax, ok, v);
}

// Operands of one 16-wide k-block: A as loaded (TA: float, or the FP64 input of the first
// pass, rounded to FP32 where the MFMA takes it, so that the next k-block's loads are
// issued before this one's values are used), B from LDS.
template <int MT, int NT, typename TA = float>
struct Frag32 {
  TA a[MT][4];
  float b[NT][4];
};

template <int MT, int NT, typename TA>
__device__ inline void mma_block32(const Frag32<MT, NT, TA> &f, flt4 (&acc)[MT][NT]) {
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int b = 0; b < NT; ++b) acc[a][b] = mfma32((float)f.a[a][t], f.b[b][t], acc[a][b]);
}

// acc = sum over the 16-wide k-blocks below kpad <= 16 KB; block kb + 1's operands are
// loaded before block kb's MFMAs, in a loop unrolled over the KB blocks with unconditional
// loads (load stays in bounds for every j0 < 16 KB), so that the compiler waits for exactly
// the loads a block needs (a rolled loop with conditional loads waited for all of them).
template <int MT, int NT, int KB, typename TA = float, typename Load>
__device__ inline void gemm32(int kpad, Load load, flt4 (&acc)[MT][NT]) {
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = flt4{0.f, 0.f, 0.f, 0.f};
  Frag32<MT, NT, TA> f[2];
  load(0, f[0]);
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    if (kb + 1 < KB) load(16 * (kb + 1), f[(kb + 1) & 1]);
    if (16 * kb < kpad) mma_block32<MT, NT>(f[kb & 1], acc);
  }
}

// Pass A / C: workgroup = (slab s, block of kNB columns); wave w owns rows
// [w*MT*16, (w+1)*MT*16) of both contractions.
//   GEMM1: Y1[i2][c] = sum_i1 X[s][i2][i1] W1[c][i1]   (W1 column tile in LDS)
//   GEMM2: Y2[k2][c] = sum_i2 W2[k2][i2] Y1[i2][c]     (Y1 in LDS, transposed)
//   2D: Y2[k2][c] /= lam2[k2] + lam1[c].
template <int WAVES, int MT, int NT, typename TI, typename TO, bool DIV, bool VEC>
__global__ __launch_bounds__(64 * WAVES) void k_slab32(const TI *__restrict__ X, TO *__restrict__ Y,
                                                       const float *__restrict__ W1, const float *__restrict__ W2,
                                                       int ldw, int n, int64_t nslab, int ncb, int xcd_remap,
                                                       const float *__restrict__ lam1, const float *__restrict__ lam2) {
  constexpr int MPAD = WAVES * MT * 16;
  constexpr int LDP = MPAD + kPad;
  constexpr int NTHR = 64 * WAVES;
  constexpr int kNB = 16 * NT;
  __shared__ float buf[kNB * LDP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  int64_t s;
  int cb;
  {
    const int64_t bid = blockIdx.x;
    if (xcd_remap) {  // the ncb workgroups of one slab share an XCD
      const int64_t xcd = bid & 7, local = bid >> 3;
      s = (local / ncb) * 8 + xcd;
      cb = (int)(local % ncb);
    } else {
      s = bid / ncb;
      cb = (int)(bid % ncb);
    }
  }
  if (s >= nslab) return;
  const int64_t n2 = (int64_t)n * n;
  const TI *__restrict__ Xs = X + s * n2;
  TO *__restrict__ Ys = Y + s * n2;
  const int c0 = cb * kNB;
  const int m0 = wave * MT * 16;
  const int kpad = (n + 15) & ~15;
  {  // W1 column tile, 4-wide: every load of the thread issued before the first LDS store
    constexpr int SIT = (kNB * (MPAD / 4) + NTHR - 1) / NTHR;
    const int q4 = kpad / 4, stot = kNB * q4;
    flt4 sv[SIT];
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
      const int e0 = (int)threadIdx.x + it * NTHR, e = e0 < stot ? e0 : stot - 1;
      const int c = e / q4, j = 4 * (e - c * q4);
      sv[it] = *reinterpret_cast<const flt4 *>(W1 + (size_t)(c0 + c) * ldw + j);
    }
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
      const int e = (int)threadIdx.x + it * NTHR;
      if (e < stot) {
        const int c = e / q4, j = 4 * (e - c * q4);
#pragma unroll
        for (int t = 0; t < 4; ++t) buf[c * LDP + j + t] = sv[it][t];
      }
    }
  }
  __syncthreads();
  flt4 acc[MT][NT];
  if constexpr (VEC) {
    // A loaded 4-wide at clamped addresses with no branch (its values are rounded to FP32
    // only where the MFMA takes them): an element beyond the slab's n columns or rows
    // meets a zero of the zero-padded W1 tile in GEMM1, and a padding row of Y1 a zero
    // column of W2 in GEMM2, so the clamped values never reach the result
    gemm32<MT, NT, MPAD / 16, TI>(kpad, [&](int j0, Frag32<MT, NT, TI> &f) {
      const int j = j0 + 4 * lg, jc = j < n ? j : n - 4;
#pragma unroll
      for (int a = 0; a < MT; ++a) {
        const int row = m0 + 16 * a + li, rowc = row < n ? row : n - 1;
        typedef typename std::conditional<sizeof(TI) == 8, dbl4, flt4>::type V4;
        const V4 x = *reinterpret_cast<const V4 *>(Xs + (int64_t)rowc * n + jc);
#pragma unroll
        for (int t = 0; t < 4; ++t) f.a[a][t] = x[t];
      }
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        const float *p = buf + (16 * b + li) * LDP + j;
        f.b[b][0] = p[0]; f.b[b][1] = p[1]; f.b[b][2] = p[2]; f.b[b][3] = p[3];
      }
    }, acc);
  } else {
    gemm32<MT, NT, MPAD / 16>(kpad, [&](int j0, Frag32<MT, NT> &f) {
      const int j = j0 + 4 * lg;
#pragma unroll
      for (int a = 0; a < MT; ++a) {
        const int row = m0 + 16 * a + li;
        load4f(Xs + (int64_t)row * n + j, j, n, row < n, f.a[a]);
      }
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        const float *p = buf + (16 * b + li) * LDP + j;
        f.b[b][0] = p[0]; f.b[b][1] = p[1]; f.b[b][2] = p[2]; f.b[b][3] = p[3];
      }
    }, acc);
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) buf[(16 * b + li) * LDP + m0 + 16 * a + 4 * lg + r] = acc[a][b][r];
  __syncthreads();
  gemm32<MT, NT, MPAD / 16>(kpad, [&](int j0, Frag32<MT, NT> &f) {
    const int j = j0 + 4 * lg;
#pragma unroll
    for (int a = 0; a < MT; ++a) {
      const float *w = W2 + (size_t)(m0 + 16 * a + li) * ldw + j;
      f.a[a][0] = w[0]; f.a[a][1] = w[1]; f.a[a][2] = w[2]; f.a[a][3] = w[3];
    }
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      const float *p = buf + (16 * b + li) * LDP + j;
      f.b[b][0] = p[0]; f.b[b][1] = p[1]; f.b[b][2] = p[2]; f.b[b][3] = p[3];
    }
  }, acc);
#pragma unroll
  for (int b = 0; b < NT; ++b) {
    const int c = c0 + 16 * b + li;
    if (c >= n) continue;
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k2 = m0 + 16 * a + 4 * lg + r;
        if (k2 < n) {
          float v = acc[a][b][r];
          if (DIV) v = v / (lam2[k2] + lam1[c]);
          Ys[(int64_t)k2 * n + c] = (TO)v;
        }
      }
  }
}

// Pass B: workgroup = (entry, block of kNB columns c of X[i3][c]); the block is staged
// transposed in LDS, then T = Wa X, T /= lam3 + lam2 + lam1, S = Wb T.
template <int WAVES, int MT, int NT, bool VEC>
__global__ __launch_bounds__(64 * WAVES) void k_fibre32(const float *__restrict__ X, float *__restrict__ Y,
                                                        const float *__restrict__ Wa, const float *__restrict__ Wb,
                                                        int ldw, int n, int ncb, const float *__restrict__ lam1,
                                                        const float *__restrict__ lam2, const float *__restrict__ lam3) {
  constexpr int MPAD = WAVES * MT * 16;
  constexpr int LDP = MPAD + kPad;
  constexpr int NTHR = 64 * WAVES;
  constexpr int kNB = 16 * NT;
  __shared__ float xt[kNB * LDP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t bidx = blockIdx.x / ncb;
  const int cb = (int)(blockIdx.x % ncb);
  const int64_t n2 = (int64_t)n * n;
  const float *__restrict__ Xb = X + bidx * n2 * n;
  float *__restrict__ Yb = Y + bidx * n2 * n;
  const int64_t c0 = (int64_t)cb * kNB;
  const int m0 = wave * MT * 16;
  const int kpad = (n + 15) & ~15;
  // the eigenvalues of the divide, loaded with the first loads of the pass (a load used
  // right after it is issued would be waited for on its own)
  float lv3[MT][4], lv2[NT], lv1[NT];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) lv3[a][r] = lam3[m0 + 16 * a + 4 * lg + r];
#pragma unroll
  for (int b = 0; b < NT; ++b) {
    const int64_t cg = c0 + 16 * b + li;
    const bool cok = cg < n2;
    lv2[b] = lam2[cok ? (int)(cg / n) : 0];
    lv1[b] = lam1[cok ? (int)(cg % n) : 0];
  }
  if (VEC) {  // n^2 % 4 == 0 and a 16-byte aligned X: four columns per load, every load of
             // the thread issued (at clamped addresses) before the first LDS store
    constexpr int Q = kNB / 4;
    constexpr int SIT = (MPAD * Q + NTHR - 1) / NTHR;
    flt4 sv[SIT];
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
      const int e = (int)threadIdx.x + it * NTHR;
      const int i3 = e / Q, q = e - i3 * Q;
      const int64_t cg = c0 + 4 * q;
      const int i3c = i3 < n ? i3 : n - 1;
      const int64_t cgc = cg < n2 ? cg : n2 - 4;
      sv[it] = *reinterpret_cast<const flt4 *>(Xb + (int64_t)i3c * n2 + cgc);
    }
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
      const int e = (int)threadIdx.x + it * NTHR;
      if (e < kpad * Q) {
        const int i3 = e / Q, q = e - i3 * Q;
        const bool ok = i3 < n && c0 + 4 * q < n2;
#pragma unroll
        for (int t = 0; t < 4; ++t) xt[(4 * q + t) * LDP + i3] = ok ? sv[it][t] : 0.0f;
      }
    }
  } else {
    for (int e = threadIdx.x; e < kpad * kNB; e += NTHR) {
      const int i3 = e / kNB, c = e % kNB;
      const int64_t cg = c0 + c;
      xt[c * LDP + i3] = (i3 < n && cg < n2) ? Xb[(int64_t)i3 * n2 + cg] : 0.0f;
    }
  }
  __syncthreads();
  flt4 acc[MT][NT];
  auto lds_gemm = [&](const float *W) {
    gemm32<MT, NT, MPAD / 16>(kpad, [&](int j0, Frag32<MT, NT> &f) {
      const int j = j0 + 4 * lg;
#pragma unroll
      for (int a = 0; a < MT; ++a) {
        const float *w = W + (size_t)(m0 + 16 * a + li) * ldw + j;
        f.a[a][0] = w[0]; f.a[a][1] = w[1]; f.a[a][2] = w[2]; f.a[a][3] = w[3];
      }
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        const float *p = xt + (16 * b + li) * LDP + j;
        f.b[b][0] = p[0]; f.b[b][1] = p[1]; f.b[b][2] = p[2]; f.b[b][3] = p[3];
      }
    }, acc);
  };
  lds_gemm(Wa);
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NT; ++b) {
    const float l12 = lv2[b] + lv1[b];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k3 = m0 + 16 * a + 4 * lg + r;
        xt[(16 * b + li) * LDP + k3] = acc[a][b][r] / (lv3[a][r] + l12);  // lam3 padded with 1
      }
  }

  __syncthreads();
  lds_gemm(Wb);
#pragma unroll
  for (int b = 0; b < NT; ++b) {
    const int64_t cg = c0 + 16 * b + li;
    if (cg >= n2) continue;
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k3 = m0 + 16 * a + 4 * lg + r;
        if (k3 < n) Yb[(int64_t)k3 * n2 + cg] = acc[a][b][r];
      }
  }
}

// Workgroup shape as for the FP64 passes (waves, 16-row tiles per wave, 16-column tiles
// per wave): 16 columns per workgroup for 3D n <= 96 and the 2D solve.
struct Shape32 {
  int waves, mt, nt;
};

Shape32 pick_shape32(int n, bool small_grid) {
  const int nt = (small_grid || n <= 96) ? 1 : 2;
  const int k = (n + 15) / 16;
  if (k <= 4) return {4, 1, nt};
  if (k <= 8) return {k, 1, nt};
  if (k <= 12) return {12, 1, nt};
  return {8, 2, nt};
}

#define FDG_SHAPES32(X)                                                                          \
  X(4, 1, 1) X(5, 1, 1) X(6, 1, 1) X(7, 1, 1) X(8, 1, 1) X(12, 1, 1) X(8, 2, 1)                  \
  X(4, 1, 2) X(5, 1, 2) X(6, 1, 2) X(7, 1, 2) X(8, 1, 2) X(12, 1, 2) X(8, 2, 2)

template <int W, int M, int NT, typename TI, typename TO>
void slab32(hipStream_t s, const TI *X, TO *Y, const float *W1, const float *W2, int ldw, int n, int64_t nslab,
            bool div, const float *lam1, const float *lam2) {
  constexpr int kNB = 16 * NT;
  const int ncb = (n + kNB - 1) / kNB;
  const int remap = (nslab % 8 == 0) ? 1 : 0;
  const dim3 grid((unsigned)(nslab * ncb)), blk(64 * W);
  const bool vec = n % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 31) == 0;
#define FDG_SLAB32(D, V)                                                                                        \
  hipLaunchKernelGGL((k_slab32<W, M, NT, TI, TO, D, V>), grid, blk, 0, s, X, Y, W1, W2, ldw, n, nslab, ncb, remap, \
                     lam1, lam2)
  if (div) {
    if (vec) FDG_SLAB32(true, true); else FDG_SLAB32(true, false);
  } else {
    if (vec) FDG_SLAB32(false, true); else FDG_SLAB32(false, false);
  }
#undef FDG_SLAB32
}

template <typename TI, typename TO>
void slab32_dispatch(hipStream_t s, const TI *X, TO *Y, const float *W1, const float *W2, int ldw, int n,
                     int64_t nslab, bool two_d, bool div, const float *lam1, const float *lam2) {
  const Shape32 sh = pick_shape32(n, two_d);
#define FDG_CASE(W, M, T)                                                        \
  if (sh.waves == W && sh.mt == M && sh.nt == T) {                              \
    slab32<W, M, T, TI, TO>(s, X, Y, W1, W2, ldw, n, nslab, div, lam1, lam2);   \
    return;                                                                     \
  }
  FDG_SHAPES32(FDG_CASE)
#undef FDG_CASE
}

void fibre32_dispatch(hipStream_t s, const float *X, float *Y, const float *Wa, const float *Wb, int ldw, int n,
                      int64_t batch, const float *lam1, const float *lam2, const float *lam3) {
  const Shape32 sh = pick_shape32(n, false);
  const int64_t n2 = (int64_t)n * n;
  const bool vec = n2 % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
#define FDG_CASE(W, M, T)                                                                                         \
  if (sh.waves == W && sh.mt == M && sh.nt == T) {                                                               \
    const int ncb = (int)((n2 + 16 * T - 1) / (16 * T));                                                         \
    if (vec)                                                                                                     \
      hipLaunchKernelGGL((k_fibre32<W, M, T, true>), dim3((unsigned)(batch * ncb)), dim3(64 * W), 0, s, X, Y, Wa, Wb,  \
                         ldw, n, ncb, lam1, lam2, lam3);                                                         \
    else                                                                                                         \
      hipLaunchKernelGGL((k_fibre32<W, M, T, false>), dim3((unsigned)(batch * ncb)), dim3(64 * W), 0, s, X, Y, Wa, Wb, \
                         ldw, n, ncb, lam1, lam2, lam3);                                                         \
    return;                                                                                                      \
  }
  FDG_SHAPES32(FDG_CASE)
#undef FDG_CASE
}

}  // namespace

void launch_fd_apply_f32(hipStream_t s, int d, int n, int64_t batch, const double *b, double *out, float *t1,
                         float *t2, const float *const *Wv, const float *const *Wu, const float *const *lam, int ldw) {
  if (d == 3) {
    const int64_t nslab = batch * n;
    slab32_dispatch<double, float>(s, b, t1, Wv[0], Wv[1], ldw, n, nslab, false, false, nullptr, nullptr);
    fibre32_dispatch(s, t1, t2, Wv[2], Wu[2], ldw, n, batch, lam[0], lam[1], lam[2]);
    slab32_dispatch<float, double>(s, t2, out, Wu[0], Wu[1], ldw, n, nslab, false, false, nullptr, nullptr);
  } else {
    slab32_dispatch<double, float>(s, b, t1, Wv[0], Wv[1], ldw, n, batch, true, true, lam[0], lam[1]);
    slab32_dispatch<float, double>(s, t1, out, Wu[0], Wu[1], ldw, n, batch, true, false, nullptr, nullptr);
  }
}

}  // namespace fdg
