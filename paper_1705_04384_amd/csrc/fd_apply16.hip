// Fused BF16 fast-diagonalization solve (eq. 4.9 / 4.7): the three passes of the FP64
// solve (slab: modes 1 and 2; fibre: mode 3, divide, mode 3; slab: modes 1 and 2) on
// v_mfma_f32_16x16x32_bf16.  Every mode-product input, factor and tensor, is rounded to
// BF16 (round to nearest even) where it enters an MFMA; products accumulate in FP32, and
// the diagonal solve and the scaling are FP32.  The intermediates between passes are
// stored already rounded to BF16: the next pass rounds each of them to BF16 where it enters
// its first MFMA, so storing the rounded value gives the same bits with half the traffic.
// The first pass reads the FP64 Krylov vector and the last one writes FP64.
//
// v_mfma_f32_16x16x32_bf16 lane layout (li = lane % 16, lg = lane / 16), per 32-wide
// block of the contraction index starting at j0:
//   A[m = li][k = j0 + 8 lg + t], B[k = j0 + 8 lg + t][n = li], t < 8 (eight BF16 per lane),
//   D[m = 4 lg + r][n = li] in register r.
// Intermediates that feed the next MFMA inside a pass are kept in LDS already rounded to
// BF16, which is the rounding the next product applies on load.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "bf16_round.h"
#include "fd_apply.h"

namespace fdg {

namespace {

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kPadB = 8;  // LDS row padding (BF16 elements: rows stay 16-byte aligned)

__device__ inline flt4 mfma16(const bf16x8 &a, const bf16x8 &b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Eight consecutive elements p[0..7] rounded to BF16, zero where j + t >= jmax or !ok.
template <typename T>
__device__ inline bf16x8 load8(const T *p, int j, int jmax, bool ok) {
  bf16x8 v;
#pragma unroll
  for (int t = 0; t < 8; ++t) v[t] = to_bf16_once((ok && j + t < jmax) ? p[t] : T(0));
  return v;
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// The same with two 4-wide loads where the whole group is in range (VEC: p is aligned to
// 4 elements, i.e. n % 4 == 0 and 32-byte aligned rows).
template <bool VEC, typename T>
__device__ inline bf16x8 load8v(const T *p, int j, int jmax, bool ok) {
  if (VEC && ok && j + 7 < jmax) {
    bf16x8 v;
    if constexpr (sizeof(T) == 8) {
      const dbl4 x0 = *reinterpret_cast<const dbl4 *>(p), x1 = *reinterpret_cast<const dbl4 *>(p + 4);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        v[t] = to_bf16_once(x0[t]);
        v[4 + t] = to_bf16_once(x1[t]);
      }
    } else if constexpr (sizeof(T) == 4) {
      const flt4 x0 = *reinterpret_cast<const flt4 *>(p), x1 = *reinterpret_cast<const flt4 *>(p + 4);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        v[t] = to_bf16_once(x0[t]);
        v[4 + t] = to_bf16_once(x1[t]);
      }
    } else {  // BF16 already: one 16-byte load (VEC: p is 16-byte aligned)
      v = *reinterpret_cast<const bf16x8 *>(p);
    }
    return v;
  }
  return load8(p, j, jmax, ok);
}

// A pass output in its stored type: FP64 and FP32 as computed, BF16 rounded to nearest even.
template <typename TO>
__device__ inline TO store_as(float v) {
  if constexpr (sizeof(TO) == 2)
    return to_bf16_once(v);
  else
    return (TO)v;
}

// Eight consecutive BF16 (16-byte aligned, always in bounds).
__device__ inline bf16x8 load8_bf(const __bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

template <int MT, int NT>
struct Frag16 {
  bf16x8 a[MT];
  bf16x8 b[NT];
};

template <int MT, int NT>
__device__ inline void mma_block16(const Frag16<MT, NT> &f, flt4 (&acc)[MT][NT]) {
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = mfma16(f.a[a], f.b[b], acc[a][b]);
}

// acc = sum over the 32-wide k-blocks j0 = 0, 32, .., kpad - 32 (kpad <= 32 KB) of
// load(j0); block kb + 1's operands are loaded before block kb's MFMAs, in a loop unrolled
// over the KB blocks with unconditional loads (load stays in bounds for every j0 < 32 KB),
// so that the compiler waits for exactly the loads a block needs (a rolled loop with
// conditional loads waited for all of them).
template <int MT, int NT, int KB, typename Load>
__device__ inline void gemm16(int kpad, Load load, flt4 (&acc)[MT][NT]) {
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = flt4{0.f, 0.f, 0.f, 0.f};
  Frag16<MT, NT> f[2];
  load(0, f[0]);
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    if (kb + 1 < KB) load(32 * (kb + 1), f[(kb + 1) & 1]);
    if (32 * kb < kpad) mma_block16<MT, NT>(f[kb & 1], acc);
  }
}

// Pass A / C: workgroup = (slab s, block of kNB columns); wave w owns rows
// [w*MT*16, (w+1)*MT*16) of both contractions.  MPAD = 16 WAVES MT is a multiple of 32
// and at least n, so the 32-wide k-blocks never leave the staged rows.
//   GEMM1: Y1[i2][c] = sum_i1 X[s][i2][i1] W1[c][i1]   (W1 column tile in LDS, BF16)
//   GEMM2: Y2[k2][c] = sum_i2 W2[k2][i2] Y1[i2][c]     (Y1 in LDS transposed, BF16)
//   2D: Y2[k2][c] /= lam2[k2] + lam1[c].
template <int WAVES, int MT, int NT, typename TI, typename TO, bool DIV, bool VEC>
__global__ __launch_bounds__(64 * WAVES) void k_slab16(const TI *__restrict__ X, TO *__restrict__ Y,
                                                       const __bf16 *__restrict__ W1, const __bf16 *__restrict__ W2,
                                                       int ldw, int n, int64_t nslab, int ncb, int xcd_remap,
                                                       const float *__restrict__ lam1, const float *__restrict__ lam2) {
  constexpr int MPAD = WAVES * MT * 16;
  static_assert(MPAD % 32 == 0, "k-blocks of 32 need MPAD a multiple of 32");
  constexpr int LDP = MPAD + kPadB;
  constexpr int NTHR = 64 * WAVES;
  constexpr int kNB = 16 * NT;
  __shared__ __attribute__((aligned(16))) __bf16 buf[kNB * LDP];
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
  const int kpad = (n + 31) & ~31;
  // the wave's whole strip of X (its MT*16 rows, every 32-wide k-block) is loaded first,
  // eight BF16 per lane and k-block (4 VGPRs), so its memory latency overlaps the W1
  // staging below
  constexpr int KB = MPAD / 32;
  bf16x8 xa[MT][KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    const int j = kb * 32 + 8 * lg;
#pragma unroll
    for (int a = 0; a < MT; ++a) {
      const int row = m0 + 16 * a + li;
      xa[a][kb] = load8v<VEC>(Xs + (int64_t)row * n + j, j, n, row < n && kb * 32 < kpad);
    }
  }
  // W1 columns c0 .. c0 + kNB (zero-padded factor rows and columns beyond n), 8 at a time
  for (int e = threadIdx.x; e < kNB * (kpad / 8); e += NTHR) {
    const int c = e / (kpad / 8), j = 8 * (e - c * (kpad / 8));
    *reinterpret_cast<bf16x8 *>(buf + c * LDP + j) = load8_bf(W1 + (size_t)(c0 + c) * ldw + j);
  }
  __syncthreads();
  flt4 acc[MT][NT];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    if (kb * 32 >= kpad) break;
    const int j = kb * 32 + 8 * lg;
    bf16x8 bv[NT];
#pragma unroll
    for (int b = 0; b < NT; ++b) bv[b] = load8_bf(buf + (16 * b + li) * LDP + j);
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int b = 0; b < NT; ++b) acc[a][b] = mfma16(xa[a][kb], bv[b], acc[a][b]);
  }
  __syncthreads();  // every wave is done with the W1 tile
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) buf[(16 * b + li) * LDP + m0 + 16 * a + 4 * lg + r] = to_bf16_once(acc[a][b][r]);
  __syncthreads();
  gemm16<MT, NT, MPAD / 32>(kpad, [&](int j0, Frag16<MT, NT> &f) {
    const int j = j0 + 8 * lg;
#pragma unroll
    for (int a = 0; a < MT; ++a) f.a[a] = load8_bf(W2 + (size_t)(m0 + 16 * a + li) * ldw + j);
#pragma unroll
    for (int b = 0; b < NT; ++b) f.b[b] = load8_bf(buf + (16 * b + li) * LDP + j);
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
          Ys[(int64_t)k2 * n + c] = store_as<TO>(v);
        }
      }
  }
}

// Pass B: workgroup = (entry, block of kNB columns c of X[i3][c]); the block is staged
// transposed in LDS (BF16), then T = Wa X, T /= lam3 + lam2 + lam1 (FP32), S = Wb T.
template <int WAVES, int MT, int NT, bool VEC, typename TI, typename TO>
__global__ __launch_bounds__(64 * WAVES) void k_fibre16(const TI *__restrict__ X, TO *__restrict__ Y,
                                                        const __bf16 *__restrict__ Wa, const __bf16 *__restrict__ Wb,
                                                        int ldw, int n, int ncb, const float *__restrict__ lam1,
                                                        const float *__restrict__ lam2, const float *__restrict__ lam3) {
  constexpr int MPAD = WAVES * MT * 16;
  static_assert(MPAD % 32 == 0, "k-blocks of 32 need MPAD a multiple of 32");
  constexpr int LDP = MPAD + kPadB;
  constexpr int NTHR = 64 * WAVES;
  constexpr int kNB = 16 * NT;
  __shared__ __attribute__((aligned(16))) __bf16 xt[kNB * LDP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t bidx = blockIdx.x / ncb;
  const int cb = (int)(blockIdx.x % ncb);
  const int64_t n2 = (int64_t)n * n;
  const TI *__restrict__ Xb = X + bidx * n2 * n;
  TO *__restrict__ Yb = Y + bidx * n2 * n;
  const int64_t c0 = (int64_t)cb * kNB;
  const int m0 = wave * MT * 16;
  const int kpad = (n + 31) & ~31;
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
  if (VEC) {  // n^2 % 4 == 0 and an aligned X: four columns per load, every load of the
             // thread issued (at clamped addresses) before the first LDS store
    typedef TI vec4 __attribute__((ext_vector_type(4)));
    constexpr int Q = kNB / 4;
    constexpr int SIT = (MPAD * Q + NTHR - 1) / NTHR;
    vec4 sv[SIT];
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
      const int e = (int)threadIdx.x + it * NTHR;
      const int i3 = e / Q, q = e - i3 * Q;
      const int64_t cg = c0 + 4 * q;
      const int i3c = i3 < n ? i3 : n - 1;
      const int64_t cgc = cg < n2 ? cg : n2 - 4;
      sv[it] = *reinterpret_cast<const vec4 *>(Xb + (int64_t)i3c * n2 + cgc);
    }
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
      const int e = (int)threadIdx.x + it * NTHR;
      if (e < kpad * Q) {
        const int i3 = e / Q, q = e - i3 * Q;
        const bool ok = i3 < n && c0 + 4 * q < n2;
#pragma unroll
        for (int t = 0; t < 4; ++t) xt[(4 * q + t) * LDP + i3] = to_bf16_once(ok ? sv[it][t] : TI(0));
      }
    }
  } else {
    for (int e = threadIdx.x; e < kpad * kNB; e += NTHR) {
      const int i3 = e / kNB, c = e % kNB;
      const int64_t cg = c0 + c;
      xt[c * LDP + i3] = to_bf16_once((i3 < n && cg < n2) ? Xb[(int64_t)i3 * n2 + cg] : TI(0));
    }
  }
  __syncthreads();
  flt4 acc[MT][NT];
  auto lds_gemm = [&](const __bf16 *W) {
    gemm16<MT, NT, MPAD / 32>(kpad, [&](int j0, Frag16<MT, NT> &f) {
      const int j = j0 + 8 * lg;
#pragma unroll
      for (int a = 0; a < MT; ++a) f.a[a] = load8_bf(W + (size_t)(m0 + 16 * a + li) * ldw + j);
#pragma unroll
      for (int b = 0; b < NT; ++b) f.b[b] = load8_bf(xt + (16 * b + li) * LDP + j);
    }, acc);
  };
  lds_gemm(Wa);
  __syncthreads();  // every wave is done with the staged block
#pragma unroll
  for (int b = 0; b < NT; ++b) {
    const float l12 = lv2[b] + lv1[b];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k3 = m0 + 16 * a + 4 * lg + r;
        // rows k3 >= n are zero (zero-padded Wa); lam3 is padded with 1
        xt[(16 * b + li) * LDP + k3] = to_bf16_once(acc[a][b][r] / (lv3[a][r] + l12));
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
        if (k3 < n) Yb[(int64_t)k3 * n2 + cg] = store_as<TO>(acc[a][b][r]);
      }
  }
}

// Workgroup shape: waves and 16-row tiles per wave with 16 WAVES MT >= roundup(n, 32) and
// a multiple of 32, and 16 NT columns per workgroup: 16 for the 2D solve and 3D n <= 64
// (more workgroups), 32 for 3D n > 192, wider in between (below).
struct Shape16 {
  int waves, mt, nt;
};

// 3D n in 65..192: wider column blocks, 64 columns per workgroup (128 in the slab passes
// for n > 160), so that fewer workgroups re-read and re-round the same rows of the slab
// (each of the ceil(n / columns) workgroups of a slab reads all of it).  Measured on
// MI355X (BF16 apply, us, 16 or 32 columns -> these): n = 96 22.7 -> 18.6, 128 30.0 ->
// 26.1, 160 77 -> 60.3, 192 112 -> 90.0 (64 columns in the slab passes: 96.1; 128 at
// n = 128 and 160: 30.2 and 75.6).
enum ShapeRole16 { kRole16Slab = 1, kRole16Fibre = 2 };
Shape16 pick_shape16(int n, bool small_grid, int role) {
  const int nt = (small_grid || n <= 96) ? 1 : 2;
  const int k = (n + 31) / 32;
  if (k <= 2) return {4, 1, nt};
  if (!small_grid && k <= 5) return {k <= 4 ? 2 * k : 12, 1, 4};
  if (!small_grid && k == 6) return {12, 1, role == kRole16Slab ? 8 : 2};
  if (k <= 4) return {2 * k, 1, nt};
  if (k <= 6) return {12, 1, nt};
  return {8, 2, nt};
}

#define FDG_SHAPES16(X)                                                                                         \
  X(4, 1, 1) X(6, 1, 1) X(8, 1, 1) X(12, 1, 1) X(8, 2, 1) X(4, 1, 2) X(6, 1, 2) X(8, 1, 2) X(12, 1, 2) X(8, 2, 2) \
  X(6, 1, 4) X(8, 1, 4) X(12, 1, 4) X(12, 1, 8)

template <int W, int M, int NT, typename TI, typename TO>
void slab16(hipStream_t s, const TI *X, TO *Y, const __bf16 *W1, const __bf16 *W2, int ldw, int n, int64_t nslab,
            bool div, const float *lam1, const float *lam2) {
  constexpr int kNB = 16 * NT;
  const int ncb = (n + kNB - 1) / kNB;
  const int remap = (nslab % 8 == 0) ? 1 : 0;
  const dim3 grid((unsigned)(nslab * ncb)), blk(64 * W);
  // 8-element loads: two 4-wide ones for FP64 / FP32 (n % 4 == 0, 32-byte aligned X), one
  // 16-byte one for BF16 (n % 8 == 0, 16-byte aligned X)
  const bool vec = sizeof(TI) == 2 ? (n % 8 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0)
                                   : (n % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 31) == 0);
#define FDG_SLAB16(D, V)                                                                                        \
  hipLaunchKernelGGL((k_slab16<W, M, NT, TI, TO, D, V>), grid, blk, 0, s, X, Y, W1, W2, ldw, n, nslab, ncb, remap, \
                     lam1, lam2)
  if (div) {
    if (vec) FDG_SLAB16(true, true); else FDG_SLAB16(true, false);
  } else {
    if (vec) FDG_SLAB16(false, true); else FDG_SLAB16(false, false);
  }
#undef FDG_SLAB16
}

template <typename TI, typename TO>
void slab16_dispatch(hipStream_t s, const TI *X, TO *Y, const __bf16 *W1, const __bf16 *W2, int ldw, int n,
                     int64_t nslab, bool two_d, bool div, const float *lam1, const float *lam2) {
  const Shape16 sh = pick_shape16(n, two_d, kRole16Slab);
#define FDG_CASE(W, M, T)                                                        \
  if (sh.waves == W && sh.mt == M && sh.nt == T) {                              \
    slab16<W, M, T, TI, TO>(s, X, Y, W1, W2, ldw, n, nslab, div, lam1, lam2);   \
    return;                                                                     \
  }
  FDG_SHAPES16(FDG_CASE)
#undef FDG_CASE
}

template <typename TI, typename TO>
void fibre16_dispatch(hipStream_t s, const TI *X, TO *Y, const __bf16 *Wa, const __bf16 *Wb, int ldw, int n,
                      int64_t batch, const float *lam1, const float *lam2, const float *lam3) {
  const Shape16 sh = pick_shape16(n, false, kRole16Fibre);
  const int64_t n2 = (int64_t)n * n;
  const bool vec = n2 % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & (4 * sizeof(TI) - 1)) == 0;
#define FDG_CASE(W, M, T)                                                                                         \
  if (sh.waves == W && sh.mt == M && sh.nt == T) {                                                               \
    const int ncb = (int)((n2 + 16 * T - 1) / (16 * T));                                                         \
    if (vec)                                                                                                     \
      hipLaunchKernelGGL((k_fibre16<W, M, T, true, TI, TO>), dim3((unsigned)(batch * ncb)), dim3(64 * W), 0, s, X, Y, \
                         Wa, Wb,                                                                               \
                         ldw, n, ncb, lam1, lam2, lam3);                                                         \
    else                                                                                                         \
      hipLaunchKernelGGL((k_fibre16<W, M, T, false, TI, TO>), dim3((unsigned)(batch * ncb)), dim3(64 * W), 0, s, X, Y, \
                         Wa, Wb,                                                                               \
                         ldw, n, ncb, lam1, lam2, lam3);                                                         \
    return;                                                                                                      \
  }
  FDG_SHAPES16(FDG_CASE)
#undef FDG_CASE
}

}  // namespace

void launch_fd_apply_bf16(hipStream_t s, int d, int n, int64_t batch, const double *b, double *out, float *t1,
                          float *t2, const void *const *Wv, const void *const *Wu, const float *const *lam, int ldw) {
  const __bf16 *V0 = (const __bf16 *)Wv[0], *V1 = (const __bf16 *)Wv[1];
  const __bf16 *U0 = (const __bf16 *)Wu[0], *U1 = (const __bf16 *)Wu[1];
  __bf16 *h1 = reinterpret_cast<__bf16 *>(t1), *h2 = reinterpret_cast<__bf16 *>(t2);  // BF16 intermediates
  if (d == 3) {
    const int64_t nslab = batch * n;
    slab16_dispatch<double, __bf16>(s, b, h1, V0, V1, ldw, n, nslab, false, false, nullptr, nullptr);
    fibre16_dispatch<__bf16, __bf16>(s, h1, h2, (const __bf16 *)Wv[2], (const __bf16 *)Wu[2], ldw, n, batch, lam[0],
                                     lam[1], lam[2]);
    slab16_dispatch<__bf16, double>(s, h2, out, U0, U1, ldw, n, nslab, false, false, nullptr, nullptr);
  } else {
    slab16_dispatch<double, __bf16>(s, b, h1, V0, V1, ldw, n, batch, true, true, lam[0], lam[1]);
    slab16_dispatch<__bf16, double>(s, h1, out, U0, U1, ldw, n, batch, true, false, nullptr, nullptr);
  }
}

}  // namespace fdg
