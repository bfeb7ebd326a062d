// Fused FP64 fast-diagonalization solve (eq. 4.9 in 3D, eq. 4.7 in 2D) on MFMA.
//
// The tensor X[b][i3][i2][i1] (i1 fastest) is processed in three passes:
//   pass A ("slab"):  per i3-slab, Y = W2 . X_slab . W1^T  -- modes 1 and 2 with V_1^T, V_2^T
//   pass B ("fibre"): per block of (i2, i1) columns, T = W3a . X_cols, T /= Lambda,
//                     S = W3b . T                        -- mode 3 with V_3^T, divide, U_3
//   pass C ("slab"):  modes 1 and 2 with U_1, U_2
// In 2D pass A also applies the divide by lambda_2[k2] + lambda_1[k1] and pass B is absent.
// Each pass reads and writes the tensor once; the intermediate of the two chained
// contractions lives in LDS.
//
// v_mfma_f64_16x16x4_f64 lane layout (li = lane % 16, lg = lane / 16):
//   A[m = li][k = lg], B[k = lg][n = li], D[m = lg + 4 r][n = li] in register r.
// The contraction index is permuted so that each lane reads four consecutive elements:
// over the four MFMAs t = 0..3 of a 16-wide k-block starting at j0, lane group lg
// supplies contraction index j0 + 4 lg + t to both operands.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch_addr.h"
#include "fd_apply.h"

namespace fdg {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

#ifndef FDG_FD_LDS_PAD
#define FDG_FD_LDS_PAD 2
#endif
// NT: 16-column MFMA tiles per wave, 16 NT columns per workgroup (a template parameter of
// every kernel: 2 at large n, 1 where fewer columns per workgroup give more workgroups)
constexpr int kPad = FDG_FD_LDS_PAD;  // LDS row padding (doubles, even: rows stay 16-byte aligned)

__device__ inline dbl4 mfma(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Four consecutive doubles p[0..3], zero where the index j + t >= jmax or !ok.
template <bool VEC>
__device__ inline void load4(gptr<const double> p, int j, int jmax, bool ok, double (&v)[4]) {
  if (VEC && ok && j + 3 < jmax) {
    const dbl4 x = *(gptr<const dbl4>)p;
    v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = (ok && j + t < jmax) ? p[t] : 0.0;
  }
}

__device__ inline void load4_pad(const double *p, double (&v)[4]) {  // always in bounds, 32-B aligned
  const dbl4 x = *reinterpret_cast<const dbl4 *>(p);
  v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
}

// Fragments of one 16-wide k-block: MT row tiles of A, NT column tiles of B (4 contraction
// indices each per lane).
template <int MT, int NT>
struct Frag {
  double a[MT][4];
  double b[NT][4];
};

template <int MT, int NT>
__device__ inline void mma_block(const Frag<MT, NT> &f, dbl4 (&acc)[MT][NT]) {
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int b = 0; b < NT; ++b) acc[a][b] = mfma(f.a[a][t], f.b[b][t], acc[a][b]);
}

// acc = sum over k-blocks j0 = 0, 16, .., kpad-16 of load(j0), for kpad <= 16 KB; the
// operands of block kb + PD are loaded before block kb's MFMAs are issued (PD + 1 register
// buffers).  The loop is unrolled over the KB blocks the workgroup shape allows and every
// load is issued unconditionally (load must stay in bounds for every j0 < 16 KB), so the
// compiler waits for exactly the loads a block needs; a rolled loop with conditional
// loads made it wait for all outstanding loads before every block.
#ifndef FDG_FD_PD
#define FDG_FD_PD 1
#endif
template <int MT, int NT, int KB, typename Load>
__device__ inline void gemm_pipelined(int kpad, Load load, dbl4 (&acc)[MT][NT]) {
  constexpr int PD = FDG_FD_PD < KB ? FDG_FD_PD : KB;
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
  Frag<MT, NT> f[PD + 1];
#pragma unroll
  for (int p = 0; p < PD; ++p) load(16 * p, f[p]);
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    if (kb + PD < KB) load(16 * (kb + PD), f[(kb + PD) % (PD + 1)]);
    if (16 * kb < kpad) mma_block<MT, NT>(f[kb % (PD + 1)], acc);
  }
}

// acc = sum over the KB k-blocks of (A fragments already in registers) x (B from load_b);
// B fragments are double-buffered.  k-blocks at or beyond kpad are skipped.
template <int MT, int NT, int KB, typename LoadB>
__device__ inline void gemm_preloaded_a(int kpad, const double (&xa)[MT][KB][4], LoadB load_b,
                                        dbl4 (&acc)[MT][NT]) {
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    if (kb * 16 >= kpad) break;
    double bv[NT][4];
    load_b(kb * 16, bv);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = mfma(xa[a][kb][t], bv[b][t], acc[a][b]);
  }
}

// The same, loading after the MFMAs of each k-block kb the A fragment kb of the next
// contraction (load_next(kb)): its loads overlap this contraction, and its registers take
// the place of the fragment just consumed.
template <int MT, int NT, int KB, typename LoadB, typename LoadNext>
__device__ inline void gemm_preloaded_a_next(int kpad, const double (&xa)[MT][KB][4], LoadB load_b,
                                             dbl4 (&acc)[MT][NT], LoadNext load_next) {
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    if (kb * 16 >= kpad) break;
    double bv[NT][4];
    load_b(kb * 16, bv);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int a = 0; a < MT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = mfma(xa[a][kb][t], bv[b][t], acc[a][b]);
    load_next(kb);
  }
}

// ------------------------------------------------------------------------------------
// Pass A / C.  Workgroup = (slab s, column block cb) with WAVES waves; wave w owns rows
// [w*MT*16, (w+1)*MT*16) of both contractions and all kNB columns.
//   GEMM1: Y1[i2][c] = sum_i1 X[s][i2][i1] W1[c][i1]   (A = X rows from HBM, B = W1 tile in LDS)
//   GEMM2: Y2[k2][c] = sum_i2 W2[k2][i2] Y1[i2][c]     (A = W2 rows from L2, B = Y1 in LDS)
//   2D divide: Y2[k2][c] /= lam2[k2] + lam1[c].
// The LDS buffer holds the W1 column tile during GEMM1 and then Y1 (transposed).
// ------------------------------------------------------------------------------------
template <int WAVES, int MT, int NT, bool VEC, bool DIV, bool PRE>
__global__ __launch_bounds__(64 * WAVES, PRE ? 2 : 1) void k_slab(CBatch X, MBatch Y,
                                                     const double *__restrict__ W1, const double *__restrict__ W2,
                                                     int ldw, int n, int64_t nslab, int spe, int ncb, int xcd_remap,
                                                     const double *__restrict__ lam1,
                                                     const double *__restrict__ lam2) {
  constexpr int MPAD = WAVES * MT * 16;
  constexpr int LDP = MPAD + kPad;
  constexpr int NTHR = 64 * WAVES;
  constexpr int kNB = 16 * NT;
  __shared__ double buf[kNB * LDP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  int64_t s;
  int cb;
  {
    const int64_t bid = blockIdx.x;
    if (xcd_remap) {  // the ncb workgroups of one slab share an XCD (and its L2)
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
  const int64_t ent = s / spe, loc = s - ent * spe;  // batch entry and slab inside it
  FDG_GLOBAL const double *__restrict__ Xs = X.gat(ent) + loc * n2;
  FDG_GLOBAL double *__restrict__ Ys = Y.gat(ent) + loc * n2;
  const int c0 = cb * kNB;
  const int m0 = wave * MT * 16;
  const int kpad = (n + 15) & ~15;

  // with PRE, the wave's whole strip of X (its MT*16 rows, all columns) is loaded into
  // registers first, together with the W1 staging below, and GEMM1 loads the W2 rows of
  // GEMM2 as it consumes the strip: the pass waits for memory about twice instead of
  // once per k-block
  constexpr int KB = PRE ? MPAD / 16 : 1;
  double xa[MT][KB][4], w2a[MT][KB][4];
  if (PRE) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int j = kb * 16 + 4 * lg;
#pragma unroll
      for (int a = 0; a < MT; ++a) {
        const int row = m0 + 16 * a + li;
        load4<VEC>(Xs + (int64_t)row * n + j, j, n, row < n, xa[a][kb]);
      }
    }
  }
  // stage W1[c0 .. c0+kNB)[0 .. kpad) (zero-padded rows and columns beyond n); every
  // thread's loads are issued before the first LDS store (addresses clamped to the tile)
  {
    constexpr int SIT = (kNB * (MPAD / 2) + NTHR - 1) / NTHR;
    const int half = kpad / 2, stot = kNB * half;
    double2 sv[SIT];
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
      const int e0 = (int)threadIdx.x + it * NTHR, e = e0 < stot ? e0 : stot - 1;
      const int c = e / half, j = 2 * (e % half);
      sv[it] = *reinterpret_cast<const double2 *>(W1 + (size_t)(c0 + c) * ldw + j);
    }
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
      const int e = (int)threadIdx.x + it * NTHR;
      if (e < stot) {
        const int c = e / half, j = 2 * (e % half);
        buf[c * LDP + j] = sv[it].x;
        buf[c * LDP + j + 1] = sv[it].y;
      }
    }
  }
  __syncthreads();

  // ---- GEMM1 ----
  dbl4 acc[MT][NT];
  if (PRE) {
    gemm_preloaded_a_next<MT, NT, KB>(kpad, xa, [&](int j0, double (&bv)[NT][4]) {
      const int j = j0 + 4 * lg;
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        const double *p = buf + (16 * b + li) * LDP + j;
        bv[b][0] = p[0]; bv[b][1] = p[1]; bv[b][2] = p[2]; bv[b][3] = p[3];
      }
    }, acc, [&](int kb) {
#pragma unroll
      for (int a = 0; a < MT; ++a)
        load4_pad(W2 + (size_t)(m0 + 16 * a + li) * ldw + kb * 16 + 4 * lg, w2a[a][kb]);
    });
  } else {
    gemm_pipelined<MT, NT, MPAD / 16>(kpad, [&](int j0, Frag<MT, NT> &f) {
      const int j = j0 + 4 * lg;
#pragma unroll
      for (int a = 0; a < MT; ++a) {
        const int row = m0 + 16 * a + li;
        if (VEC) {
          // 4-wide at clamped addresses, no branch: an element beyond the slab's n columns
          // meets a zero of the zero-padded W1 tile, and a padding row of Y1 a zero column
          // of W2 in GEMM2, so clamped values never reach the result
          const int rowc = row < n ? row : n - 1, jc = j < n ? j : n - 4;
          const dbl4 x = *(gptr<const dbl4>)(Xs + (int64_t)rowc * n + jc);
          f.a[a][0] = x[0]; f.a[a][1] = x[1]; f.a[a][2] = x[2]; f.a[a][3] = x[3];
        } else {
          load4<VEC>(Xs + (int64_t)row * n + j, j, n, row < n, f.a[a]);
        }
      }
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        const double *p = buf + (16 * b + li) * LDP + j;
        f.b[b][0] = p[0]; f.b[b][1] = p[1]; f.b[b][2] = p[2]; f.b[b][3] = p[3];
      }
    }, acc);
  }
  __syncthreads();  // all waves are done with the W1 tile
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) buf[(16 * b + li) * LDP + m0 + 16 * a + lg + 4 * r] = acc[a][b][r];
  __syncthreads();

  // ---- GEMM2 ----
  if (PRE) {
    gemm_preloaded_a<MT, NT, KB>(kpad, w2a, [&](int j0, double (&bv)[NT][4]) {
      const int j = j0 + 4 * lg;
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        const double *p = buf + (16 * b + li) * LDP + j;
        bv[b][0] = p[0]; bv[b][1] = p[1]; bv[b][2] = p[2]; bv[b][3] = p[3];
      }
    }, acc);
  } else {
    gemm_pipelined<MT, NT, MPAD / 16>(kpad, [&](int j0, Frag<MT, NT> &f) {
      const int j = j0 + 4 * lg;
#pragma unroll
      for (int a = 0; a < MT; ++a) load4_pad(W2 + (size_t)(m0 + 16 * a + li) * ldw + j, f.a[a]);
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        const double *p = buf + (16 * b + li) * LDP + j;
        f.b[b][0] = p[0]; f.b[b][1] = p[1]; f.b[b][2] = p[2]; f.b[b][3] = p[3];
      }
    }, acc);
  }
#pragma unroll
  for (int b = 0; b < NT; ++b) {
    const int c = c0 + 16 * b + li;
    if (c >= n) continue;
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k2 = m0 + 16 * a + lg + 4 * r;
        if (k2 < n) {
          double v = acc[a][b][r];
          if (DIV) v = v / (lam2[k2] + lam1[c]);
          Ys[(int64_t)k2 * n + c] = v;
        }
      }
  }
}

// ------------------------------------------------------------------------------------
// Pass B.  Workgroup = (batch entry b, block of kNB columns c of the n x n^2 matrix
// X[b][i3][c]).  The column block is staged in LDS transposed (xt[c][i3]); then
//   GEMM1: T[k3][c] = sum_i3 Wa[k3][i3] X[i3][c];   T /= lam3[k3] + lam2[i2] + lam1[i1]
//   GEMM2: S[k3][c] = sum_k Wb[k3][k] T[k][c]        (T back in LDS, transposed)
// ------------------------------------------------------------------------------------
template <int WAVES, int MT, int NT, bool VEC, bool PRE>
__global__ __launch_bounds__(64 * WAVES) void k_fibre(CBatch X, MBatch Y,
                                                      const double *__restrict__ Wa, const double *__restrict__ Wb,
                                                      int ldw, int n, int ncb, const double *__restrict__ lam1,
                                                      const double *__restrict__ lam2,
                                                      const double *__restrict__ lam3) {
  constexpr int MPAD = WAVES * MT * 16;
  constexpr int LDP = MPAD + kPad;
  constexpr int NTHR = 64 * WAVES;
  constexpr int kNB = 16 * NT;
  __shared__ double xt[kNB * LDP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t bidx = blockIdx.x / ncb;
  const int cb = (int)(blockIdx.x % ncb);
  const int64_t n2 = (int64_t)n * n;
  FDG_GLOBAL const double *__restrict__ Xb = X.gat(bidx);
  FDG_GLOBAL double *__restrict__ Yb = Y.gat(bidx);
  const int64_t c0 = (int64_t)cb * kNB;
  const int m0 = wave * MT * 16;
  const int kpad = (n + 15) & ~15;
  // the eigenvalues of the divide, loaded with the first loads of the pass (a load used
  // right after it is issued would be waited for on its own)
  double lv3[MT][4], lv2[NT], lv1[NT];
#pragma unroll
  for (int a = 0; a < MT; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) lv3[a][r] = lam3[m0 + 16 * a + lg + 4 * r];
#pragma unroll
  for (int b = 0; b < NT; ++b) {
    const int64_t cg = c0 + 16 * b + li;
    const bool cok = cg < n2;
    lv2[b] = lam2[cok ? (int)(cg / n) : 0];
    lv1[b] = lam1[cok ? (int)(cg % n) : 0];
  }
  // with PRE, the wave's rows of Wa and Wb (the A operands of both contractions) are
  // loaded into registers together with the staging loads below
  constexpr int KB = PRE ? MPAD / 16 : 1;
  double wa[MT][KB][4], wb[MT][KB][4];
  if (PRE) {  // Wa now; Wb while GEMM1 consumes Wa
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int a = 0; a < MT; ++a)
        load4_pad(Wa + (size_t)(m0 + 16 * a + li) * ldw + kb * 16 + 4 * lg, wa[a][kb]);
  }
  // stage X[i3][c0 .. c0+kNB) -> xt[c][i3], zero beyond n or n^2 (VEC: n^2 % 4 == 0 and
  // 32-byte aligned entries, four columns per load; every thread's loads are issued at
  // clamped addresses before the first LDS store)
  if (VEC) {
    constexpr int Q = kNB / 4;
    constexpr int SIT = (MPAD * Q + NTHR - 1) / NTHR;
    dbl4 sv[SIT];
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
      const int e = (int)threadIdx.x + it * NTHR;
      const int i3 = e / Q, q = e - i3 * Q;
      const int64_t cg = c0 + 4 * q;
      const int i3c = i3 < n ? i3 : n - 1;
      const int64_t cgc = cg < n2 ? cg : n2 - 4;
      sv[it] = *(gptr<const dbl4>)(Xb + (int64_t)i3c * n2 + cgc);
    }
#pragma unroll
    for (int it = 0; it < SIT; ++it) {
      const int e = (int)threadIdx.x + it * NTHR;
      if (e < kpad * Q) {
        const int i3 = e / Q, q = e - i3 * Q;
        const bool ok = i3 < n && c0 + 4 * q < n2;
#pragma unroll
        for (int t = 0; t < 4; ++t) xt[(4 * q + t) * LDP + i3] = ok ? sv[it][t] : 0.0;
      }
    }
  } else {
    for (int e = threadIdx.x; e < kpad * kNB; e += NTHR) {
      const int i3 = e / kNB, c = e % kNB;
      const int64_t cg = c0 + c;
      xt[c * LDP + i3] = (i3 < n && cg < n2) ? Xb[(int64_t)i3 * n2 + cg] : 0.0;
    }
  }
  __syncthreads();
  dbl4 acc[MT][NT];
  auto lds_b = [&](int j0, double (&bv)[NT][4]) {
    const int j = j0 + 4 * lg;
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      const double *p = xt + (16 * b + li) * LDP + j;
      bv[b][0] = p[0]; bv[b][1] = p[1]; bv[b][2] = p[2]; bv[b][3] = p[3];
    }
  };
  auto lds_gemm = [&](const double *W) {
    gemm_pipelined<MT, NT, MPAD / 16>(kpad, [&](int j0, Frag<MT, NT> &f) {
      const int j = j0 + 4 * lg;
#pragma unroll
      for (int a = 0; a < MT; ++a) load4_pad(W + (size_t)(m0 + 16 * a + li) * ldw + j, f.a[a]);
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        const double *p = xt + (16 * b + li) * LDP + j;
        f.b[b][0] = p[0]; f.b[b][1] = p[1]; f.b[b][2] = p[2]; f.b[b][3] = p[3];
      }
    }, acc);
  };
  if (PRE)
    gemm_preloaded_a_next<MT, NT, KB>(kpad, wa, lds_b, acc, [&](int kb) {
#pragma unroll
      for (int a = 0; a < MT; ++a)
        load4_pad(Wb + (size_t)(m0 + 16 * a + li) * ldw + kb * 16 + 4 * lg, wb[a][kb]);
    });
  else
    lds_gemm(Wa);
  __syncthreads();  // every wave has finished reading xt
#pragma unroll
  for (int b = 0; b < NT; ++b) {
    const double l12 = lv2[b] + lv1[b];
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k3 = m0 + 16 * a + lg + 4 * r;
        // rows k3 >= n are zero (zero-padded Wa); lam3 is padded with 1
        xt[(16 * b + li) * LDP + k3] = acc[a][b][r] / (lv3[a][r] + l12);
      }
  }
  __syncthreads();
  if (PRE)
    gemm_preloaded_a<MT, NT, KB>(kpad, wb, lds_b, acc);
  else
    lds_gemm(Wb);
#pragma unroll
  for (int b = 0; b < NT; ++b) {
    const int64_t cg = c0 + 16 * b + li;
    if (cg >= n2) continue;
#pragma unroll
    for (int a = 0; a < MT; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k3 = m0 + 16 * a + lg + 4 * r;
        if (k3 < n) Yb[(int64_t)k3 * n2 + cg] = acc[a][b][r];
      }
  }
}

// Launch on stream s, with dispatch-recorded events when ev0 is given.
template <typename K, typename... Args>
void launch_timed(K kernel, dim3 grid, dim3 blk, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, Args... args) {
  if (ev0)
    hipExtLaunchKernelGGL(kernel, grid, blk, 0, s, ev0, ev1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, blk, 0, s, args...);
}

// The preloading forms (the A operands of a pass in registers, about two waits for memory
// per pass instead of one per k-block) for the 16-column workgroups of n <= 64.  Measured
// on MI355X (FP64 apply, us, pipelined -> preloading): 3D n = 32: 12.3 -> 11.4, 48: 14.6
// -> 13.0, 64: 18.0 -> 16.1; n = 80: 31.8 -> 32.8 and 96: 55.5 -> 59.5 (there every
// wave of a pass reaches its MFMAs at the same time, and the waits the preloading removes
// were already overlapped by other workgroups).
#ifndef FDG_FD_PRE_MAXN
#define FDG_FD_PRE_MAXN 64
#endif
#ifndef FDG_FD_PRE_FIBRE_MAXN
#define FDG_FD_PRE_FIBRE_MAXN 64
#endif
inline bool pre_ok(int n) { return n <= FDG_FD_PRE_MAXN; }
inline bool pre_fibre_ok(int n) { return n <= FDG_FD_PRE_FIBRE_MAXN; }

template <int WAVES, int MT, int NT>
void slab_launch(hipStream_t s, CBatch X, MBatch Y, const double *W1, const double *W2, int ldw, int n,
                 int64_t nslab, int spe, bool div, const double *lam1, const double *lam2, bool aligned32,
                 hipEvent_t ev0, hipEvent_t ev1) {
  constexpr int kNB = 16 * NT;
  const int ncb = (n + kNB - 1) / kNB;
  const int64_t nwg = nslab * ncb;
  const int remap = (nslab % 8 == 0) ? 1 : 0;
  const bool vec = (n % 4 == 0) && aligned32;
  const dim3 grid((unsigned)nwg), blk(64 * WAVES);
  if (NT == 1 && pre_ok(n)) {
    constexpr bool P = NT == 1 && WAVES * MT * 16 <= 96;
    if (div) {
      if (vec)
        launch_timed(k_slab<WAVES, MT, NT, true, true, P>, grid, blk, s, ev0, ev1, X, Y, W1, W2, ldw, n, nslab, spe,
                     ncb, remap, lam1, lam2);
      else
        launch_timed(k_slab<WAVES, MT, NT, false, true, P>, grid, blk, s, ev0, ev1, X, Y, W1, W2, ldw, n, nslab, spe,
                     ncb, remap, lam1, lam2);
    } else {
      if (vec)
        launch_timed(k_slab<WAVES, MT, NT, true, false, P>, grid, blk, s, ev0, ev1, X, Y, W1, W2, ldw, n, nslab, spe,
                     ncb, remap, lam1, lam2);
      else
        launch_timed(k_slab<WAVES, MT, NT, false, false, P>, grid, blk, s, ev0, ev1, X, Y, W1, W2, ldw, n, nslab, spe,
                     ncb, remap, lam1, lam2);
    }
    return;
  }
  if (div) {
    if (vec)
      launch_timed(k_slab<WAVES, MT, NT, true, true, false>, grid, blk, s, ev0, ev1, X, Y, W1, W2, ldw, n, nslab, spe,
                   ncb, remap, lam1, lam2);
    else
      launch_timed(k_slab<WAVES, MT, NT, false, true, false>, grid, blk, s, ev0, ev1, X, Y, W1, W2, ldw, n, nslab, spe,
                   ncb, remap, lam1, lam2);
  } else {
    if (vec)
      launch_timed(k_slab<WAVES, MT, NT, true, false, false>, grid, blk, s, ev0, ev1, X, Y, W1, W2, ldw, n, nslab, spe,
                   ncb, remap, lam1, lam2);
    else
      launch_timed(k_slab<WAVES, MT, NT, false, false, false>, grid, blk, s, ev0, ev1, X, Y, W1, W2, ldw, n, nslab,
                   spe, ncb, remap, lam1, lam2);
  }
}

template <int WAVES, int MT, int NT>
void fibre_launch(hipStream_t s, CBatch X, MBatch Y, const double *Wa, const double *Wb, int ldw, int n,
                  int64_t batch, const double *lam1, const double *lam2, const double *lam3, hipEvent_t ev0,
                  hipEvent_t ev1) {
  constexpr int kNB = 16 * NT;
  const int64_t n2 = (int64_t)n * n;
  const int ncb = (int)((n2 + kNB - 1) / kNB);
  const dim3 grid((unsigned)(batch * ncb)), blk(64 * WAVES);
  // 4-wide staging loads: every entry and every i3 row 32-byte aligned
  const bool vec = n2 % 4 == 0 && !X.ptrs && (reinterpret_cast<uintptr_t>(X.base) & 31) == 0 &&
                   (batch == 1 || X.stride % 4 == 0);
  if (NT == 1 && pre_fibre_ok(n)) {
    constexpr bool P = NT == 1 && WAVES * MT * 16 <= 96;
    if (vec)
      launch_timed(k_fibre<WAVES, MT, NT, true, P>, grid, blk, s, ev0, ev1, X, Y, Wa, Wb, ldw, n, ncb, lam1, lam2,
                   lam3);
    else
      launch_timed(k_fibre<WAVES, MT, NT, false, P>, grid, blk, s, ev0, ev1, X, Y, Wa, Wb, ldw, n, ncb, lam1, lam2,
                   lam3);
    return;
  }
  if (vec)
    launch_timed(k_fibre<WAVES, MT, NT, true, false>, grid, blk, s, ev0, ev1, X, Y, Wa, Wb, ldw, n, ncb, lam1, lam2,
                 lam3);
  else
    launch_timed(k_fibre<WAVES, MT, NT, false, false>, grid, blk, s, ev0, ev1, X, Y, Wa, Wb, ldw, n, ncb, lam1, lam2,
                 lam3);
}

}  // namespace

bool fd_fused_supported(int n) { return n >= 1 && n <= 256; }

// Workgroup shape (waves, 16-row tiles per wave, 16-column tiles per wave) for a given n:
// MPAD = 16 * waves * MT covers roundup(n, 16) with little padding (MPAD <= ldw always
// holds).  NT = 1 (16 columns per workgroup, twice the workgroups) where the passes would
// otherwise leave compute units idle: 3D n <= 96 and the 2D solve (one slab per entry).
// Measured (FP64 apply, us, NT = 2 -> 1): 3D n = 32: 16.8 -> 13.0, 64: 25.1 -> 19.3,
// 96: 61 -> 57; 2D n = 256: 90 -> 70; 3D n = 128: 85 -> 113 (kept at NT = 2).
struct Shape {
  int waves, mt, nt;
};

// With 32 columns per workgroup (3D, n > 96), two or three 16-row tiles per wave: from
// n = 97 on 4 waves of 2 tiles in both passes, from n = 129 on 4 waves of 3 tiles in the
// slab passes (the fibre pass keeps 12 waves of one tile).  Measured on MI355X (3D FP64
// apply, us, one tile per wave -> these): n = 112 64.6 -> 62.3, 128 72.5 -> 70.2, 144 172
// -> 164, 160 233 -> 221, 176 286 -> 264, 192 328 -> 308; the fibre pass with 4 x 3 at
// n = 192: 340.
enum ShapeRole { kRoleSlab = 1, kRoleFibre = 2 };
static Shape pick_shape(int n, bool small_grid, int role) {
#if defined(FDG_FD_FORCE_W) && defined(FDG_FD_FORCE_MT) && defined(FDG_FD_FORCE_NT)
  if (16 * FDG_FD_FORCE_W * FDG_FD_FORCE_MT >= ((n + 15) & ~15) &&
      16 * FDG_FD_FORCE_W * FDG_FD_FORCE_MT <= ((n + 63) / 64) * 64)
    return {FDG_FD_FORCE_W, FDG_FD_FORCE_MT, FDG_FD_FORCE_NT};
#endif
  const int nt = (small_grid || n <= 96) ? 1 : 2;
  const int k = (n + 15) / 16;  // 16-row tiles needed
  if (k <= 4) return {4, 1, nt};
  if (nt == 2 && k <= 8) return {4, 2, 2};
  if (k <= 8) return {k, 1, nt};  // 5..8 waves, one tile each
  if (nt == 2 && k <= 12 && role == kRoleSlab) return {4, 3, 2};
  if (k <= 12) return {12, 1, nt};
  return {8, 2, nt};
}

#define FDG_SHAPES(X)                                                                             \
  X(4, 1, 1) X(5, 1, 1) X(6, 1, 1) X(7, 1, 1) X(8, 1, 1) X(8, 2, 1) X(12, 1, 1) \
  X(4, 1, 2) X(5, 1, 2) X(6, 1, 2) X(7, 1, 2) X(8, 1, 2) X(4, 2, 2) X(6, 2, 2) X(8, 2, 2) X(4, 3, 2) X(12, 1, 2)

void launch_slab_f64(hipStream_t s, CBatch X, MBatch Y, const double *W1, const double *W2, int ldw, int n,
                     int64_t nentries, int spe, bool divide, const double *lam1, const double *lam2, bool aligned32,
                     hipEvent_t ev0, hipEvent_t ev1) {
  const Shape sh = pick_shape(n, spe == 1, kRoleSlab);
  const int64_t nslab = nentries * spe;
#define FDG_CASE(W, M, T)                                                                  \
  if (sh.waves == W && sh.mt == M && sh.nt == T) {                                       \
    slab_launch<W, M, T>(s, X, Y, W1, W2, ldw, n, nslab, spe, divide, lam1, lam2, aligned32, ev0, ev1); \
    return;                                                                              \
  }
  FDG_SHAPES(FDG_CASE)
#undef FDG_CASE
}

void launch_fibre_f64(hipStream_t s, CBatch X, MBatch Y, const double *Wa, const double *Wb, int ldw, int n,
                      int64_t batch, const double *lam1, const double *lam2, const double *lam3, hipEvent_t ev0,
                      hipEvent_t ev1) {
  const Shape sh = pick_shape(n, false, kRoleFibre);
#define FDG_CASE(W, M, T)                                                               \
  if (sh.waves == W && sh.mt == M && sh.nt == T) {                                    \
    fibre_launch<W, M, T>(s, X, Y, Wa, Wb, ldw, n, batch, lam1, lam2, lam3, ev0, ev1); \
    return;                                                                           \
  }
  FDG_SHAPES(FDG_CASE)
#undef FDG_CASE
}

}  // namespace fdg
