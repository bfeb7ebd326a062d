// Host FP64 factorisation of one univariate pencil for the nonsymmetric FD method.
//
// eq. 4.6: M^{-1} K U = U D with D real (Remark 1), then V = (M U)^{-T} (the definition
// right after eq. 4.6), so that M = V^{-T} U^{-1} and K = V^{-T} D U^{-1}.
//
// Method (no LAPACK in the image): A = M^{-1} K by LU with partial pivoting, Householder
// reduction to upper Hessenberg form, Francis implicit double-shift QR iterations to
// a real Schur form T = Z^T A Z (accumulating Z), 2x2 blocks with real eigenvalues split
// by a rotation; eigenvectors of the triangular T by back-substitution; U = Z Y.
// A pencil with complex eigenvalues (Sec. 4, the remark after eq. 4.7) keeps each pair's
// 2x2 block in T; its eigenvector z = u + i v (complex back-substitution through the
// quasi-triangular T) gives the two real columns u, v of U, and D gets the real 2x2
// block [[a, b], [-b, a]] for the pair a +- ib (fdg_factor_pencil_blocks).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.h"

namespace fdg {
namespace {

struct Mat {
  int n;
  std::vector<double> a;
  explicit Mat(int n_) : n(n_), a((size_t)n_ * n_, 0.0) {}
  double &operator()(int i, int j) { return a[(size_t)i * n + j]; }
  double operator()(int i, int j) const { return a[(size_t)i * n + j]; }
};

// LU with partial pivoting in place; piv[i] = row swapped with i.  Returns false if singular.
bool lu_factor(Mat &A, std::vector<int> &piv) {
  const int n = A.n;
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(A(k, k));
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A(i, k)) > best) { best = std::fabs(A(i, k)); p = i; }
    piv[k] = p;
    if (best == 0.0 || !std::isfinite(best)) return false;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(A(k, j), A(p, j));
    const double inv = 1.0 / A(k, k);
    for (int i = k + 1; i < n; ++i) {
      const double l = A(i, k) * inv;
      A(i, k) = l;
      if (l != 0.0)
        for (int j = k + 1; j < n; ++j) A(i, j) -= l * A(k, j);
    }
  }
  return true;
}

// Solves LU X = B in place for B (n x nrhs, row-major).
void lu_solve(const Mat &LU, const std::vector<int> &piv, std::vector<double> &B, int nrhs) {
  const int n = LU.n;
  for (int k = 0; k < n; ++k)
    if (piv[k] != k)
      for (int c = 0; c < nrhs; ++c) std::swap(B[(size_t)k * nrhs + c], B[(size_t)piv[k] * nrhs + c]);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < i; ++k) {
      const double l = LU(i, k);
      if (l != 0.0)
        for (int c = 0; c < nrhs; ++c) B[(size_t)i * nrhs + c] -= l * B[(size_t)k * nrhs + c];
    }
  for (int i = n - 1; i >= 0; --i) {
    for (int k = i + 1; k < n; ++k) {
      const double u = LU(i, k);
      if (u != 0.0)
        for (int c = 0; c < nrhs; ++c) B[(size_t)i * nrhs + c] -= u * B[(size_t)k * nrhs + c];
    }
    const double inv = 1.0 / LU(i, i);
    for (int c = 0; c < nrhs; ++c) B[(size_t)i * nrhs + c] *= inv;
  }
}

// Householder reduction to upper Hessenberg form, H = Z^T A Z, Z accumulated (stored
// transposed in Zt, so its updates run along contiguous rows).
void hessenberg(Mat &H, Mat &Zt) {
  const int n = H.n;
  std::vector<double> v(n), w(n);
  for (int k = 0; k + 2 < n; ++k) {
    double alpha = 0.0;
    for (int i = k + 1; i < n; ++i) alpha += H(i, k) * H(i, k);
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    if (H(k + 1, k) > 0) alpha = -alpha;
    // v = x - alpha e1 on rows k+1..n-1
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    v[k + 1] = H(k + 1, k) - alpha;
    for (int i = k + 2; i < n; ++i) v[i] = H(i, k);
    double vv = 0.0;
    for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    // left: H = (I - beta v v^T) H on rows k+1.., columns k.. (row-major sweeps:
    // w = H^T v accumulated row by row, then the rank-one update row by row)
    std::fill(w.begin(), w.end(), 0.0);
    for (int i = k + 1; i < n; ++i) {
      const double vi = v[i];
      const double *h = &H(i, 0);
      for (int j = k; j < n; ++j) w[j] += vi * h[j];
    }
    for (int i = k + 1; i < n; ++i) {
      const double bv = beta * v[i];
      double *h = &H(i, 0);
      for (int j = k; j < n; ++j) h[j] -= bv * w[j];
    }
    // right: H = H (I - beta v v^T) on all rows, columns k+1..
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += H(i, j) * v[j];
      s *= beta;
      for (int j = k + 1; j < n; ++j) H(i, j) -= s * v[j];
    }
    // Z = Z (I - beta v v^T), Z stored transposed (Zt(j, i) = Z(i, j))
    std::fill(w.begin(), w.end(), 0.0);
    for (int j = k + 1; j < n; ++j) {
      const double vj = v[j];
      const double *z = &Zt(j, 0);
      for (int i = 0; i < n; ++i) w[i] += vj * z[i];
    }
    for (int j = k + 1; j < n; ++j) {
      const double bv = beta * v[j];
      double *z = &Zt(j, 0);
      for (int i = 0; i < n; ++i) z[i] -= bv * w[i];
    }
    H(k + 1, k) = alpha;
    for (int i = k + 2; i < n; ++i) H(i, k) = 0.0;
  }
}

// Applies the reflector I - beta v v^T (v of length m = 2 or 3 at rows/cols
// r0..r0+m-1) to H from both sides within the given ranges, and to Z from the right
// (Z stored transposed in Zt).
void apply_reflector(Mat &H, Mat &Zt, int r0, int m, const double *v, double beta, int col_lo,
                     int row_hi) {
  const int n = H.n;
  for (int j = col_lo; j < n; ++j) {
    double s = 0.0;
    for (int t = 0; t < m; ++t) s += v[t] * H(r0 + t, j);
    s *= beta;
    for (int t = 0; t < m; ++t) H(r0 + t, j) -= s * v[t];
  }
  for (int i = 0; i <= row_hi; ++i) {
    double s = 0.0;
    for (int t = 0; t < m; ++t) s += H(i, r0 + t) * v[t];
    s *= beta;
    for (int t = 0; t < m; ++t) H(i, r0 + t) -= s * v[t];
  }
  // Z = Z (I - beta v v^T) with Z stored transposed: rows r0..r0+m-1 of Zt
  double *z0 = &Zt(r0, 0);
  double *z1 = m > 1 ? &Zt(r0 + 1, 0) : nullptr;
  double *z2 = m > 2 ? &Zt(r0 + 2, 0) : nullptr;
  if (m == 3) {
    for (int i = 0; i < n; ++i) {
      const double s = beta * (v[0] * z0[i] + v[1] * z1[i] + v[2] * z2[i]);
      z0[i] -= s * v[0];
      z1[i] -= s * v[1];
      z2[i] -= s * v[2];
    }
  } else {
    for (int i = 0; i < n; ++i) {
      const double s = beta * (v[0] * z0[i] + v[1] * z1[i]);
      z0[i] -= s * v[0];
      z1[i] -= s * v[1];
    }
  }
}

// Reflector mapping x (length m) to a multiple of e1: returns beta, fills v.
double make_reflector(const double *x, int m, double *v) {
  double nrm = 0.0;
  for (int t = 0; t < m; ++t) nrm += x[t] * x[t];
  nrm = std::sqrt(nrm);
  if (nrm == 0.0) {
    for (int t = 0; t < m; ++t) v[t] = 0.0;
    return 0.0;
  }
  const double alpha = x[0] > 0 ? -nrm : nrm;
  v[0] = x[0] - alpha;
  for (int t = 1; t < m; ++t) v[t] = x[t];
  double vv = 0.0;
  for (int t = 0; t < m; ++t) vv += v[t] * v[t];
  return vv == 0.0 ? 0.0 : 2.0 / vv;
}

// Rotates the 2x2 diagonal block at (p, p+1), whose eigenvalues are real, to upper
// triangular form.  Returns false if the block's eigenvalues are genuinely complex.
bool split_block(Mat &H, Mat &Zt, int p, double *ev0, double *ev1) {
  const int n = H.n, q = p + 1;
  const double a = H(p, p), b = H(p, q), c = H(q, p), d = H(q, q);
  const double half = 0.5 * (a - d);
  double disc = half * half + b * c;
  const double scale = std::fabs(a) + std::fabs(d) + std::fabs(b) + std::fabs(c);
  if (disc < 0.0) {
    if (std::sqrt(-disc) > 1e-10 * scale) return false;
    disc = 0.0;
  }
  const double r = std::sqrt(disc);
  const double mid = 0.5 * (a + d);
  // eigenvalue of larger distance from d first, computed without cancellation
  const double lam = half >= 0 ? mid + r : mid - r;
  // eigenvector (b, lam - a) or (lam - d, c), whichever is larger
  double x0 = b, x1 = lam - a;
  const double y0 = lam - d, y1 = c;
  if (std::hypot(y0, y1) > std::hypot(x0, x1)) { x0 = y0; x1 = y1; }
  const double nv = std::hypot(x0, x1);
  double cs = 1.0, sn = 0.0;
  if (nv > 0.0) { cs = x0 / nv; sn = x1 / nv; }
  // Q2 = [[cs, -sn], [sn, cs]];  H <- Q2^T H Q2 on rows/cols p, q
  for (int j = p; j < n; ++j) {
    const double h0 = H(p, j), h1 = H(q, j);
    H(p, j) = cs * h0 + sn * h1;
    H(q, j) = -sn * h0 + cs * h1;
  }
  for (int i = 0; i <= q; ++i) {
    const double h0 = H(i, p), h1 = H(i, q);
    H(i, p) = cs * h0 + sn * h1;
    H(i, q) = -sn * h0 + cs * h1;
  }
  double *zp = &Zt(p, 0), *zq = &Zt(q, 0);  // columns p, q of Z
  for (int i = 0; i < n; ++i) {
    const double z0 = zp[i], z1 = zq[i];
    zp[i] = cs * z0 + sn * z1;
    zq[i] = -sn * z0 + cs * z1;
  }
  H(q, p) = 0.0;
  *ev0 = H(p, p);
  *ev1 = H(q, q);
  return true;
}

// Francis double-shift QR on the Hessenberg H to real Schur form.  Real eigenvalues end on
// the diagonal (2x2 blocks with real eigenvalues are split by a rotation); a 2x2 block with
// a complex-conjugate pair a +- ib is kept when allow_complex (ev = a, evi = +b on its
// first row and -b on its second), and is an error otherwise.
int schur_real(Mat &H, Mat &Zt, std::vector<double> &ev, std::vector<double> &evi, bool allow_complex) {
  const int n = H.n;
  const double eps = 2.220446049250313e-16;
  double anorm = 0.0;
  for (double x : H.a) anorm = std::max(anorm, std::fabs(x));
  if (anorm == 0.0) anorm = 1.0;
  ev.assign(n, 0.0);
  evi.assign(n, 0.0);
  int hi = n - 1;
  int iter = 0, total = 0;
  const int max_total = 60 * std::max(n, 10);
  double v[3];
  while (hi >= 0) {
    int l = hi;
    for (; l > 0; --l) {
      double s = std::fabs(H(l - 1, l - 1)) + std::fabs(H(l, l));
      if (s == 0.0) s = anorm;
      if (std::fabs(H(l, l - 1)) <= eps * s) {
        H(l, l - 1) = 0.0;
        break;
      }
    }
    if (l == hi) {
      ev[hi] = H(hi, hi);
      --hi;
      iter = 0;
      continue;
    }
    if (l == hi - 1) {
      double e0, e1;
      if (!split_block(H, Zt, hi - 1, &e0, &e1)) {
        if (!allow_complex) return set_error(FDG_ECOMPLEX, "factor_pencil: complex eigenvalue pair");
        const double a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
        const double half = 0.5 * (a - d);
        const double im = std::sqrt(-(half * half + b * c));
        ev[hi - 1] = ev[hi] = 0.5 * (a + d);
        evi[hi - 1] = im;
        evi[hi] = -im;
      } else {
        ev[hi - 1] = e0;
        ev[hi] = e1;
      }
      hi -= 2;
      iter = 0;
      continue;
    }
    if (++total > max_total) return set_error(FDG_ENOCONV, "factor_pencil: QR iteration did not converge");
    ++iter;
    double s, t;
    if (iter % 11 == 10) {  // exceptional shift against stagnation
      const double w = std::fabs(H(hi, hi - 1)) + std::fabs(H(hi - 1, hi - 2));
      s = 1.5 * w + H(hi, hi);
      t = w * w;
    } else {
      s = H(hi - 1, hi - 1) + H(hi, hi);
      t = H(hi - 1, hi - 1) * H(hi, hi) - H(hi - 1, hi) * H(hi, hi - 1);
    }
    double x = H(l, l) * H(l, l) + H(l, l + 1) * H(l + 1, l) - s * H(l, l) + t;
    double y = H(l + 1, l) * (H(l, l) + H(l + 1, l + 1) - s);
    double z = H(l + 1, l) * H(l + 2, l + 1);
    for (int k = l; k <= hi - 2; ++k) {
      const double xv[3] = {x, y, z};
      const double beta = make_reflector(xv, 3, v);
      if (beta != 0.0) {
        apply_reflector(H, Zt, k, 3, v, beta, std::max(l, k - 1), std::min(k + 3, hi));
        if (k > l) {
          H(k + 1, k - 1) = 0.0;
          H(k + 2, k - 1) = 0.0;
        }
      }
      x = H(k + 1, k);
      y = H(k + 2, k);
      if (k < hi - 2) z = H(k + 3, k);
    }
    const double xv[2] = {x, y};
    const double beta = make_reflector(xv, 2, v);
    if (beta != 0.0) {
      apply_reflector(H, Zt, hi - 1, 2, v, beta, std::max(l, hi - 2), hi);
      if (hi - 2 >= l) H(hi, hi - 2) = 0.0;
    }
  }
  return FDG_OK;
}

}  // namespace
}  // namespace fdg

using namespace fdg;


namespace {

typedef std::complex<double> cplx;

// Solution of the 2x2 system [[a, b], [c, d]] [x0, x1] = [r0, r1] by Cramer's rule, the
// determinant moved away from zero by smin (nearly equal eigenvalues).
template <typename T>
void solve2(T a, T b, T c, T d, T r0, T r1, double smin, T &x0, T &x1) {
  T det = a * d - b * c;
  if (std::abs(det) < smin) det = det == T(0) ? T(smin) : det * (smin / std::abs(det));
  x0 = (r0 * d - b * r1) / det;
  x1 = (a * r1 - c * r0) / det;
}

// Eigenvalues, Schur vectors and quasi-triangular T -> U (eigenvectors, real; a complex
// pair z = u + i v is stored as the columns u, v), V = (M U)^{-T}, lambda (real parts),
// mu (0, or +b and -b on the two columns of a pair a +- ib), ordered by real part.
int factor_impl(int n, const double *K, const double *M, bool allow_complex, double *U, double *V, double *lambda,
                double *mu, double *cond_u) {
  if (n < 1 || n > 4096 || !K || !M || !U || !V || !lambda)
    return set_error(FDG_EINVAL, "factor_pencil: bad arguments (n=%d)", n);
  const size_t nn = (size_t)n * n;
  for (size_t i = 0; i < nn; ++i)
    if (!std::isfinite(K[i]) || !std::isfinite(M[i]))
      return set_error(FDG_EINVAL, "factor_pencil: non-finite input");
  // A = M^{-1} K
  Mat LU(n);
  std::memcpy(LU.a.data(), M, nn * sizeof(double));
  std::vector<int> piv;
  if (!lu_factor(LU, piv)) return set_error(FDG_EINVAL, "factor_pencil: M is singular");
  std::vector<double> A(K, K + nn);
  lu_solve(LU, piv, A, n);
  Mat H(n), Zt(n);  // Zt = Z^T, the Schur vectors as rows
  H.a = A;
  for (int i = 0; i < n; ++i) Zt(i, i) = 1.0;
  hessenberg(H, Zt);
  std::vector<double> ev, evi;
  int st = schur_real(H, Zt, ev, evi, allow_complex);
  if (st != FDG_OK) return st;
  for (double e : ev)
    if (!(e > 0.0)) return set_error(FDG_ECOMPLEX, "factor_pencil: eigenvalue with non-positive real part %g", e);
  // first[i]: rows i, i+1 of T form a 2x2 block (a complex pair)
  std::vector<char> first(n, 0);
  for (int i = 0; i + 1 < n; ++i)
    if (evi[i] > 0.0) first[i] = 1;
  auto in_block_second = [&](int i) { return i >= 1 && first[i - 1]; };
  // Eigenvectors of the quasi-triangular T = H by back-substitution, kept as rows of Yt
  // (row k: eigenvector of a real eigenvalue; rows k, k+1: real and imaginary parts of
  // the eigenvector of the pair's eigenvalue a + ib) so inner products run over rows.
  const double ulp = 2.220446049250313e-16;
  Mat Yt(n);
  std::vector<cplx> yc(n);
  for (int k = n - 1; k >= 0; --k) {
    if (in_block_second(k)) continue;  // handled with the pair's first row
    if (first[k]) {                    // complex pair at rows k, k+1
      const cplx lk(ev[k], evi[k]);
      const double smin = std::max(ulp * std::abs(lk), 1e-300);
      std::fill(yc.begin(), yc.end(), cplx(0.0));
      yc[k] = H(k, k + 1);
      yc[k + 1] = lk - H(k, k);
      int i = k - 1;
      while (i >= 0) {
        if (in_block_second(i)) {  // rows i-1, i: a 2x2 block
          cplx s0 = 0.0, s1 = 0.0;
          for (int j = i + 1; j <= k + 1; ++j) {
            s0 += H(i - 1, j) * yc[j];
            s1 += H(i, j) * yc[j];
          }
          solve2<cplx>(H(i - 1, i - 1) - lk, H(i - 1, i), H(i, i - 1), H(i, i) - lk, -s0, -s1, smin, yc[i - 1],
                       yc[i]);
          i -= 2;
        } else {
          cplx s = 0.0;
          for (int j = i + 1; j <= k + 1; ++j) s += H(i, j) * yc[j];
          cplx den = H(i, i) - lk;
          if (std::abs(den) < smin) den = smin;
          yc[i] = -s / den;
          i -= 1;
        }
      }
      double *yr = &Yt(k, 0), *yi = &Yt(k + 1, 0);
      for (int j = 0; j <= k + 1; ++j) {
        yr[j] = yc[j].real();
        yi[j] = yc[j].imag();
      }
      continue;
    }
    const double lk = H(k, k);
    const double smin = std::max(ulp * std::fabs(lk), 1e-300);
    double *y = &Yt(k, 0);
    y[k] = 1.0;
    int i = k - 1;
    while (i >= 0) {
      if (in_block_second(i)) {  // rows i-1, i: a 2x2 block of a complex pair
        double s0 = 0.0, s1 = 0.0;
        for (int j = i + 1; j <= k; ++j) {
          s0 += H(i - 1, j) * y[j];
          s1 += H(i, j) * y[j];
        }
        solve2<double>(H(i - 1, i - 1) - lk, H(i - 1, i), H(i, i - 1), H(i, i) - lk, -s0, -s1, smin, y[i - 1], y[i]);
        i -= 2;
        continue;
      }
      const double *h = &H(i, 0);
      double s = 0.0;
      for (int j = i + 1; j <= k; ++j) s += h[j] * y[j];
      double den = H(i, i) - lk;
      double yi;
      if (std::fabs(den) < smin) {
        // equal eigenvalues (the double outlier of Remark 1): when the coupling is at
        // rounding level the Schur vector itself is an eigenvector of the cluster;
        // otherwise perturb the divisor as for nearby eigenvalues.
        double ymax = 0.0;
        for (int j = i + 1; j <= k; ++j) ymax = std::max(ymax, std::fabs(y[j]));
        if (std::fabs(s) <= 1e-10 * std::fabs(lk) * ymax) {
          yi = 0.0;
        } else {
          den = den >= 0 ? smin : -smin;
          yi = -s / den;
        }
      } else {
        yi = -s / den;
      }
      y[i] = yi;
      if (std::fabs(yi) > 1e150) {  // rescale the partial vector
        for (int j = i; j <= k; ++j) y[j] *= 1e-150;
      }
      i -= 1;
    }
  }
  // U = Z Y (column k of U = sum_j Y(j, k) Z(:, j), accumulated as row k of Ut)
  Mat Ut(n);
  for (int k = 0; k < n; ++k) {
    const double *y = &Yt(k, 0);
    double *u = &Ut(k, 0);
    const int jmax = (first[k] || in_block_second(k)) ? std::min(n - 1, k + 1) : k;
    for (int j = 0; j <= jmax; ++j) {
      const double yj = y[j];
      if (yj == 0.0) continue;
      const double *z = &Zt(j, 0);
      for (int i = 0; i < n; ++i) u[i] += yj * z[i];
    }
  }
  // units (a real eigenvalue or a pair) in ascending order of the real part
  std::vector<int> units;
  for (int k = 0; k < n; ++k)
    if (!in_block_second(k)) units.push_back(k);
  std::stable_sort(units.begin(), units.end(), [&](int a, int b) { return ev[a] < ev[b]; });
  int c = 0;
  for (int k : units) {
    if (first[k]) {
      // z = u + i v: rotate the phase so that u and v are orthogonal, unit 2-norm of z
      double *u = &Ut(k, 0), *v = &Ut(k + 1, 0);
      double uu = 0.0, vv = 0.0, uv = 0.0;
      for (int i = 0; i < n; ++i) {
        uu += u[i] * u[i];
        vv += v[i] * v[i];
        uv += u[i] * v[i];
      }
      const double th = 0.5 * std::atan2(-2.0 * uv, uu - vv);
      const double cs = std::cos(th), sn = std::sin(th);
      const double nrm = std::sqrt(uu + vv);
      if (!(nrm > 0.0) || !std::isfinite(nrm)) return set_error(FDG_ENOCONV, "factor_pencil: degenerate eigenvector");
      for (int i = 0; i < n; ++i) {
        U[(size_t)i * n + c] = (cs * u[i] - sn * v[i]) / nrm;
        U[(size_t)i * n + c + 1] = (sn * u[i] + cs * v[i]) / nrm;
      }
      lambda[c] = lambda[c + 1] = ev[k];
      if (mu) {
        mu[c] = evi[k];
        mu[c + 1] = -evi[k];
      }
      c += 2;
    } else {
      double nrm = 0.0;
      for (int i = 0; i < n; ++i) nrm += Ut(k, i) * Ut(k, i);
      nrm = std::sqrt(nrm);
      if (!(nrm > 0.0) || !std::isfinite(nrm)) return set_error(FDG_ENOCONV, "factor_pencil: degenerate eigenvector");
      for (int i = 0; i < n; ++i) U[(size_t)i * n + c] = Ut(k, i) / nrm;
      lambda[c] = ev[k];
      if (mu) mu[c] = 0.0;
      c += 1;
    }
  }
  // V = (M U)^{-T}
  Mat MU(n);
  for (int i = 0; i < n; ++i) {
    double *mrow = &MU(i, 0);
    for (int j = 0; j < n; ++j) {
      const double m = M[(size_t)i * n + j];
      if (m == 0.0) continue;
      const double *u = U + (size_t)j * n;
      for (int k = 0; k < n; ++k) mrow[k] += m * u[k];
    }
  }
  std::vector<int> piv2;
  if (!lu_factor(MU, piv2)) return set_error(FDG_EINVAL, "factor_pencil: M U is singular");
  std::vector<double> inv(nn, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  lu_solve(MU, piv2, inv, n);  // inv = (M U)^{-1}
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) V[(size_t)i * n + k] = inv[(size_t)k * n + i];
  if (cond_u) {
    Mat LUu(n);
    std::memcpy(LUu.a.data(), U, nn * sizeof(double));
    std::vector<int> p3;
    double c1 = 0.0;
    for (int k = 0; k < n; ++k) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += std::fabs(U[(size_t)i * n + k]);
      c1 = std::max(c1, s);
    }
    if (!lu_factor(LUu, p3)) {
      *cond_u = INFINITY;
    } else {
      std::vector<double> ui(nn, 0.0);
      for (int i = 0; i < n; ++i) ui[(size_t)i * n + i] = 1.0;
      lu_solve(LUu, p3, ui, n);
      double c2 = 0.0;
      for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += std::fabs(ui[(size_t)i * n + k]);
        c2 = std::max(c2, s);
      }
      *cond_u = c1 * c2;
    }
  }
  return FDG_OK;
}

}  // namespace

extern "C" int fdg_factor_pencil(int n, const double *K, const double *M, double *U, double *V,
                                 double *lambda, double *cond_u) {
  clear_error();
  return factor_impl(n, K, M, false, U, V, lambda, nullptr, cond_u);
}

extern "C" int fdg_factor_pencil_blocks(int n, const double *K, const double *M, double *U, double *V,
                                        double *lambda, double *mu, double *cond_u) {
  clear_error();
  if (!mu) return set_error(FDG_EINVAL, "factor_pencil_blocks: mu is NULL");
  return factor_impl(n, K, M, true, U, V, lambda, mu, cond_u);
}
