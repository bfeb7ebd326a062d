"""Galerkin matrices for the oracle (test infrastructure only; see package header).

Sec. 3.2 adapts the preconditioner to the convection-diffusion operator
L_w = -Lap + w . grad (eq. 3.6) under an isogeometric Galerkin discretization
whose integrals are taken by standard Gaussian quadrature.  The preconditioner
is the same discretization on the unit cube with the wind either dropped
(eq. 3.7, univariate factors of eq. 3.8: symmetric positive definite, so the
symmetric FD of Sec. 4 applies, V_l = U_l) or replaced by univariate
approximations w~_l(zeta_l) (eq. 3.9: K_l becomes K_l + H_l with
(H_l)_ij = int w~_l B_i B'_j, nonsymmetric, so the nonsymmetric FD applies).
The same factors with the wind dropped are the Galerkin preconditioner P_G of
Sec. 3, which equals the weighted-quadrature one (P_wq = P_G).

Readings where the paper is silent:
* Quadrature: p + 1 Gauss-Legendre points on every knot span (exact for M, K
  and for H with an affine wind; the paper ignores the quadrature error of a
  general wind, and so does this module).
* Test problem: the paper does not explore convection-diffusion numerically.
  The system matrix here is the Galerkin matrix of -Lap u + w . grad u with
  homogeneous Dirichlet conditions on F([0,1]^3) (the smooth map of
  ``colloc.deform_map``; amp = 0 is the unit cube), pulled back to the
  parametric cube:
      A_ij = sum_q omega_q [ grad B_i^T Q grad B_j + B_i b^T grad B_j ](xi_q),
      Q = det(J) J^{-1} J^{-T}  (eq. 2.10 with K = I),  b = det(J) J^{-1} w(F(xi)),
  with the tensor (p+1)^3-point Gauss rule of every element, the interior
  functions of eq. 2.3 (i_1 fastest) and the wind
      w_l(x) = c_l (1 + x_l) (1 + beta cos(2 pi x_{l+1}) cos(2 pi x_{l+2}))
  (indices cyclic), whose average over the other two coordinates on the unit
  cube is the affine univariate wind w~_l(zeta) = c_l (1 + zeta) used in
  eq. 3.9.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import bspline
from .colloc import deform_map, kron_chain


def gauss_rule(p, n):
    """(p+1)-point Gauss-Legendre rule on every span [e/E, (e+1)/E] of the uniform
    open knot vector with E = n + 2 - p spans (Sec. 2.1); points ascending."""
    E = bspline.n_spans(p, n)
    g, w = np.polynomial.legendre.leggauss(p + 1)
    x = ((np.arange(E)[:, None] + 0.5 * (g[None, :] + 1.0)) / E).ravel()
    wt = np.tile(0.5 * w / E, E)
    return x, wt


def basis_at(p, n, x):
    """Interior B-splines B_1..B_n (eq. 2.3) and their first derivatives at points x
    strictly inside spans: arrays (len(x), n), [q, j] = B_j(x_q), B'_j(x_q)."""
    E = bspline.n_spans(p, n)
    xi = bspline.knots(p, E)
    D = bspline.basis_derivs(xi, p, np.asarray(x, dtype=np.float64), nder=1)
    return D[0, 1:n + 1, :].T.copy(), D[1, 1:n + 1, :].T.copy()


def galerkin_factors(p, n, wind=None):
    """Univariate Galerkin factors of eq. 3.8 and, for a univariate wind w~ (callable),
    the convection factor after eq. 3.9:
        (M)_ij = int B_i B_j,  (K)_ij = int B'_i B'_j,  (H)_ij = int w~ B_i B'_j,
    i, j = 1..n (row = test function), by the Gauss rule of ``gauss_rule``.
    Returns (M, K, H) with H None when wind is None."""
    x, w = gauss_rule(p, n)
    B, dB = basis_at(p, n, x)
    M = B.T @ (w[:, None] * B)
    K = dB.T @ (w[:, None] * dB)
    H = None
    if wind is not None:
        H = B.T @ ((w * np.asarray(wind(x), dtype=np.float64))[:, None] * dB)
    return M, K, H


def affine_wind(c):
    """The univariate wind w~(zeta) = c (1 + zeta) (see module docstring)."""
    return lambda z: c * (1.0 + np.asarray(z))


def factor_pencil_sym(K, M):
    """Symmetric FD factors (Sec. 4, after eq. 4.6): for K symmetric and M symmetric
    positive definite the eigenvectors of M^{-1} K can be taken M-orthonormal, and then
    V = (M U)^{-T} = U.  Returns (U, lam) with lam ascending and U^T M U = I."""
    lam, U = sla.eigh(K, M)
    return U, lam


def wind_field(x, c, beta):
    """w(x) of the module docstring at physical points x (..., 3); c = (c_1, c_2, c_3)."""
    out = np.empty_like(x)
    tp = 2.0 * np.pi
    for a in range(3):
        b1, b2 = (a + 1) % 3, (a + 2) % 3
        out[..., a] = c[a] * (1.0 + x[..., a]) * (1.0 + beta * np.cos(tp * x[..., b1]) * np.cos(tp * x[..., b2]))
    return out


def galerkin_operator(p, n, amp=0.0, c=(0.0, 0.0, 0.0), beta=0.0):
    """Galerkin matrix of -Lap u + w . grad u on F([0,1]^3) (module docstring), CSR,
    rows = test functions, i_1 fastest.

    Written as sums of diagonally scaled Kronecker products: with B_l, G_l the
    values and derivatives of direction l's interior functions at the 1D Gauss points,
    the value of B_j at the tensor point q is (B x B x B)[q, j] and its derivative in
    direction a replaces that direction's factor by G (``kron_chain`` order), so
        A = sum_a Grad_a^T (sum_b diag(omega Q_ab) Grad_b) + Val^T (sum_b diag(omega b_b) Grad_b)."""
    x1, w1 = gauss_rule(p, n)
    B, G = basis_at(p, n, x1)
    grids = np.meshgrid(x1, x1, x1, indexing="ij")               # axes (q3, q2, q1)
    xi = np.stack([grids[2].ravel(), grids[1].ravel(), grids[0].ravel()], axis=-1)
    wg = np.meshgrid(w1, w1, w1, indexing="ij")
    omega = (wg[0] * wg[1] * wg[2]).ravel()
    F, J, _ = deform_map(amp)
    Jx = J(xi)
    det = np.linalg.det(Jx)
    Ji = np.linalg.inv(Jx)
    Q = det[:, None, None] * (Ji @ np.swapaxes(Ji, -1, -2))
    bvec = det[:, None] * np.einsum("qab,qb->qa", Ji, wind_field(F(xi), c, beta))
    val = kron_chain([B, B, B])
    grad = [kron_chain([G if q == a else B for q in range(3)]) for a in range(3)]
    # the inner sums over b first (same sparsity for every b), then one product per a
    A = None
    for a in range(3):
        S = sum(sp.diags(omega * Q[:, a, b]) @ grad[b] for b in range(3))
        T = grad[a].T @ S
        A = T if A is None else A + T
    if any(ci != 0.0 for ci in c):
        S = sum(sp.diags(omega * bvec[:, b]) @ grad[b] for b in range(3))
        A = A + val.T @ S
    A = A.tocsr()
    A.sort_indices()
    return A


def galerkin_load(p, n, f, amp=0.0):
    """Load vector F_i = int_Omega (B_i o F^{-1}) f dx = sum_q omega_q det J(xi_q) B_i(xi_q)
    f(xi_q) on Omega = F([0,1]^3) by the same tensor Gauss rule, for f given as a callable
    of the parametric points xi (..., 3) -- the right-hand side of the Galerkin system."""
    x1, w1 = gauss_rule(p, n)
    B, _ = basis_at(p, n, x1)
    grids = np.meshgrid(x1, x1, x1, indexing="ij")
    xi = np.stack([grids[2].ravel(), grids[1].ravel(), grids[0].ravel()], axis=-1)
    wg = np.meshgrid(w1, w1, w1, indexing="ij")
    omega = (wg[0] * wg[1] * wg[2]).ravel()
    det = np.linalg.det(deform_map(amp)[1](xi))
    return kron_chain([B, B, B]).T @ (omega * det * f(xi))
