"""Pins of the Galerkin oracle (Sec. 3.2, eq. 3.6-3.9; symmetric FD of Sec. 4).

Each test checks ``oracle.galerkin`` against something other than itself: closed
forms of linear splines, adaptive quadrature of scipy's B-splines, integration by
parts, the min-max principle, Kronecker reductions, brute-force dense solves and
the convergence order of a manufactured solution."""
import numpy as np
import pytest
import scipy.integrate as si
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.interpolate import BSpline

from oracle import bspline, colloc, fd
from oracle import galerkin as G


def _scipy_basis(p, n):
    E = bspline.n_spans(p, n)
    t = bspline.knots(p, E)
    m = n + 2
    funcs = []
    for j in range(1, n + 1):
        c = np.zeros(m)
        c[j] = 1.0
        funcs.append(BSpline(t, c, p, extrapolate=False))
    return t, funcs


def test_linear_splines_closed_form():
    # p = 1: hat functions on h = 1/E; M = h/6 tridiag(1, 4, 1), K = tridiag(-1, 2, -1)/h
    for n in (1, 4, 9):
        M, K, _ = G.galerkin_factors(1, n)
        h = 1.0 / (n + 1)
        I = np.eye(n)
        off = np.eye(n, k=1) + np.eye(n, k=-1)
        assert np.allclose(M, h / 6 * (4 * I + off), rtol=0, atol=1e-15)
        assert np.allclose(K, (2 * I - off) / h, rtol=0, atol=1e-12)


@pytest.mark.parametrize("p,n", [(2, 6), (3, 7)])
def test_factors_match_adaptive_quadrature(p, n):
    # every entry against scipy's BSpline integrated by adaptive quadrature span by span
    wind = lambda z: 2.0 + 3.0 * z
    M, K, H = G.galerkin_factors(p, n, wind)
    t, B = _scipy_basis(p, n)
    dB = [b.derivative() for b in B]
    brk = np.unique(t)
    def integ(f):
        return sum(si.quad(lambda z: np.nan_to_num(f(z)), a, b, epsabs=1e-14, epsrel=1e-13)[0]
                   for a, b in zip(brk[:-1], brk[1:]))
    for i in range(n):
        for j in range(n):
            assert abs(M[i, j] - integ(lambda z: B[i](z) * B[j](z))) <= 1e-13
            assert abs(K[i, j] - integ(lambda z: dB[i](z) * dB[j](z))) <= 1e-11
            assert abs(H[i, j] - integ(lambda z: wind(z) * B[i](z) * dB[j](z))) <= 1e-12


@pytest.mark.parametrize("p,n", [(2, 8), (3, 11), (5, 9)])
def test_convection_factor_integration_by_parts(p, n):
    # interior functions vanish at 0 and 1: int w (B_i B_j)' = -int w' B_i B_j, so
    # H + H^T = 0 for a constant wind and H + H^T = -M for w(z) = z
    M, _, H1 = G.galerkin_factors(p, n, lambda z: np.ones_like(z))
    assert np.abs(H1 + H1.T).max() <= 1e-14
    _, _, Hz = G.galerkin_factors(p, n, lambda z: z)
    assert np.abs(Hz + Hz.T + M).max() <= 1e-14


@pytest.mark.parametrize("p,n", [(2, 9), (4, 10)])
def test_quadratic_in_spline_space(p, n):
    # u = z - z^2 is in the space for p >= 2 (coefficients from the blossom: the mean of
    # the p interior knots of B_j minus the mean of their pairwise products).  Then
    # (K c)_i = int B_i' u' = -int B_i u'' = 2 int B_i = 2 (xi_{i+p+1} - xi_i) / (p+1),
    # and (H c)_i = int B_i u' for a constant wind, checked by adaptive quadrature.
    E = bspline.n_spans(p, n)
    t = bspline.knots(p, E)
    c = np.zeros(n)
    for j in range(1, n + 1):
        a = t[j + 1:j + p + 1]
        pairs = [a[r] * a[s] for r in range(p) for s in range(r + 1, p)]
        c[j - 1] = a.mean() - np.mean(pairs)
    M, K, H = G.galerkin_factors(p, n, lambda z: np.ones_like(z))
    integral = np.array([(t[i + p + 1] - t[i]) / (p + 1) for i in range(1, n + 1)])
    assert np.abs(K @ c - 2.0 * integral).max() <= 1e-13
    _, B = _scipy_basis(p, n)
    brk = np.unique(t)
    for i in range(n):
        ref = sum(si.quad(lambda z: np.nan_to_num(B[i](z)) * (1 - 2 * z), a, b, epsabs=1e-15)[0]
                  for a, b in zip(brk[:-1], brk[1:]))
        assert abs((H @ c)[i] - ref) <= 1e-13


@pytest.mark.parametrize("p,n", [(2, 16), (3, 33), (4, 40)])
def test_symmetric_pencil(p, n):
    # U^T M U = I, K U = M U diag(lam), V = (M U)^{-T} = U (Sec. 4 after eq. 4.6); Galerkin
    # eigenvalues bound the Dirichlet Laplacian's (k pi)^2 from above (min-max principle)
    M, K, _ = G.galerkin_factors(p, n)
    U, lam = G.factor_pencil_sym(K, M)
    assert np.abs(U.T @ M @ U - np.eye(n)).max() <= 1e-12
    assert np.abs(K @ U - M @ U * lam).max() <= 1e-10 * lam.max()
    V = np.linalg.inv(M @ U).T
    assert np.abs(V - U).max() <= 1e-10 * np.abs(U).max()
    k = np.arange(1, 6)
    assert np.all(lam[:5] >= (k * np.pi) ** 2 * (1 - 1e-13))
    assert abs(lam[0] - np.pi ** 2) <= 1e-3 * np.pi ** 2


@pytest.mark.parametrize("d,p,n", [(2, 2, 6), (3, 3, 5)])
def test_symmetric_fd_brute_force(d, p, n):
    # symmetric FD (V = U) = dense solve of the Kronecker sum of eq. 3.7, and equals the
    # nonsymmetric FD of the same pencil (they differ only in the eigenvector scaling)
    M, K, _ = G.galerkin_factors(p, n)
    U, lam = G.factor_pencil_sym(K, M)
    P = colloc.unit_operator([M] * d, [K] * d).toarray()
    b = np.random.default_rng(5).standard_normal(n ** d)
    s = fd.fd_apply([U] * d, [U] * d, [lam] * d, b)
    assert np.abs(s - np.linalg.solve(P, b)).max() <= 1e-12 * np.abs(s).max()
    Un, Vn, ln = fd.factor_pencil(K, M)
    s2 = fd.fd_apply([Un] * d, [Vn] * d, [ln] * d, b)
    assert np.abs(s - s2).max() <= 1e-12 * np.abs(s).max()


def test_convection_fd_brute_force():
    # eq. 3.9: P = (K_3 + H_3) x M x M + ... with per-direction winds; the nonsymmetric FD
    # of the pencils (K_l + H_l, M_l) against a dense solve
    p, n = 3, 5
    facs = [G.galerkin_factors(p, n, G.affine_wind(c)) for c in (2.0, 4.0, 6.0)]
    Ms = [f[0] for f in facs]
    KHs = [f[1] + f[2] for f in facs]
    P = colloc.unit_operator(Ms, KHs).toarray()
    fac = [fd.factor_pencil(KH, M) for KH, M in zip(KHs, Ms)]
    b = np.random.default_rng(6).standard_normal(n ** 3)
    s = fd.fd_apply([f[0] for f in fac], [f[1] for f in fac], [f[2] for f in fac], b)
    assert np.abs(s - np.linalg.solve(P, b)).max() <= 1e-12 * np.abs(s).max()


def test_convection_pencils_real_for_configured_wind():
    # Remark 1's assumption (real eigenvalues) holds for the winds the tests and
    # measurements use (c <= 10 with n >= 16, p <= 4: mesh Peclet number c h below ~1);
    # coarser meshes give complex pairs, outside the method as built
    for p in (2, 3, 4):
        for n in (16, 48):
            M, K, H = G.galerkin_factors(p, n, G.affine_wind(10.0))
            fd.factor_pencil(K + H, M)   # raises ComplexPencilError otherwise
    M, K, H = G.galerkin_factors(3, 8, G.affine_wind(10.0))
    with pytest.raises(fd.ComplexPencilError):
        fd.factor_pencil(K + H, M)


def test_operator_unit_cube_reduces_to_kronecker():
    # F = id, no wind: the Galerkin matrix is the Kronecker sum of eq. 3.7 with eq. 3.8
    # factors; F = id with beta = 0: the wind c_l (1 + x_l) adds c_l times the Kronecker
    # product with H of w~ = 1 + z in direction l
    p, n = 2, 5
    M, K, H = G.galerkin_factors(p, n, G.affine_wind(1.0))
    A0 = G.galerkin_operator(p, n)
    P = colloc.unit_operator([M] * 3, [K] * 3)
    assert abs(A0 - P).max() <= 1e-14 * abs(P).max()
    c = (1.5, -2.0, 3.0)
    A1 = G.galerkin_operator(p, n, 0.0, c, 0.0)
    ref = P.copy()
    for l in range(3):
        ref = ref + c[l] * colloc.kron_chain([H if q == l else M for q in range(3)])
    assert abs(A1 - ref).max() <= 1e-13 * abs(ref).max()


def test_operator_deformed_symmetric_positive_definite():
    # no wind: A_ij = int grad B_i^T Q grad B_j with Q = det J J^{-1} J^{-T} SPD
    A = G.galerkin_operator(2, 5, amp=0.1).toarray()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0.0


def _manufactured_f(xi, amp, c, beta):
    # f = -Lap_x u + w . grad_x u for u = u_hat o F^{-1}, u_hat = prod sin(pi xi_l); the
    # Laplacian by the chain rule of the collocation oracle (pinned separately),
    # grad_x u = J^{-T} grad_xi u_hat
    C, g = colloc.deformed_coefficients(xi, amp)
    s, co = np.sin(np.pi * xi), np.cos(np.pi * xi)
    grad = np.zeros_like(xi)
    hess = np.zeros(xi.shape + (3,))
    for k in range(3):
        o1, o2 = [q for q in range(3) if q != k]
        grad[:, k] = np.pi * co[:, k] * s[:, o1] * s[:, o2]
        hess[:, k, k] = -np.pi ** 2 * s[:, 0] * s[:, 1] * s[:, 2]
        for l in range(3):
            if l != k:
                hess[:, k, l] = np.pi ** 2 * co[:, k] * co[:, l] * s[:, 3 - k - l]
    f = -(np.einsum("nkl,nkl->n", C, hess) + np.einsum("nk,nk->n", g, grad))
    F, J, _ = colloc.deform_map(amp)
    gx = np.einsum("nka,nk->na", np.linalg.inv(J(xi)), grad)
    return f + np.einsum("na,na->n", G.wind_field(F(xi), c, beta), gx)


def test_manufactured_solution_converges():
    # Galerkin error of a smooth solution on the deformed cube with variable wind decays
    # like h^{p+1}; a wrong metric Q, wind transform or orientation stalls it
    p, amp, c, beta = 2, 0.1, (2.0, 3.0, 4.0), 0.5
    pts = np.random.default_rng(0).uniform(0.05, 0.95, (200, 3))
    errs, Es = [], []
    for n in (6, 10):
        A = G.galerkin_operator(p, n, amp, c, beta)
        b = G.galerkin_load(p, n, lambda xi: _manufactured_f(xi, amp, c, beta), amp)
        x = spla.spsolve(sp.csc_matrix(A), b)
        E = bspline.n_spans(p, n)
        kn = bspline.knots(p, E)
        Bs = [bspline.basis_derivs(kn, p, pts[:, l], nder=0)[0, 1:n + 1, :].T for l in range(3)]
        uh = np.einsum("qc,qb,qa,cba->q", Bs[2], Bs[1], Bs[0], x.reshape(n, n, n))
        errs.append(np.abs(uh - np.prod(np.sin(np.pi * pts), axis=1)).max())
        Es.append(E)
    rate = np.log(errs[0] / errs[1]) / np.log(Es[1] / Es[0])
    assert errs[1] < 1e-3
    assert rate >= p + 0.5, (errs, rate)


@pytest.mark.parametrize("d,p,n,c", [(2, 3, 8, 10.0), (3, 3, 6, 12.0), (3, 2, 7, 20.0)])
def test_complex_pencil_fd_brute_force(d, p, n, c):
    # Sec. 4 after eq. 4.7: a pencil with complex eigenvalues (strong wind on a coarse
    # mesh) is still diagonalized, in complex arithmetic; the FD then equals a dense solve
    # of the Kronecker sum of eq. 3.9 and the result is real
    M, K, H = G.galerkin_factors(p, n, G.affine_wind(c))
    U, V, lam = fd.factor_pencil(K + H, M, allow_complex=True)
    assert np.abs(lam.imag).max() > 1e-3 * np.abs(lam).max()        # genuinely complex
    assert np.abs((K + H) @ U - M @ U * lam).max() <= 1e-10 * np.abs(lam).max()
    P = colloc.unit_operator([M] * d, [K + H] * d).toarray()
    b = np.random.default_rng(7).standard_normal(n ** d)
    shape = [n] * d
    X = b.reshape(shape).astype(complex)
    for l in range(d):
        X = fd.mode_product(X, V.T, l + 1)
    X = X / fd.eig_sum([lam] * d)
    for l in range(d):
        X = fd.mode_product(X, U, l + 1)
    assert np.abs(X.imag).max() <= 1e-12 * np.abs(X.real).max()
    s = fd.fd_apply([U] * d, [V] * d, [lam] * d, b)
    assert np.abs(s - np.linalg.solve(P, b)).max() <= 1e-11 * np.abs(s).max()
