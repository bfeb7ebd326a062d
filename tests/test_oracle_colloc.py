"""Pins of the oracle's collocation operators (unit and deformed cube).

* The unit-domain operator (eq. 2.7 / 2.9) applied to random spline
  coefficients equals -Laplacian of that spline at the Greville grid, computed
  with scipy.interpolate.NdBSpline (independent library).
* Manufactured-solution convergence at order >= p - 1 (unit square/cube).
* Deformed cube: amp = 0 reduces to the unit operator; the chain-rule
  coefficients (C, g) reproduce the Laplacian of a polynomial/trigonometric test
  function computed by finite differences in parameter space; A applied to
  spline coefficients equals the chain rule applied to NdBSpline derivatives;
  manufactured convergence on the deformed cube.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
from scipy.interpolate import NdBSpline

from oracle import bspline, colloc


def _ndspline(p, n, d, coef_interior):
    E = bspline.n_spans(p, n)
    xi = bspline.knots(p, E)
    m = n + 2
    c = np.zeros([m] * d)
    c[tuple([slice(1, m - 1)] * d)] = coef_interior.reshape([n] * d)   # axes (i_d, ..., i_1)
    return NdBSpline(tuple([xi] * d), c, p)


def _grid_points(p, n, d):
    tau = bspline.greville(p, n)
    g = np.meshgrid(*([tau] * d), indexing="ij")        # axis 0 <-> i_d
    return np.stack([gi.ravel() for gi in g], axis=-1)  # columns ordered (x_d, ..., x_1)


@pytest.mark.parametrize("d,p,n", [(2, 3, 9), (2, 2, 7), (3, 4, 7), (3, 3, 6), (2, 5, 10)])
def test_unit_operator_is_minus_laplacian(d, p, n):
    M, K, _, _ = colloc.colloc_factors(p, n)
    P = colloc.unit_operator([M] * d, [K] * d)
    c = np.random.default_rng(d * 10 + p).standard_normal(n ** d)
    s = _ndspline(p, n, d, c)
    pts = _grid_points(p, n, d)
    lap = np.zeros(len(pts))
    for a in range(d):
        nu = [0] * d
        nu[a] = 2
        lap += s(pts, nu=nu)
    assert np.allclose(P @ c, -lap, rtol=1e-11, atol=1e-11 * np.abs(lap).max())


def _unit_error(p, n, d):
    M, K, _, tau = colloc.colloc_factors(p, n)
    P = colloc.unit_operator([M] * d, [K] * d).tocsc()
    f = colloc.manufactured_rhs(p, n, d)
    c = spla.spsolve(P, f)
    uh = colloc.kron_chain([M] * d) @ c
    coords = colloc.tensor_grid([tau] * d)
    u = np.ones_like(coords[0])
    for x in coords:
        u = u * np.sin(np.pi * x)
    return np.abs(uh - u.ravel()).max()


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_unit_square_manufactured_order(p):
    ns = [14, 22, 30]
    errs = [_unit_error(p, n, 2) for n in ns]
    hs = [1.0 / bspline.n_spans(p, n) for n in ns]
    order = np.log(errs[-2] / errs[-1]) / np.log(hs[-2] / hs[-1])
    assert order >= p - 1 - 0.1, (errs, order)


def test_config_small_2d_error_level():
    # p = 3, 32 spans: the collocation error of the manufactured solution is O(h^2)
    err = _unit_error(3, 33, 2)
    assert 1e-4 < err < 3e-3


def test_deformed_reduces_to_unit():
    p, n = 3, 6
    M, K, _, _ = colloc.colloc_factors(p, n)
    P = colloc.unit_operator([M] * 3, [K] * 3)
    A = colloc.deformed_operator(p, n, 0.0)
    assert abs(A - P).max() <= 1e-12 * abs(P).max()


def test_chain_rule_coefficients_by_finite_differences():
    """-Lap_x u at x = F(xi) from (C, g) and parameter-space derivatives of u o F."""
    amp = 0.1
    F, _, _ = colloc.deform_map(amp)

    def u(x):
        return x[..., 0] ** 2 * x[..., 1] + np.sin(x[..., 2]) + x[..., 0] * x[..., 2] ** 3

    def lap_u(x):
        return 2 * x[..., 1] - np.sin(x[..., 2]) + 6 * x[..., 0] * x[..., 2]

    rng = np.random.default_rng(3)
    xi = rng.uniform(0.05, 0.95, size=(20, 3))
    C, g = colloc.deformed_coefficients(xi, amp)
    h = 2e-4
    uhat = lambda z: u(F(z))
    grad = np.zeros((20, 3))
    hess = np.zeros((20, 3, 3))
    E = np.eye(3)
    for k in range(3):
        grad[:, k] = (uhat(xi + h * E[k]) - uhat(xi - h * E[k])) / (2 * h)
        for l in range(3):
            hess[:, k, l] = (uhat(xi + h * E[k] + h * E[l]) - uhat(xi + h * E[k] - h * E[l])
                             - uhat(xi - h * E[k] + h * E[l]) + uhat(xi - h * E[k] - h * E[l])) / (4 * h * h)
    lhs = np.einsum("nkl,nkl->n", C, hess) + np.einsum("nk,nk->n", g, grad)
    assert np.allclose(lhs, lap_u(F(xi)), atol=2e-5)


def test_deformed_operator_matches_chain_rule_on_splines():
    p, n, amp = 3, 6, 0.1
    A = colloc.deformed_operator(p, n, amp)
    c = np.random.default_rng(11).standard_normal(n ** 3)
    s = _ndspline(p, n, 3, c)
    pts = _grid_points(p, n, 3)               # columns (x_3, x_2, x_1)
    xi = pts[:, ::-1]                          # (xi_1, xi_2, xi_3)
    C, g = colloc.deformed_coefficients(xi, amp)

    def der(orders):                            # orders by direction 1..3
        return s(pts, nu=list(reversed(orders)))

    lap = np.zeros(len(pts))
    for k in range(3):
        for l in range(3):
            o = [0, 0, 0]
            o[k] += 1
            o[l] += 1
            lap += C[:, k, l] * der(o)
        o = [0, 0, 0]
        o[k] = 1
        lap += g[:, k] * der(o)
    assert np.allclose(A @ c, -lap, rtol=1e-10, atol=1e-10 * np.abs(lap).max())


def test_deformed_pattern_27_per_row_for_cubic():
    A = colloc.deformed_operator(3, 8, 0.1)
    nnz = np.diff(A.indptr)
    assert nnz.max() == 27


def test_deformed_manufactured_order():
    p, amp = 3, 0.1
    errs, hs = [], []
    for n in (10, 14, 18):
        A = colloc.deformed_operator(p, n, amp).tocsc()
        f = colloc.deformed_manufactured_rhs(p, n, amp)
        c = spla.spsolve(A, f)
        M, _, _, tau = colloc.colloc_factors(p, n)
        uh = colloc.kron_chain([M] * 3) @ c
        coords = colloc.tensor_grid([tau] * 3)
        u = np.sin(np.pi * coords[0]) * np.sin(np.pi * coords[1]) * np.sin(np.pi * coords[2])
        errs.append(np.abs(uh - u.ravel()).max())
        hs.append(1.0 / bspline.n_spans(p, n))
    order = np.log(errs[-2] / errs[-1]) / np.log(hs[-2] / hs[-1])
    assert order >= p - 1 - 0.1, (errs, order)


@pytest.mark.parametrize("d,p,n", [(2, 3, 11), (3, 4, 9), (3, 2, 7)])
def test_unit_matvec_equals_sparse_operator(d, p, n):
    M, K, _, _ = colloc.colloc_factors(p, n)
    x = np.random.default_rng(1).standard_normal(n ** d)
    P = colloc.unit_operator([M] * d, [K] * d)
    assert np.allclose(colloc.unit_matvec([M] * d, [K] * d, x), P @ x, rtol=1e-13, atol=1e-13 * abs(P @ x).max())
