"""Pins of the oracle's B-spline layer against things other than itself.

* partition of unity and linear precision (textbook B-spline identities);
* values and derivatives against scipy.interpolate.BSpline (an independent library);
* closed-form values of uniform quadratic/cubic B-splines (golden file);
* the support count of B-splines at Greville points (p at a simple knot, p+1
  inside a span).
"""
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import bspline, colloc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("p,E", [(2, 5), (3, 7), (4, 9), (5, 6), (6, 11)])
def test_partition_of_unity_and_linear_precision(p, E):
    xi = bspline.knots(p, E)
    rng = np.random.default_rng(p * 100 + E)
    x = np.concatenate([rng.uniform(0, 1, 50), xi, [0.0, 1.0]])
    D = bspline.basis_derivs(xi, p, x, nder=2)
    assert np.allclose(D[0].sum(axis=0), 1.0, atol=1e-14)
    assert np.allclose(D[1].sum(axis=0), 0.0, atol=1e-10 * E)
    assert np.allclose(D[2].sum(axis=0), 0.0, atol=1e-9 * E * E)
    # linear precision: the Greville abscissae are the coefficients of x
    g = bspline.greville_all(p, E)
    assert np.allclose(g @ D[0], x, atol=1e-14)
    assert np.allclose(g @ D[1], 1.0, atol=1e-12)
    assert np.allclose(g @ D[2], 0.0, atol=1e-9 * E * E)


@pytest.mark.parametrize("p,E", [(2, 6), (3, 8), (4, 5), (6, 9)])
def test_against_scipy_bspline(p, E):
    xi = bspline.knots(p, E)
    m = E + p
    rng = np.random.default_rng(7 + p)
    x = np.concatenate([rng.uniform(0, 1, 40), bspline.greville(p, m - 2)])
    D = bspline.basis_derivs(xi, p, x, nder=2)
    for j in range(m):
        c = np.zeros(m)
        c[j] = 1.0
        s = BSpline(xi, c, p)
        for r in range(3):
            ref = s.derivative(r)(x) if r else s(x)
            assert np.allclose(D[r, j], ref, rtol=1e-12, atol=1e-12 * E ** r), (j, r)


def _read_golden(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            rows[key] = np.array([float(Fraction(v)) for v in vals])
    return rows


def test_closed_form_uniform_cubic_and_quadratic():
    """Interior rows of M, K, D1 against the classical uniform B-spline values (golden file)."""
    g = _read_golden("uniform_bspline_rows.txt")
    # cubic: Greville points of interior functions are knots; h = 1/E
    p, n = 3, 20
    E = bspline.n_spans(p, n)
    M, K, D1, _ = colloc.colloc_factors(p, n)
    i = n // 2
    assert np.allclose(M[i, i - 1:i + 2], g["cubic_value"], atol=1e-15)
    assert np.allclose(D1[i, i - 1:i + 2] / E, g["cubic_d1"], atol=1e-13)
    assert np.allclose(-K[i, i - 1:i + 2] / E ** 2, g["cubic_d2"], atol=1e-11)
    # quadratic: Greville points are span midpoints
    p, n = 2, 20
    E = bspline.n_spans(p, n)
    M, K, D1, _ = colloc.colloc_factors(p, n)
    assert np.allclose(M[i, i - 1:i + 2], g["quadratic_value"], atol=1e-15)
    assert np.allclose(-K[i, i - 1:i + 2] / E ** 2, g["quadratic_d2"], atol=1e-11)
    assert np.allclose(M[0, 0:2], g["quadratic_value_first_row"], atol=1e-15)


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6])
def test_support_count_at_greville_points(p):
    """A point inside a span meets p+1 non-zero B-splines, a simple knot p (for p >= 2)."""
    n = 40
    M, K, D1, tau = colloc.colloc_factors(p, n)
    nnz = (M != 0).sum(axis=1)
    nnzK = (K != 0).sum(axis=1)
    interior = slice(p + 1, n - p - 1)
    expect = p if p % 2 == 1 else p + 1       # odd p: Greville points of interior functions are knots
    assert np.all(nnz[interior] == expect)
    assert np.all(nnzK[interior] <= expect)
    assert np.all(nnz <= p + 1)


def test_greville_exact_knots_for_odd_degree():
    p, n = 3, 33
    E = bspline.n_spans(p, n)
    tau = bspline.greville(p, n)
    xi = bspline.knots(p, E)
    interior_knots = set(xi[p + 1:-p - 1].tolist())
    hits = sum(t in interior_knots for t in tau)
    assert hits == n - 2          # all but the two boundary-adjacent points sit exactly on knots
