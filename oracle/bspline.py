"""Univariate B-splines for the oracle (test infrastructure only; see package header).

Follows Sec. 2.1 (open knot vectors with p+1 repeated end knots, interior
knots of multiplicity one for maximal C^{p-1} regularity; basis functions
B_i, i = 0..m-1; interior functions i = 1..m-2 span the Dirichlet space of
eq. 2.3, so n = m - 2) and Sec. 2.2, eq. 2.4 (Greville abscissae).

Readings where the paper is silent:
* The uniform open knot vector with E spans has the interior knots k/E; they are
  kept as integer numerators so the Greville points are one rational division
  (for odd p the interior Greville points then coincide exactly with knots).
* "n unknowns per direction" fixes E = n + 2 - p.
* Spans are half-open [xi_k, xi_{k+1}), the last non-empty span is closed at 1.
"""
import numpy as np


def n_spans(p, n):
    """Number of uniform knot spans E for degree p and n interior unknowns.

    From m = E + p basis functions (Sec. 2.1) and n = m - 2 (eq. 2.3)."""
    E = n + 2 - p
    if p < 1 or E < 1:
        raise ValueError("need p >= 1 and n >= p - 1")
    return E


def knot_numerators(p, E):
    """Integer numerators k_j of the open uniform knot vector xi_j = k_j / E.

    Sec. 2.1: p+1 knots at 0, the interior knots once each, p+1 knots at 1;
    m + p + 1 = E + 2p + 1 knots in total."""
    return np.concatenate([np.zeros(p + 1, dtype=np.int64),
                           np.arange(1, E, dtype=np.int64),
                           np.full(p + 1, E, dtype=np.int64)])


def knots(p, E):
    """The open uniform knot vector as floats (each entry k_j / E correctly rounded)."""
    return knot_numerators(p, E).astype(np.float64) / float(E)


def greville(p, n):
    """Greville abscissae tau_i, i = 1..n, of the interior basis functions (eq. 2.4).

    With the paper's 1-based knot indices, tau_i is the mean of xi_{i+2}..xi_{i+p+1};
    in 0-based storage that is entries i+1..i+p.  The p numerators are summed as
    integers and divided once by p*E."""
    E = n_spans(p, n)
    k = knot_numerators(p, E)
    tau = np.empty(n, dtype=np.float64)
    for i in range(1, n + 1):
        tau[i - 1] = float(k[i + 1:i + p + 1].sum()) / float(p * E)
    return tau


def greville_all(p, E):
    """Greville abscissae of all m = E + p basis functions (used by the linear-precision pin)."""
    k = knot_numerators(p, E)
    m = E + p
    return np.array([float(k[i + 1:i + p + 1].sum()) / float(p * E) for i in range(m)])


def basis_derivs(xi, p, x, nder=2):
    """Values and derivatives of every B-spline of degree p on knot vector xi at points x.

    Returns an array D of shape (nder+1, m, len(x)) with D[r, j, q] = B_j^{(r)}(x_q),
    m = len(xi) - p - 1.  Cox-de Boor recursion
        B_{j,0}(x) = 1 on [xi_j, xi_{j+1}) (last non-empty span closed at its right end),
        B_{j,q} = (x - xi_j)/(xi_{j+q} - xi_j) B_{j,q-1} + (xi_{j+q+1} - x)/(xi_{j+q+1} - xi_{j+1}) B_{j+1,q-1},
    and the derivative rule
        B_{j,q}^{(r)} = q/(xi_{j+q} - xi_j) B_{j,q-1}^{(r-1)} - q/(xi_{j+q+1} - xi_{j+1}) B_{j+1,q-1}^{(r-1)},
    with every 0/0 quotient read as 0 (repeated knots)."""
    xi = np.asarray(xi, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    L = len(xi)
    m = L - p - 1
    # degree-0 indicators, one per knot interval
    b0 = np.zeros((L - 1, len(x)))
    for j in range(L - 1):
        if xi[j] < xi[j + 1]:
            b0[j] = (xi[j] <= x) & (x < xi[j + 1])
    last = max(j for j in range(L - 1) if xi[j] < xi[j + 1])
    b0[last] = np.where(x == xi[last + 1], 1.0, b0[last])

    def ratio(num, den):
        return num / den if den != 0.0 else 0.0 * num

    # vals[q] has L-1-q rows: all B_{j,q}
    vals = [b0]
    for q in range(1, p + 1):
        prev = vals[-1]
        cur = np.zeros((L - 1 - q, len(x)))
        for j in range(L - 1 - q):
            cur[j] = (ratio(x - xi[j], xi[j + q] - xi[j]) * prev[j]
                      + ratio(xi[j + q + 1] - x, xi[j + q + 1] - xi[j + 1]) * prev[j + 1])
        vals.append(cur)
    # der[r][q]: r-th derivative of all B_{j,q}
    der = [vals]
    for r in range(1, nder + 1):
        lower = der[r - 1]
        cur_r = [None] * (p + 1)
        for q in range(r, p + 1):
            prev = lower[q - 1]
            cur = np.zeros((L - 1 - q, len(x)))
            for j in range(L - 1 - q):
                a = xi[j + q] - xi[j]
                c = xi[j + q + 1] - xi[j + 1]
                t = np.zeros(len(x))
                if a != 0.0:
                    t = t + (q / a) * prev[j]
                if c != 0.0:
                    t = t - (q / c) * prev[j + 1]
                cur[j] = t
            cur_r[q] = cur
        for q in range(0, r):
            cur_r[q] = np.zeros((L - 1 - q, len(x)))
        der.append(cur_r)
    out = np.zeros((nder + 1, m, len(x)))
    for r in range(nder + 1):
        out[r] = der[r][p][:m]
    return out
