"""Collocation matrices for the oracle (test infrastructure only; see package header).

Sec. 2.2: collocation of -div(K grad u) = f (eq. 2.1, K = I as in all the
paper's experiments, Sec. 5) at the Greville points (eq. 2.4); unknowns are
ordered with i_1 fastest (Sec. 2.1, after eq. 2.3).  On the unit domain the
matrix is the Kronecker sum of eq. 2.7 (2D) / eq. 2.9 (3D) with the univariate
factors of eq. 2.8.  On a deformed domain the paper does not print the matrix
(Sec. 2.2 says only that it is complicated); it is derived here from the chain
rule for u = u_hat o F^{-1}:

    -Lap_x u = -sum_{k,l} C_kl d_k d_l u_hat - sum_k g_k d_k u_hat,
    C = J^{-1} J^{-T},   g_k = -sum_a (J^{-1})_{ka} sum_{l,m} (d_l d_m F_a) C_lm,

with J the Jacobian of F, all evaluated at the parametric collocation point.
"""
import numpy as np
import scipy.sparse as sp

from . import bspline


def colloc_factors(p, n):
    """Univariate collocation factors on the uniform open knot vector (eq. 2.8).

    Returns (M, K, D1, tau): (M)_{ij} = B_j(tau_i), (K)_{ij} = -B''_j(tau_i),
    (D1)_{ij} = B'_j(tau_i), for interior functions j = 1..n and Greville
    points tau_i, i = 1..n (eq. 2.3 drops B_0 and B_{m-1})."""
    E = bspline.n_spans(p, n)
    xi = bspline.knots(p, E)
    tau = bspline.greville(p, n)
    D = bspline.basis_derivs(xi, p, tau, nder=2)      # (3, m, n): D[r, j, i] = B_j^{(r)}(tau_i)
    M = D[0, 1:n + 1, :].T.copy()
    D1 = D[1, 1:n + 1, :].T.copy()
    K = -D[2, 1:n + 1, :].T.copy()
    return M, K, D1, tau


def kron_chain(mats):
    """Kronecker product F_d x ... x F_1 given mats = [F_1, ..., F_d] (F_1 acts on i_1, the fastest index)."""
    out = sp.csr_matrix(mats[-1])
    for F in reversed(mats[:-1]):
        out = sp.kron(out, sp.csr_matrix(F), format="csr")
    return out


def unit_operator(Ms, Ks):
    """Unit-domain collocation operator as a sparse matrix.

    eq. 2.7 (d = 2): K_2 x M_1 + M_2 x K_1;  eq. 2.9 (d = 3): K_3 x M_2 x M_1 +
    M_3 x K_2 x M_1 + M_3 x M_2 x K_1.  Ms, Ks list the factors by direction
    l = 1..d.  The same formula is the preconditioner P (Sec. 3: the same
    discretization on the unit cube)."""
    d = len(Ms)
    A = None
    for l in range(d):
        mats = [Ks[q] if q == l else Ms[q] for q in range(d)]
        T = kron_chain(mats)
        A = T if A is None else A + T
    return A.tocsr()


def unit_matvec(Ms, Ks, x):
    """y = P x for the unit-domain operator of eq. 2.7 / 2.9 without forming P: each
    Kronecker term is applied as one mode product per direction (dense factors)."""
    d = len(Ms)
    shape = [Ms[l].shape[0] for l in reversed(range(d))]
    X = np.asarray(x, dtype=np.float64).reshape(shape)
    Y = np.zeros_like(X)
    for l in range(d):
        T = X
        for q in range(d):
            F = Ks[q] if q == l else Ms[q]
            axis = d - 1 - q
            T = np.moveaxis(np.tensordot(F, T, axes=([1], [axis])), 0, axis)
        Y = Y + T
    return Y.ravel()


def tensor_grid(vals_by_dir):
    """Tensor of shape (n_d, ..., n_1) holding the listed per-direction 1D arrays,
    returned as a list of d arrays (coordinate l+1 broadcast over the grid); flattening
    in C order gives the paper's i_1-fastest numbering."""
    d = len(vals_by_dir)
    grids = np.meshgrid(*reversed(vals_by_dir), indexing="ij")   # axes (i_d, ..., i_1)
    return [grids[d - 1 - l] for l in range(d)]


def manufactured_rhs(p, n, d):
    """Right-hand side f(tau) for u = prod_l sin(pi x_l) on the unit domain.

    -Lap u = d pi^2 u, evaluated at the tensor Greville grid (eq. 2.6), i_1 fastest."""
    tau = bspline.greville(p, n)
    coords = tensor_grid([tau] * d)
    u = np.ones_like(coords[0])
    for c in coords:
        u = u * np.sin(np.pi * c)
    return (d * np.pi ** 2 * u).ravel()


# ---------------------------------------------------------------------------
# Deformed cube
# ---------------------------------------------------------------------------

def deform_map(amp):
    """The smooth map F(xi)_a = xi_a + amp sin(2 pi xi_{a+1}) sin(2 pi xi_{a+2}) (indices cyclic mod 3).

    Returns callables (F, J, H) on arrays xi of shape (..., 3):
      F -> (..., 3), J -> (..., 3, 3) with J[a, b] = dF_a/dxi_b,
      H -> (..., 3, 3, 3) with H[a, k, l] = d^2 F_a / dxi_k dxi_l."""
    w = 2.0 * np.pi

    def F(xi):
        out = np.array(xi, dtype=np.float64, copy=True)
        for a in range(3):
            b1, b2 = (a + 1) % 3, (a + 2) % 3
            out[..., a] += amp * np.sin(w * xi[..., b1]) * np.sin(w * xi[..., b2])
        return out

    def J(xi):
        out = np.zeros(xi.shape[:-1] + (3, 3))
        for a in range(3):
            b1, b2 = (a + 1) % 3, (a + 2) % 3
            out[..., a, a] = 1.0
            out[..., a, b1] = amp * w * np.cos(w * xi[..., b1]) * np.sin(w * xi[..., b2])
            out[..., a, b2] = amp * w * np.sin(w * xi[..., b1]) * np.cos(w * xi[..., b2])
        return out

    def H(xi):
        out = np.zeros(xi.shape[:-1] + (3, 3, 3))
        for a in range(3):
            b1, b2 = (a + 1) % 3, (a + 2) % 3
            ss = np.sin(w * xi[..., b1]) * np.sin(w * xi[..., b2])
            cc = np.cos(w * xi[..., b1]) * np.cos(w * xi[..., b2])
            out[..., a, b1, b1] = -amp * w * w * ss
            out[..., a, b2, b2] = -amp * w * w * ss
            out[..., a, b1, b2] = amp * w * w * cc
            out[..., a, b2, b1] = amp * w * w * cc
        return out

    return F, J, H


def deformed_coefficients(xi, amp):
    """Chain-rule coefficients of -Lap_x at parametric points xi (..., 3).

    Returns (C, g): C (..., 3, 3) = J^{-1} J^{-T} and
    g (..., 3) = -J^{-1} [sum_{l,m} H[:, l, m] C_lm]  (see module docstring)."""
    _, J, H = deform_map(amp)
    Jx = J(xi)
    Ji = np.linalg.inv(Jx)
    C = Ji @ np.swapaxes(Ji, -1, -2)
    Hx = H(xi)
    t = np.einsum("...alm,...lm->...a", Hx, C)
    g = -np.einsum("...ka,...a->...k", Ji, t)
    return C, g


def deformed_operator(p, n, amp):
    """Collocation matrix of -Lap on the deformed cube F([0,1]^3), CSR, i_1 fastest.

    Row i (collocation point tau_i) of A is
        -sum_{k,l} C_kl(tau_i) d_k d_l B_j(tau_i) - sum_k g_k(tau_i) d_k B_j(tau_i),
    and every term is a diagonal scaling of a Kronecker product of the 1D
    matrices {M, D1, -K} of eq. 2.8 (derivative order per direction).
    With amp = 0 this is eq. 2.9."""
    M, K, D1, tau = colloc_factors(p, n)
    by_order = [M, D1, -K]
    coords = tensor_grid([tau] * 3)
    xi = np.stack([c.ravel() for c in coords], axis=-1)          # (N, 3), row = collocation point
    C, g = deformed_coefficients(xi, amp)
    N = n ** 3
    A = sp.csr_matrix((N, N))
    for k in range(3):
        for l in range(3):
            orders = [int(q == k) + int(q == l) for q in range(3)]
            T = kron_chain([by_order[orders[q]] for q in range(3)])
            A = A - sp.diags(C[:, k, l]) @ T
    for k in range(3):
        orders = [int(q == k) for q in range(3)]
        T = kron_chain([by_order[orders[q]] for q in range(3)])
        A = A - sp.diags(g[:, k]) @ T
    A = A.tocsr()
    A.eliminate_zeros()
    A.sort_indices()
    return A


def deformed_manufactured_rhs(p, n, amp):
    """f at F(tau_i) for the exact solution u = u_hat o F^{-1}, u_hat = prod_l sin(pi xi_l).

    f = -Lap_x u, written with the same chain rule and the exact derivatives of u_hat."""
    tau = bspline.greville(p, n)
    coords = tensor_grid([tau] * 3)
    xi = np.stack([c.ravel() for c in coords], axis=-1)
    C, g = deformed_coefficients(xi, amp)
    s = np.sin(np.pi * xi)
    c = np.cos(np.pi * xi)
    grad = np.zeros_like(xi)
    hess = np.zeros(xi.shape + (3,))
    for k in range(3):
        o1, o2 = [q for q in range(3) if q != k]
        grad[:, k] = np.pi * c[:, k] * s[:, o1] * s[:, o2]
        hess[:, k, k] = -np.pi ** 2 * s[:, 0] * s[:, 1] * s[:, 2]
    for k in range(3):
        for l in range(3):
            if k != l:
                o = 3 - k - l
                hess[:, k, l] = np.pi ** 2 * c[:, k] * c[:, l] * s[:, o]
    return -(np.einsum("nkl,nkl->n", C, hess) + np.einsum("nk,nk->n", g, grad))
