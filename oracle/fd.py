"""Fast-diagonalization solve for the oracle (test infrastructure only; see package header).

Sec. 4: the preconditioning system P s = b (eq. 4.1) with P a Kronecker sum of
univariate pencils (K_l, M_l).  The nonsymmetric FD method takes the
eigendecomposition M_l^{-1} K_l U_l = U_l D_l (eq. 4.6), sets
V_l = (M_l U_l)^{-T}, and applies
    s = (U_d x ... x U_1) (sum_l I x D_l x I)^{-1} (V_d x ... x V_1)^T b
(eq. 4.7 for d = 2, eq. 4.9 for d = 3).

Readings where the paper is silent:
* Eigenvalues must be real (Remark 1 assumes it); the oracle rejects a pencil
  whose eigenvalues have an imaginary part above 1e-10 of the largest modulus or
  a non-positive real part (the block-diagonal complex variant is not built).
* Column scaling and order of U are free (they cancel in the product); the
  oracle sorts eigenvalues ascending and scales each column of U to unit 2-norm.
"""
import numpy as np
import scipy.linalg as sla


class ComplexPencilError(ValueError):
    """The pencil has non-real or non-positive eigenvalues (outside Remark 1's assumption)."""


def factor_pencil(K, M, allow_complex=False):
    """U, V, lam for the pencil (K, M): K U = M U diag(lam), V = (M U)^{-T} (eq. 4.6 and the line after it).

    With allow_complex, a pencil with complex-conjugate eigenvalue pairs is accepted
    (Sec. 4 after eq. 4.7: the decomposition then needs complex arithmetic, or 2 x 2
    real blocks in D); U, V and lam are returned complex, ordered by real part, and every
    real part must be positive."""
    lam, U = sla.eig(K, M)
    scale = np.max(np.abs(lam))
    is_complex = np.max(np.abs(lam.imag)) > 1e-10 * scale
    if is_complex and not allow_complex:
        raise ComplexPencilError("pencil has complex eigenvalues")
    if np.min(lam.real) <= 0.0:
        raise ComplexPencilError("pencil has eigenvalues with non-positive real part")
    if is_complex:
        order = np.lexsort((lam.imag, lam.real))
        U = U[:, order]
        U = U / np.linalg.norm(U, axis=0)
        return U, np.linalg.inv(M @ U).T, lam[order]
    lam = lam.real
    U = U.real
    order = np.argsort(lam, kind="stable")
    lam = lam[order]
    U = U[:, order]
    U = _cluster_eigenvectors(K, M, lam, U)
    U = U / np.linalg.norm(U, axis=0)
    V = np.linalg.inv(M @ U).T
    return U, V, lam


def _cluster_eigenvectors(K, M, lam, U, rel=1e-10):
    """Eigenvectors for clusters of (numerically) equal eigenvalues.

    Remark 1 notes an outlier eigenvalue of algebraic multiplicity two and assumes the
    pencil is diagonalizable; the two outlier modes live at opposite ends of the
    interval and their eigenvalues agree to rounding once n is moderate, where the
    QZ eigenvector step may return one vector twice.  For each cluster of eigenvalues
    within rel * max|lam| of each other, the columns are replaced by an orthonormal
    basis of the cluster's invariant subspace of M^{-1} K (ordered real Schur form),
    combined by the eigenvectors of the cluster's Schur block unless that block is a
    multiple of the identity to rounding.  Pairs that are merely close (the gap well
    above rounding) keep their QZ eigenvectors, which are accurate there.  A cluster whose block is far from diagonalizable is
    rejected."""
    tol = rel * np.max(np.abs(lam))
    n = len(lam)
    i = 0
    A = None
    while i < n:
        j = i + 1
        while j < n and lam[j] - lam[j - 1] <= tol:
            j += 1
        k = j - i
        if k > 1:
            if A is None:
                A = np.linalg.solve(M, K)
            lo, hi = lam[i] - tol, lam[j - 1] + tol
            T, Z, sdim = sla.schur(A, output="real", sort=lambda re, im: (re >= lo) & (re <= hi))
            if sdim != k:
                raise ComplexPencilError("eigenvalue cluster not separable")
            T11 = T[:k, :k]
            spread = np.abs(T11 - np.mean(np.diag(T11)) * np.eye(k)).max()
            if spread <= 1e-12 * np.abs(lam[i]):        # a scalar block to rounding
                W = np.eye(k)
            else:
                w, W = np.linalg.eig(T11)
                if np.max(np.abs(w.imag)) > 0 or np.linalg.cond(W) > 1e8:
                    raise ComplexPencilError("eigenvalue cluster is not diagonalizable")
                W = W[:, np.argsort(w.real)].real
            U[:, i:j] = Z[:, :k] @ W
        i = j
    return U


def mode_product(X, A, l):
    """X x_l A for a tensor X of shape (n_d, ..., n_1): Y[.., k, ..] = sum_j A[k, j] X[.., j, ..]
    along direction l (1-based; direction 1 is the last, fastest axis)."""
    axis = X.ndim - l
    Y = np.tensordot(A, X, axes=([1], [axis]))        # new axis 0
    return np.moveaxis(Y, 0, axis)


def eig_sum(lams):
    """Lambda[i_d, ..., i_1] = sum_l lam_l[i_l], the diagonal of sum_l I x D_l x I."""
    d = len(lams)
    out = np.zeros([len(lams[l]) for l in reversed(range(d))])
    for l in range(d):
        shape = [1] * d
        shape[d - 1 - l] = len(lams[l])
        out = out + lams[l].reshape(shape)
    return out


def fd_apply(Us, Vs, lams, b):
    """s = P^{-1} b by eq. 4.7 / 4.9.  Us, Vs, lams are per direction l = 1..d; b is i_1-fastest.
    With complex factors (conjugate-closed spectra) the arithmetic is complex and the
    result, real up to rounding, is returned as its real part."""
    d = len(Us)
    shape = [len(lams[l]) for l in reversed(range(d))]
    X = np.asarray(b, dtype=np.float64).reshape(shape)
    for l in range(d):                              # (V_d x ... x V_1)^T b
        X = mode_product(X, Vs[l].T, l + 1)
    X = X / eig_sum(lams)                           # diagonal solve
    for l in range(d):                              # (U_d x ... x U_1) s~
        X = mode_product(X, Us[l], l + 1)
    if np.iscomplexobj(X):
        X = X.real
    return X.ravel()


def fd_flops(d, n):
    """Algorithmic flop count of one apply: 2d mode products of 2 n^{d+1} flops each
    (Sec. 4.1: 8 n^3 in 2D, 12 n^4 in 3D)."""
    return 4 * d * n ** (d + 1)
