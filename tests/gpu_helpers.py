"""Shared helpers of the GPU tests: device selection and oracle-side problem builders."""
import numpy as np

from oracle import colloc, fd


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def to_dev(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def oracle_unit(p, n, d):
    """Oracle factors and operator for the unit-domain problem."""
    M, K, D1, tau = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    P = colloc.unit_operator([M] * d, [K] * d)
    prec = lambda v: fd.fd_apply([U] * d, [V] * d, [lam] * d, v)
    return P, prec


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def maxrel(a, b):
    """Largest element-wise difference relative to the largest element of b."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
