"""Seeded synthetic inputs shared by the library's callers and its checkers.

This module draws random numbers only; it holds none of the solver's arithmetic.
Vectors are flat float64 arrays in the i_1-fastest unknown order.
"""
import numpy as np

SEED_NOISE_128 = 1      # 3D p=4, 128^3 unit cube, N(0,1) right-hand side
SEED_DEFORMED_96 = 2    # 3D p=3, 96^3 deformed cube, U[-1,1] right-hand side
SEED_SWEEP_192 = 3      # 3D p=6, 192^3 unit cube, N(0,1) right-hand side
SEED_ARRIVALS = 7       # serving arrival process
SEED_REQUEST_BASE = 1000  # serving request r draws from seed 1000 + r


def rhs_normal(seed, N):
    """N(0, 1) right-hand side of length N."""
    return np.random.default_rng(seed).standard_normal(N)


def rhs_uniform(seed, N):
    """U[-1, 1] right-hand side of length N."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, N)


def serving_requests(count, rate_per_s, seed=SEED_ARRIVALS):
    """A Poisson arrival stream of solve requests with a mixed shape distribution.

    Returns a list of dicts (arrival time in seconds, d, p, n, rhs seed):
    d in {2, 3} with equal probability, p uniform in {2..6}, n uniform in
    [32, 256] for d = 2 and in [16, 128] for d = 3 (n counts unknowns per
    direction, so every request has E = n + 2 - p >= 12 knot spans).  The
    shapes do not depend on the rate: the gaps are unit-rate draws scaled by it."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(count):
        d = int(rng.integers(2, 4))
        p = int(rng.integers(2, 7))
        lo, hi = (32, 256) if d == 2 else (16, 128)
        n = int(rng.integers(lo, hi + 1))
        out.append(dict(id=r, t=float(t[r]), d=d, p=p, n=n, seed=SEED_REQUEST_BASE + r))
    return out
