"""Pins of the oracle's reduced-precision FD solve (oracle/reduced.py) against what does
not depend on it: the BF16 format's definition (a textbook round-half-even written with
frexp), torch's FP32 -> BF16 conversion (library routine), exact integer arithmetic, the
FP64 FD solve, and planted mistakes that the GPU parity tolerances must catch."""
import math

import numpy as np
import pytest

from oracle import colloc, fd, reduced
from paper_1705_04384_amd import inputs


def _bf16_textbook(x):
    """Nearest value with an 8-bit significand, ties to even, by frexp and Python's
    round-half-even on the exactly scaled significand."""
    out = np.empty(len(x))
    for i, v in enumerate(np.asarray(x, dtype=np.float64)):
        if v == 0.0:
            out[i] = v
            continue
        m, e = math.frexp(v)                  # v = m 2^e, 0.5 <= |m| < 1
        out[i] = math.ldexp(round(m * 256.0), e - 8)   # exact scaling; round() is half-even
    return out


def test_bf16_from_fp64_is_the_textbook_rounding():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 255.5, 256.5, 257.0,
                                  1.0 + 2.0 ** -8 + 2.0 ** -40, 1.0 + 2.0 ** -8 - 2.0 ** -40, 0.0, -0.0])])
    got = reduced.bf16_from_fp64(x).astype(np.float64)
    assert np.array_equal(got, _bf16_textbook(x))
    # ties go to even; just above a tie rounds up, where FP64 -> FP32 -> BF16 would not
    assert got[-10] == 1.0 and got[-9] == 1.0 + 2.0 ** -6 and got[-8] == -1.0
    assert got[-4] == 1.0 + 2.0 ** -7 and got[-3] == 1.0
    assert reduced.bf16_from_fp32(np.float32(1.0 + 2.0 ** -8 + 2.0 ** -40)) == 1.0   # the double rounding


def test_bf16_from_fp32_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    x = (rng.standard_normal(50000) * 10.0 ** rng.integers(-20, 20, 50000)).astype(np.float32)
    x = np.concatenate([x, np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 3.0e38], dtype=np.float32)])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(reduced.bf16_from_fp32(x), want)


@pytest.mark.parametrize("d,n", [(2, 9), (3, 7)])
@pytest.mark.parametrize("mode", ["fp32", "bf16"])
def test_identity_factors_round_the_input_once(d, n, mode):
    """U = V = I, lambda = (1, 1, 2): every product is exact, so the result is the input
    rounded once to the mode's precision and divided by Lambda (= 2 in 2D, 4 in 3D)."""
    b = inputs.rhs_normal(11, n ** d) * 3.0
    I = np.eye(n)
    lams = [np.ones(n), np.ones(n), 2.0 * np.ones(n)][:d]
    got = reduced.fd_apply_reduced([I] * d, [I] * d, lams, b, mode)
    lam_sum = 4.0 if d == 3 else 2.0
    want = (_bf16_textbook(b) if mode == "bf16" else b.astype(np.float32).astype(np.float64)) / lam_sum
    assert np.array_equal(got, want)


def _ternary_problem(d, n, seed):
    rng = np.random.default_rng(seed)
    Us = [rng.choice([-1.0, 0.0, 0.0, 1.0], size=(n, n)) for _ in range(d)]
    Vs = [rng.choice([-1.0, 0.0, 0.0, 1.0], size=(n, n)) for _ in range(d)]
    lams = [np.ones(n), np.ones(n), 2.0 * np.ones(n)][:d]
    b = rng.integers(-3, 4, size=n ** d).astype(np.float64)
    return Us, Vs, lams, b


def _exact_chain(Us, Vs, lams, b, rnd):
    """The same chain in exact arithmetic (small integers and quarters, exact in FP64),
    each product input passed through rnd, written with the oracle's FP64 mode product."""
    d = len(Us)
    n = len(lams[0])
    X = b.reshape([n] * d)
    for l in range(d):
        X = fd.mode_product(rnd(X), Vs[l].T, l + 1)
    X = X / (4.0 if d == 3 else 2.0)
    for l in reduced.u_order(d):
        X = fd.mode_product(rnd(X), Us[l - 1], l)
        assert np.max(np.abs(X)) < 2.0 ** 22          # still exact in FP32
    return X.ravel()


@pytest.mark.parametrize("d,n", [(2, 40), (3, 17)])
def test_integer_chain_is_exact(d, n):
    """Ternary factors, integer input, lambda (1, 1, 2): FP32 accumulation is exact, so
    the FP32 mode equals exact arithmetic, and the BF16 mode equals exact arithmetic with
    every product input rounded to 8 significant bits (intermediates outgrow 256)."""
    Us, Vs, lams, b = _ternary_problem(d, n, 21)
    assert np.array_equal(reduced.fd_apply_reduced(Us, Vs, lams, b, "fp32"), _exact_chain(Us, Vs, lams, b, lambda X: X))
    bf = reduced.fd_apply_reduced(Us, Vs, lams, b, "bf16")
    want = _exact_chain(Us, Vs, lams, b, lambda X: _bf16_textbook(X.ravel()).reshape(X.shape))
    assert np.array_equal(bf, want)
    assert not np.array_equal(bf, _exact_chain(Us, Vs, lams, b, lambda X: X))


def _real_problem(d, p, n, seed=7):
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    return [U] * d, [V] * d, [lam] * d, inputs.rhs_normal(seed, n ** d)


@pytest.mark.parametrize("d,p,n", [(3, 3, 33), (2, 4, 130), (3, 6, 24)])
def test_reduced_modes_approach_the_fp64_solve(d, p, n):
    """FP32 lands at the FP32 rounding level of the FP64 solve, BF16 at the BF16 level:
    about 2^-24 and 2^-9 times the conditioning of the chain."""
    Us, Vs, lams, b = _real_problem(d, p, n)
    s64 = fd.fd_apply(Us, Vs, lams, b)
    e32 = np.linalg.norm(reduced.fd_apply_reduced(Us, Vs, lams, b, "fp32") - s64) / np.linalg.norm(s64)
    e16 = np.linalg.norm(reduced.fd_apply_reduced(Us, Vs, lams, b, "bf16") - s64) / np.linalg.norm(s64)
    assert 1e-9 < e32 < 1e-5
    assert 1e-4 < e16 < 5e-2
    assert e16 > 100 * e32


# Tolerances of the GPU comparison of the reduced-precision kernels with this oracle
# (tests/test_gpu_reduced.py): max-abs and 2-norm distance relative to the oracle result.
GPU_TOL = {"fp32": (2e-5, 5e-6), "bf16": (4e-3, 1.5e-3)}


@pytest.mark.parametrize("d,p,n", [(3, 3, 33), (3, 6, 65), (2, 4, 130), (2, 3, 47)])
def test_gpu_tolerances_catch_planted_mistakes(d, p, n):
    """A valid implementation may accumulate in another order; that changes the result by
    FP32 accumulation error plus, in BF16, the rare product input whose BF16 rounding
    flips.  Emulated here by FP32 (not exact) sums: it stays inside the GPU tolerances.
    Planted mistakes must not: a dropped last term of every contraction (the last k-block
    at n = 33 is one term), a BF16 chain computed in FP32, and the U products in another
    order (the last two are also caught bit for bit by the integer-chain GPU test)."""
    Us, Vs, lams, b = _real_problem(d, p, n)
    ref = {m: reduced.fd_apply_reduced(Us, Vs, lams, b, m) for m in ("fp32", "bf16")}

    def dist(a, r):
        return np.max(np.abs(a - r)) / np.max(np.abs(r)), np.linalg.norm(a - r) / np.linalg.norm(r)

    orig = reduced._mode_product_fp32

    def fp32_sums(X, W, l):
        axis = X.ndim - l
        return np.moveaxis(np.tensordot(W.astype(np.float32), X.astype(np.float32), axes=([1], [axis])), 0, axis)

    def dropped_last(X, W, l):
        W = W.copy()
        W[:, -1] = 0.0
        return orig(X, W, l)

    try:
        reduced._mode_product_fp32 = fp32_sums
        for m in ("fp32", "bf16"):
            mx, nm = dist(reduced.fd_apply_reduced(Us, Vs, lams, b, m), ref[m])
            assert mx <= GPU_TOL[m][0] / 2 and nm <= GPU_TOL[m][1] / 2, (m, mx, nm)
        reduced._mode_product_fp32 = dropped_last
        for m in ("fp32", "bf16"):
            mx, nm = dist(reduced.fd_apply_reduced(Us, Vs, lams, b, m), ref[m])
            assert mx > 3 * GPU_TOL[m][0] and nm > 3 * GPU_TOL[m][1], (m, mx, nm)
    finally:
        reduced._mode_product_fp32 = orig
    mx, nm = dist(ref["fp32"], ref["bf16"])                 # BF16 kernel that skipped the BF16 roundings
    assert nm > 1.8 * GPU_TOL["bf16"][1], (mx, nm)
    if d == 3:
        orig_order = reduced.u_order
        try:
            reduced.u_order = lambda dd: [1, 2, 3]
            mx, nm = dist(reduced.fd_apply_reduced(Us, Vs, lams, b, "bf16"), ref["bf16"])
            assert nm > 1.8 * GPU_TOL["bf16"][1], (mx, nm)
        finally:
            reduced.u_order = orig_order


@pytest.mark.parametrize("d,p,n", [(3, 6, 24), (2, 6, 96)])
def test_column_balancing_leaves_the_bf16_error(d, p, n):
    """The FD is invariant under U_l -> U_l S^-1, V_l -> V_l S for diagonal S, so the
    columns of U and V could be balanced before the BF16 rounding.  BF16 keeps FP32's
    exponent range and rounds each value relative to its own magnitude, so balancing does
    not lower the BF16 error of the apply (it moves it by -10% to +30% here, while the
    columns of V span a factor of about 10 in 2-norm): it cannot cut the BF16 iteration
    count."""
    Us, Vs, lams, b = _real_problem(d, p, n)
    U, V, lam = Us[0], Vs[0], lams[0]
    s64 = fd.fd_apply(Us, Vs, lams, b)
    e0 = np.linalg.norm(reduced.fd_apply_reduced(Us, Vs, lams, b, "bf16") - s64) / np.linalg.norm(s64)
    for sc in (1.0 / np.linalg.norm(V, axis=0), np.sqrt(np.linalg.norm(U, axis=0) / np.linalg.norm(V, axis=0))):
        Ub, Vb = U / sc, V * sc
        assert np.linalg.norm(fd.fd_apply([Ub] * d, [Vb] * d, lams, b) - s64) <= 1e-13 * np.linalg.norm(s64)
        e = np.linalg.norm(reduced.fd_apply_reduced([Ub] * d, [Vb] * d, lams, b, "bf16") - s64) / np.linalg.norm(s64)
        assert 0.9 * e0 <= e <= 1.5 * e0, (e, e0)
