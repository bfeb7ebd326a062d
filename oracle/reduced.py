"""Reduced-precision fast-diagonalization solve for the oracle (test infrastructure only;
see the package header).

The paper computes in FP64 throughout and states no reduced-precision variant.  The
preconditioner P^{-1} of eq. 4.7 / 4.9 is a chain of mode products (Sec. 4.1 counts them
as separate BLAS-3 calls) around a diagonal solve, and a flexible Krylov method accepts
an inexact P^{-1}; this module defines that inexact P^{-1} exactly, so that a
reduced-precision implementation can be compared with it element by element.  Readings
(the paper is silent on all of them):

* Factors W = V_l^T and U_l are rounded once from FP64, to nearest even, to FP32 ("fp32")
  or BF16 ("bf16"); the eigenvalues are rounded to FP32 in both modes.
* Every mode-product input is rounded from its stored precision to the mode's input
  precision, to nearest even, once: FP64 -> FP32 in "fp32"; FP64 -> BF16 and FP32 -> BF16
  in "bf16" (a direct rounding, never FP64 -> FP32 -> BF16).
* Products accumulate in FP32: each mode product's output is the FP32 rounding of the
  exact sum of the exact products of its rounded inputs (the most accurate FP32
  accumulation; an implementation that accumulates in another order differs from it by
  at most the FP32 accumulation error of that sum).
* The diagonal solve divides in FP32 by Lambda = fl32(lam_3 + fl32(lam_2 + lam_1))
  (d = 3) or fl32(lam_2 + lam_1) (d = 2), rounded to FP32.
* Order of the products (where the roundings fall): the V^T products in directions
  1, 2, (3); after the divide the U products in directions 3, 1, 2 for d = 3 and 1, 2
  for d = 2.
* The output is the last product's FP32 result, widened to FP64.
"""
import numpy as np

_SHIFT64 = np.uint64(45)            # 52 - 7 fraction bits dropped from FP64 to BF16
_HALF64 = np.uint64((1 << 44) - 1)
_MASK64 = ~np.uint64((1 << 45) - 1)


def bf16_from_fp64(x):
    """FP64 -> BF16, round to nearest (ties to even), one rounding; returned as float32
    (every BF16 value is an FP32 value).  Finite inputs in the FP32 normal range."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    u = x.view(np.uint64).copy()
    u += _HALF64 + ((u >> _SHIFT64) & np.uint64(1))
    u &= _MASK64
    return u.view(np.float64).astype(np.float32)      # exact: 8 significant bits


def bf16_from_fp32(x):
    """FP32 -> BF16, round to nearest (ties to even); returned as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).copy()
    u += np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))
    u &= np.uint32(0xFFFF0000)
    return u.view(np.float32)


def fp32_from_fp64(x):
    """FP64 -> FP32, round to nearest (ties to even)."""
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def round_input(x, mode):
    """A mode-product input rounded to the mode's input precision (FP32 values)."""
    if mode == "fp32":
        return fp32_from_fp64(x) if x.dtype == np.float64 else np.asarray(x, dtype=np.float32)
    if mode == "bf16":
        return bf16_from_fp64(x) if x.dtype == np.float64 else bf16_from_fp32(x)
    raise ValueError(mode)


def _mode_product_fp32(X, W, l):
    """X x_l W with rounded operands: exact products summed in FP64 (exact enough that one
    rounding to FP32 gives the FP32 rounding of the exact sum for these operand sizes)."""
    axis = X.ndim - l
    Y = np.tensordot(W.astype(np.float64), X.astype(np.float64), axes=([1], [axis]))
    return np.moveaxis(Y, 0, axis).astype(np.float32)


def u_order(d):
    """Directions (1-based) of the U products after the divide, in the order taken."""
    return [3, 1, 2] if d == 3 else [1, 2]


def fd_apply_reduced(Us, Vs, lams, b, mode):
    """P~^{-1} b in the reduced-precision arithmetic of the module header ("fp32" or
    "bf16"): eq. 4.9 (d = 3) / eq. 4.7 (d = 2) with the roundings stated there.  Us, Vs,
    lams per direction l = 1..d (FP64); b is i_1-fastest FP64.  Returns FP64."""
    d = len(Us)
    shape = [len(lams[l]) for l in reversed(range(d))]
    rf = bf16_from_fp64 if mode == "bf16" else fp32_from_fp64
    X = np.asarray(b, dtype=np.float64).reshape(shape)
    for l in range(d):                                  # (V_d x .. x V_1)^T b
        X = _mode_product_fp32(round_input(X, mode), rf(np.asarray(Vs[l]).T), l + 1)
    lam32 = [fp32_from_fp64(lm) for lm in lams]
    if d == 3:
        L = lam32[2][:, None, None] + (lam32[1][:, None] + lam32[0][None, :]).astype(np.float32)[None, :, :]
    else:
        L = lam32[1][:, None] + lam32[0][None, :]
    X = (X / L.astype(np.float32)).astype(np.float32)    # FP32 divide
    for l in u_order(d):                                # (U_d x .. x U_1) s~
        X = _mode_product_fp32(round_input(X, mode), rf(np.asarray(Us[l - 1])), l)
    return X.astype(np.float64).ravel()
