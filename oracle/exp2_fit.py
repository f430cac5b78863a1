"""Coefficients of the FP32 form's polynomial for 2^f, |f| <= 1/2.

The FP32 Metropolis test evaluates 2^t = 2^k 2^f with k = rint(t) and
f = t - k.  2^f comes from p(f) = 1 + c1 f + ... + c6 f^6: the constant term is
exactly 1 (so p(0) = 1 and 2^k is exact at integer t), and c1..c6 minimise the
largest relative error |p(f) - 2^f| / 2^f on [-1/2, 1/2].  The minimax fit is
found by Lawson's iteratively reweighted least squares on 4001 Chebyshev
points; its relative error before rounding the coefficients to float is
2.0e-9, and the polynomial evaluated by Horner's rule with float fused
multiply-adds (the oracle's `oracle_pexp2_32`, and the GPU kernels) is within
0.952 float ulp of 2^f for every float f in [-1/2, 1/2] (checked
exhaustively).  Test infrastructure: it documents where the oracle's constants
come from, and a CPU test re-runs it.

    python -m oracle.exp2_fit
"""
from __future__ import annotations

import numpy as np

DEGREE = 6


def fit(degree: int = DEGREE, points: int = 4001, iters: int = 200) -> tuple[list[float], float]:
    """(coefficients c0..c_degree rounded to float, relative error of the
    unrounded fit on the grid)."""
    x = 0.5 * np.cos(np.linspace(0.0, np.pi, points))
    y = np.exp2(x)
    # relative error of 1 + sum_k c_k x^k: (1 + A c - y) / y = A' c - b
    a = np.stack([x ** k for k in range(1, degree + 1)], axis=1) / y[:, None]
    b = (y - 1.0) / y
    w = np.full(points, 1.0 / points)
    c = np.zeros(degree)
    for _ in range(iters):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(a * sw[:, None], b * sw, rcond=None)
        r = np.abs(a @ c - b)
        w = w * r
        w /= w.sum()
    err = float(np.max(np.abs(a @ c - b)))
    return [1.0] + [float(np.float32(v)) for v in c], err


if __name__ == "__main__":
    coefs, err = fit()
    print(f"relative error of the fit {err:.3e}")
    for k, v in enumerate(coefs):
        print(f"c{k} = {v.hex()}")
