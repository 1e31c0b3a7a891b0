"""Coefficients of the division-free normal tail used by ``half_erfc_fast``
(device_common.h).

For y >= 0 the tail T(y) = 1 - Phi(y) is written as 2^(-1 - P(y)) with
P(y) = a1 y + ... + a7 y^7 (no constant term, so T(0) = 1/2 exactly).  The
coefficients minimise max_y |T(y) ln 2 * (P(y) - G(y))| on a dense grid of
[0, 6], G(y) = -log2(2 T(y)): to first order the absolute error of the tail.
The minimax problem is a linear programme.  Beyond 6 the kernels clamp the
argument.  Run ``python fit_normal_tail.py`` to print the coefficients (as
FP32 literals) and the error of the FP32 evaluation.
"""
import numpy as np
from scipy.optimize import linprog
from scipy.special import ndtr

Y_MAX = 6.0
DEGREE = 7


def fit(y_max=Y_MAX, degree=DEGREE, npts=6000):
    y = np.linspace(0.0, y_max, npts)
    t = ndtr(-y)
    g = -np.log2(2.0 * t)
    v = np.stack([y ** k for k in range(1, degree + 1)], 1)
    w = t * np.log(2.0)
    ones = np.ones((npts, 1))
    a_ub = np.vstack([np.hstack([w[:, None] * v, -ones]), np.hstack([-w[:, None] * v, -ones])])
    b_ub = np.concatenate([w * g, -w * g])
    cost = np.zeros(degree + 1)
    cost[-1] = 1.0
    res = linprog(cost, A_ub=a_ub, b_ub=b_ub, bounds=[(None, None)] * degree + [(0, None)], method="highs")
    if not res.success:
        raise RuntimeError(res.message)
    return [float(np.float32(c)) for c in res.x[:degree]]


def tail_fp32(y, a):
    """The kernels' evaluation: FP32 multiply-adds (each rounded once) on
    x = min(|y|, Y_MAX), then 2^x (rounded to FP32)."""
    x = np.minimum(np.abs(np.asarray(y, np.float32)), np.float32(Y_MAX))
    fma = lambda p, q, r: (np.float64(p) * np.float64(q) + np.float64(r)).astype(np.float32)
    q = np.full_like(x, np.float32(-a[-1]))
    for k in range(len(a) - 2, -1, -1):
        q = fma(x, q, np.float32(-a[k]))
    return np.exp2(fma(x, q, np.float32(-1.0)).astype(np.float64)).astype(np.float32)


if __name__ == "__main__":
    a = fit()
    y = np.linspace(0.0, 9.0, 2000001).astype(np.float32)
    h = tail_fp32(y, a)
    e_tail = np.abs(h.astype(np.float64) - ndtr(-y.astype(np.float64))).max()
    e_body = np.abs((np.float32(1.0) - h).astype(np.float64) - ndtr(y.astype(np.float64))).max()
    print("-a_k, k = 7 .. 1 (the Horner order of the kernel):")
    for c in a[::-1]:
        print(f"  {-c:.9e}f")
    print(f"max |error| of T: {e_tail:.3e}; of 1 - T: {e_body:.3e}")
