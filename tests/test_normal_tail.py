"""The division-free normal tail of the GPU loaders (``half_erfc_fast`` in
device_common.h), checked on the CPU against scipy's normal CDF: the
coefficients are read from the header and evaluated the way the kernels do
(FP32 multiply-adds, FP32 2^x).  The Gaussian isovalue model of Sec. 3.5
turns every value f into Phi((c - f) / sigma) or its complement; these paths
rely on that value being within 2e-7 of the exact one."""
import os
import re

import numpy as np
from scipy.special import ndtr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_2512_15187_amd", "csrc", "device_common.h")


def header_coefficients():
    src = open(HEADER).read()
    body = src[src.index("float half_erfc_fast("):]
    body = body[:body.index("return")]
    lits = [float(x) for x in re.findall(r"([-+]?\d\.\d+e[-+]\d+)f", body)]
    clamp = float(re.search(r"fminf\(fabsf\(y\), ([\d.]+)f\)", body).group(1))
    return lits, clamp   # lits: -a7 .. -a1 in Horner order


def tail_fp32(y, neg_a, clamp):
    x = np.minimum(np.abs(np.asarray(y, np.float32)), np.float32(clamp))
    fma = lambda p, q, r: (np.float64(p) * np.float64(q) + np.float64(r)).astype(np.float32)
    q = np.full_like(x, np.float32(neg_a[0]))
    for c in neg_a[1:]:
        q = fma(x, q, np.float32(c))
    return np.exp2(fma(x, q, np.float32(-1.0)).astype(np.float64)).astype(np.float32)


def test_tail_and_body_within_bound():
    neg_a, clamp = header_coefficients()
    assert len(neg_a) == 7 and clamp == 6.0
    y = np.linspace(0.0, 12.0, 1200001).astype(np.float32)
    h = tail_fp32(y, neg_a, clamp)
    exact_tail = ndtr(-y.astype(np.float64))
    assert np.abs(h - exact_tail).max() <= 1.2e-7
    body = (np.float32(1.0) - h).astype(np.float64)
    assert np.abs(body - ndtr(y.astype(np.float64))).max() <= 1.5e-7


def test_tail_special_values():
    neg_a, clamp = header_coefficients()
    h = tail_fp32(np.array([0.0, 1.0, 1.959963985, 6.0, 40.0], np.float32), neg_a, clamp)
    assert h[0] == np.float32(0.5)                       # T(0) = 1/2 exactly (no constant term)
    assert abs(h[1] - 0.15865525393) < 1.2e-7            # 1 - Phi(1)
    assert abs(h[2] - 0.025) < 1.2e-7                    # the two-sided 5 % point
    assert 0.0 < h[3] < 1.2e-7 and h[4] == h[3]          # clamped beyond 6
    # monotone non-increasing in |y| (a rank-preserving model)
    y = np.linspace(0.0, 8.0, 80001).astype(np.float32)
    assert np.all(np.diff(tail_fp32(y, neg_a, clamp).astype(np.float64)) <= 0.0)
