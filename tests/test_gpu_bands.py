"""GPU parity of the contour-boxplot bands (pid_bands, through the C ABI)
against the FP64 oracle: every output byte compared, seeded inputs with
ragged tails, strided rows, the three extraction models, the edge cases
N = 1, M = 1, k = 1, k = N, and an order entry outside 0..N-1."""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_15187_amd as pid
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _soft(n, m, seed, dtype, thr):
    U = synth.random_soft(n, m, seed, dtype=torch.float64).to(dtype)
    # plant values equal to the threshold (inside by the >= reading)
    rng = _rng(seed + 1)
    idx = rng.integers(0, n * m, size=max(1, n * m // 97))
    U.view(-1)[torch.from_numpy(idx)] = torch.tensor(thr, dtype=torch.float64).to(dtype)
    return U


def _order(n, seed):
    return _rng(seed).permutation(n).astype(np.int32)


def _run(U_host, order, ki, ko, thr, iso=None, U_dev=None):
    U_dev = U_host.to(DEV) if U_dev is None else U_dev
    code = pid.pid_bands(U_dev, torch.from_numpy(order).to(DEV), ki, ko, thr, iso=iso)
    torch.cuda.synchronize()
    return code.cpu().numpy()


CASES = [
    # (n, m, dtype, k_inner, k_outer, threshold)
    (50, 16384 + 37, torch.float32, 25, 50, 0.5),      # rows not 16-byte aligned: element loads
    (50, 16384 + 36, torch.float32, 25, 50, 0.5),      # aligned rows: 16-byte loads
    (31, 5000, torch.float16, 16, 31, 0.5),
    (20, 3001, torch.bfloat16, 10, 20, 0.02),          # density threshold
    (40, 4099, torch.float64, 20, 40, 0.5),
    (12, 1000, torch.float32, 1, 12, 0.5),             # inner band of one member
    (12, 1000, torch.float32, 12, 12, 0.5),
    (1, 100, torch.float32, 1, 1, 0.5),                # N = 1
    (9, 1, torch.float32, 3, 9, 0.5),                  # M = 1
    (300, 2053, torch.float32, 150, 290, 0.5),         # k_outer < N, many rounds of loads
]


@pytest.mark.parametrize("n,m,dtype,ki,ko,thr", CASES)
def test_bands_soft(n, m, dtype, ki, ko, thr):
    U = _soft(n, m, 900 + n + m, dtype, thr)
    order = _order(n, 70 + n)
    code = _run(U, order, ki, ko, thr)
    ref = oracle.boxplot_bands(U.to(torch.float64).numpy(), order, ki, ko, thr)
    assert np.array_equal(code, ref["code"]), np.flatnonzero(code != ref["code"])[:10]


def test_bands_binary_u8():
    n, m = 33, 7777
    B = synth.random_binary(n, m, 41)
    order = _order(n, 42)
    code = _run(B, order, 17, 33, 0.5)
    ref = oracle.boxplot_bands(B.numpy().astype(np.float64), order, 17, 33, 0.5)
    assert np.array_equal(code, ref["code"])


@pytest.mark.parametrize("m,ld,dtype", [(999, 1003, torch.float32),    # not 16-byte aligned rows
                                         (1001, 1004, torch.float32),   # aligned rows, ragged last chunk
                                         (1013, 1024, torch.float16)])
def test_bands_strided_rows(m, ld, dtype):
    n = 17
    big = _soft(n, ld, 43 + m, dtype, 0.5)
    order = _order(n, 44)
    view = big.to(DEV)[:, :m]
    code = _run(None, order, 8, 17, 0.5, U_dev=view)
    ref = oracle.boxplot_bands(big[:, :m].to(torch.float64).numpy(), order, 8, 17, 0.5)
    assert np.array_equal(code, ref["code"])


def test_bands_step_isovalue():
    n, m = 64, 64 * 300 + 11
    F = torch.from_numpy(_rng(45).normal(0.5, 0.08, size=(n, m)).astype(np.float32))
    iso = dict(kind="step", c=0.5, side=-1)
    order = _order(n, 46)
    code = _run(F, order, 32, 64, 0.5, iso=iso)
    ref = oracle.boxplot_bands(oracle.extract(F.numpy(), iso), order, 32, 64, 0.5)
    assert np.array_equal(code, ref["code"])


def test_bands_gaussian_isovalue():
    """Phi is evaluated in FP64 on both sides by different routines, so a point
    whose probability lies within 1e-12 of the threshold may fall either way:
    those points are excluded (and counted); all others must agree."""
    n, m = 48, 20000
    F = torch.from_numpy(_rng(47).normal(0.5, 0.08, size=(n, m)).astype(np.float32))
    iso = dict(kind="gaussian", c=0.5, sigma=0.05, side=1)
    order = _order(n, 48)
    code = _run(F, order, 24, 48, 0.5, iso=iso)
    u = oracle.extract(F.numpy(), iso)
    ref = oracle.boxplot_bands(u, order, 24, 48, 0.5)
    ambiguous = np.any(np.abs(u[order[:48]] - 0.5) < 1e-12, axis=0)
    assert ambiguous.sum() < 5
    ok = ~ambiguous
    assert np.array_equal(code[ok], ref["code"][ok])


def test_bands_order_entry_out_of_range():
    """An order entry outside 0..N-1 is skipped (never read) and flags every
    point with bit 128; the other bits are those of the remaining members."""
    n, m = 10, 3000
    U = _soft(n, m, 49, torch.float32, 0.5)
    order = _order(n, 50)
    bad = order.copy()
    bad[9] = n                                   # the last member of the outer band
    code = _run(U, bad, 5, 10, 0.5)
    ref = oracle.boxplot_bands(U.to(torch.float64).numpy(), order[:9], 5, 9, 0.5)
    assert np.all(code & 128)
    assert np.array_equal(code & 127, ref["code"])


def test_bands_headline_size_sampled():
    """N = 256 soft masks on 512 x 512 (the headline workload's shape), the
    50 % and 100 % groups of an order: every point compared with the oracle
    on a sample of 8192 points."""
    n, m = 256, 512 * 512
    U = synth.random_soft(n, m, 51, dtype=torch.float32)
    order = _order(n, 52)
    code = _run(U, order, 128, 256, 0.5)
    pts = np.sort(_rng(53).choice(m, size=8192, replace=False))
    ref = oracle.boxplot_bands(U[:, torch.from_numpy(pts)].to(torch.float64).numpy(), order, 128, 256, 0.5)
    assert np.array_equal(code[pts], ref["code"])

