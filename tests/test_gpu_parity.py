"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle on
seeded inputs that span several tiles and ragged tails, plus edge cases."""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_15187_amd as pid
import synth
from tests.gpu_helpers import (TOL_F32, TOL_F64, TOL_MIXED, assert_bitwise, assert_close,
                               assert_ranks, np64)

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _dev(t):
    return t.to(DEV)


def _soft(n, m, seed, dtype):
    return synth.random_soft(n, m, seed, dtype=torch.float64).to(dtype)


def _fields(n, m, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return torch.from_numpy(rng.normal(0.5, 0.08, size=(n, m)).astype(np.float32))


def _weights(m, seed):
    return synth.volume_weights(m, seed)


def _ref_input(U):
    """Exactly the stored values, widened to float64."""
    return U.to(torch.float64).numpy()


TOL_OF = {"f16": TOL_MIXED, "bf16": 3e-3, "bf16_split": TOL_MIXED, "f32": TOL_F32, "f64": TOL_F64}


# ------------------------------------------------------------------ extraction
@pytest.mark.parametrize("side", [1, -1])
def test_extract_gaussian_f32(side):
    F = _fields(7, 3001, 1)
    iso = dict(kind="gaussian", c=0.5, sigma=0.05, side=side)
    u = pid.pid_extract(_dev(F), iso, torch.float32)
    ref = oracle.extract(F.numpy(), iso)
    err = np.max(np.abs(np64(u) - ref))
    assert err < 1e-6, err


def test_extract_step_exact_and_f64():
    F = _fields(5, 2000, 2)
    F[0, :10] = 0.5                      # ties at the isovalue are outside
    for side in (1, -1):
        iso = dict(kind="step", c=0.5, side=side)
        u = pid.pid_extract(_dev(F), iso, torch.float32)
        assert (np64(u) == oracle.extract(F.numpy(), iso)).all()
    F64 = F.to(torch.float64)
    iso = dict(kind="gaussian", c=0.5, sigma=0.05, side=1)
    u = pid.pid_extract(_dev(F64), iso, torch.float64)
    assert np.max(np.abs(np64(u) - oracle.extract(F64.numpy(), iso))) < 1e-15


# ------------------------------------------------------------------ PID-mean
MEAN_CASES = [
    # (name, n, m, dtype, weighted, tol)
    ("f32_w", 37, 5003, torch.float32, True, TOL_MIXED),
    ("f16", 64, 8191, torch.float16, False, TOL_MIXED),
    ("f16_w", 64, 8192 + 513, torch.float16, True, TOL_MIXED),
    ("bf16", 20, 3000, torch.bfloat16, False, TOL_MIXED),
    ("f64", 50, 4097, torch.float64, False, TOL_F64),
    ("f64_w", 9, 777, torch.float64, True, TOL_F64),
    ("f32_n1", 1, 999, torch.float32, False, TOL_MIXED),
    ("f32_m1", 6, 1, torch.float32, False, TOL_MIXED),
    ("f16_n200", 200, 4000, torch.float16, True, TOL_MIXED),
    ("f16_twopass", 300, 4001, torch.float16, False, TOL_MIXED),
    ("f32_twopass_w", 280, 2100, torch.float32, True, TOL_MIXED),
    # several tiles per workgroup in the pipelined kernel: an odd count (the
    # last pair reads past the end), a ragged tile, rows past N in the last wave
    ("f32_pipe_oddK", 200, 64 * 256 * 3 + 37, torch.float32, False, TOL_F32),
    ("f32_pipe_oddK_w", 200, 64 * 256 * 3 + 37, torch.float32, True, TOL_F32),
    ("f16_pipe_w", 100, 256 * 256 * 6 + 100, torch.float16, True, TOL_MIXED),
    ("f64_pipe", 70, 128 * 256 * 5 + 3, torch.float64, True, TOL_F64),
    # LDS-staged kernel (rows end on 16-byte boundaries): ragged last tile,
    # rows past N in the last wave, weights, every element type
    ("f32_lds", 150, 32 * 1000 + 12, torch.float32, False, TOL_F32),
    ("f32_lds_w", 256, 32 * 777 + 20, torch.float32, True, TOL_F32),
    ("f16_lds_w", 64, 64 * 513 + 8, torch.float16, True, TOL_MIXED),
    ("bf16_lds", 100, 64 * 300 + 24, torch.bfloat16, False, TOL_MIXED),
    ("f64_lds_w", 40, 16 * 777 + 2, torch.float64, True, TOL_F64),
]


@pytest.mark.parametrize("name,n,m,dtype,weighted,tol", MEAN_CASES, ids=[c[0] for c in MEAN_CASES])
def test_pid_mean_soft(name, n, m, dtype, weighted, tol):
    U = _soft(n, m, 100 + n, dtype)
    w = _weights(m, 5) if weighted else None
    res = pid.pid_mean(_dev(U), None if w is None else _dev(w))
    ref = oracle.pid_mean(_ref_input(U), None if w is None else w.numpy())
    assert_close(res, ref, tol, label=name)
    assert_ranks(res["rank"], ref["depth"], tol, label=name)


def test_pid_mean_gaussian_fields():
    F = _fields(128, 4096 + 7, 3)
    iso = dict(kind="gaussian", c=0.5, sigma=0.05, side=1)
    res = pid.pid_mean(_dev(F), iso=iso)
    ref = oracle.pid_mean(oracle.extract(F.numpy(), iso))
    assert_close(res, ref, TOL_MIXED, label="gauss")


@pytest.mark.parametrize("n,m,kind", [(33, 3001, "step"), (70, 2000, "u8"), (5, 17, "u8"),
                                      (300, 1500, "u8"), (260, 999, "step")])
def test_pid_mean_binary_bitexact(n, m, kind):
    if kind == "u8":
        B = synth.random_binary(n, m, 7 + n)
        res = pid.pid_mean(_dev(B))
    else:
        F = _fields(n, m, 8 + n)
        iso = dict(kind="step", c=0.5, side=1)
        res = pid.pid_mean(_dev(F), iso=iso)
        B = torch.from_numpy(oracle.extract(F.numpy(), iso).astype(np.uint8))
    ref = oracle.binary_pid_mean(B.numpy())
    assert_bitwise(res, ref, keys=("in_in", "in_out", "depth", "mass"), label=f"mean-bin {kind}")
    assert_ranks(res["rank"], ref["depth"], 0)


# ------------------------------------------------------------------ all-pairs
PAIR_CASES = [
    # (n, m, dtype, weighted, scheme)
    (5, 300, torch.float32, False, "f16"),
    (33, 5003, torch.float32, True, "f16"),
    (70, 2049, torch.float32, False, "bf16_split"),
    (70, 2049, torch.float32, True, "f32"),
    (100, 3000, torch.float32, False, "bf16"),
    (130, 1000, torch.float64, False, "f64"),
    (40, 1500, torch.float64, True, "f64"),
    (256, 4096, torch.float16, False, "f16"),
    (230, 3333, torch.float16, True, "f16"),
    (300, 2000, torch.float32, False, "f16"),
    (300, 2000, torch.float32, True, "f32"),
    (41, 1111, torch.bfloat16, False, "bf16"),
    (1, 500, torch.float32, False, "f16"),
    (7, 1, torch.float32, False, "f32"),
]


@pytest.mark.parametrize("n,m,dtype,weighted,scheme", PAIR_CASES,
                         ids=[f"{c[0]}x{c[1]}-{str(c[2])[6:]}-{'w' if c[3] else 'u'}-{c[4]}" for c in PAIR_CASES])
def test_all_pairs_soft(n, m, dtype, weighted, scheme):
    U = _soft(n, m, 200 + n + m, dtype)
    w = _weights(m, 6) if weighted else None
    res = pid.pid_all_pairs(_dev(U), None if w is None else _dev(w), gemm=scheme)
    ref = oracle.pid(_ref_input(U), None if w is None else w.numpy())
    tol = TOL_OF[scheme]
    if scheme == "bf16" and dtype == torch.bfloat16:
        tol = TOL_MIXED          # exact BF16 inputs: only accumulation error
    assert_close(res, ref, tol, label=f"pairs {scheme}")
    assert_ranks(res["rank"], ref["depth"], tol, label=f"pairs {scheme}")


@pytest.mark.parametrize("scheme", ["f16", "bf16_split", "f32"])
def test_all_pairs_gaussian_fields(scheme):
    F = _fields(96, 3000 + 5, 9)
    iso = dict(kind="gaussian", c=0.5, sigma=0.05, side=-1)
    w = _weights(3005, 4)
    res = pid.pid_all_pairs(_dev(F), _dev(w), iso=iso, gemm=scheme)
    ref = oracle.pid(oracle.extract(F.numpy(), iso), w.numpy())
    assert_close(res, ref, TOL_OF[scheme], label=f"gauss {scheme}")


@pytest.mark.parametrize("n,m,kind", [(3, 100, "u8"), (40, 5000, "u8"), (129, 3001, "step"),
                                      (300, 1700, "u8"), (257, 2222, "step")])
def test_all_pairs_binary_bitexact(n, m, kind):
    if kind == "u8":
        B = synth.random_binary(n, m, 30 + n)
        res = pid.pid_all_pairs(_dev(B), gemm="i8")
    else:
        F = _fields(n, m, 31 + n)
        iso = dict(kind="step", c=0.5, side=1)
        res = pid.pid_all_pairs(_dev(F), iso=iso)          # AUTO -> INT8
        B = torch.from_numpy(oracle.extract(F.numpy(), iso).astype(np.uint8))
    ref = oracle.binary_pid(B.numpy())
    assert_bitwise(res, ref, label=f"pairs-bin {kind}")
    assert_ranks(res["rank"], ref["depth"], 0)


# Rows ending on a 16-byte boundary take the LDS-staged Gram kernel in its
# field variants: the Gaussian model in two 8-wave workgroups per CU (N <= 128),
# the linear models and thresholds on 256-byte row segments (N <= 128), INT8
# tiles for thresholded values on 128-byte segments (N > 128, grouped sub-tiles
# for eight row blocks, several super-tiles past 256 rows; FP16 fields).  The
# cases cover ragged N, a tail of M inside the last slab and point weights.
STAGED_FIELD_CASES = [
    # (kind, n, m, dtype, weighted, scheme of the soft kinds)
    ("gaussian", 100, 4132, torch.float32, True, "f16"),
    ("gaussian", 37, 2052, torch.float32, False, "f16"),
    ("gaussian", 160, 2056, torch.float32, True, "f16"),
    ("gaussian", 100, 4132, torch.float32, True, "bf16_split"),
    ("tent", 100, 4132, torch.float32, True, "f16"),
    ("tent", 100, 4132, torch.float32, False, "bf16_split"),
    ("step", 100, 4132, torch.float32, False, None),
    ("step", 200, 2056, torch.float32, False, None),
    ("step", 250, 2048, torch.float32, False, None),
    ("step", 300, 1028, torch.float32, False, None),
    ("step", 90, 4104, torch.float16, False, None),
]


@pytest.mark.parametrize("kind,n,m,dtype,weighted,scheme", STAGED_FIELD_CASES,
                         ids=[f"{c[0]}-{c[1]}x{c[2]}-{str(c[3])[6:]}{'-w' if c[4] else ''}{'-' + c[5] if c[5] else ''}"
                              for c in STAGED_FIELD_CASES])
def test_all_pairs_staged_fields(kind, n, m, dtype, weighted, scheme):
    F = _fields(n, m, 500 + n).to(dtype)
    Fh = F.to(torch.float64).numpy()
    if kind == "step":
        iso = dict(kind="step", c=0.5, side=1)
        res = pid.pid_all_pairs(_dev(F), iso=iso)           # AUTO -> INT8
        B = oracle.extract(Fh, iso).astype(np.uint8)
        ref = oracle.binary_pid(B)
        assert_bitwise(res, ref, label=f"staged {kind}")
        assert_ranks(res["rank"], ref["depth"], 0)
        return
    iso = (dict(kind="gaussian", c=0.5, sigma=0.05, side=-1) if kind == "gaussian"
           else dict(kind="tent", c=0.5, width=0.1))
    w = _weights(m, 7 + n) if weighted else None
    res = pid.pid_all_pairs(_dev(F), None if w is None else _dev(w), iso=iso, gemm=scheme)
    ref = oracle.pid(oracle.extract(Fh, iso), None if w is None else w.numpy())
    assert_close(res, ref, TOL_OF[scheme], label=f"staged {kind} {scheme}")
    assert_ranks(res["rank"], ref["depth"], TOL_MIXED, label=f"staged {kind}")


def test_binary_reduces_to_eid_on_gpu():
    B = synth.random_binary(12, 700, 77)
    res = pid.pid_all_pairs(_dev(B))
    _, _, edep = oracle.eid_sets(B.numpy())
    assert np.max(np.abs(np64(res["depth"]) - np.array([float(v) for v in edep]))) < 1e-15


# ------------------------------------------------------------------ edge cases
def test_strided_and_unaligned_rows():
    base = _soft(40, 1203, 41, torch.float32)
    big = torch.zeros(40, 1301, dtype=torch.float32)
    big[:, :1203] = base
    view = _dev(big)[:, :1203]                     # ld = 1301: rows not 16-byte aligned
    ref = oracle.pid(_ref_input(base))
    assert_close(pid.pid_all_pairs(view, gemm="f16"), ref, TOL_MIXED, label="strided pairs")
    refm = oracle.pid_mean(_ref_input(base))
    assert_close(pid.pid_mean(view), refm, TOL_MIXED, label="strided mean")


def test_zero_mass_and_identical_members():
    U = _soft(10, 900, 51, torch.float32)
    U[3] = 0.0
    U[7] = U[2]
    for scheme in ("f16", "f32"):
        res = pid.pid_all_pairs(_dev(U), gemm=scheme)
        ref = oracle.pid(_ref_input(U))
        assert_close(res, ref, TOL_OF[scheme], label="zero-mass")
        assert np64(res["depth"])[3] == 0.0 and np64(res["in_in"])[3] == 0.0
    rm = pid.pid_mean(_dev(U))
    assert np64(rm["depth"])[3] == 0.0
    Z = torch.zeros(4, 64)
    rz = pid.pid_mean(_dev(Z))
    assert (np64(rz["depth"]) == 0).all()
    rz = pid.pid_all_pairs(_dev(Z))
    assert (np64(rz["depth"]) == 0).all()


@pytest.mark.parametrize("case", ["f16_pairs_mean", "f32_both_gauss", "weighted_f32", "u8_bits", "fields_models"])
def test_deterministic_repeat(case):
    """Ten runs of each call give the same bits (split-K partials, column-sum
    groups and tile partials are all reduced in a fixed order), with the
    caller's streams and other work in between."""
    runs = []
    for r in range(10):
        if case == "f16_pairs_mean":
            U = _dev(_soft(200, 20000, 61, torch.float16))
            a, b = pid.pid_all_pairs(U), pid.pid_mean(U)
            out = [a["inclusion"], a["depth"], a["in_in"], a["in_out"], b["depth"], b["in_in"], b["in_out"]]
        elif case == "f32_both_gauss":
            F = _dev(_fields(256, 4096 * 3 + 17, 62))
            p, m = pid.pid_both(F, iso=dict(kind="gaussian", c=0.5, sigma=0.05, side=1))
            out = [p["inclusion"], p["depth"], m["depth"], m["in_out"]]
        elif case == "weighted_f32":
            U = _dev(_soft(300, 9000, 63, torch.float32))
            w = _dev(_weights(9000, 64))
            a = pid.pid_mean(U, w)
            c = pid.pid_pairs_depths(U, w)
            out = [a["depth"], a["in_in"], c["depth"], c["in_out"]]
        elif case == "u8_bits":
            B = _dev(synth.random_binary(3000, 20000, 65))
            out = [pid.pid_mean(B)["depth"], pid.pid_mean(pid.pid_pack_bits(B))["depth"]]
        else:
            F = _dev(_fields(96, 7001, 66))
            a = pid.pid_all_pairs(F, iso=dict(kind="tent", c=0.5, width=0.1))
            b = pid.pid_mean_weighted(F, _dev(torch.linspace(0.0, 1.0, 96, dtype=torch.float64)),
                                      iso=dict(kind="ramp", c=0.5, width=0.1, side=1))
            out = [a["inclusion"], a["depth"], b["depth"]]
        torch.cuda.synchronize()
        runs.append([t.cpu() for t in out])
        if r % 3 == 1:      # other work on the device between runs
            torch.randn(1 << 20, device=DEV).sum().item()
    for r in runs[1:]:
        for x, y in zip(runs[0], r):
            assert torch.equal(x, y), case


def test_validate_flag():
    U = _soft(4, 100, 71, torch.float32)
    U[1, 5] = 1.5
    with pytest.raises(pid.PidError) as ei:
        pid.pid_mean(_dev(U), validate=True)
    assert ei.value.status == pid.PID_ERR_VALUE_RANGE
    B = synth.random_binary(4, 100, 72)
    B[0, 0] = 3
    with pytest.raises(pid.PidError):
        pid.pid_all_pairs(_dev(B), validate=True)
    ok = pid.pid_mean(_dev(_soft(4, 100, 73, torch.float32)), validate=True)
    assert np.isfinite(np64(ok["depth"])).all()


def test_scheme_errors():
    U = _dev(_soft(4, 100, 81, torch.float32))
    with pytest.raises(pid.PidError) as ei:
        pid.pid_all_pairs(U, gemm="i8")
    assert ei.value.status == pid.PID_ERR_INVALID_ARG
    with pytest.raises(pid.PidError) as ei:
        pid.pid_all_pairs(_dev(synth.random_binary(4, 100, 3)), weights=_dev(_weights(100, 1)), gemm="i8")
    assert ei.value.status == pid.PID_ERR_INVALID_ARG


def test_rank_entry_point():
    d = torch.tensor([0.5, 0.7, 0.5, 0.9, 0.1, 0.7], dtype=torch.float64)
    rank, order = pid.pid_rank(_dev(d))
    r, o = oracle.rank_order(d.numpy())
    assert rank.cpu().tolist() == r.tolist() and order.cpu().tolist() == o.tolist()


@pytest.mark.parametrize("n", [2048, 2049, 5003, 40000])
def test_rank_large(n):
    """pid_rank on large ensembles (no workspace: the comparison kernel, depth
    tiles in LDS): exact ranks, with ties (depths drawn from 600 values) broken
    by the member index."""
    rng = np.random.Generator(np.random.PCG64(n))
    d = torch.from_numpy(rng.integers(0, 600, size=n) / 600.0)
    rank, order = pid.pid_rank(_dev(d))
    r, o = oracle.rank_order(d.numpy())
    assert np.array_equal(rank.cpu().numpy(), r) and np.array_equal(order.cpu().numpy(), o)


# ------------------------------------------------------------------ both in one call
BOTH_CASES = [
    # (n, m, dtype, weighted, gemm)
    (256, 32 * 1000, torch.float32, False, "f16"),
    (200, 32 * 777 + 20, torch.float32, True, "f16"),
    (64, 64 * 300, torch.float16, True, "f16"),
    (130, 32 * 500, torch.float32, False, "bf16_split"),
    (300, 4000, torch.float16, False, "f16"),      # several super-tiles
    (37, 5003, torch.float32, True, "f16"),        # row ends not on 16 bytes
    (50, 4096, torch.float64, False, "f64"),       # FP64 scheme
]


@pytest.mark.parametrize("n,m,dtype,weighted,gemm", BOTH_CASES,
                         ids=[f"{c[0]}x{c[1]}-{str(c[2])[6:]}-{'w' if c[3] else 'u'}-{c[4]}" for c in BOTH_CASES])
def test_pid_both(n, m, dtype, weighted, gemm):
    """pid_both: all-pairs results bitwise those of pid_all_pairs; PID-mean
    from the Gram row sums, within the tolerance of the Gram's scheme, with
    IN_in and the masses equal to the all-pairs ones (recall identity)."""
    U = _soft(n, m, 400 + n, dtype)
    w = _weights(m, 9) if weighted else None
    Ud, wd = _dev(U), (None if w is None else _dev(w))
    rp, rm = pid.pid_both(Ud, wd, gemm=gemm)
    alone = pid.pid_all_pairs(Ud, wd, gemm=gemm)
    for key in ("inclusion", "mass", "in_in", "in_out", "depth", "rank", "order"):
        assert torch.equal(rp[key], alone[key]), key
    assert torch.equal(rm["in_in"], rp["in_in"]) and torch.equal(rm["mass"], rp["mass"])
    ref = oracle.pid_mean(_ref_input(U), None if w is None else w.numpy())
    assert_close(rm, ref, TOL_OF[gemm], label=f"both mean {n}x{m}")
    assert_ranks(rm["rank"], ref["depth"], TOL_OF[gemm], label="both mean")


# ------------------------------------------------- all-pairs depths, O(N M)
# Tolerance: t(x) = sum_j u_j / m_j and the tile sums of B_i = sum_x w u_i t are
# FP32 (N and up to 16 x 1024 positive terms, relative error ~1e-6 typical,
# N * 6e-8 at worst), so 1e-5 absolute on the depths; FP64 input sums in FP64.
LIN_CASES = [
    # (n, m, dtype, weighted)
    (64, 64 * 300, torch.float32, False),
    (200, 32 * 777 + 20, torch.float32, True),
    (300, 4000, torch.float16, False),      # members in several groups
    (37, 5003, torch.float32, True),        # rows not 16-byte aligned
    (9, 100, torch.bfloat16, False),
    (50, 4096, torch.float64, False),
    (600, 6000, torch.float32, True),       # member groups in both column-sum passes
]


@pytest.mark.parametrize("n,m,dtype,weighted", LIN_CASES,
                         ids=[f"{c[0]}x{c[1]}-{str(c[2])[6:]}-{'w' if c[3] else 'u'}" for c in LIN_CASES])
def test_pairs_depths_linear(n, m, dtype, weighted):
    """pid_pairs_depths against the all-pairs oracle (no inclusion matrix)."""
    U = _soft(n, m, 500 + n, dtype)
    w = _weights(m, 11) if weighted else None
    res = pid.pid_pairs_depths(_dev(U), None if w is None else _dev(w))
    ref = oracle.pid(_ref_input(U), None if w is None else w.numpy())
    tol = TOL_F64 if dtype == torch.float64 else 1e-5
    assert_close(res, ref, tol, keys=("mass_rel", "in_in", "in_out", "depth"), label=f"linear {n}x{m}")
    assert_ranks(res["rank"], ref["depth"], tol, label="linear")


def test_pairs_depths_linear_fields_and_binary():
    """Gaussian fields, and binary input (IN_in exact; IN_out in soft arithmetic)."""
    F = _fields(48, 3001, 71)
    iso = dict(kind="gaussian", c=0.5, sigma=0.05, side=1)
    res = pid.pid_pairs_depths(_dev(F), iso=iso)
    ref = oracle.pid(oracle.extract(F.numpy(), iso))
    assert_close(res, ref, 1e-5, keys=("mass_rel", "in_in", "in_out", "depth"), label="linear gauss")
    B = synth.random_binary(70, 2000, 72)
    rb = pid.pid_pairs_depths(_dev(B))
    refb = oracle.binary_pid(B.numpy())
    assert np.array_equal(np64(rb["in_in"]), refb["in_in"]), "binary IN_in not exact"
    assert_close(rb, refb, 1e-5, keys=("mass_rel", "in_in", "in_out", "depth"), label="linear binary")


@pytest.mark.parametrize("n,m,kind", [(40, 5000, "u8"), (257, 2222, "step")])
def test_pid_both_binary_bitexact(n, m, kind):
    """Binary input through INT8: both depth kinds bitwise equal to the
    oracle's integer forms."""
    if kind == "u8":
        B = synth.random_binary(n, m, 60 + n)
        rp, rm = pid.pid_both(_dev(B), gemm="i8")
    else:
        F = _fields(n, m, 61 + n)
        iso = dict(kind="step", c=0.5, side=1)
        rp, rm = pid.pid_both(_dev(F), iso=iso)
        B = torch.from_numpy(oracle.extract(F.numpy(), iso).astype(np.uint8))
    assert_bitwise(rp, oracle.binary_pid(B.numpy()), label=f"both-bin pairs {kind}")
    refm = oracle.binary_pid_mean(B.numpy())
    assert_bitwise(rm, refm, keys=("in_in", "in_out", "depth", "mass"), label=f"both-bin mean {kind}")
    assert_ranks(rm["rank"], refm["depth"], 0)
