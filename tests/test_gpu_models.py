"""GPU parity of the further probability models (uniform isovalue ramp,
Sec. 3.5; level-centred tent, Sec. 3.6; normalised density, Sec. 6.3), of
PID-mean against a reliability-weighted mean contour (Sec. 4.1) and of the
field maximum, against the FP64 oracle on the same stored values, through the
C ABI: every depth call that takes an isovalue model, several tiles and ragged
tails, aligned and unaligned rows, weights, both sides of the ramp."""
import numpy as np
import pytest
import torch

import oracle
import paper_2512_15187_amd as pid
import synth
from tests.gpu_helpers import TOL_F32, TOL_F64, TOL_MIXED, assert_close, assert_ranks, np64

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _fields(n, m, seed, dtype=torch.float32):
    rng = np.random.Generator(np.random.PCG64(seed))
    return torch.from_numpy(rng.normal(0.5, 0.08, size=(n, m))).to(dtype)


def _models(fmax):
    return {"ramp_up": dict(kind="ramp", c=0.5, width=0.06, side=1),
            "ramp_down": dict(kind="ramp", c=0.48, width=0.1, side=-1),
            "tent": dict(kind="tent", c=0.52, width=0.07),
            "density": dict(kind="density", c=float(fmax))}


MODEL_NAMES = ("ramp_up", "ramp_down", "tent", "density")


def _ref(F, iso, w=None):
    return oracle.extract(F.to(torch.float64).numpy(), iso), None if w is None else w.numpy()


# ------------------------------------------------------------------ extraction
@pytest.mark.parametrize("model", MODEL_NAMES)
@pytest.mark.parametrize("dtype,out_dtype,tol", [(torch.float32, torch.float32, 1e-6),
                                                 (torch.float64, torch.float64, 1e-15),
                                                 (torch.float16, torch.float32, 1e-6)])
def test_extract_models(model, dtype, out_dtype, tol):
    # FP32 evaluates t = (f - c) * a with c and a rounded to FP32: the error
    # is about a * |c| * 2^-24 + 2^-24 (a = 1 / width up to 17 here), below 1e-6
    F = _fields(6, 2501, 1, dtype)
    iso = _models(F.to(torch.float64).max().item())[model]
    u = pid.pid_extract(F.to(DEV), iso, out_dtype)
    ref = oracle.extract(F.to(torch.float64).numpy(), iso)
    err = np.max(np.abs(np64(u) - ref))
    assert err <= tol, (model, err)


def test_field_max():
    for dtype in (torch.float32, torch.float64, torch.float16, torch.bfloat16):
        F = _fields(9, 1003, 2, dtype) - 0.3
        F[4, 100] = float("nan")
        got = pid.pid_field_max(F.to(DEV)).item()
        assert got == float(torch.nan_to_num(F.to(torch.float64), nan=-1e300).max()), dtype
    B = synth.random_binary(5, 777, 3)
    assert pid.pid_field_max(B.to(DEV)).item() == 1.0
    Z = torch.full((3, 50), -2.5, dtype=torch.float32)
    assert pid.pid_field_max(Z.to(DEV)).item() == -2.5
    # a strided view: only the first m values of each row count
    W = torch.zeros((4, 64), dtype=torch.float32)
    W[:, 40:] = 9.0
    V = W.to(DEV)[:, :40]
    assert pid.pid_field_max(V).item() == 0.0


# ------------------------------------------------------------------ PID-mean
MEAN_MODEL_CASES = [
    # (n, m, dtype, weighted, tol): pipelined (FP32 / FP64), unpipelined (FP16,
    # unaligned rows), two-pass (N > 256)
    (40, 64 * 256 * 2 + 77, torch.float32, True, TOL_F32),
    (100, 5003, torch.float32, False, TOL_F32),
    (37, 4096 + 5, torch.float64, True, TOL_F64),
    (64, 8192 + 513, torch.float16, True, TOL_MIXED),
    (300, 4001, torch.float32, True, TOL_F32),
]


@pytest.mark.parametrize("model", MODEL_NAMES)
@pytest.mark.parametrize("n,m,dtype,weighted,tol", MEAN_MODEL_CASES,
                         ids=[f"{c[0]}x{c[1]}-{str(c[2])[6:]}-{'w' if c[3] else 'u'}" for c in MEAN_MODEL_CASES])
def test_pid_mean_models(model, n, m, dtype, weighted, tol):
    F = _fields(n, m, 10 + n, dtype)
    w = synth.volume_weights(m, 5) if weighted else None
    iso = _models(F.to(torch.float64).max().item())[model]
    res = pid.pid_mean(F.to(DEV), None if w is None else w.to(DEV), iso=iso)
    U, wr = _ref(F, iso, w)
    ref = oracle.pid_mean(U, wr)
    assert_close(res, ref, tol, label=f"mean {model}")
    assert_ranks(res["rank"], ref["depth"], tol, label=f"mean {model}")


# ------------------------------------------------------------------ all-pairs
PAIR_MODEL_CASES = [
    # (n, m, dtype, weighted, scheme, tol): LDS-staged FP16 MFMA (aligned rows),
    # register-fed FP16 (ragged rows), the BF16 split, the FP32 and FP64 comparators
    (64, 4096, torch.float32, False, "f16", TOL_MIXED),
    (33, 5003, torch.float32, True, "f16", TOL_MIXED),
    (256, 2048, torch.float32, True, "f16", TOL_MIXED),
    (70, 2049, torch.float32, False, "bf16_split", TOL_MIXED),
    (70, 2049, torch.float32, True, "f32", TOL_F32),
    (100, 3000, torch.float16, False, "f16", TOL_MIXED),
    (40, 1500, torch.float64, True, "f64", TOL_F64),
]


@pytest.mark.parametrize("model", MODEL_NAMES)
@pytest.mark.parametrize("n,m,dtype,weighted,scheme,tol", PAIR_MODEL_CASES,
                         ids=[f"{c[0]}x{c[1]}-{str(c[2])[6:]}-{'w' if c[3] else 'u'}-{c[4]}"
                              for c in PAIR_MODEL_CASES])
def test_pid_pairs_models(model, n, m, dtype, weighted, scheme, tol):
    F = _fields(n, m, 20 + n, dtype)
    w = synth.volume_weights(m, 6) if weighted else None
    iso = _models(F.to(torch.float64).max().item())[model]
    res = pid.pid_all_pairs(F.to(DEV), None if w is None else w.to(DEV), iso=iso, gemm=scheme)
    U, wr = _ref(F, iso, w)
    ref = oracle.pid(U, wr)
    assert_close(res, ref, tol, label=f"pairs {model} {scheme}")
    assert_ranks(res["rank"], ref["depth"], tol, label=f"pairs {model}")
    if scheme == "f16":
        dp, dm = pid.pid_both(F.to(DEV), None if w is None else w.to(DEV), iso=iso, gemm=scheme)
        assert_close(dp, ref, tol, label=f"both pairs {model}")
        assert_close(dm, oracle.pid_mean(U, wr), tol, label=f"both mean {model}")


@pytest.mark.parametrize("model", MODEL_NAMES)
def test_pairs_depths_models(model):
    F = _fields(180, 6001, 31)
    iso = _models(F.to(torch.float64).max().item())[model]
    res = pid.pid_pairs_depths(F.to(DEV), iso=iso)
    U, _ = _ref(F, iso)
    ref = oracle.pid(U)
    assert_close(res, ref, 1e-5, keys=("mass_rel", "in_in", "in_out", "depth"), label=f"depths {model}")


def test_bands_density_threshold():
    """Boxplot bands of normalised densities thresholded at 0.02 (the value
    of the smoke-plume example); points whose oracle probability lies within
    1e-12 of the threshold are left out (the two sides round the model
    differently there)."""
    F = _fields(48, 9001, 41) - 0.35
    fmax = pid.pid_field_max(F.to(DEV)).item()
    iso = dict(kind="density", c=fmax)
    order = torch.from_numpy(np.random.Generator(np.random.PCG64(3)).permutation(48).astype(np.int32))
    code = pid.pid_bands(F.to(DEV), order.to(DEV), 24, 48, 0.02, iso=iso).cpu().numpy()
    U = oracle.extract(F.to(torch.float64).numpy(), iso)
    ref = oracle.boxplot_bands(U, order.numpy(), 24, 48, 0.02)["code"]
    near = np.any(np.abs(U - 0.02) < 1e-12, axis=0)
    assert (code[~near] == ref[~near]).all()


# ------------------------------------------------------- reliability weights
WEIGHTED_CASES = [
    # (name, n, m, dtype, point weights, iso, tol)
    ("f32_soft_unaligned", 45, 3001, torch.float32, False, None, TOL_F32),
    ("f16_soft_w", 130, 8192 + 64, torch.float16, True, None, TOL_MIXED),
    ("f64_soft_w", 30, 2000, torch.float64, True, None, TOL_F64),
    ("u8_binary", 70, 4099, torch.uint8, False, None, TOL_F32),
    ("f32_gauss", 60, 4096, torch.float32, False, dict(kind="gaussian", c=0.5, sigma=0.05, side=1), TOL_MIXED),
    ("f32_tent_w", 300, 2500, torch.float32, True, dict(kind="tent", c=0.5, width=0.08), TOL_F32),
]


@pytest.mark.parametrize("name,n,m,dtype,weighted,iso,tol", WEIGHTED_CASES, ids=[c[0] for c in WEIGHTED_CASES])
def test_pid_mean_weighted(name, n, m, dtype, weighted, iso, tol):
    rng = np.random.Generator(np.random.PCG64(n + m))
    if dtype == torch.uint8:
        U = synth.random_binary(n, m, 9)
    elif iso is None:
        U = synth.random_soft(n, m, 40 + n, dtype=torch.float64).to(dtype)
    else:
        U = _fields(n, m, 50 + n, dtype)
    w = synth.volume_weights(m, 7) if weighted else None
    r = rng.uniform(0.0, 2.0, size=n)
    r[rng.permutation(n)[: max(1, n // 10)]] = 0.0            # some members carry no weight
    res = pid.pid_mean_weighted(U.to(DEV), torch.from_numpy(r).to(DEV), None if w is None else w.to(DEV), iso=iso)
    Uref = oracle.extract(U.to(torch.float64).numpy(), iso)
    ref = oracle.pid_mean_weighted(Uref, r, None if w is None else w.numpy())
    assert_close(res, ref, tol, label=name)
    assert_ranks(res["rank"], ref["depth"], tol, label=name)
    # unit weights: the values of pid_mean
    one = pid.pid_mean_weighted(U.to(DEV), torch.ones(n, dtype=torch.float64, device=DEV),
                                None if w is None else w.to(DEV), iso=iso)
    plain = oracle.pid_mean(Uref, None if w is None else w.numpy())
    assert_close(one, plain, tol, label=name + " unit")


def test_pid_mean_weighted_degenerate():
    U = synth.random_soft(12, 777, 3, dtype=torch.float64).to(torch.float32)
    z = pid.pid_mean_weighted(U.to(DEV), torch.zeros(12, dtype=torch.float64, device=DEV))
    assert (z["depth"].cpu() == 0).all() and (z["in_in"].cpu() == 0).all()
    # one-hot weights: the mean contour is that member
    e = torch.zeros(12, dtype=torch.float64)
    e[5] = 2.0
    r = pid.pid_mean_weighted(U.to(DEV), e.to(DEV))
    Uh = U.to(torch.float64).numpy()
    for i in range(12):
        assert abs(r["in_in"][i].item() - oracle.incl(Uh[i], Uh[5])) < TOL_F32
        assert abs(r["in_out"][i].item() - oracle.incl(Uh[5], Uh[i])) < TOL_F32
