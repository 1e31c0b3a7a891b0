"""pid_both_static (the workspace in the library's fixed device array) gives
the results of pid_both with a caller workspace: called through the C ABI on
two inputs in a row, the second smaller, each compared bitwise with pid_both
on the same input (the same kernels and launch plan) and with the FP64 oracle
within the mixed-precision tolerance."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2512_15187_amd as pid
import synth
from tests.gpu_helpers import TOL_MIXED, assert_close, assert_ranks

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
KEYS = ("mass", "in_in", "in_out", "depth", "rank", "order")


def _outputs(n, inclusion):
    d = {k: torch.full((n,), -7.0, dtype=torch.float64, device=DEV) for k in ("mass", "in_in", "in_out", "depth")}
    d["rank"] = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    d["order"] = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    if inclusion:
        d["inclusion"] = torch.full((n, n), -7.0, dtype=torch.float64, device=DEV)
    o = pid.pid_out(d["inclusion"].data_ptr() if inclusion else None, d["mass"].data_ptr(), d["in_in"].data_ptr(),
                    d["in_out"].data_ptr(), d["depth"].data_ptr(), d["rank"].data_ptr(), d["order"].data_ptr())
    return d, o


def _static_call(U, gemm):
    lib = pid.load_library()
    fn = lib.pid_both_static
    fn.argtypes = [ctypes.POINTER(pid.pid_ensemble), ctypes.POINTER(pid.pid_iso), ctypes.c_int,
                   ctypes.POINTER(pid.pid_out), ctypes.POINTER(pid.pid_out), ctypes.c_void_p]
    fn.restype = ctypes.c_int
    e, i = pid.make_ensemble(U), pid.make_iso(None)
    n = U.shape[0]
    dp, op = _outputs(n, True)
    dm, om = _outputs(n, False)
    st = fn(ctypes.byref(e), ctypes.byref(i), pid.GEMM[gemm], ctypes.byref(op), ctypes.byref(om),
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == pid.PID_OK, lib.pid_last_error().decode()
    return dp, dm


def test_static_scratch_matches_pid_both_twice():
    big, _ = synth.config1(device=DEV)                              # 256 x 512^2 FP32
    small, _ = synth.config1(device=DEV, res=96, n=40)              # 40 x 96^2, a smaller second call
    for U in (big, small):
        sp, sm = _static_call(U, "f16")
        rp, rm = pid.pid_both(U, gemm="f16")
        torch.cuda.synchronize()
        for k in KEYS + ("inclusion",):
            assert torch.equal(sp[k], rp[k]), ("pairs", tuple(U.shape), k)
        for k in KEYS:
            assert torch.equal(sm[k], rm[k]), ("mean", tuple(U.shape), k)
        host = U.cpu().numpy()
        ref = oracle.pid_large(host)
        refm = oracle.pid_mean_large(host)
        assert_close(sp, ref, TOL_MIXED, label=f"static pairs {tuple(U.shape)}")
        assert_close(sm, refm, TOL_MIXED, label=f"static mean {tuple(U.shape)}")
        assert_ranks(sp["rank"], ref["depth"], TOL_MIXED)
        assert_ranks(sm["rank"], refm["depth"], TOL_MIXED)


def test_static_scratch_binary_bitwise_and_limit():
    B = synth.random_binary(60, 50001, 7).to(DEV)
    sp, sm = _static_call(B, "i8")
    ref = oracle.binary_pid(B.cpu().numpy())
    refm = oracle.binary_pid_mean(B.cpu().numpy())
    for k in ("in_in", "in_out", "depth", "inclusion"):
        assert np.array_equal(sp[k].cpu().numpy(), ref[k]), k
    for k in ("in_in", "in_out", "depth"):
        assert np.array_equal(sm[k].cpu().numpy(), refm[k]), k
    # a call whose workspace exceeds the array is refused before any launch
    lib = pid.load_library()
    e = pid.pid_ensemble(4096, 1 << 22, 1 << 22, pid.PID_F16, 0, 0x1000, None)
    i = pid.make_iso(None)
    o = pid.pid_out()
    st = lib.pid_both_static(ctypes.byref(e), ctypes.byref(i), pid.GEMM["f16"], ctypes.byref(o), ctypes.byref(o),
                             None)
    assert st == pid.PID_ERR_UNSUPPORTED
    assert b"static scratch" in lib.pid_last_error()
