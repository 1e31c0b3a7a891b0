"""Serving loop on the GPU: requests of uneven size admitted while others run.

Every served result is checked against the FP64 oracle (the definitions of
Sec. 3.2 Eq. pid and Sec. 4.1 on the same stored FP16 values) and bitwise
against the same request run alone; requests overlap on the device (per
request timing events on the slot streams); a request that fits the arena
alone waits for memory while another runs; the footprint budget serialises
requests; errors of a failed request reach the client with their text;
over-budget and cancelled requests are reported."""
import threading

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


@pytest.fixture(scope="module")
def pool():
    return {("2d", 128): synth.serving_pool("2d", 128, 96, device=DEV),
            ("2d", 320): synth.serving_pool("2d", 320, 300, device=DEV),
            ("3d", 48): synth.serving_pool("3d", 48, 64, device=DEV)}


@pytest.fixture(scope="module")
def big():
    """All-pairs request of 512 members on 1024 x 1024 (the longest of the mix)."""
    return synth.serving_pool("2d", 1024, 512, device=DEV)


def _oracle(U, variant):
    host = U.detach().cpu().numpy()          # the stored FP16 values, widened exactly below
    if variant == "pairs":
        return oracle.pid_large(host)
    if variant == "depths":
        r = oracle.pid_large(host)
        r.pop("inclusion")
        return r
    return oracle.pid_mean_large(host)


def _check_against_oracle(U, variant, out, label):
    ref = _oracle(U, variant)
    keys = ("mass_rel", "in_in", "in_out", "depth") + (("inclusion",) if "inclusion" in out else ())
    assert_close(out, ref, TOL_MIXED, keys=keys, label=label)
    assert_ranks(out["rank"], ref["depth"], TOL_MIXED, label=label)


def _alone(U, variant):
    if variant == "pairs":
        return pid.pid_all_pairs(U)
    if variant == "depths":
        return pid.pid_pairs_depths(U)
    return pid.pid_mean(U)


def _overlapping(intervals):
    """True if some two (start, end) intervals intersect."""
    for a, (sa, ea) in enumerate(intervals):
        for b, (sb, eb) in enumerate(intervals):
            if a != b and sa < eb and sb < ea:
                return True
    return False


def test_mixed_equals_alone_and_oracle(pool, big):
    rng = np.random.Generator(np.random.PCG64(5))
    srv = pid.PidServer(512 << 20, max_slots=3)
    # a long request first, so that the following ones are admitted while it runs
    t_big, out_big = srv.pid_submit(big, variant="pairs")
    jobs = [(big, "pairs", t_big, out_big)]
    variants = ("pairs", "mean", "depths")
    for k in range(18):
        key = list(pool)[k % 3]
        n = int(rng.integers(8, pool[key].shape[0] + 1))
        variant = variants[k % 3]
        U = pool[key][:n]
        t, out = srv.pid_submit(U, variant=variant, inclusion=(variant == "pairs"))
        jobs.append((U, variant, t, out))
    for U, variant, t, out in jobs:
        assert srv.pid_wait(t) == pid.PID_OK, srv.last_error()
    torch.cuda.synchronize()
    dev = [srv.pid_request_device_times(t) for _, _, t, _ in jobs]
    assert all(e >= s >= 0 for s, e in dev)
    assert _overlapping(dev), "no two requests were on the device at the same time"
    for U, variant, t, out in jobs:
        label = f"served {variant} {tuple(U.shape)}"
        alone = _alone(U, variant)
        for key in KEYS + (("inclusion",) if "inclusion" in out else ()):
            assert torch.equal(out[key], alone[key]), (label, key)
        _check_against_oracle(U, variant, out, label)
        srv.release(t)
    with pytest.raises(pid.PidError):
        srv.pid_poll(t_big)                    # released tickets are unknown
    srv.pid_server_destroy()


def test_waits_for_arena_memory(pool, big):
    """Each request fits the arena alone, not both together: the second one
    starts on the device only after the first has finished, although a slot
    is free, and both results are right."""
    U2 = pool[("2d", 320)][:200]
    w1 = pid.pid_workspace_size(big, variant=0)
    w2 = pid.pid_workspace_size(U2, variant=0)
    arena = max(w1, w2) + min(w1, w2) // 2
    srv = pid.PidServer(arena, max_slots=4)
    t1, o1 = srv.pid_submit(big, variant="pairs")
    t2, o2 = srv.pid_submit(U2, variant="pairs")
    assert srv.pid_wait(t1) == pid.PID_OK and srv.pid_wait(t2) == pid.PID_OK
    (s1, e1), (s2, e2) = srv.pid_request_device_times(t1), srv.pid_request_device_times(t2)
    assert s2 >= e1, (s1, e1, s2, e2)
    _, start2, _ = srv.pid_request_times(t2)
    _, _, done1 = srv.pid_request_times(t1)
    assert start2 >= done1
    for U, out in ((big, o1), (U2, o2)):
        alone = pid.pid_all_pairs(U, inclusion=False)
        for key in KEYS:
            assert torch.equal(out[key], alone[key]), key
    _check_against_oracle(U2, "pairs", o2, "waited for memory")
    srv.pid_server_destroy()


def test_footprint_budget_serialises(pool):
    """A footprint budget that holds one request at a time: no overlap."""
    Ua, Ub = pool[("3d", 48)][:64], pool[("3d", 48)][:50]
    srv = pid.PidServer(256 << 20, max_slots=4)
    fa = Ua.numel() * 2 + pid.pid_workspace_size(Ua, variant=1) + 6 * 8 * 64
    srv.pid_server_set_budget(int(fa * 1.5))
    tickets = [srv.pid_submit(U, variant="mean")[0] for U in (Ua, Ub, Ua, Ub)]
    for t in tickets:
        assert srv.pid_wait(t) == pid.PID_OK
    dev = [srv.pid_request_device_times(t) for t in tickets]
    assert not _overlapping(dev), dev
    # a request whose footprint alone exceeds the budget is refused at once
    srv.pid_server_set_budget(1 << 10)
    with pytest.raises(pid.PidError) as ei:
        srv.pid_submit(Ua, variant="mean")
    assert ei.value.status == pid.PID_ERR_OVER_BUDGET
    srv.pid_server_destroy()


def test_failed_request_reports_its_error(pool):
    """A request that fails its value check ends with PID_ERR_VALUE_RANGE and
    its error text; requests around it complete normally."""
    U = pool[("2d", 128)][:40].clone()
    bad = U.clone()
    bad[3, 17] = float("nan")
    srv = pid.PidServer(64 << 20, max_slots=2)
    t0, out0 = srv.pid_submit(U, variant="mean")
    t1, _ = srv.pid_submit(bad, variant="mean", validate=True)
    t2, out2 = srv.pid_submit(U, variant="mean", validate=True)
    assert srv.pid_wait(t1) == pid.PID_ERR_VALUE_RANGE
    assert "probability" in srv.last_error()
    assert srv.pid_wait(t0) == pid.PID_OK and srv.pid_wait(t2) == pid.PID_OK
    alone = pid.pid_mean(U)
    for key in KEYS:
        assert torch.equal(out0[key], alone[key]) and torch.equal(out2[key], alone[key]), key
    srv.pid_server_destroy()


def test_over_budget_and_cancel(pool):
    srv = pid.PidServer(1 << 16, max_slots=1)
    with pytest.raises(pid.PidError) as ei:
        srv.pid_submit(pool[("2d", 320)], variant="pairs")
    assert ei.value.status == pid.PID_ERR_OVER_BUDGET
    srv.pid_server_destroy()
    # destroying the server while requests are queued returns promptly: the
    # running request finishes, the queued ones are cancelled
    srv = pid.PidServer(64 << 20, max_slots=1)
    for _ in range(30):
        srv.pid_submit(pool[("3d", 48)][:40], variant="mean")
    th = threading.Thread(target=srv.pid_server_destroy)
    th.start()
    th.join(timeout=60)
    assert not th.is_alive() and srv.h is None


def test_binary_requests_served(pool):
    """Binary PID-mean requests of the three input forms (U8 masks, bit-packed
    masks, thresholded FP16 masks) served beside soft requests: bitwise the
    oracle's integer results and the same call run alone."""
    srv = pid.PidServer(256 << 20, max_slots=3)
    B = synth.ellipsoids_3d(300, 40, 21, device=DEV)                  # U8 0/1, 64,000 points
    P = pid.pid_pack_bits(B[:200])
    F = pool[("2d", 128)][:90]
    step = dict(kind="step", c=0.5, side=1)
    reqs = [(B, None), (P, None), (F, step), (B[:37], None), (pool[("3d", 48)][:30], None)]
    jobs = []
    for U, iso in reqs:
        t, out = srv.pid_submit(U, variant="mean", iso=iso)
        jobs.append((U, iso, t, out))
    for U, iso, t, out in jobs:
        assert srv.pid_wait(t) == pid.PID_OK, srv.last_error()
    torch.cuda.synchronize()
    for U, iso, t, out in jobs:
        alone = pid.pid_mean(U, iso=iso)
        for key in KEYS:
            assert torch.equal(out[key], alone[key]), key
        if isinstance(U, pid.PackedMasks):
            bits = B[:200].cpu().numpy()
        elif iso is not None:
            bits = oracle.extract(U.cpu().to(torch.float64).numpy(), iso).astype(np.uint8)
        elif U.dtype == torch.uint8:
            bits = U.cpu().numpy()
        else:
            _check_against_oracle(U, "mean", out, "served soft mean")
            continue
        ref = oracle.binary_pid_mean(bits)
        for key in ("mass", "in_in", "in_out", "depth"):
            assert np.array_equal(out[key].cpu().numpy(), ref[key]), key
        srv.release(t)
    srv.pid_server_destroy()
