"""Serving loop: requests of uneven size admitted while others run give
bitwise the same results as the same requests run alone; over-budget and
cancelled requests are reported."""
import numpy as np
import pytest
import torch

import paper_2512_15187_amd as pid
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
KEYS = ("mass", "in_in", "in_out", "depth", "rank", "order")


@pytest.fixture(scope="module")
def pool():
    return {("2d", 128): synth.serving_pool("2d", 128, 96, device=DEV),
            ("2d", 320): synth.serving_pool("2d", 320, 300, device=DEV),
            ("3d", 48): synth.serving_pool("3d", 48, 64, device=DEV)}


def _overlap(times):
    """True if some two requests were on the device at the same time."""
    for a, (_, sa, da) in enumerate(times):
        for b, (_, sb, db) in enumerate(times):
            if a != b and sa < db and sb < da:
                return True
    return False


def test_mixed_equals_alone(pool, big):
    rng = np.random.Generator(np.random.PCG64(5))
    srv = pid.PidServer(512 << 20, max_slots=3)
    # a long request first, so that the following ones are admitted while it runs
    t_big, out_big = srv.pid_submit(big, variant="pairs")
    jobs = [(big, "pairs", t_big, out_big)]
    for k in range(16):
        key = list(pool)[k % 3]
        n = int(rng.integers(8, pool[key].shape[0] + 1))
        variant = "pairs" if k % 2 == 0 else "mean"
        U = pool[key][:n]
        t, out = srv.pid_submit(U, variant=variant, inclusion=(variant == "pairs"))
        jobs.append((U, variant, t, out))
    for U, variant, t, out in jobs:
        assert srv.pid_wait(t) == pid.PID_OK
    torch.cuda.synchronize()
    times = [srv.pid_request_times(t) for _, _, t, _ in jobs]
    assert _overlap(times), "no two requests were in flight together"
    for U, variant, t, out in jobs:
        alone = pid.pid_all_pairs(U) if variant == "pairs" else pid.pid_mean(U)
        for key in KEYS + (("inclusion",) if variant == "pairs" and "inclusion" in out else ()):
            assert torch.equal(out[key], alone[key]), (variant, tuple(U.shape), key)
    srv.pid_server_destroy()


@pytest.fixture(scope="module")
def big():
    """All-pairs request of 512 members on 1024 x 1024 (several milliseconds)."""
    return synth.serving_pool("2d", 1024, 512, device=DEV)


def test_over_budget_and_cancel(pool):
    srv = pid.PidServer(1 << 16, max_slots=1)
    with pytest.raises(pid.PidError) as ei:
        srv.pid_submit(pool[("2d", 320)], variant="pairs")
    assert ei.value.status == pid.PID_ERR_OVER_BUDGET
    srv.pid_server_destroy()
    # destroying the server while requests are queued returns promptly: the
    # running request finishes, the queued ones are cancelled
    import threading
    srv = pid.PidServer(64 << 20, max_slots=1)
    for _ in range(30):
        srv.pid_submit(pool[("3d", 48)][:40], variant="mean")
    th = threading.Thread(target=srv.pid_server_destroy)
    th.start()
    th.join(timeout=60)
    assert not th.is_alive() and srv.h is None
