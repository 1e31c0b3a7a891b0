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


def test_mixed_equals_alone(pool):
    rng = np.random.Generator(np.random.PCG64(5))
    srv = pid.PidServer(256 << 20, max_slots=3)
    jobs = []
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
    starts = sorted(srv.pid_request_times(t)[1] for _, _, t, _ in jobs)
    ends = sorted(srv.pid_request_times(t)[2] for _, _, t, _ in jobs)
    assert starts[1] < ends[0] or len(jobs) == 1, "no two requests were in flight together"
    for U, variant, t, out in jobs:
        alone = pid.pid_all_pairs(U) if variant == "pairs" else pid.pid_mean(U)
        for key in KEYS + (("inclusion",) if variant == "pairs" else ()):
            assert torch.equal(out[key], alone[key]), (variant, tuple(U.shape), key)
    srv.pid_server_destroy()


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
