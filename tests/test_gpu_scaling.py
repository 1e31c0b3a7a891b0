"""GPU parity at the shapes of the paper's scalability study (Sec. 5.2):
binary 3D ellipsoid ensembles through the exact integer PID-mean path."""
import numpy as np
import pytest

import oracle
import paper_2512_15187_amd as pid
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("n,res", [(2000, 50), (50, 128)])
def test_pid_mean_ellipsoids_bitexact(n, res):
    """Binary 3D ellipsoid ensembles (80 % normal, 20 % outliers) at the
    shapes of the scalability study: PID-mean through the exact integer path
    bitwise equal to the oracle's integer form."""
    B = synth.ellipsoids_3d(n, res, 60 + n + res)
    res_gpu = pid.pid_mean(B.to(DEV))
    ref = oracle.binary_pid_mean(B.numpy())
    for k in ("in_in", "in_out", "depth", "mass"):
        a = res_gpu[k].cpu().numpy()
        assert np.array_equal(a, ref[k]), (k, np.flatnonzero(a != ref[k])[:5])
