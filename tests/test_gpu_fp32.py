"""FP32-bulk path (FP64 kept for flagged pressure recovery, dt and sums)
against the FP64 oracle: both start from the same FP32-rounded state and use
the same time steps; L1 and Linf per field are checked against stated bounds."""
import numpy as np
import pytest

from mhd_inputs import problems as P
from tests.gpu_util import gpu_sim, host_state, needs_gpu
from tests.helpers import oracle_of

pytestmark = [pytest.mark.gpu, needs_gpu]


def _run(pb, nsteps):
    pb = pb.astype("float32")
    o = oracle_of(pb)
    s = gpu_sim(pb, precision=1)
    dts = []
    for _ in range(nsteps):
        dts.append(o.dt())
        o.step(dts[-1])
    s.step(nsteps, dt=dts)
    g = host_state(s)
    r = o.get_state()
    l1 = {}
    for m, nm in enumerate(("rho", "Mx", "My", "Mz", "E")):
        l1[nm] = float(np.abs(g[0][m] - r[0][m]).mean() / np.abs(r[0][m]).mean())
    d = s.diag()
    return l1, d, g, r


def test_fp32_random_box():
    l1, d, g, r = _run(P.random_smooth((48, 40, 32), seed=41), 10)
    assert l1["rho"] <= 1e-6, l1
    assert l1["E"] <= 1e-6, l1
    assert d["status"] == 0


def test_fp32_turbulent_box():
    """64^3 box from the turbulent-ISM generator (rougher than at 256^3:
    the k <= 16 spectrum is resolved by 4 cells)."""
    l1, d, g, r = _run(P.turbulent_ism(64, seed=2), 20)
    assert l1["rho"] <= 1e-5, l1
    assert d["status"] == 0


def test_fp32_alfven():
    l1, d, g, r = _run(P.alfven(32), 10)
    assert l1["rho"] <= 1e-6, l1
    for m in (1, 2, 3):
        assert l1[("rho", "Mx", "My", "Mz")[m]] <= 1e-5, l1
