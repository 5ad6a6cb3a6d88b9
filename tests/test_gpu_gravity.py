"""Self-gravity on the GPU (periodic FFT Poisson solve feeding S) against
the oracle, whose potential is the discrete Fourier transform written out
from its definition: potential and gradient after a step, whole-state parity
over several steps (FP64 <= 1e-11), the FP32 path, and the Jeans linear
theory at any size."""
import math

import numpy as np
import pytest

from mhd_inputs import problems as P
from tests.gpu_util import field_errors, gpu_sim, host_state, needs_gpu
from tests.helpers import oracle_of

pytestmark = [pytest.mark.gpu, needs_gpu]


def _gravity_box(shape, seed, G=2.0):
    pb = P.random_smooth(shape, seed=seed)
    pb.source, pb.src = P.SRC_SELF_GRAVITY, (G, 0.0, 0.0, 0.0)
    return pb


@pytest.mark.parametrize("shape", [(16, 8, 32), (32, 4, 1), (8, 8, 8), (1024, 2, 4), (4, 512, 2),
                                   (2, 4, 256), (128, 64, 2)])
def test_potential_and_state_match_oracle(shape):
    """Every FFT line length from 2 to 1024 (each splits n = R1 R2
    differently) along each axis."""
    pb = _gravity_box(shape, seed=41)
    o = oracle_of(pb)
    s = gpu_sim(pb)
    dts = []
    for _ in range(3):
        dts.append(o.dt())
        o.step(dts[-1])
    s.step(3, dt=dts)
    # potential and gradient of the last (corrector) stage, interior cells
    sl = (slice(2, 2 + pb.nz), slice(2, 2 + pb.ny), slice(2, 2 + pb.nx))
    for gw, ow in ((35, 41), (36, 42), (37, 43), (38, 44)):
        g = s.debug_array(gw).cpu().numpy()[sl]
        r = o.debug_array(ow)[sl]
        sc = np.abs(r).max()
        if sc == 0:  # a single-cell axis has no gradient
            assert np.abs(g).max() == 0
            continue
        assert np.abs(g - r).max() <= 1e-11 * sc, (gw, np.abs(g - r).max() / sc)
    err = field_errors(host_state(s), o.get_state())
    assert max(err.values()) <= 1e-11, err


def test_fp32_gravity_close_to_fp64_oracle():
    pb = _gravity_box((32, 16, 16), seed=42).astype("float32")
    o = oracle_of(pb)
    s = gpu_sim(pb, precision=1)
    dts = []
    for _ in range(5):
        dts.append(o.dt())
        o.step(dts[-1])
    s.step(5, dt=dts)
    g, r = host_state(s), o.get_state()
    l1 = float(np.abs(g[0][0] - r[0][0]).mean() / np.abs(r[0][0]).mean())
    assert l1 <= 1e-6, l1


@pytest.mark.parametrize("k_over_kj", [0.5, 2.0])
def test_jeans_linear_theory_on_device(k_over_kj):
    """Same as the oracle pin: growth as cosh(g t) below the Jeans scale,
    oscillation as cos(w t) above it, laid along z this time."""
    n, t = 64, 0.25
    pb = P.jeans(n, axis=2, k_over_kj=k_over_kj)
    s = gpu_sim(pb)

    def amp():
        rho = s.get_state()[0][0].double().cpu().numpy().reshape(-1)
        x = (np.arange(n) + 0.5) / n
        return 2.0 * float(np.mean((rho - rho.mean()) * np.cos(2.0 * math.pi * x)))

    a0 = amp()
    tt = 0.0
    while tt < t * (1 - 1e-14):
        dt = min(s.dt(), t - tt)
        s.step(1, dt=dt)
        tt += dt
    r = pb.extra["rate"]
    want = math.cosh(r * t) if pb.extra["growing"] else math.cos(r * t)
    assert abs(amp() / a0 - want) <= 0.03 * max(1.0, abs(want))
