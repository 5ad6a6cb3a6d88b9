"""Pins of the oracle's CFL step and of its fixed-potential sources, by values
that do not come from the oracle's own formulas.

* CFL (reading R9: the paper gives no time-step rule): hand-worked values of
  dt = C min_cells min_a d_a / (|v_a| + c_f,a) for uniform states with unequal
  cell sizes, oblique velocity and oblique field, from the textbook form of
  the fast speed (tests/golden/cfl_dt_hand.json).
* Source S of Eq. 2 (section 2.1), S = (0, -rho grad Phi, -rho v.grad Phi, 0):
  gas at rest with uniform pressure has uniform fluxes, so one very short
  step changes the momentum by -rho grad Phi dt at each cell centre.  grad Phi
  is taken here by a central difference of the potential as printed: the
  disc's logarithmic potential (section 4) and the Gaussian well of the bow
  shock test (section 3).
"""
import json
import math
import os

import numpy as np
import pytest

from mhd_inputs import problems as P
from tests.helpers import oracle_of

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cfl_dt_hand.json")


def _cfl_problem(case):
    nx, ny, nz = case["n"]
    pb = P.uniform((nx, ny, nz), rho=case["rho"], v=tuple(case["v"]), p=case["p"],
                   b=tuple(case["b"]), d=tuple(case["d"]))
    fc = case.get("fast_cell")
    if fc:
        i, j, k = fc["ijk"]
        rho, p = case["rho"], case["p"]
        v = fc["v"]
        b2 = sum(x * x for x in case["b"])
        pb.cell5[1:4, k, j, i] = [rho * v[0], rho * v[1], rho * v[2]]
        pb.cell5[4, k, j, i] = p / (pb.gamma - 1.0) + 0.5 * rho * sum(x * x for x in v) + 0.5 * b2
    return pb


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_cfl_dt_hand_values(case):
    pb = _cfl_problem(case)
    assert pb.cfl == 0.4 and abs(pb.gamma - 5.0 / 3.0) < 1e-15
    o = oracle_of(pb)
    assert o.dt() == pytest.approx(case["dt"], rel=1e-14)


def test_cfl_dt_scales_with_courant_number():
    """dt is linear in the Courant number (same state, C = 0.4 and 0.25)."""
    case = _cases()[1]
    pb = _cfl_problem(case)
    o = oracle_of(pb, cfl=0.25)
    assert o.dt() == pytest.approx(case["dt"] * 0.25 / 0.4, rel=1e-14)


# ------------------------------------------------------------------ source --

def _phi_logpot(x, y, z, v0, rc, q):
    """Disc potential as printed: Phi = v0^2/2 ln(Rc^2 + R^2 + z^2/q^2)."""
    return 0.5 * v0 * v0 * np.log(rc * rc + x * x + y * y + z * z / (q * q))


def _phi_gauss(x, y, z, A, w):
    """Bow-shock well as printed: Phi = -A exp(-(x/w)^2)."""
    return -A * np.exp(-(x / w) ** 2) + 0.0 * (y + z)


def _central_grad(phi, X, Y, Z, h):
    return (
        (phi(X + h, Y, Z) - phi(X - h, Y, Z)) / (2 * h),
        (phi(X, Y + h, Z) - phi(X, Y - h, Z)) / (2 * h),
        (phi(X, Y, Z + h) - phi(X, Y, Z - h)) / (2 * h),
    )


def _rest_box(n, d, x0, rho, p, b=(0.0, 0.0, 0.0)):
    pb = P.uniform(n, rho=rho, v=(0.0, 0.0, 0.0), p=p, b=b, d=d, bc=(P.OUTFLOW,) * 6)
    pb.x0, pb.y0, pb.z0 = x0
    return pb


def _momentum_rate(pb, dt):
    o = oracle_of(pb)
    o.step(dt)
    c5, *_ = o.get_state()
    return [c5[1 + a] / dt for a in range(3)], (c5[4] - pb.cell5[4]) / dt


@pytest.mark.parametrize("q", [1.0, 0.7])
def test_logpot_source_is_minus_rho_grad_phi(q):
    """Uniform gas at rest in the disc potential (v0 = 200, Rc = 0.5, q): after
    one step of 1e-9 the momentum equals -rho grad Phi dt (all three
    components, both signs of every coordinate), energy stays at rest."""
    v0, rc = 200.0, 0.5
    rho, p = 1.3, 1.0
    pb = _rest_box((8, 6, 4), (1.0, 0.9, 0.45), (-3.1, -2.2, -0.85), rho, p, b=(0.1, -0.2, 0.05))
    pb.source, pb.src = P.SRC_LOGPOT, (v0, rc, q, 0.0)
    dt = 1e-9
    rate, erate = _momentum_rate(pb, dt)
    X, Y, Z = P.cell_centres(pb)
    g = _central_grad(lambda x, y, z: _phi_logpot(x, y, z, v0, rc, q), X, Y, Z, 1e-4)
    scale = max(np.max(np.abs(rho * gi)) for gi in g)
    for a in range(3):
        np.testing.assert_allclose(rate[a], -rho * g[a], rtol=0, atol=1e-6 * scale)
    # the energy gained is the kinetic energy of the velocity the step gave:
    # second order in dt
    assert np.max(np.abs(erate)) < dt * scale * scale / rho


def test_gaussian_well_source_is_minus_rho_grad_phi():
    """Gas at rest over the bow-shock well Phi = -5 exp(-(x/0.1)^2) (section 3):
    momentum after one step of 1e-9 is -rho dPhi/dx dt along x (towards the
    well's centre on both sides), zero along y and z."""
    A, w = 5.0, 0.1
    rho, p = 1.0, 1.0
    pb = _rest_box((30, 2, 2), (0.02, 0.02, 0.02), (-0.3, 0.0, 0.0), rho, p)
    pb.source, pb.src = P.SRC_GAUSS_X, (A, w, 0.0, 0.0)
    dt = 1e-9
    rate, erate = _momentum_rate(pb, dt)
    X, Y, Z = P.cell_centres(pb)
    g = _central_grad(lambda x, y, z: _phi_gauss(x, y, z, A, w), X, Y, Z, 1e-5)
    scale = np.max(np.abs(rho * g[0]))
    assert scale > 10.0
    np.testing.assert_allclose(rate[0], -rho * g[0], rtol=0, atol=1e-6 * scale)
    # gas left of the centre is pulled to +x, right of it to -x
    assert np.all(rate[0][X < 0] > 0) and np.all(rate[0][X > 0] < 0)
    assert np.max(np.abs(rate[1])) == 0.0 and np.max(np.abs(rate[2])) == 0.0
    assert np.max(np.abs(erate)) < dt * scale * scale / rho


def test_logpot_energy_source_moving_gas():
    """Gas moving uniformly through the potential: a uniform stream has
    uniform fluxes, so over one short step the energy changes by the source
    -rho v.grad Phi dt, up to terms of second order in dt (the step's own
    velocity change; dt = 1e-11 keeps them below 1e-6 of the source)."""
    v0, rc, q = 200.0, 0.5, 1.0
    rho, p, v = 0.8, 1.0, (1.5, -0.7, 0.4)
    pb = P.uniform((6, 6, 4), rho=rho, v=v, p=p, b=(0.0, 0.0, 0.0), d=(1.0, 1.0, 0.5),
                   bc=(P.OUTFLOW,) * 6)
    pb.x0, pb.y0, pb.z0 = -2.7, 0.4, -1.1
    pb.source, pb.src = P.SRC_LOGPOT, (v0, rc, q, 0.0)
    dt = 1e-11
    o = oracle_of(pb)
    o.step(dt)
    c5, *_ = o.get_state()
    X, Y, Z = P.cell_centres(pb)
    g = _central_grad(lambda x, y, z: _phi_logpot(x, y, z, v0, rc, q), X, Y, Z, 1e-4)
    expect = -rho * (v[0] * g[0] + v[1] * g[1] + v[2] * g[2])
    got = (c5[4] - pb.cell5[4]) / dt
    scale = np.max(np.abs(expect))
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-5 * scale)
    assert math.isfinite(scale) and scale > 1e3
