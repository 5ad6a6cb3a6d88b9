"""Pins of the synthetic galactic-disc slab (the disc workloads' input):
what its generator's model fixes, checked by routes other than the
generator's own formulas.

* The rotation balances the logarithmic potential of the source term:
  v_phi^2 / R equals dPhi/dR, with the derivative taken by central
  differences of Phi itself; the flow is purely azimuthal.
* The field is divergence-free on the faces (it comes from a vector
  potential) and toroidal, and the plasma beta 2P / |B|^2 is the same
  everywhere, since B^2 and P share the profile exp(-R/rd) sech^2(z/h).
* The gas is isothermal (P = rho cs^2), its density the exponential,
  sech^2 profile with 1 % multiplicative noise clipped at 3 sigma, floored.
"""
import math

import numpy as np
import pytest

from mhd_inputs import problems as P

NX, NY, NZ = 64, 64, 16


@pytest.fixture(scope="module")
def disc():
    pb = P.disc(NX, NY, NZ)
    X, Y, Z = P.cell_centres(pb)
    return pb, X, Y, Z


def _prims(pb):
    c5 = pb.cell5
    rho = c5[0]
    v = [c5[1 + a] / rho for a in range(3)]
    bc = [0.5 * (pb.bx[:, :, :-1] + pb.bx[:, :, 1:]), 0.5 * (pb.by[:, :-1, :] + pb.by[:, 1:, :]),
          0.5 * (pb.bz[:-1] + pb.bz[1:])]
    ke = 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    me = 0.5 * (bc[0] ** 2 + bc[1] ** 2 + bc[2] ** 2)
    p = (pb.gamma - 1.0) * (c5[4] - ke - me)
    return rho, v, bc, p


def test_rotation_balances_the_log_potential(disc):
    pb, X, Y, Z = disc
    v0, rc, q = pb.src[0], pb.src[1], pb.src[2]
    _, v, _, _ = _prims(pb)
    R = np.sqrt(X ** 2 + Y ** 2)

    def phi(r, z):
        return 0.5 * v0 * v0 * np.log(rc * rc + r * r + (z / q) ** 2)

    dr = 1e-4
    dphi = (phi(R + dr, Z) - phi(R - dr, Z)) / (2 * dr)
    vphi = (-Y * v[0] + X * v[1]) / R
    np.testing.assert_allclose(vphi ** 2 / R, dphi, rtol=1e-6)
    vr = (X * v[0] + Y * v[1]) / R
    assert np.abs(vr).max() <= 1e-9 * v0
    assert np.abs(v[2]).max() == 0.0


def test_field_divergence_free_toroidal_constant_beta(disc):
    pb, X, Y, Z = disc
    rho, _, bc, p = _prims(pb)
    div = ((pb.bx[:, :, 1:] - pb.bx[:, :, :-1]) / pb.dx + (pb.by[:, 1:, :] - pb.by[:, :-1, :]) / pb.dy
           + (pb.bz[1:] - pb.bz[:-1]) / pb.dz)
    bmax = max(np.abs(pb.bx).max(), np.abs(pb.by).max())
    assert np.abs(div).max() * pb.dx <= 1e-12 * bmax
    assert np.abs(pb.bz).max() == 0.0
    R = np.sqrt(X ** 2 + Y ** 2)
    b2 = bc[0] ** 2 + bc[1] ** 2
    # toroidal: the radial component is a discretisation remainder
    br = (X * bc[0] + Y * bc[1]) / R
    far = R > 4 * pb.dx
    assert np.abs(br[far]).max() <= 0.01 * np.sqrt(b2[far]).max()
    # beta = 2 P / B^2 is the configured 10 wherever the noise and the
    # floor leave the profile (inside the disc, away from the axis)
    body = far & (np.abs(Z) < 0.4) & (R < 9.0)
    beta = 2.0 * p[body] / b2[body]
    assert abs(np.median(beta) - 10.0) < 0.2
    assert np.percentile(np.abs(beta / 10.0 - 1.0), 90) < 0.06


def test_isothermal_density_profile_with_noise(disc):
    pb, X, Y, Z = disc
    rho, _, _, p = _prims(pb)
    cs, rd, h, noise = 10.0, 3.0, 0.2, 0.01
    floor = pb.rho_floor
    R = np.sqrt(X ** 2 + Y ** 2)
    model = np.exp(-R / rd) / np.cosh(Z / h) ** 2
    above = model * (1 - 3 * noise) > floor
    xi = (rho[above] / model[above] - 1.0) / noise
    assert abs(xi.mean()) < 0.05
    assert abs(xi.std() - 1.0) < 0.05
    assert np.abs(xi).max() <= 3.0 + 1e-9
    np.testing.assert_allclose(p[above], rho[above] * cs * cs, rtol=1e-9)
    assert rho.min() >= floor
    assert math.isclose(pb.p_floor, floor * cs * cs)
