"""Pins of the oracle's N-body particles (section 2.1: particle-in-cell
dynamics with the "flip-flop" integrator and a mass-conserving
second-order mass assignment), sharing the periodic FFT potential.

What fixes them independently of the oracle:
* the deposit equals the definition it restates -- the volume of a
  one-cell cube around the particle that falls into each cell -- computed
  here as products of 1-D interval overlaps, including across the periodic
  wrap, and conserves mass;
* interpolation reproduces linear fields and constants;
* two particles, or a cloud, keep their total momentum to rounding (same
  weights both ways, a symmetric gradient); with the gas coupled, gas plus
  particles keep the total;
* the integrator is time-reversible: flipping the velocities retraces the
  orbit;
* a cold plane wave grows as cosh(gamma t) with the closed-form growth
  rate of the discrete operators, gamma^2 = 4 pi G rho0 cos^2(k h / 2)
  (deposit sin(kh/2)/(h/2)-weighted, 7-point Laplacian, central gradient
  and interpolation to the lattice combined), within 1e-4 (and within 2 %
  of the continuum rate);
* a Plummer sphere in equilibrium keeps its total energy.
"""
import math

import numpy as np
import pytest

from mhd_inputs import problems as P
from oracle import pyorc as O
from tests.helpers import orc_config


def _oracle(pb, x, v, m):
    cfg = orc_config(pb)
    cfg.npart = x.shape[1]
    o = O.Oracle(cfg)
    assert o.set_state(pb.cell5, pb.bx, pb.by, pb.bz) == 0
    o.set_particles(x, v, m)
    return o


def _overlap_deposit(pb, x, m):
    """rho of each cell = sum over particles of m * (volume of the cube
    [x - d/2, x + d/2] inside the cell, over the box's periodic images) / dV^2."""
    n = (pb.nx, pb.ny, pb.nz)
    d = (pb.dx, pb.dy, pb.dz)
    lo = (pb.x0, pb.y0, pb.z0)
    rho = np.zeros((pb.nz, pb.ny, pb.nx))
    for q in range(x.shape[1]):
        ov = []
        for a in range(3):
            L = n[a] * d[a]
            edges = lo[a] + np.arange(n[a] + 1) * d[a]
            o1 = np.zeros(n[a])
            for img in (-L, 0.0, L):
                c0, c1 = x[a, q] + img - 0.5 * d[a], x[a, q] + img + 0.5 * d[a]
                o1 += np.clip(np.minimum(edges[1:], c1) - np.maximum(edges[:-1], c0), 0.0, None)
            ov.append(o1)
        rho += m[q] * np.einsum("k,j,i->kji", ov[2], ov[1], ov[0])
    return rho / (pb.dx * pb.dy * pb.dz) ** 2


def test_deposit_is_the_volume_overlap_and_conserves_mass():
    pb = P.gravity_box((8, 6, 5), d=(0.1, 0.2, 0.15))
    rng = np.random.default_rng(1)
    n = 60
    L = np.array([0.8, 1.2, 0.75])
    x = rng.uniform(0, 1, (3, n)) * L[:, None]
    # particles on cell centres, faces and the periodic seam
    x[:, 0] = [0.05, 0.1, 0.075]
    x[:, 1] = [0.0, 0.0, 0.0]
    x[:, 2] = [0.8 - 1e-12, 0.6, 0.74]
    m = rng.uniform(0.5, 2.0, n)
    o = _oracle(pb, x, np.zeros_like(x), m)
    rho = o.particle_deposit(x)
    want = _overlap_deposit(pb, x, m)
    assert np.abs(rho - want).max() <= 1e-12 * want.max()
    assert abs(rho.sum() * 0.1 * 0.2 * 0.15 - m.sum()) <= 1e-13 * m.sum()
    # a particle on a cell centre puts all its mass into that cell
    r1 = o.particle_deposit(np.repeat([[0.05], [0.1], [0.075]], n, axis=1))
    assert r1[0, 0, 0] == pytest.approx(m.sum() / (0.1 * 0.2 * 0.15), rel=1e-14)
    assert np.count_nonzero(r1) == 1


def test_interpolation_reproduces_linear_fields():
    pb = P.gravity_box((10, 8, 6), d=(0.1, 0.125, 0.2))
    rng = np.random.default_rng(2)
    Xc, Yc, Zc = P.cell_centres(pb)
    f = 0.3 + 1.5 * Xc - 2.0 * Yc + 0.7 * Zc
    # inside the span of the cell centres (no wrap): exact
    lo = np.array([0.05, 0.0625, 0.1])
    hi = np.array([0.95, 0.9375, 1.1])
    x = lo[:, None] + rng.uniform(0, 1, (3, 200)) * (hi - lo)[:, None]
    o = _oracle(pb, x[:, :5], np.zeros((3, 5)), np.ones(5))
    got = o.particle_interp(f, x)
    want = 0.3 + 1.5 * x[0] - 2.0 * x[1] + 0.7 * x[2]
    assert np.abs(got - want).max() <= 1e-13
    assert np.abs(o.particle_interp(np.full_like(f, 2.5), rng.uniform(0, 1, (3, 50)))
                  - 2.5).max() <= 1e-14


def test_two_particles_conserve_momentum():
    pb = P.gravity_box((16, 16, 16))
    x = np.array([[0.31, 0.62], [0.44, 0.52], [0.5, 0.47]])
    v = np.array([[0.1, -0.2], [0.0, 0.05], [0.02, 0.0]])
    m = np.array([1.0, 0.4])
    o = _oracle(pb, x, v, m)
    p0 = (v * m).sum(axis=1)
    for _ in range(30):
        o.step(0.01)
    x1, v1 = o.get_particles()
    p1 = (v1 * m).sum(axis=1)
    assert np.abs(p1 - p0).max() <= 1e-13
    # they attract: the separation along x shrank
    assert abs(x1[0, 1] - x1[0, 0]) < abs(0.62 - 0.31) + 30 * 0.01 * 0.3


def test_gas_and_particles_conserve_total_momentum():
    """Coupled: the gas feels and sources the potential; the corrector's
    potential moves gas and particles alike, so the total is constant."""
    pb = P.random_smooth((16, 16, 16), seed=3)
    pb.source, pb.src = P.SRC_SELF_GRAVITY, (0.5, 0.0, 0.0, 0.0)
    x, v, m = P.particles_plummer(pb, 300, seed=4, scale=0.1, mass_total=2.0, G=0.5)
    o = _oracle(pb, x, v, m)
    dv = pb.dx * pb.dy * pb.dz

    def total():
        c5, *_ = o.get_state()
        _, vv = o.get_particles()
        return np.array([c5[1 + a].sum() * dv for a in range(3)]) + (vv * m).sum(axis=1)

    p0 = total()
    for _ in range(5):
        o.step()
    p1 = total()
    assert np.abs(p1 - p0).max() <= 1e-12 * (np.abs(x).max() + 1.0)
    _, v1 = o.get_particles()
    assert np.abs(v1 - v).max() > 1e-3


def test_flip_flop_is_time_reversible():
    pb = P.gravity_box((16, 16, 16))
    x, v, m = P.particles_plummer(pb, 200, seed=5, scale=0.1)
    o = _oracle(pb, x, v, m)
    for _ in range(40):
        o.step(0.005)
    x1, v1 = o.get_particles()
    o2 = _oracle(pb, x1, -v1, m)
    for _ in range(40):
        o2.step(0.005)
    x2, v2 = o2.get_particles()
    dx = x2 - x
    dx -= np.round(dx)   # unit periodic box
    assert np.abs(dx).max() <= 1e-10
    assert np.abs(-v2 - v).max() <= 1e-9 * np.abs(v).max()
    assert np.abs(x1 - x).max() > 1e-2  # it did move


def test_cold_plane_wave_grows_at_the_discrete_rate():
    n = (32, 4, 4)
    rho0 = 1.0
    G = 1.0 / (4.0 * math.pi * rho0)   # continuum gamma = 1
    pb = P.gravity_box(n, G=G)
    amp = 0.01
    x, v, m = P.particles_plane_wave(pb, amp=amp, mass_total=rho0)   # unit box: mass = rho0
    lat = np.round(x[0] / pb.dx) * pb.dx   # the lattice (displacements << a cell)
    o = _oracle(pb, x, v, m)
    t_end, dt = 2.0, 0.005
    for _ in range(int(round(t_end / dt))):
        o.step(dt)
    x1, _ = o.get_particles()
    disp = x1[0] - lat
    disp -= np.round(disp)
    a1 = 2.0 * np.mean(disp * np.sin(2 * math.pi * lat))
    a0 = amp * pb.dx
    kh = 2 * math.pi * pb.dx
    g_disc = math.cos(0.5 * kh)
    assert a1 / a0 == pytest.approx(math.cosh(g_disc * t_end), rel=1e-4)
    assert a1 / a0 == pytest.approx(math.cosh(t_end), rel=2e-2)


def test_plummer_sphere_keeps_its_energy():
    pb = P.gravity_box((32, 32, 32))
    x, v, m = P.particles_plummer(pb, 3000, seed=6, scale=0.08)
    o = _oracle(pb, x, v, m)
    dv = pb.dx * pb.dy * pb.dz

    def energy():
        xx, vv = o.get_particles()
        rho = o.particle_deposit(xx)
        psi = O.poisson_periodic(rho, (pb.dx, pb.dy, pb.dz), 1.0)
        return 0.5 * (m * (vv ** 2).sum(axis=0)).sum(), 0.5 * (rho * psi).sum() * dv

    k0, w0 = energy()
    for _ in range(60):
        o.step()
    k1, w1 = energy()
    assert abs((k1 + w1) - (k0 + w0)) <= 0.01 * abs(w0)
    assert k0 + w0 < 0.0   # bound (the mesh softens W below the point-mass value)
