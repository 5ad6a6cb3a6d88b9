"""GPU parity of the N-body particles (cloud-in-cell deposit and force,
leapfrog with the corrector's potential, particle CFL) against the FP64
oracle -- same seeded inputs, same time steps, positions (modulo the
periodic box), velocities and the gas state element by element, 1e-11 of
their scales in FP64 -- plus the cold plane wave's closed-form growth on the
device, momentum conservation, and at full size (256^3 box, 2^21
particles) the Poisson equation and the kick checked on sampled cells and
particles."""
import math

import numpy as np
import pytest

from mhd_inputs import problems as P
from oracle import pyorc as O
from tests.gpu_util import field_errors, host_state, needs_gpu, rel_err
from tests.helpers import orc_config

pytestmark = [pytest.mark.gpu, needs_gpu]

TOL = 1e-11


def _pair(pb, x, v, m, precision=0):
    from paper_1502_02935_amd import Sim, config_from_problem
    cfg = orc_config(pb)
    cfg.npart = x.shape[1]
    o = O.Oracle(cfg)
    assert o.set_state(pb.cell5, pb.bx, pb.by, pb.bz) == 0
    o.set_particles(x, v, m)
    s = Sim(config_from_problem(pb, precision=precision, npart=x.shape[1]), pb.cell5, pb.bx,
            pb.by, pb.bz)
    s.set_particles(x, v, m)
    return o, s


def _box(pb):
    return np.array([pb.nx * pb.dx, pb.ny * pb.dy, pb.nz * pb.dz])


def _particle_errors(s, o, pb):
    xg, vg = (t.double().cpu().numpy() for t in s.get_particles())
    xo, vo = o.get_particles()
    L = _box(pb)[:, None]
    dx = xg - xo
    dx -= L * np.round(dx / L)
    return float(np.abs(dx).max() / L.max()), rel_err(vg, vo)


def _run_both(o, s, nsteps, dt=None):
    dts = []
    for _ in range(nsteps):
        dts.append(o.dt() if dt is None else dt)
        o.step(dts[-1])
    s.step(nsteps, dt=dts)


def test_set_get_roundtrip_and_errors():
    from paper_1502_02935_amd import _lib as L
    pb = P.gravity_box((8, 8, 8))
    x, v, m = P.particles_plummer(pb, 100, seed=1, scale=0.1)
    _, s = _pair(pb, x, v, m)
    xg, vg = (t.cpu().numpy() for t in s.get_particles())
    xw = x - np.floor(x)   # unit box
    assert np.abs(xg - xw).max() <= 1e-15 and np.array_equal(vg, v)
    assert s.L.mhd_get_particles(s.ctx, None, None) == L.MHD_E_ARG


def test_two_particles_parity_and_momentum():
    pb = P.gravity_box((16, 16, 16))
    x = np.array([[0.31, 0.62], [0.44, 0.52], [0.5, 0.47]])
    v = np.array([[0.1, -0.2], [0.0, 0.05], [0.02, 0.0]])
    m = np.array([1.0, 0.4])
    o, s = _pair(pb, x, v, m)
    _run_both(o, s, 30, dt=0.01)
    ex, ev = _particle_errors(s, o, pb)
    assert ex <= TOL and ev <= TOL, (ex, ev)
    _, vg = (t.double().cpu().numpy() for t in s.get_particles())
    assert np.abs((vg * m).sum(axis=1) - (v * m).sum(axis=1)).max() <= 1e-13


@pytest.mark.parametrize("device_dt", [False, True])
def test_plummer_with_coupled_gas_parity(device_dt):
    """Gas that sources and feels the potential, 2000 particles, ragged
    32 x 16 x 8 box; the device's own CFL dt (cells and particles) too."""
    pb = P.random_smooth((32, 16, 8), seed=3, d=(1 / 32, 1 / 16, 1 / 8))
    pb.source, pb.src = P.SRC_SELF_GRAVITY, (0.5, 0.0, 0.0, 0.0)
    x, v, m = P.particles_plummer(pb, 2000, seed=4, scale=0.12, mass_total=2.0, G=0.5)
    o, s = _pair(pb, x, v, m)
    if device_dt:
        assert abs(s.dt() - o.dt()) <= 1e-13 * o.dt()
        for _ in range(4):
            o.step()
        s.step(4)
    else:
        _run_both(o, s, 4)
    ex, ev = _particle_errors(s, o, pb)
    assert ex <= TOL and ev <= TOL, (ex, ev)
    err = field_errors(host_state(s), o.get_state())
    assert max(err.values()) <= TOL, err


def test_total_momentum_gas_and_particles():
    pb = P.random_smooth((16, 16, 16), seed=5)
    pb.source, pb.src = P.SRC_SELF_GRAVITY, (0.5, 0.0, 0.0, 0.0)
    x, v, m = P.particles_plummer(pb, 500, seed=6, scale=0.1, mass_total=2.0, G=0.5)
    _, s = _pair(pb, x, v, m)
    dv = pb.dx * pb.dy * pb.dz

    def total():
        c5 = s.get_state()[0].double().cpu().numpy()
        vv = s.get_particles()[1].double().cpu().numpy()
        return np.array([c5[1 + a].sum() * dv for a in range(3)]) + (vv * m).sum(axis=1)

    p0 = total()
    s.step(6)
    assert np.abs(total() - p0).max() <= 1e-12


@pytest.mark.parametrize("precision,tol", [(0, 1e-4), (1, 2e-3)])
def test_cold_plane_wave_growth_on_device(precision, tol):
    n = (32, 4, 4)
    pb = P.gravity_box(n, G=1.0 / (4.0 * math.pi))
    amp = 0.01
    x, v, m = P.particles_plane_wave(pb, amp=amp, mass_total=1.0)
    lat = np.round(x[0] / pb.dx) * pb.dx
    from paper_1502_02935_amd import Sim, config_from_problem
    s = Sim(config_from_problem(pb, precision=precision, npart=x.shape[1]), pb.cell5, pb.bx,
            pb.by, pb.bz)
    s.set_particles(x, v, m)
    s.step(400, dt=0.005)
    x1 = s.get_particles()[0].double().cpu().numpy()
    disp = x1[0] - lat
    disp -= np.round(disp)
    a1 = 2.0 * np.mean(disp * np.sin(2 * math.pi * lat))
    g_disc = math.cos(0.5 * 2 * math.pi * pb.dx)
    assert a1 / (amp * pb.dx) == pytest.approx(math.cosh(g_disc * 2.0), rel=tol)


def test_fp32_against_fp64_oracle():
    pb = P.random_smooth((16, 16, 16), seed=7).astype("float32")
    pb.source, pb.src = P.SRC_SELF_GRAVITY, (0.5, 0.0, 0.0, 0.0)
    x, v, m = P.particles_plummer(pb, 1000, seed=8, scale=0.1, mass_total=1.0, G=0.5)
    x, v, m = (a.astype(np.float32).astype(np.float64) for a in (x, v, m))
    o, s = _pair(pb, x, v, m, precision=1)
    _run_both(o, s, 5)
    ex, ev = _particle_errors(s, o, pb)
    assert ex <= 1e-6 and ev <= 1e-4, (ex, ev)


def test_fullsize_poisson_and_kick_sampled():
    """256^3 turbulent box (coupled gas, G = 1) with 2^21 Plummer particles,
    FP64: after one step with a fixed dt, (a) the corrector's potential
    satisfies the 7-point Poisson equation with the gas density of W* plus
    the oracle's cloud-in-cell deposit of the particles at x + dt/2 v, at
    sampled cells; (b) each sampled particle's velocity changed by -dt
    times the oracle's interpolation of the device's gradient at x_h."""
    import torch
    from paper_1502_02935_amd import Sim, config_from_problem
    N, npart, dt, G = 256, 1 << 21, 1e-4, 1.0
    pb = P.turbulent_ism(N, seed=1)
    pb.source, pb.src = P.SRC_SELF_GRAVITY, (G, 0.0, 0.0, 0.0)
    x, v, m = P.particles_plummer(pb, npart, seed=9, scale=0.1, mass_total=1.0, G=G)
    s = Sim(config_from_problem(pb, precision=0, npart=npart), pb.cell5, pb.bx, pb.by, pb.bz)
    s.set_particles(x, v, m)
    s.step(1, dt=dt)
    psi = s.debug_array(35).double().cpu().numpy()[2:2 + N, 2:2 + N, 2:2 + N]
    grad = [s.debug_array(36 + a).double().cpu().numpy()[2:2 + N, 2:2 + N, 2:2 + N]
            for a in range(3)]
    rho_gas = s.debug_array(27).double().cpu().numpy()[2:2 + N, 2:2 + N, 2:2 + N]
    x1, v1 = (t.double().cpu().numpy() for t in s.get_particles())
    s.close()
    torch.cuda.empty_cache()
    xh = x + 0.5 * dt * v
    xh -= np.floor(xh)
    cfg = orc_config(P.gravity_box((N, N, N)))
    cfg.npart = npart
    o = O.Oracle(cfg)
    o.set_particles(xh, np.zeros_like(xh), m)
    rho = rho_gas + o.particle_deposit(xh)
    assert abs(o.particle_deposit(xh).sum() / N ** 3 - m.sum()) <= 1e-12
    h = 1.0 / N
    rng = np.random.default_rng(10)
    cells = rng.integers(0, N, (400, 3))
    k, j, i = cells[:, 2], cells[:, 1], cells[:, 0]
    lap = sum(np.roll(psi, -1, ax)[k, j, i] + np.roll(psi, 1, ax)[k, j, i] for ax in (0, 1, 2))
    lap = (lap - 6.0 * psi[k, j, i]) / (h * h)
    want = 4.0 * math.pi * G * (rho[k, j, i] - rho.mean())
    assert np.abs(lap - want).max() <= 1e-9 * np.abs(want).max()
    sel = rng.choice(npart, 2000, replace=False)
    for a in range(3):
        acc = o.particle_interp(grad[a], xh[:, sel])
        got = v1[a, sel]
        assert np.abs(got - (v[a, sel] - dt * acc)).max() <= 1e-12 * (np.abs(v[a]).max() + 1.0)


def test_gas_scalars_particles_together_parity():
    """Everything at once, FP64: coupled self-gravity, two passive scalars
    and 800 particles on a ragged 32 x 16 x 8 box, 4 steps with the oracle's
    steps: gas state, scalars and particles within 1e-11."""
    from paper_1502_02935_amd import Sim, config_from_problem
    pb = P.random_smooth((32, 16, 8), seed=11, d=(1 / 32, 1 / 16, 1 / 8))
    pb.source, pb.src = P.SRC_SELF_GRAVITY, (0.7, 0.0, 0.0, 0.0)
    x, v, m = P.particles_plummer(pb, 800, seed=12, scale=0.15, mass_total=1.5, G=0.7)
    rx = P.mass_fractions(pb, 2, "random", seed=13)
    cfg = orc_config(pb)
    cfg.npart, cfg.nscalar = x.shape[1], 2
    o = O.Oracle(cfg)
    assert o.set_state(pb.cell5, pb.bx, pb.by, pb.bz) == 0
    o.set_particles(x, v, m)
    o.set_scalars(rx)
    s = Sim(config_from_problem(pb, precision=0, npart=x.shape[1], nscalar=2), pb.cell5, pb.bx,
            pb.by, pb.bz)
    s.set_particles(x, v, m)
    s.set_scalars(rx)
    _run_both(o, s, 4)
    ex, ev = _particle_errors(s, o, pb)
    assert ex <= TOL and ev <= TOL, (ex, ev)
    err = field_errors(host_state(s), o.get_state())
    assert max(err.values()) <= TOL, err
    g = s.get_scalars().double().cpu().numpy()
    r = o.get_scalars()
    assert max(rel_err(g[k], r[k]) for k in range(2)) <= TOL
