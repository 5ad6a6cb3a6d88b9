"""Pins of the oracle's density and pressure floors (no GPU).  The floors
are a reading of the method, not part of the paper's equations: after each
stage's conservative and CT update, rho is raised to rho_floor, then E is
raised so that the gas pressure of the updated cell (with the cell-centred
B of its updated faces) reaches p_floor.  What that definition fixes
independently of the oracle's code: on a uniform state every flux
difference is exactly zero, so the step reduces to the floors alone and
the end state has a closed form; floors below every value change nothing."""
import numpy as np
import pytest

from mhd_inputs import problems as P
from tests.helpers import oracle_of

GAMMA = 5.0 / 3.0
V = (0.3, -0.2, 0.1)
B = (0.5, -0.4, 0.3)


def _pressure(c5, bx, by, bz, gamma=GAMMA):
    """Textbook gas pressure of the conserved state, with the cell-centred
    field the mean of the two faces (periodic: the upper face of the last
    cell is the first face)."""
    bcx = 0.5 * (bx + np.roll(bx, -1, axis=2))
    bcy = 0.5 * (by + np.roll(by, -1, axis=1))
    bcz = 0.5 * (bz + np.roll(bz, -1, axis=0))
    rho, mx, my, mz, e = c5
    return (gamma - 1.0) * (e - 0.5 * (mx * mx + my * my + mz * mz) / rho
                            - 0.5 * (bcx * bcx + bcy * bcy + bcz * bcz))


def test_density_floor_uniform():
    """rho below its floor, P well above: both stages floor every cell, the
    momenta, E and B are left as they were (the floor adds mass at rest in
    the moving frame's momentum, not energy)."""
    pb = P.uniform((6, 5, 4), rho=0.5, v=V, p=0.7, b=B)
    pb.rho_floor = 0.8
    o = oracle_of(pb)
    o.step(0.01)
    c5, bx, by, bz = o.get_state()
    assert np.all(c5[0] == 0.8)
    np.testing.assert_array_equal(c5[1:], pb.cell5[1:])
    np.testing.assert_array_equal(bx, pb.bx)
    np.testing.assert_array_equal(by, pb.by)
    np.testing.assert_array_equal(bz, pb.bz)
    d = o.diag()
    assert d["n_floor"] == 2 * pb.ncell  # predictor and corrector
    assert np.all(_pressure(c5, bx, by, bz) > 0.7)


@pytest.mark.parametrize("b", [B, (0.0, 0.0, 0.0)])
def test_pressure_floor_uniform(b):
    """P below its floor: the pressure of the end state equals the floor
    (magnetic energy counted), E grows by exactly (p_floor - P)/(gamma - 1)
    and nothing else moves."""
    p0, pf = 0.3, 0.9
    pb = P.uniform((6, 5, 4), rho=1.2, v=V, p=p0, b=b)
    pb.p_floor = pf
    o = oracle_of(pb)
    o.step(0.01)
    c5, bx, by, bz = o.get_state()
    np.testing.assert_array_equal(c5[:4], pb.cell5[:4])
    np.testing.assert_array_equal(bx, pb.bx)
    np.testing.assert_allclose(_pressure(c5, bx, by, bz), pf, rtol=1e-13)
    np.testing.assert_allclose(c5[4] - pb.cell5[4], (pf - p0) / (GAMMA - 1.0), rtol=1e-13)
    assert o.diag()["n_floor"] == 2 * pb.ncell


def test_both_floors_uniform():
    """Both floors at once: rho first, then P from the floored rho (a
    larger rho lowers the kinetic energy, so P rises before the pressure
    floor is checked)."""
    rho0, p0, rf, pf = 0.5, 0.2, 0.8, 0.6
    pb = P.uniform((4, 4, 4), rho=rho0, v=V, p=p0, b=B)
    pb.rho_floor, pb.p_floor = rf, pf
    o = oracle_of(pb)
    o.step(0.01)
    c5, bx, by, bz = o.get_state()
    assert np.all(c5[0] == rf)
    np.testing.assert_array_equal(c5[1:4], pb.cell5[1:4])
    ke0 = 0.5 * rho0 * sum(x * x for x in V)
    p_after_rho = p0 + (GAMMA - 1.0) * (ke0 - ke0 * rho0 / rf)
    assert p_after_rho < pf
    np.testing.assert_allclose(_pressure(c5, bx, by, bz), pf, rtol=1e-13)


def test_floors_below_every_value_change_nothing():
    """A smooth random state with floors far below its density and pressure
    gives bitwise the run without floors, and no floor hit."""
    pb = P.random_smooth((12, 10, 8), seed=5)
    o0 = oracle_of(pb)
    pb.rho_floor, pb.p_floor = 1e-6, 1e-6
    o1 = oracle_of(pb)
    for _ in range(3):
        dt = o0.dt()
        o0.step(dt)
        o1.step(dt)
    for a0, a1 in zip(o0.get_state(), o1.get_state()):
        np.testing.assert_array_equal(a0, a1)
    assert o1.diag()["n_floor"] == 0


def test_floors_bound_a_rarefied_region():
    """Two strongly diverging streams empty the middle of the box: with the
    floors on, no interior cell ends below either floor (to the pressure's
    rounding), and the floors act in some cells."""
    pb = P.uniform((32, 2, 2), rho=1e-3, v=(0.0, 0.0, 0.0), p=1e-4, b=(0.0, 0.0, 0.0))
    x = (np.arange(32) + 0.5) / 32
    c5 = pb.cell5.copy()
    c5[1] = np.where(x < 0.5, -1.0, 1.0)[None, None, :] * c5[0] * 5.0
    c5[4] = 1e-4 / (GAMMA - 1.0) + 0.5 * c5[1] ** 2 / c5[0]
    pb.cell5 = c5
    pb.rho_floor, pb.p_floor = 8e-4, 5e-5
    o = oracle_of(pb)
    for _ in range(6):
        o.step(0.5 * o.dt())
        s = o.get_state()
        assert np.all(s[0][0] >= pb.rho_floor)
        assert np.all(_pressure(*s) >= pb.p_floor * (1 - 1e-12))
    assert o.diag()["n_floor"] > 0
