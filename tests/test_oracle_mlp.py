"""Pins of the oracle's learned flux correction (a 32-64-64-8 MLP with GELU,
gated and clipped, added to the corrector fluxes before constrained
transport)."""
import math

import numpy as np
import pytest

from mhd_inputs import problems as P
from oracle import pyorc as O
from tests.helpers import oracle_of


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, scale, O.MLP_NPARAM)
    return p


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 3, 2000), [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0]])
    t = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([O.bf16(v) for v in x])
    np.testing.assert_array_equal(got, t)
    assert O.bf16(1.0 + 2 ** -8) == 1.0            # tie -> even
    assert O.bf16(1.0 + 3 * 2 ** -9) == 1.0 + 2 ** -7


def test_gelu_values():
    """A 1-unit network exposes GELU: y = gelu(a) with a chosen by b1."""
    p = np.zeros(O.MLP_NPARAM)
    W2, B2, W3 = 2048 + 64, 2048 + 64 + 4096, 2048 + 64 + 4096 + 64
    for a in (-3.0, -1.0, 0.0, 0.5, 2.0):
        p[:] = 0.0
        p[2048 + 0] = a            # b1[0] = a
        p[W2 + 0 * 64 + 0] = 1.0   # a2[0] = h1[0]
        p[W3 + 0 * 64 + 0] = 1.0   # y[0] = h2[0]
        y = O.mlp_forward(p, np.zeros((1, 32)))[0, 0]
        g1 = 0.5 * a * (1 + math.erf(a / math.sqrt(2)))
        assert y == pytest.approx(0.5 * g1 * (1 + math.erf(g1 / math.sqrt(2))), rel=1e-14, abs=1e-16)


def test_mlp_backward_finite_differences():
    """Central differences (h = 1e-6) of sum(dy . y) against the analytic
    backward pass, full FP64."""
    rng = np.random.default_rng(1)
    p = _params(2)
    x = rng.normal(size=(5, 32))
    dy = rng.normal(size=(5, 8))
    g = O.mlp_backward(p, x, dy)
    idx = rng.choice(O.MLP_NPARAM, 300, replace=False)
    idx = np.concatenate([idx, [0, 2047, 2048, 2111, 2112, 6207, 6208, 6271, 6272, 6783, 6784, 6791]])
    h = 1e-6
    for i in idx:
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd = (np.sum(dy * O.mlp_forward(pp, x)) - np.sum(dy * O.mlp_forward(pm, x))) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_features_of_a_uniform_state():
    """rho/rho_m = 1, (v - v_m)/c = 0, P/(rho c^2) = 1/gamma, B/(sqrt(rho) c)."""
    g = 5.0 / 3.0
    rho, p = 2.0, 0.7
    v = [0.3, -0.2, 0.5]
    b = [0.4, 0.1, -0.6]
    w8 = np.array([rho, *v, p, *b] * 4)
    x = O.mlp_features(w8, g)
    c = math.sqrt(g * p / rho)
    want = [1.0, 0, 0, 0, 1.0 / g] + [bb / (math.sqrt(rho) * c) for bb in b]
    np.testing.assert_allclose(x, want * 4, rtol=1e-14, atol=1e-15)


def test_output_flux_round_trip_and_galilean_rows():
    rng = np.random.default_rng(3)
    g = 1.4
    for _ in range(50):
        w8 = np.concatenate([[np.exp(rng.normal()), *rng.normal(size=3), np.exp(rng.normal()),
                              *rng.normal(size=3)] for _ in range(4)])
        y = rng.normal(size=8)
        y[5] = 0.0
        df = O.mlp_out_to_flux(w8, g, y)
        np.testing.assert_allclose(O.mlp_flux_to_out(w8, g, df), y, rtol=1e-12, atol=1e-12)
    # a pure mass-flux correction carries momentum v_m dm and energy |v_m|^2 dm / 2
    w8 = np.array([1.0, 0.2, 0.4, -0.1, 1.0, 0.0, 0.0, 0.0] * 4)
    y = np.zeros(8)
    y[0] = 0.25
    df = O.mlp_out_to_flux(w8, g, y)
    c = math.sqrt(g)
    dm = c * 0.25
    np.testing.assert_allclose(df, [dm, 0.2 * dm, 0.4 * dm, -0.1 * dm,
                                    0.5 * (0.04 + 0.16 + 0.01) * dm, 0, 0], rtol=1e-14, atol=1e-16)


def test_zero_network_is_the_plain_step():
    pb = P.random_smooth((12, 10, 8), seed=5)
    a = oracle_of(pb)
    b = oracle_of(pb)
    b.set_mlp(np.zeros(O.MLP_NPARAM))
    for _ in range(3):
        dt = a.dt()
        a.step(dt)
        b.step(dt)
    for x, y in zip(a.get_state(), b.get_state()):
        np.testing.assert_array_equal(x, y)
    assert b.diag()["n_mlp_faces"] > 0


def test_corrected_step_conserves_and_keeps_div_b():
    """The correction is added to face fluxes before CT: totals stay constant
    on a periodic box and div_h B stays at rounding level."""
    pb = P.random_smooth((12, 10, 8), seed=6)
    o = oracle_of(pb)
    o.set_mlp(_params(7, 0.05), tau=0.5, jump=0.5, tau_flux=0.5)
    d0 = o.diag()
    c0, *_ = o.get_state()
    for _ in range(5):
        o.step()
    d1 = o.diag()
    c1, *_ = o.get_state()
    for m in range(5):
        assert abs(c1[m].sum() - c0[m].sum()) <= 1e-13 * np.abs(c0[m]).sum()
    assert d1["divb_max"] < 1e-12
    assert d1["n_mlp_faces"] > 0


@pytest.mark.parametrize("make,gated", [(P.sod, True), (P.brio_wu, True), (P.ryu_jones, False)])
def test_shock_cells_gate_the_correction(make, gated):
    """Faces touching a cell with a > 50 % pressure jump and converging flow
    keep the plain flux (Sod, Brio-Wu); the Ryu-Jones jumps are all below
    that threshold."""
    o = oracle_of(make(64))
    o.set_mlp(_params(8, 0.05), tau=0.5, jump=0.5, tau_flux=0.5)
    for _ in range(3):
        o.step()
    d = o.diag()
    assert d["n_mlp_faces"] > 0
    assert (d["n_mlp_gated"] > 0) == gated


@pytest.mark.parametrize("bc", [(P.PERIODIC,) * 6, (P.OUTFLOW,) * 6])
def test_coarsening_keeps_mass_and_div_b(bc):
    """The 2x coarse-graining (plain definition) keeps the total of every
    cell field (volume means of 2^3 cells) and, for a discretely
    divergence-free face field, a coarse field that is divergence-free on the
    coarse grid (the face means telescope); on a non-periodic axis the
    boundary faces carry over."""
    pb = P.random_smooth((12, 8, 6), seed=5, bc=bc)
    c5, bx, by, bz = O.coarsen(pb.cell5, pb.bx, pb.by, pb.bz)
    for m in range(5):
        assert abs(c5[m].sum() * 8 - pb.cell5[m].sum()) <= 1e-12 * np.abs(pb.cell5[m]).sum()
    dx, dy, dz = 2 * pb.dx, 2 * pb.dy, 2 * pb.dz
    nz, ny, nx = c5.shape[1:]
    if bc[0] == P.PERIODIC:
        div = ((np.roll(bx, -1, 2) - bx) / dx + (np.roll(by, -1, 1) - by) / dy +
               (np.roll(bz, -1, 0) - bz) / dz)
    else:
        assert bx.shape == (nz, ny, nx + 1) and by.shape == (nz, ny + 1, nx)
        assert bz.shape == (nz + 1, ny, nx)
        div = (np.diff(bx, axis=2) / dx + np.diff(by, axis=1) / dy + np.diff(bz, axis=0) / dz)
        np.testing.assert_allclose(bx[:, :, -1], pb.bx[:, :, -1].reshape(nz, 2, ny, 2).mean(axis=(1, 3)))
    bs = max(np.abs(bx).max(), np.abs(by).max(), np.abs(bz).max())
    assert np.abs(div).max() * min(dx, dy, dz) <= 1e-13 * bs
