"""Oracle pins for the self-gravity source (the paper's Poisson equation,
Lap Psi = 4 pi G rho, periodic box: rho - <rho> sources it): discrete
Fourier modes in closed form, an independent FFT, and the Jeans linear
theory of the coupled step."""
import math

import numpy as np
import pytest

from helpers import oracle_of, run_to
from mhd_inputs import problems as P
from oracle import pyorc as O


def _lam(m, n, d):
    """Eigenvalue of the 1-D 3-point Laplacian for mode m of n cells."""
    return (2.0 * math.cos(2.0 * math.pi * m / n) - 2.0) / (d * d)


def test_single_mode_closed_form():
    """rho = rho0 + A cos(2 pi (mx x + my y + mz z)): Psi = 4 pi G A cos(...)
    / lambda, lambda the 7-point Laplacian's eigenvalue; the mean drops out."""
    nx, ny, nz = 12, 8, 6
    d = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    G, A = 0.7, 0.3
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    z = (np.arange(nz) + 0.5) / nz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    for m in [(1, 0, 0), (0, 2, 0), (1, 1, 1), (3, 2, 1)]:
        ph = 2.0 * math.pi * (m[0] * X + m[1] * Y + m[2] * Z)
        rho = 5.0 + A * np.cos(ph)
        lam = _lam(m[0], nx, d[0]) + _lam(m[1], ny, d[1]) + _lam(m[2], nz, d[2])
        want = 4.0 * math.pi * G * A * np.cos(ph) / lam
        got = O.poisson_periodic(rho, d, G)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), m


def test_random_density_against_numpy_fft_and_laplacian():
    """A random density: the oracle's Psi equals the spectral solution by an
    independent FFT (numpy), has zero mean, and its 7-point Laplacian gives
    back 4 pi G (rho - <rho>)."""
    rng = np.random.default_rng(3)
    nz, ny, nx = 6, 10, 8
    d = (0.1, 0.07, 0.13)
    G = 1.3
    rho = 1.0 + 0.2 * rng.normal(size=(nz, ny, nx))
    psi = O.poisson_periodic(rho, d, G)
    kx = np.array([_lam(m, nx, d[0]) for m in range(nx)])
    ky = np.array([_lam(m, ny, d[1]) for m in range(ny)])
    kz = np.array([_lam(m, nz, d[2]) for m in range(nz)])
    lam = kz[:, None, None] + ky[None, :, None] + kx[None, None, :]
    lam[0, 0, 0] = 1.0
    rh = np.fft.fftn(rho)
    rh[0, 0, 0] = 0.0
    ref = np.real(np.fft.ifftn(4.0 * math.pi * G * rh / lam))
    assert np.abs(psi - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(psi.mean()) <= 1e-13 * np.abs(psi).max()
    lap = sum((np.roll(psi, -1, ax) - 2 * psi + np.roll(psi, 1, ax)) / (dd * dd)
              for ax, dd in ((2, d[0]), (1, d[1]), (0, d[2])))
    np.testing.assert_allclose(lap, 4.0 * math.pi * G * (rho - rho.mean()), rtol=0,
                               atol=1e-10 * np.abs(lap).max())


def _mode_amplitude(o, n):
    rho = o.get_state()[0][0].reshape(-1)
    x = (np.arange(n) + 0.5) / n
    return 2.0 * float(np.mean((rho - rho.mean()) * np.cos(2.0 * math.pi * x)))


@pytest.mark.parametrize("k_over_kj", [0.5, 2.0])
def test_jeans_linear_theory(k_over_kj):
    """A small adiabatic density wave at rest in a self-gravitating uniform
    gas: below the Jeans scale (k < k_J) it grows as cosh(g t) with
    g^2 = 4 pi G rho0 - cs^2 k^2; above it oscillates as cos(w t) with
    w^2 = cs^2 k^2 - 4 pi G rho0.  64 cells per wavelength, t = 0.25."""
    n = 64
    pb = P.jeans(n, k_over_kj=k_over_kj)
    o = oracle_of(pb)
    a0 = _mode_amplitude(o, n)
    t = 0.25
    run_to(o, t)
    a = _mode_amplitude(o, n)
    r = pb.extra["rate"]
    want = math.cosh(r * t) if pb.extra["growing"] else math.cos(r * t)
    assert abs(a / a0 - want) <= 0.03 * max(1.0, abs(want)), (a / a0, want)
