"""Seeded synthetic initial conditions for the ideal-MHD step.

This module holds input definitions only (initial states and their
parameters); it contains none of the solver's arithmetic.  Both the GPU
library's tests/benchmark and the FP64 CPU oracle take their inputs from here.

Every generator returns a :class:`Problem`: grid geometry, boundary
conditions, source model and the initial conserved state in the interior
layout used across the project:

* ``cell5``: float64 ``[5][nz][ny][nx]`` = rho, Mx, My, Mz, E (x fastest)
* ``bx``: ``[nz][ny][nx+ox]``, ``by``: ``[nz][ny+oy][nx]``, ``bz``: ``[nz+oz][ny][nx]``
  where ``o = 0`` on a periodic axis and 1 otherwise; face ``i`` of ``bx`` is
  at ``x0 + i*dx``.

Energy follows Eq. 3 of the paper: E = P/(gamma-1) + rho v^2/2 + B^2/2 with
the cell-centred B taken as the mean of the two faces (Eq. 6), in rationalised
units (B^2/2 magnetic pressure).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

PERIODIC, OUTFLOW, INFLOW = 0, 1, 2
SRC_NONE, SRC_LOGPOT, SRC_UNIFORM, SRC_GAUSS_X, SRC_SELF_GRAVITY = 0, 1, 2, 3, 4


@dataclass
class Problem:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    x0: float
    y0: float
    z0: float
    gamma: float
    bc: tuple
    cell5: np.ndarray
    bx: np.ndarray
    by: np.ndarray
    bz: np.ndarray
    cfl: float = 0.4
    source: int = SRC_NONE
    src: tuple = (0.0, 0.0, 0.0, 0.0)
    rho_floor: float = 0.0
    p_floor: float = 0.0
    inflow: tuple = (0.0,) * 8
    t_end: float = 0.0
    extra: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    def astype(self, dtype) -> "Problem":
        """Same problem with the state rounded to ``dtype`` and back to float64
        (so two precisions can start from one representable state)."""
        f = lambda a: np.asarray(a, dtype=dtype).astype(np.float64)
        return replace(self, cell5=f(self.cell5), bx=f(self.bx), by=f(self.by), bz=f(self.bz))


def _face_counts(bc, nx, ny, nz):
    ox = 0 if bc[0] == PERIODIC else 1
    oy = 0 if bc[2] == PERIODIC else 1
    oz = 0 if bc[4] == PERIODIC else 1
    return ox, oy, oz


def energy_from(rho, vx, vy, vz, P, bx, by, bz, gamma, bc):
    """Total energy (Eq. 3) with cell-centred B from the face means (Eq. 6)."""
    def centre(b, axis, periodic):
        if periodic:
            return 0.5 * (b + np.roll(b, -1, axis=axis))
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(None, -1)
        hi[axis] = slice(1, None)
        return 0.5 * (b[tuple(lo)] + b[tuple(hi)])

    bcx = centre(bx, 2, bc[0] == PERIODIC)
    bcy = centre(by, 1, bc[2] == PERIODIC)
    bcz = centre(bz, 0, bc[4] == PERIODIC)
    M = (rho * vx, rho * vy, rho * vz)
    ke = 0.5 * (M[0] * M[0] + M[1] * M[1] + M[2] * M[2]) / rho
    me = 0.5 * (bcx * bcx + bcy * bcy + bcz * bcz)
    return P / (gamma - 1.0) + ke + me


def _pack(rho, vx, vy, vz, P, bx, by, bz, gamma, bc):
    E = energy_from(rho, vx, vy, vz, P, bx, by, bz, gamma, bc)
    cell5 = np.stack([rho, rho * vx, rho * vy, rho * vz, E]).astype(np.float64)
    return np.ascontiguousarray(cell5)


# ---------------------------------------------------------------------------
# Circularly polarised Alfven wave (plain-method FP64 box)
# ---------------------------------------------------------------------------

def _alfven_basis():
    n = np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0)
    e1 = np.array([-1.0, 1.0, 0.0]) / math.sqrt(2.0)
    e2 = np.cross(n, e1)
    return n, e1, e2


def alfven_exact(n: int, t: float, *, rho=1.0, p=0.1, b_par=1.0, b_perp=0.1, gamma=5.0 / 3.0):
    """Exact cell averages of v and the phase at time t for the travelling
    circularly polarised wave with k = 2 pi (1,1,1) on the unit periodic cube.
    Returns (vx, vy, vz) each [n][n][n]."""
    nh, e1, e2 = _alfven_basis()
    h = 1.0 / n
    kv = 2.0 * math.pi * np.array([1.0, 1.0, 1.0])
    kmag = float(np.linalg.norm(kv))
    va = b_par / math.sqrt(rho)
    omega = kmag * va
    c = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    ph = kv[0] * x + kv[1] * y + kv[2] * z - omega * t
    sinc = 1.0
    for kd in kv:
        a = 0.5 * kd * h
        sinc *= math.sin(a) / a
    amp = -(b_perp / math.sqrt(rho)) * sinc
    cs, sn = np.cos(ph), np.sin(ph)
    return tuple(amp * (cs * e1[d] + sn * e2[d]) for d in range(3))


def alfven(n: int = 64, *, rho=1.0, p=0.1, b_par=1.0, b_perp=0.1, gamma=5.0 / 3.0,
           cfl=0.4, t=0.0) -> Problem:
    """Circularly polarised Alfven wave travelling along (1,1,1)/sqrt(3) at
    v_A = b_par/sqrt(rho) on [0,1)^3, periodic.  Face B is the uniform part
    plus the exact face average of curl A with A = -dB/|k|, computed from
    closed-form edge line integrals, so div_h B vanishes to rounding."""
    nh, e1, e2 = _alfven_basis()
    h = 1.0 / n
    kv = 2.0 * math.pi * np.array([1.0, 1.0, 1.0])
    kmag = float(np.linalg.norm(kv))
    omega = kmag * b_par / math.sqrt(rho)
    eA = -(b_perp / kmag)  # A = eA (cos(ph) e1 + sin(ph) e2)
    idx = np.arange(n)
    lo = idx * h            # lower faces / edges
    cen = (idx + 0.5) * h   # centres

    def line_int(comp, axis, X, Y, Z):
        """Integral of A_comp along +axis over one cell length starting at
        (X, Y, Z) (the along-axis coordinate of the start is in X/Y/Z)."""
        ph0 = kv[0] * X + kv[1] * Y + kv[2] * Z - omega * t
        ph1 = ph0 + kv[axis] * h
        ka = kv[axis]
        int_cos = (np.sin(ph1) - np.sin(ph0)) / ka
        int_sin = -(np.cos(ph1) - np.cos(ph0)) / ka
        return eA * (int_cos * e1[comp] + int_sin * e2[comp])

    Z, Y, X = np.meshgrid(lo, lo, lo, indexing="ij")
    # z-edge at (x_{i-1/2}, y_{j-1/2}) spanning z_{k-1/2}..z_{k+1/2}: integral of A_z
    LAz = line_int(2, 2, X, Y, Z)
    LAy = line_int(1, 1, X, Y, Z)
    LAx = line_int(0, 0, X, Y, Z)
    r = lambda a, ax: np.roll(a, -1, axis=ax)  # value at index +1 (periodic)
    bx = ((r(LAz, 1) - LAz) - (r(LAy, 0) - LAy)) / (h * h) + b_par * nh[0]
    by = ((r(LAx, 0) - LAx) - (r(LAz, 2) - LAz)) / (h * h) + b_par * nh[1]
    bz = ((r(LAy, 2) - LAy) - (r(LAx, 1) - LAx)) / (h * h) + b_par * nh[2]
    vx, vy, vz = alfven_exact(n, t, rho=rho, p=p, b_par=b_par, b_perp=b_perp, gamma=gamma)
    rh = np.full((n, n, n), rho)
    P = np.full((n, n, n), p)
    bc = (PERIODIC,) * 6
    cell5 = _pack(rh, vx, vy, vz, P, bx, by, bz, gamma, bc)
    return Problem("alfven", n, n, n, h, h, h, 0.0, 0.0, 0.0, gamma, bc, cell5,
                   np.ascontiguousarray(bx), np.ascontiguousarray(by), np.ascontiguousarray(bz),
                   cfl=cfl, extra=dict(rho=rho, p=p, b_par=b_par, b_perp=b_perp))


# ---------------------------------------------------------------------------
# Turbulent ISM box (precision form)
# ---------------------------------------------------------------------------

def gaussian_random_field(rng, n: int, kmin=1.0, kmax=16.0, slope=-4.0) -> np.ndarray:
    """Zero-mean, unit-variance periodic Gaussian field on n^3 with per-mode
    power |k|^slope on integer shells kmin <= |k| <= kmax."""
    white = rng.standard_normal((n, n, n))
    F = np.fft.rfftn(white)
    kz = np.fft.fftfreq(n, d=1.0 / n)
    ky = np.fft.fftfreq(n, d=1.0 / n)
    kx = np.fft.rfftfreq(n, d=1.0 / n)
    K = np.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    filt = np.zeros_like(K)
    sel = (K >= kmin) & (K <= kmax)
    filt[sel] = K[sel] ** (0.5 * slope)
    g = np.fft.irfftn(F * filt, s=(n, n, n), axes=(0, 1, 2))
    g -= g.mean()
    g /= g.std()
    return g


def turbulent_ism(n: int = 256, seed: int = 1, *, sigma_lnrho=1.0, mach=3.0, c_iso2=0.1,
                  beta=1.0, gamma=5.0 / 3.0, cfl=0.4) -> Problem:
    """Periodic [0,1)^3 box: lognormal density (sigma_lnrho, <rho> = 1),
    k^-4 Gaussian random velocity on 1 <= |k| <= 16 scaled to rms Mach
    `mach` against c_iso, P = c_iso^2 rho, uniform B along x with plasma
    beta <P>/(B^2/2) = beta."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    g = gaussian_random_field(rng, n)
    e = np.exp(sigma_lnrho * g)
    rho = e / e.mean()
    v = [gaussian_random_field(rng, n) for _ in range(3)]
    for a in v:
        a -= a.mean()
    vrms = math.sqrt(float(np.mean(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)))
    scale = mach * math.sqrt(c_iso2) / vrms
    vx, vy, vz = (a * scale for a in v)
    P = c_iso2 * rho
    b0 = math.sqrt(2.0 * c_iso2 / beta)
    bx = np.full((n, n, n), b0)
    by = np.zeros((n, n, n))
    bz = np.zeros((n, n, n))
    bc = (PERIODIC,) * 6
    cell5 = _pack(rho, vx, vy, vz, P, bx, by, bz, gamma, bc)
    return Problem("turbulent_ism", n, n, n, h, h, h, 0.0, 0.0, 0.0, gamma, bc, cell5,
                   bx, by, bz, cfl=cfl, extra=dict(seed=seed))


# ---------------------------------------------------------------------------
# Galactic disc slab (precision form, disc)
# ---------------------------------------------------------------------------

def _gd(u):
    """Gudermannian: integral of sech from 0 to u."""
    return 2.0 * np.arctan(np.tanh(0.5 * u))


def disc(nx: int = 512, ny: int = 512, nz: int = 128, *, lx=24.0, ly=24.0, lz=6.0, seed=1,
         rho0=1.0, rd=3.0, h=0.2, cs=10.0, v0=200.0, rc=0.5, q=1.0, beta=10.0,
         noise=0.01, rho_floor_rel=1e-5, gamma=5.0 / 3.0, cfl=0.4) -> Problem:
    """Cartesian slab disc centred on the origin, units kpc and km/s:
    rho = rho0 exp(-R/rd) sech^2(z/h) (1 + noise xi) (xi ~ N(0,1) clipped to
    +-3, floored), isothermal P = rho cs^2, rotation balancing the logarithmic
    potential Phi = v0^2/2 ln(rc^2 + R^2 + z^2/q^2), toroidal B from
    A_z = -B0 sech(z/h) 2 rd (1 - exp(-R/(2 rd))) with B0 = sqrt(2 rho0 cs^2/beta)
    (midplane beta = `beta`), outflow on all sides."""
    rng = np.random.default_rng(seed)
    dx, dy, dz = lx / nx, ly / ny, lz / nz
    x0, y0, z0 = -0.5 * lx, -0.5 * ly, -0.5 * lz
    xc = x0 + (np.arange(nx) + 0.5) * dx
    yc = y0 + (np.arange(ny) + 0.5) * dy
    zc = z0 + (np.arange(nz) + 0.5) * dz
    rho_floor = rho_floor_rel * rho0
    p_floor = rho_floor * cs * cs
    R2 = (xc[None, :] ** 2 + yc[:, None] ** 2)            # [ny][nx]
    R = np.sqrt(R2)
    sech2 = 1.0 / np.cosh(zc / h) ** 2                     # [nz]
    xi = np.clip(rng.standard_normal((nz, ny, nx)), -3.0, 3.0)
    rho = rho0 * np.exp(-R / rd)[None] * sech2[:, None, None] * (1.0 + noise * xi)
    np.maximum(rho, rho_floor, out=rho)
    P = rho * cs * cs
    den = np.sqrt(rc * rc + R2[None] + (zc[:, None, None] / q) ** 2)
    vx = -v0 * yc[None, :, None] / den
    vy = v0 * xc[None, None, :] / den
    vz = np.zeros_like(rho)
    del den
    b0 = math.sqrt(2.0 * rho0 * cs * cs / beta)
    # z-edge line integrals of A_z at the cell corners (x_{i-1/2}, y_{j-1/2})
    xe = x0 + np.arange(nx + 1) * dx
    ye = y0 + np.arange(ny + 1) * dy
    Re = np.sqrt(xe[None, :] ** 2 + ye[:, None] ** 2)      # [ny+1][nx+1]
    fR = -b0 * 2.0 * rd * (1.0 - np.exp(-Re / (2.0 * rd)))
    ze = z0 + np.arange(nz + 1) * dz
    gz = h * (_gd(ze[1:] / h) - _gd(ze[:-1] / h))            # [nz]
    LAz = gz[:, None, None] * fR[None]                     # [nz][ny+1][nx+1]
    bx = (LAz[:, 1:, :] - LAz[:, :-1, :]) / (dy * dz)      # [nz][ny][nx+1]
    by = -(LAz[:, :, 1:] - LAz[:, :, :-1]) / (dz * dx)     # [nz][ny+1][nx]
    bz = np.zeros((nz + 1, ny, nx))
    bc = (OUTFLOW,) * 6
    cell5 = _pack(rho, vx, vy, vz, P, bx, by, bz, gamma, bc)
    return Problem("disc", nx, ny, nz, dx, dy, dz, x0, y0, z0, gamma, bc, cell5,
                   np.ascontiguousarray(bx), np.ascontiguousarray(by), bz, cfl=cfl,
                   source=SRC_LOGPOT, src=(v0, rc, q, 0.0), rho_floor=rho_floor, p_floor=p_floor,
                   extra=dict(seed=seed))


# ---------------------------------------------------------------------------
# One-dimensional Riemann problems (paper section 3) on an n x 1 x 1 grid
# ---------------------------------------------------------------------------

def _cyc(v, axis):
    """Cyclically permute an (x, y, z) triple so that the x entry goes to
    `axis`."""
    v = list(v)
    return tuple(v[(d - axis) % 3] for d in range(3))


def riemann_1d(left, right, n: int, *, xlo=-0.5, xhi=0.5, gamma=5.0 / 3.0, axis=0,
               name="riemann", t_end=0.0, cfl=0.4, bc_lohi=(OUTFLOW, OUTFLOW), x_split=0.0,
               right_rho=None) -> Problem:
    """Two constant states (rho, vx, vy, vz, P, Bx, By, Bz) split at x_split
    on [xlo, xhi] with n cells, outflow along the problem axis and periodic
    (one cell) across it; right_rho(x), if given, replaces the right state's
    density at the cell centres.  `axis` lays the problem along x, y or z
    with the vector components permuted cyclically."""
    L = np.asarray(left, dtype=np.float64)
    R = np.asarray(right, dtype=np.float64)
    if L[5] != R[5]:
        raise ValueError("normal B must be continuous")
    h = (xhi - xlo) / n
    xc = xlo + (np.arange(n) + 0.5) * h
    sel = xc < x_split
    q = np.where(sel[:, None], L[None, :], R[None, :])   # [n][8]
    if right_rho is not None:
        q[:, 0] = np.where(sel, L[0], right_rho(xc))
    # 1-D arrays along the problem axis
    rho, vx, vy, vz, P = (q[:, m] for m in range(5))
    nfn = n if bc_lohi[0] == PERIODIC else n + 1  # faces along the problem axis
    b_n = np.full(nfn, L[5])
    b_t1 = q[:, 6]
    b_t2 = q[:, 7]
    shape = [1, 1, 1]
    shape[2 - axis] = n
    shp = tuple(shape)  # (nz, ny, nx)
    vel = _cyc((vx, vy, vz), axis)
    comps = [rho.reshape(shp), *(c.reshape(shp) for c in vel), P.reshape(shp)]
    # face arrays: the normal one has n+1 faces along the axis (n if it is
    # periodic), transverse ones are one per cell (periodic single-cell axes)
    bfield = _cyc((b_n, b_t1, b_t2), axis)
    faces = []
    for d in range(3):
        fs = list(shp)
        if d == axis:
            fs[2 - d] = nfn
        faces.append(np.ascontiguousarray(bfield[d].reshape(fs)))
    bc = [PERIODIC] * 6
    bc[2 * axis], bc[2 * axis + 1] = bc_lohi
    bc = tuple(bc)
    cell5 = _pack(*comps, *faces, gamma, bc)
    d = [1.0, 1.0, 1.0]
    d[axis] = h
    o = [0.0, 0.0, 0.0]
    o[axis] = xlo
    nxyz = [1, 1, 1]
    nxyz[axis] = n
    return Problem(name, nxyz[0], nxyz[1], nxyz[2], d[0], d[1], d[2], o[0], o[1], o[2], gamma,
                   bc, cell5, faces[0], faces[1], faces[2], cfl=cfl, t_end=t_end,
                   extra=dict(left=L, right=R, axis=axis, h=h, xlo=xlo))


def sod(n=200, axis=0) -> Problem:
    """Sod shock tube: {rho, v, P} = {1, 0, 1} | {0.125, 0, 0.1}, gamma 1.4,
    [-1, 1], t = 0.5."""
    return riemann_1d((1, 0, 0, 0, 1, 0, 0, 0), (0.125, 0, 0, 0, 0.1, 0, 0, 0), n, xlo=-1.0,
                      xhi=1.0, gamma=1.4, axis=axis, name="sod", t_end=0.5)


def jeans(n=64, axis=0, k_over_kj=0.5, amp=1e-4, cs=1.0, gamma=5.0 / 3.0) -> Problem:
    """Jeans problem on a periodic unit box laid along `axis` (one cell
    across): rho = 1 + amp cos(2 pi x), adiabatic P = P0 (rho/rho0)^gamma with
    sound speed cs, at rest, B = 0; self-gravity with G such that the mode
    k = 2 pi sits at k/k_J = k_over_kj (k_J^2 = 4 pi G rho0 / cs^2).  extra:
    the linear rate, growth (k < k_J) or angular frequency (k > k_J)."""
    rho0, k = 1.0, 2.0 * math.pi
    G = cs * cs * k * k / (4.0 * math.pi * rho0 * k_over_kj ** 2)
    p0 = rho0 * cs * cs / gamma
    pb = riemann_1d((rho0, 0, 0, 0, p0, 0, 0, 0), (rho0, 0, 0, 0, p0, 0, 0, 0), n, xlo=0.0, xhi=1.0,
                    gamma=gamma, axis=axis, name="jeans", bc_lohi=(PERIODIC, PERIODIC),
                    x_split=-1.0, right_rho=lambda x: rho0 + amp * np.cos(k * x))
    # adiabatic pressure of the perturbed density
    shp = pb.cell5.shape[1:]
    rho = pb.cell5[0]
    P = p0 * (rho / rho0) ** gamma
    pb.cell5[4] = P / (gamma - 1.0)  # at rest, B = 0
    pb.source, pb.src = SRC_SELF_GRAVITY, (G, 0.0, 0.0, 0.0)
    w2 = 4.0 * math.pi * G * rho0 - cs * cs * k * k
    pb.extra.update(G=G, rate=math.sqrt(abs(w2)), growing=w2 > 0, amp=amp, k=k)
    return pb


def collapse(n=128, *, G=1.0, mass=1.0, radius=1.0, u=0.05, rho_bg=1e-3, gamma=5.0 / 3.0,
             cfl=0.4) -> Problem:
    """Self-gravitating gas sphere on the periodic box [-1, 1]^3 (section 3,
    spherical collapse): rho = M / (2 pi R^2 r) inside R (the 1/r profile of
    the paper, normalised as in the adiabatic-collapse test of Evrard 1988),
    rho_bg outside, at rest, specific internal energy u everywhere, B = 0,
    self-gravity with constant G (readings: the paper names the profile, the
    box and 100^3 cells; the FFT solver takes 2^k cells per axis)."""
    h = 2.0 / n
    c = -1.0 + (np.arange(n) + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    rho = np.where(r <= radius, mass / (2.0 * math.pi * radius * radius * np.maximum(r, 1e-300)),
                   rho_bg)
    P = (gamma - 1.0) * rho * u
    zero = np.zeros_like(rho)
    bc = (PERIODIC,) * 6
    bx, by, bz = zero.copy(), zero.copy(), zero.copy()
    cell5 = _pack(rho, zero, zero, zero, P, bx, by, bz, gamma, bc)
    pb = Problem("collapse", n, n, n, h, h, h, -1.0, -1.0, -1.0, gamma, bc, cell5, bx, by, bz,
                 cfl=cfl, t_end=1.0)
    pb.source, pb.src = SRC_SELF_GRAVITY, (G, 0.0, 0.0, 0.0)
    return pb


def shu_osher(n=200, axis=0) -> Problem:
    """Shu-Osher (section 3): a Mach-3 shock, {rho, u, P} = {3.857143,
    2.629369, 10.33333} for x < 0.125, running into rho = 1 + 0.2 sin(16 pi x),
    u = 0, P = 1; gamma 1.4 on [0, 1] (reading: the paper gives the split
    point and t = 0.18, not the domain), outflow ends, t = 0.18."""
    return riemann_1d((3.857143, 2.629369, 0, 0, 10.33333, 0, 0, 0), (1, 0, 0, 0, 1, 0, 0, 0), n,
                      xlo=0.0, xhi=1.0, gamma=1.4, axis=axis, name="shu_osher", t_end=0.18,
                      x_split=0.125, right_rho=lambda x: 1.0 + 0.2 * np.sin(16.0 * np.pi * x))


def brio_wu(n=200, axis=0) -> Problem:
    """Brio-Wu: {rho, P, By} = {1, 1, 1} | {0.125, 0.1, -1}, Bx = 0.75,
    gamma 2, [-0.5, 0.5], t = 0.1."""
    return riemann_1d((1, 0, 0, 0, 1, 0.75, 1, 0), (0.125, 0, 0, 0, 0.1, 0.75, -1, 0), n,
                      gamma=2.0, axis=axis, name="brio_wu", t_end=0.1)


def ryu_jones(n=200, axis=0) -> Problem:
    """Ryu-Jones 2a (seven waves), gamma 5/3, [-0.5, 0.5], t = 0.2; B given
    in Gaussian form divided by sqrt(4 pi)."""
    s = 1.0 / math.sqrt(4.0 * math.pi)
    L = (1.08, 1.2, 0.01, 0.5, 0.95, 4 * s, 3.6 * s, 2 * s)
    R = (1.0, 0.0, 0.0, 0.0, 1.0, 4 * s, 4 * s, 2 * s)
    return riemann_1d(L, R, n, gamma=5.0 / 3.0, axis=axis, name="ryu_jones", t_end=0.2)


def uniform(n=(8, 8, 8), *, rho=1.0, v=(0.3, -0.2, 0.1), p=0.7, b=(0.5, -0.4, 0.3),
            gamma=5.0 / 3.0, bc=(PERIODIC,) * 6, d=(0.1, 0.1, 0.1)) -> Problem:
    """Uniform state on an nx x ny x nz box."""
    nx, ny, nz = n
    ox, oy, oz = _face_counts(bc, nx, ny, nz)
    shp = (nz, ny, nx)
    bx = np.full((nz, ny, nx + ox), float(b[0]))
    by = np.full((nz, ny + oy, nx), float(b[1]))
    bz = np.full((nz + oz, ny, nx), float(b[2]))
    rho_a = np.full(shp, float(rho))
    cell5 = _pack(rho_a, np.full(shp, v[0]), np.full(shp, v[1]), np.full(shp, v[2]),
                  np.full(shp, float(p)), bx, by, bz, gamma, bc)
    return Problem("uniform", nx, ny, nz, d[0], d[1], d[2], 0.0, 0.0, 0.0, gamma, tuple(bc),
                   cell5, bx, by, bz)


def random_smooth(n=(16, 12, 10), seed=0, *, amp=0.3, gamma=5.0 / 3.0, bc=(PERIODIC,) * 6,
                  b0=(0.6, 0.3, -0.2), d=None, b_amp=0.05) -> Problem:
    """Random periodic-ish smooth state for parity tests: a few random Fourier
    modes in rho, P, v and a divergence-free B from a random vector potential
    of amplitude b_amp (discrete curl of edge values, so div_h B is zero to
    rounding) on the uniform field b0 (b_amp = 0 and b0 = 0: no field).  Works for
    any boundary conditions (the potential is sampled, not assumed periodic)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    if d is None:
        d = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    ox, oy, oz = _face_counts(bc, nx, ny, nz)

    def field_at(X, Y, Z, nm=3):
        f = np.zeros_like(X)
        for _ in range(nm):
            k = rng.integers(-2, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi)
            a = rng.standard_normal()
            f += a * np.cos(2 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
        return f

    xc = (np.arange(nx) + 0.5) * d[0]
    yc = (np.arange(ny) + 0.5) * d[1]
    zc = (np.arange(nz) + 0.5) * d[2]
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    rho = np.exp(amp * field_at(X, Y, Z))
    P = 0.5 * np.exp(amp * field_at(X, Y, Z))
    vx, vy, vz = (amp * field_at(X, Y, Z) for _ in range(3))
    # vector potential on edges (sampled at edge midpoints, times edge length)
    xe = np.arange(nx + 2) * d[0]
    ye = np.arange(ny + 2) * d[1]
    ze = np.arange(nz + 2) * d[2]
    Ze, Ye, Xe = np.meshgrid(ze, ye, xe, indexing="ij")
    Ax = b_amp * field_at(Xe + 0.5 * d[0], Ye, Ze) * d[0]
    Ay = b_amp * field_at(Xe, Ye + 0.5 * d[1], Ze) * d[1]
    Az = b_amp * field_at(Xe, Ye, Ze + 0.5 * d[2]) * d[2]
    if bc[0] == PERIODIC:  # wrap so the curl is periodic
        Ax[:, :, nx:] = Ax[:, :, :2]; Ay[:, :, nx:] = Ay[:, :, :2]; Az[:, :, nx:] = Az[:, :, :2]
    if bc[2] == PERIODIC:
        Ax[:, ny:, :] = Ax[:, :2, :]; Ay[:, ny:, :] = Ay[:, :2, :]; Az[:, ny:, :] = Az[:, :2, :]
    if bc[4] == PERIODIC:
        Ax[nz:, :, :] = Ax[:2, :, :]; Ay[nz:, :, :] = Ay[:2, :, :]; Az[nz:, :, :] = Az[:2, :, :]
    bx = ((Az[:nz, 1:ny + 1, :nx + ox] - Az[:nz, :ny, :nx + ox])
          - (Ay[1:nz + 1, :ny, :nx + ox] - Ay[:nz, :ny, :nx + ox])) / (d[1] * d[2]) + b0[0]
    by = ((Ax[1:nz + 1, :ny + oy, :nx] - Ax[:nz, :ny + oy, :nx])
          - (Az[:nz, :ny + oy, 1:nx + 1] - Az[:nz, :ny + oy, :nx])) / (d[2] * d[0]) + b0[1]
    bz = ((Ay[:nz + oz, :ny, 1:nx + 1] - Ay[:nz + oz, :ny, :nx])
          - (Ax[:nz + oz, 1:ny + 1, :nx] - Ax[:nz + oz, :ny, :nx])) / (d[0] * d[1]) + b0[2]
    cell5 = _pack(rho, vx, vy, vz, P, bx, by, bz, gamma, bc)
    return Problem("random_smooth", nx, ny, nz, d[0], d[1], d[2], 0.0, 0.0, 0.0, gamma,
                   tuple(bc), cell5, np.ascontiguousarray(bx), np.ascontiguousarray(by),
                   np.ascontiguousarray(bz), extra=dict(seed=seed))


def random_face_states(m: int, seed: int = 0, *, gamma=5.0 / 3.0, shock_frac=0.3):
    """m random (W_L, W_R, Bn) face-frame states for Riemann-solver tests:
    rho, P lognormal, v and B normal; a fraction get strong jumps.
    Returns wl [m][7], wr [m][7], bn [m]."""
    rng = np.random.default_rng(seed)

    def draw():
        rho = np.exp(rng.normal(0.0, 0.7, m))
        p = np.exp(rng.normal(-0.5, 0.8, m))
        v = rng.normal(0.0, 1.0, (3, m))
        b = rng.normal(0.0, 0.8, (2, m))
        return np.stack([rho, v[0], v[1], v[2], p, b[0], b[1]], axis=1)

    wl = draw()
    wr = draw()
    near = rng.uniform(size=m) > shock_frac
    # most faces: small jumps (smooth flow); the rest: arbitrary jumps
    wr[near] = wl[near] * (1.0 + 0.05 * rng.standard_normal((int(near.sum()), 7)))
    bn = rng.normal(0.0, 0.8, m)
    bn[rng.uniform(size=m) < 0.05] = 0.0
    return np.ascontiguousarray(wl), np.ascontiguousarray(wr), bn


# ---------------------------------------------------------------------------
# Passive scalars (mass fractions carried by the flow)
# ---------------------------------------------------------------------------

def cell_centres(pb: Problem):
    """Cell-centre coordinate arrays X, Y, Z of shape (nz, ny, nx)."""
    xc = pb.x0 + (np.arange(pb.nx) + 0.5) * pb.dx
    yc = pb.y0 + (np.arange(pb.ny) + 0.5) * pb.dy
    zc = pb.z0 + (np.arange(pb.nz) + 0.5) * pb.dz
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    return X, Y, Z


def mass_fractions(pb: Problem, ns: int, kind: str = "random", *, seed: int = 0, axis: int = 0,
                   x_split: float = 0.0, amp: float = 0.3, const: float = 0.25) -> np.ndarray:
    """Conserved passive scalars rho X_s, float64 [ns][nz][ny][nx], for the
    state of `pb` (rho from its cell5).

    kind: "const"  X_s = const (s + 1) / ns;
          "step"   X_s = 1 left of x_split along `axis`, 0 right of it (scalar
                   s > 0: the complement 1 - X_0 for even s);
          "sine"   X_s = 0.5 + amp sin(2 pi (s + 1) x / L) along `axis` (L the
                   box length);
          "random" X_s in (0, 1): logistic of a few random Fourier modes of the
                   box (periodic), seeded."""
    rho = pb.cell5[0]
    X, Y, Z = cell_centres(pb)
    coord = (X, Y, Z)[axis]
    lo = (pb.x0, pb.y0, pb.z0)[axis]
    L = (pb.nx * pb.dx, pb.ny * pb.dy, pb.nz * pb.dz)
    out = np.empty((ns,) + rho.shape)
    rng = np.random.default_rng(seed)
    for s in range(ns):
        if kind == "const":
            x = np.full(rho.shape, const * (s + 1) / ns)
        elif kind == "step":
            x = np.where(coord < x_split, 1.0, 0.0)
            if s % 2 == 1:
                x = 1.0 - x
        elif kind == "sine":
            x = 0.5 + amp * np.sin(2.0 * math.pi * (s + 1) * (coord - lo) / L[axis])
        elif kind == "random":
            f = np.zeros(rho.shape)
            for _ in range(4):
                k = rng.integers(-3, 4, size=3)
                ph = rng.uniform(0.0, 2.0 * math.pi)
                f += rng.standard_normal() * np.cos(
                    2.0 * math.pi * (k[0] * (X - pb.x0) / L[0] + k[1] * (Y - pb.y0) / L[1]
                                     + k[2] * (Z - pb.z0) / L[2]) + ph)
            x = 1.0 / (1.0 + np.exp(-2.0 * f))
        else:
            raise ValueError(kind)
        out[s] = rho * x
    return out


# ---------------------------------------------------------------------------
# N-body particles (positions and velocities [3][n], masses [n])
# ---------------------------------------------------------------------------

def gravity_box(n=(32, 32, 32), *, G=1.0, couple_gas=False, rho=1e-6, p=1e-9,
                d=None) -> Problem:
    """Periodic box for particle runs: a uniform gas at rest without field
    (rho, p), self-gravity with constant G; couple_gas False sets src[1] = 1
    (the gas neither sources nor feels the potential: particles only)."""
    nx, ny, nz = n
    if d is None:
        d = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    pb = uniform(n, rho=rho, v=(0.0, 0.0, 0.0), p=p, b=(0.0, 0.0, 0.0), d=d)
    return replace(pb, name="gravity_box", source=SRC_SELF_GRAVITY,
                   src=(G, 0.0 if couple_gas else 1.0, 0.0, 0.0))


def particles_plane_wave(pb: Problem, *, amp=0.01, axis=0, mass_total=1.0, per_cell=1):
    """Cold lattice (per_cell^3 particles per cell, at the cell corners and
    their subdivisions) displaced along `axis` by amp * d sin(2 pi x / L),
    at rest; equal masses summing to mass_total."""
    nc = (pb.nx, pb.ny, pb.nz)
    d = (pb.dx, pb.dy, pb.dz)
    lo = (pb.x0, pb.y0, pb.z0)
    axes = [lo[a] + np.arange(nc[a] * per_cell) * d[a] / per_cell for a in range(3)]
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    L = nc[axis] * d[axis]
    x[axis] += amp * d[axis] * np.sin(2.0 * math.pi * (x[axis] - lo[axis]) / L)
    n = x.shape[1]
    return x, np.zeros_like(x), np.full(n, mass_total / n)


def particles_plummer(pb: Problem, n: int, *, seed=0, scale=0.08, mass_total=1.0, G=1.0,
                      centre=None, virial=True, rmax=None):
    """Plummer sphere of n equal-mass particles (scale radius `scale`, total
    mass mass_total) centred in the box, truncated at rmax (5 scale radii);
    velocities from the Plummer distribution function by rejection sampling
    (virial=True) or at rest."""
    rng = np.random.default_rng(seed)
    if centre is None:
        centre = (pb.x0 + 0.5 * pb.nx * pb.dx, pb.y0 + 0.5 * pb.ny * pb.dy,
                  pb.z0 + 0.5 * pb.nz * pb.dz)
    r = np.empty(n)
    k = 0
    while k < n:
        u = rng.uniform(0.0, 1.0, n)
        rr = scale / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        rr = rr[rr < (5.0 * scale if rmax is None else rmax)]
        take = min(len(rr), n - k)
        r[k:k + take] = rr[:take]
        k += take
    mu = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(1.0 - mu * mu)
    x = np.stack([r * s * np.cos(ph), r * s * np.sin(ph), r * mu])
    for a in range(3):
        x[a] += centre[a]
    v = np.zeros_like(x)
    if virial:
        vesc = np.sqrt(2.0 * G * mass_total) * (r * r + scale * scale) ** -0.25
        q = np.empty(n)
        k = 0
        while k < n:
            qq = rng.uniform(0.0, 1.0, 4 * n)
            yy = rng.uniform(0.0, 0.1, 4 * n)
            ok = qq[yy < qq * qq * (1.0 - qq * qq) ** 3.5]
            take = min(len(ok), n - k)
            q[k:k + take] = ok[:take]
            k += take
        sp = q * vesc
        mu = rng.uniform(-1.0, 1.0, n)
        ph = rng.uniform(0.0, 2.0 * math.pi, n)
        s = np.sqrt(1.0 - mu * mu)
        v = np.stack([sp * s * np.cos(ph), sp * s * np.sin(ph), sp * mu])
    return x, v, np.full(n, mass_total / n)
