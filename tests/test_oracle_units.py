"""Pins of the oracle's single-face building blocks against what the paper and
the mathematics fix (no GPU).  Section 2.1: Eq. 3 fluxes, Eq. 12-14 MUSCL with
minmod, and the HLLD solver the paper cites (Miyoshi & Kusano 2005)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import pyorc as O
from mhd_inputs.problems import random_face_states

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- Eq. 3 -----

def test_phys_flux_hand_values():
    with open(os.path.join(GOLD, "phys_flux_eq3.json")) as f:
        g = json.load(f)
    for c in g["cases"]:
        u = O.prim_to_cons(c["w"], c["bn"], c["gamma"])
        f = O.phys_flux(c["w"], c["bn"], c["gamma"])
        np.testing.assert_allclose(u, c["cons"], rtol=0, atol=1e-14)
        np.testing.assert_allclose(f, c["flux"], rtol=0, atol=1e-13)


def test_fast_speed_textbook_form():
    """Non-negative discriminant form equals the textbook
    c_f^2 = ((a^2+b^2) + sqrt((a^2+b^2)^2 - 4 a^2 bn^2/rho)) / 2."""
    wl, wr, bn = random_face_states(2000, seed=3)
    g = 5.0 / 3.0
    for w, b in zip(wl, bn):
        a2 = g * w[4] / w[0]
        B2 = (b * b + w[5] ** 2 + w[6] ** 2) / w[0]
        cf2 = 0.5 * ((a2 + B2) + math.sqrt(max((a2 + B2) ** 2 - 4 * a2 * b * b / w[0], 0.0)))
        assert abs(O.fast_speed(w, b, g) - math.sqrt(cf2)) <= 1e-10 * math.sqrt(cf2)
    # pure gas: the sound speed
    assert O.fast_speed([1.3, 0, 0, 0, 0.7, 0, 0], 0.0, 1.4) == pytest.approx(
        math.sqrt(1.4 * 0.7 / 1.3), rel=1e-15)


# -------------------------------------------------------------- minmod -----

def test_minmod_properties():
    rng = np.random.default_rng(0)
    vals = list(rng.normal(size=400)) + [0.0, -0.0, 1.0, -1.0, 2.0, -2.0]
    for a in vals[:60]:
        for b in vals[::7]:
            m = O.minmod(a, b)
            assert m == O.minmod(b, a)                       # symmetric
            assert abs(m) <= min(abs(a), abs(b))             # never larger
            assert m in (a, b, 0.0)                          # picks an argument or 0
            if a * b <= 0:
                assert m == 0.0                              # opposite signs or a zero
            else:
                assert m == (a if abs(a) <= abs(b) else b)
            assert O.minmod(3.0 * a, 3.0 * b) == pytest.approx(3.0 * m, rel=1e-15)
    assert O.minmod(1e-200, 1e-200) == 1e-200  # sign by comparison, no underflow


def test_minmod_is_median_with_zero():
    """minmod(a, b) equals the median of (a, b, 0): the form the GPU kernels
    evaluate with one med3 instruction."""
    rng = np.random.default_rng(4)
    vals = np.concatenate([rng.normal(size=300), [0.0, -0.0, 1e-300, -1e-300, 5.0, -5.0]])
    for a in vals[::3]:
        for b in vals[::5]:
            assert O.minmod(a, b) == float(np.median([a, b, 0.0]))


# ---------------------------------------------------------- Eq. 12-14 -----

def _phi_paper(r):
    """Closed form of the paper's Eq. 13 at kappa = 1/3, derived by hand:
    dW = d0 [K2 min(r,1) + K1 min(1, 4 r)] for r = dm/d0 > 0."""
    if r <= 0:
        return 0.0
    if r < 0.25:
        return 2.0 * r
    if r <= 1.0:
        return 2.0 * r / 3.0 + 1.0 / 3.0
    return 1.0


def _phi_kappa(r):
    """Textbook kappa = 1/3 scheme, limited with b = 4."""
    if r <= 0:
        return 0.0
    if r < 0.25:
        return 3.0 * r
    if r <= 4.0:
        return r / 3.0 + 2.0 / 3.0
    return 2.0


@pytest.mark.parametrize("recon,phi", [(O.RECON_PAPER, _phi_paper), (O.RECON_KAPPA, _phi_kappa)])
def test_muscl_limiter_closed_form(recon, phi):
    rng = np.random.default_rng(1)
    for _ in range(3000):
        w1 = rng.normal()
        d0 = rng.choice([-1, 1]) * np.exp(rng.normal())
        r = rng.choice([rng.uniform(-2, 0), rng.uniform(0, 0.25), rng.uniform(0.25, 1),
                        rng.uniform(1, 4), rng.uniform(4, 20)])
        w0 = w1 - r * d0
        w2 = w1 + d0
        # right-hand stencil mirrored so the right state sees the same ratio
        w3 = w2 + d0 / r if r != 0 else w2 + 1e3
        wl, wr = O.recon([w0, w1, w2, w3], recon)
        assert wl - w1 == pytest.approx(0.5 * phi(r) * d0, rel=1e-13, abs=1e-15)
        rr = (w3 - w2) / d0  # dw_{i+1} / dw_i
        assert w2 - wr == pytest.approx(0.5 * phi(rr) * d0, rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("recon", [O.RECON_PAPER, O.RECON_KAPPA])
def test_muscl_linear_exact_and_bounded(recon):
    rng = np.random.default_rng(2)
    for _ in range(500):
        a, b = rng.normal(size=2)
        w = [a + b * i for i in range(4)]
        wl, wr = O.recon(w, recon)
        mid = a + 1.5 * b
        assert wl == pytest.approx(mid, abs=1e-14 * (1 + abs(mid)))
        assert wr == pytest.approx(mid, abs=1e-14 * (1 + abs(mid)))
        # random data: interface values stay between the two adjacent cells
        w = rng.normal(size=4)
        wl, wr = O.recon(w, recon)
        lo, hi = min(w[1], w[2]), max(w[1], w[2])
        assert lo - 1e-15 <= wl <= hi + 1e-15
        assert lo - 1e-15 <= wr <= hi + 1e-15


def test_muscl_quadratic():
    """Cell averages of x^2 on unit cells: the textbook kappa = 1/3 scheme
    returns the exact point value (i+1/2)^2 where the limiter is inactive
    (third order); the paper's printed form does not (second order)."""
    for i in range(3, 12):
        avg = [(m) ** 2 + 1.0 / 12.0 for m in (i - 1, i, i + 1, i + 2)]
        wl_k, wr_k = O.recon(avg, O.RECON_KAPPA)
        assert wl_k == pytest.approx((i + 0.5) ** 2, rel=1e-14)
        assert wr_k == pytest.approx((i + 0.5) ** 2, rel=1e-14)
        wl_p, _ = O.recon(avg, O.RECON_PAPER)
        assert abs(wl_p - (i + 0.5) ** 2) > 1e-3


def test_first_order_recon():
    assert O.recon([1.0, 2.0, 5.0, 7.0], O.RECON_FIRST) == (2.0, 5.0)


# ---------------------------------------------------------------- HLLD -----

def test_hlld_consistency():
    """F_HLLD(U, U) = F(U) (Eq. 3)."""
    wl, _, bn = random_face_states(3000, seed=4)
    for w, b in zip(wl, bn):
        f, code = O.hlld(w, w, b, 5.0 / 3.0)
        fp = O.phys_flux(w, b, 5.0 / 3.0)
        scale = np.abs(fp).max() + O.prim_to_cons(w, b, 5.0 / 3.0)[4]
        assert np.abs(f - fp).max() <= 1e-14 * scale
        assert code & 1 == 0


def test_hlld_stationary_contact():
    """Density jump at rest with equal P and B: contact speed 0, no mass
    flux, flux = (0, P* - Bn^2, -Bn Bt1, -Bn Bt2, 0, 0, 0)."""
    rng = np.random.default_rng(5)
    for _ in range(300):
        p = np.exp(rng.normal())
        bt = rng.normal(size=2)
        b = rng.normal()
        wl = [np.exp(rng.normal()), 0, 0, 0, p, bt[0], bt[1]]
        wr = [np.exp(rng.normal()), 0, 0, 0, p, bt[0], bt[1]]
        f, _ = O.hlld(wl, wr, b, 5.0 / 3.0)
        pt = p + 0.5 * (b * b + bt[0] ** 2 + bt[1] ** 2)
        want = [0, pt - b * b, -b * bt[0], -b * bt[1], 0, 0, 0]
        np.testing.assert_allclose(f, want, rtol=0, atol=1e-14 * (1 + pt))
        assert abs(f[0]) <= 1e-14 * wl[0]  # zero to rounding


def test_hlld_stationary_rotational_discontinuity():
    """A rotational discontinuity standing still (u = Bn/sqrt(rho), equal rho,
    P, |Bt|, v_t = Bt/sqrt(rho) + c) is resolved exactly: F = F(U_L) = F(U_R)."""
    rng = np.random.default_rng(6)
    g = 5.0 / 3.0
    for _ in range(200):
        rho = np.exp(rng.normal(0, 0.5))
        p = np.exp(rng.normal(0, 0.5))
        bn = abs(rng.normal()) + 0.2
        bmag = abs(rng.normal()) + 0.1
        th = rng.uniform(0, 2 * np.pi, 2)
        btl = bmag * np.array([np.cos(th[0]), np.sin(th[0])])
        btr = bmag * np.array([np.cos(th[1]), np.sin(th[1])])
        c = rng.normal(0, 0.3, 2)
        u = bn / np.sqrt(rho)
        vtl = btl / np.sqrt(rho) + c
        vtr = btr / np.sqrt(rho) + c
        wl = [rho, u, vtl[0], vtl[1], p, btl[0], btl[1]]
        wr = [rho, u, vtr[0], vtr[1], p, btr[0], btr[1]]
        fl = O.phys_flux(wl, bn, g)
        fr = O.phys_flux(wr, bn, g)
        scale = np.abs(fl).max()
        assert np.abs(fl - fr).max() <= 1e-13 * scale  # the jump conditions hold
        f, code = O.hlld(wl, wr, bn, g)
        assert np.abs(f - fl).max() <= 1e-12 * scale, (f, fl)


def _hllc_toro(wl, wr, g):
    """Textbook HLLC (Toro ch. 10) for B = 0, with the same outer wave speeds
    (min/max of u -/+ the larger sound speed)."""
    def cons(w):
        return np.array([w[0], w[0] * w[1], w[0] * w[2], w[0] * w[3],
                         w[4] / (g - 1) + 0.5 * w[0] * (w[1] ** 2 + w[2] ** 2 + w[3] ** 2)])

    def flux(w):
        U = cons(w)
        return np.array([U[1], U[1] * w[1] + w[4], U[2] * w[1], U[3] * w[1], (U[4] + w[4]) * w[1]])

    cl, cr = math.sqrt(g * wl[4] / wl[0]), math.sqrt(g * wr[4] / wr[0])
    sl = min(wl[1], wr[1]) - max(cl, cr)
    sr = max(wl[1], wr[1]) + max(cl, cr)
    rl, ul, pl = wl[0], wl[1], wl[4]
    rr, ur, pr = wr[0], wr[1], wr[4]
    ss = (pr - pl + rl * ul * (sl - ul) - rr * ur * (sr - ur)) / (rl * (sl - ul) - rr * (sr - ur))
    if sl >= 0:
        return flux(wl)
    if sr <= 0:
        return flux(wr)

    def ustar(w, s):
        U = cons(w)
        f = w[0] * (s - w[1]) / (s - ss)
        return f * np.array([1.0, ss, w[2], w[3],
                             U[4] / w[0] + (ss - w[1]) * (ss + w[4] / (w[0] * (s - w[1])))])

    if ss >= 0:
        return flux(wl) + sl * (ustar(wl, sl) - cons(wl))
    return flux(wr) + sr * (ustar(wr, sr) - cons(wr))


def test_hlld_reduces_to_hllc_without_field():
    wl, wr, _ = random_face_states(3000, seed=7)
    for g in (1.4, 5.0 / 3.0):
        for a, b in zip(wl, wr):
            a = a.copy(); b = b.copy()
            a[5:] = 0; b[5:] = 0
            f, code = O.hlld(a, b, 0.0, g)
            h = _hllc_toro(a, b, g)
            scale = np.abs(h).max() + 1.0
            np.testing.assert_allclose(f[:5], h, rtol=0, atol=1e-13 * scale)
            assert f[5] == 0 and f[6] == 0


def test_hlld_mirror_symmetry():
    """x -> -x (u, Bn -> -u, -Bn; L <-> R) flips the sign of every flux
    component but the normal momentum."""
    wl, wr, bn = random_face_states(3000, seed=8)
    sgn = np.array([-1, 1, -1, -1, -1, -1, -1.0])
    for a, b, n in zip(wl, wr, bn):
        f, _ = O.hlld(a, b, n, 5.0 / 3.0)
        ra = a.copy(); ra[1] = -ra[1]
        rb = b.copy(); rb[1] = -rb[1]
        g, _ = O.hlld(rb, ra, -n, 5.0 / 3.0)
        scale = np.abs(f).max() + 1.0
        np.testing.assert_allclose(g, sgn * f, rtol=0, atol=1e-13 * scale)


def test_hlld_transverse_rotation_invariance():
    """Rotating the transverse frame (t1, t2) by an angle rotates the
    transverse flux components the same way."""
    wl, wr, bn = random_face_states(1000, seed=9)
    rng = np.random.default_rng(9)
    for a, b, n in zip(wl, wr, bn):
        th = rng.uniform(0, 2 * np.pi)
        c, s = math.cos(th), math.sin(th)

        def rot(w):
            w = w.copy()
            w[2], w[3] = c * w[2] - s * w[3], s * w[2] + c * w[3]
            w[5], w[6] = c * w[5] - s * w[6], s * w[5] + c * w[6]
            return w

        f, _ = O.hlld(a, b, n, 5.0 / 3.0)
        g, _ = O.hlld(rot(a), rot(b), n, 5.0 / 3.0)
        scale = np.abs(f).max() + 1.0
        np.testing.assert_allclose(g, rot(f), rtol=0, atol=1e-12 * scale)


def test_hlld_supersonic_upwind():
    """All waves moving right: the flux is the left physical flux."""
    w = [1.0, 10.0, 0.1, 0.2, 0.5, 0.3, 0.1]
    w2 = [0.8, 10.5, 0.0, 0.1, 0.4, 0.2, 0.3]
    f, _ = O.hlld(w, w2, 0.4, 5.0 / 3.0)
    np.testing.assert_array_equal(f, O.phys_flux(w, 0.4, 5.0 / 3.0))


def test_hlld_positive_mass_flux_sign_matches_contact():
    """The sign of the HLLD mass flux equals the sign of the contact speed
    S_M (the flux is rho* S_M in both star regions)."""
    wl, wr, bn = random_face_states(3000, seed=10)
    g = 5.0 / 3.0
    for a, b, n in zip(wl, wr, bn):
        f, code = O.hlld(a, b, n, g)
        if code & 1:
            continue
        ul, ur = O.prim_to_cons(a, n, g), O.prim_to_cons(b, n, g)
        cf = max(O.fast_speed(a, n, g), O.fast_speed(b, n, g))
        SL, SR = min(a[1], b[1]) - cf, max(a[1], b[1]) + cf
        if SL > 0 or SR < 0:
            continue
        ptl = a[4] + 0.5 * (n * n + a[5] ** 2 + a[6] ** 2)
        ptr = b[4] + 0.5 * (n * n + b[5] ** 2 + b[6] ** 2)
        al, ar = a[0] * (SL - a[1]), b[0] * (SR - b[1])
        SM = (ar * b[1] - al * a[1] - ptr + ptl) / (ar - al)
        if abs(SM) > 1e-9:
            assert np.sign(f[0]) == np.sign(SM)


def _hll(wl, wr, bn, g):
    ul, ur = O.prim_to_cons(wl, bn, g), O.prim_to_cons(wr, bn, g)
    fl, fr = O.phys_flux(wl, bn, g), O.phys_flux(wr, bn, g)
    cf = max(O.fast_speed(wl, bn, g), O.fast_speed(wr, bn, g))
    SL, SR = min(wl[1], wr[1]) - cf, max(wl[1], wr[1]) + cf
    if SL >= 0:
        return fl, SL, SR, ul, ur
    if SR <= 0:
        return fr, SL, SR, ul, ur
    return (SR * fl - SL * fr + SL * SR * (ur - ul)) / (SR - SL), SL, SR, ul, ur


def _near_degenerate_family():
    """Faces where the outer fast-speed estimate meets the star-region
    Alfven speed (B_t small, Alfven faster than sound): the HLLD star
    denominator rho (S-u)(S-S_M) - Bn^2 sweeps through zero."""
    wl0 = np.array([0.83473414, 0.58323446, -0.51729512, 0.23096148, 0.0958191, 0.02840005,
                    0.00290113])
    wr = np.array([0.9708816, 0.57485266, -0.48631529, 0.22997715, 0.11259915, 0.03746497,
                   -0.0052574])
    for s in np.linspace(-3e-3, 3e-3, 6001):
        wl = wl0.copy()
        wl[0] *= 1.0 + s
        yield wl, wr, 0.5452541031186486


def test_hlld_bounded_near_degenerate_star_states():
    """Both HLL and HLLD satisfy the integral form over the same fan
    [S_L, S_R]; their fluxes can differ by at most about max|S| |U_R - U_L|.
    Near a degenerate star state the printed MK05 star formulas divide by
    a vanishing denominator (v* . B* ~ 1/den^2); the degenerate treatment
    must take over before that term swamps the flux."""
    g = 5.0 / 3.0
    rng = np.random.default_rng(12)
    cases = list(_near_degenerate_family())
    wl, wr, bn = random_face_states(20000, seed=13)
    cases += list(zip(wl, wr, bn))
    for a, b, n in cases:
        f, _ = O.hlld(a, b, n, g)
        h, SL, SR, ul, ur = _hll(a, b, n, g)
        bound = 2.0 * max(abs(SL), abs(SR)) * np.abs(ur - ul).max() + 1e-12 * (np.abs(h).max() + 1)
        assert np.abs(f - h).max() <= bound, (a, b, n, f, h)
