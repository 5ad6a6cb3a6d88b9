"""Full-step parity of the HIP path (FP64) against the FP64 oracle: same
seeded inputs, same time steps, element by element over every interior cell
and face (relative to the field's max), tolerance 1e-11."""
import numpy as np
import pytest

from mhd_inputs import problems as P
from oracle import pyorc as O
from tests.gpu_util import (field_errors, field_errors_group, gpu_sim, host_state, needs_gpu,
                             rel_err)
from tests.helpers import oracle_of

pytestmark = [pytest.mark.gpu, needs_gpu]

TOL = 1e-11


def _parity(pb, nsteps, recon=O.RECON_PAPER, tol=TOL, check_dt=True, kappa=1.0 / 3.0,
            riemann=O.RIEMANN_HLLD, zero=()):
    o = oracle_of(pb, recon=recon, kappa=kappa, riemann=riemann)
    s = gpu_sim(pb, precision=0, recon=recon, kappa=kappa, riemann=riemann)
    if check_dt:
        dto, dtg = o.dt(), s.dt()
        assert abs(dtg - dto) <= 1e-13 * dto, (dtg, dto)
    dts = []
    for _ in range(nsteps):
        dt = o.dt()
        dts.append(dt)
        o.step(dt)
    s.step(nsteps, dt=dts)
    got, ref = host_state(s), o.get_state()
    err = field_errors(got, ref, zero=zero)
    bad = {k: v for k, v in err.items() if v > tol}
    assert not bad, (err, field_errors_group(got, ref))
    dg, do = s.diag(), o.diag()
    assert dg["n_hll_fallback"] == do["n_hll_fallback"]
    assert dg["t"] == pytest.approx(do["t"], rel=1e-14)
    assert dg["step"] == nsteps
    return s, o, err


def test_alfven_64_fp64_10_steps():
    """Plain method, FP64, 64^3 Alfven wave, CFL 0.4, 10 steps."""
    pb = P.alfven(64)
    s, o, err = _parity(pb, 10)
    d = s.diag()
    assert d["n_hll_fallback"] == 0
    assert abs(d["mass"] - 1.0) < 1e-13
    assert d["divb_max"] < 1e-12


def test_alfven_self_dt():
    """The device CFL dt (no host sync) gives the same run as injected dts."""
    pb = P.alfven(32)
    o = oracle_of(pb)
    s = gpu_sim(pb)
    for _ in range(5):
        o.step()
    s.step(5)
    err = field_errors(host_state(s), o.get_state())
    assert max(err.values()) <= TOL, err
    assert s.diag()["t"] == pytest.approx(o.diag()["t"], rel=1e-13)


@pytest.mark.parametrize("bc", [(P.PERIODIC,) * 6, (P.OUTFLOW,) * 6,
                                (P.OUTFLOW, P.OUTFLOW, P.PERIODIC, P.PERIODIC, P.OUTFLOW,
                                 P.OUTFLOW)])
def test_random_box_ragged(bc):
    """Several 64-wide tiles in x plus a ragged tail; odd y and z."""
    pb = P.random_smooth((70, 37, 21), seed=31, bc=bc)
    _parity(pb, 4)


@pytest.mark.parametrize("recon", [O.RECON_KAPPA, O.RECON_FIRST])
def test_recon_variants(recon):
    pb = P.random_smooth((40, 18, 12), seed=32)
    _parity(pb, 3, recon=recon)


@pytest.mark.parametrize("kappa", [-1.0, 0.0])
@pytest.mark.parametrize("recon", [O.RECON_PAPER, O.RECON_KAPPA])
def test_other_kappas(recon, kappa):
    """Eq. 12-14 with kappa = -1 (fully upwind) and 0 (upwind biased)."""
    pb = P.random_smooth((40, 18, 12), seed=33)
    _parity(pb, 3, recon=recon, kappa=kappa)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("riemann", [O.RIEMANN_HLL, O.RIEMANN_HLLC])
def test_gas_solvers_sod_each_axis(riemann, axis):
    """The paper's gas-dynamic solvers on the Sod tube laid along each axis."""
    _parity(P.sod(100, axis=axis), 30, riemann=riemann)


@pytest.mark.parametrize("riemann", [O.RIEMANN_HLLD, O.RIEMANN_HLLC])
def test_shu_osher(riemann):
    """Shu-Osher (Mach-3 shock into a density sine), 200 cells, 100 steps."""
    _parity(P.shu_osher(200), 100, riemann=riemann)


def test_hll_with_field():
    """HLL keeps the HLLD wave speeds and is valid with a field: Ryu-Jones
    and a random magnetised box under mixed boundaries."""
    _parity(P.ryu_jones(100), 30, riemann=O.RIEMANN_HLL)
    pb = P.random_smooth((34, 20, 14), seed=35,
                         bc=(P.OUTFLOW, P.OUTFLOW, P.PERIODIC, P.PERIODIC, P.OUTFLOW, P.OUTFLOW))
    _parity(pb, 4, riemann=O.RIEMANN_HLL)


def test_hllc_gas_box():
    """HLLC on a 3-D gas-dynamic box: a random smooth state with the field
    removed (its energy stays, as extra gas pressure)."""
    pb = P.random_smooth((36, 22, 10), seed=36, b0=(0.0, 0.0, 0.0))
    pb.bx[:] = 0.0
    pb.by[:] = 0.0
    pb.bz[:] = 0.0
    _parity(pb, 4, riemann=O.RIEMANN_HLLC)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_brio_wu_each_axis(axis):
    """1-D MHD Riemann problem (shocks, HLLD branches, minmod clipping) laid
    along each axis; the transverse axes have one cell."""
    pb = P.brio_wu(96, axis=axis)
    # v and B have no component along the frame's second transverse axis:
    # those two fields are zero in exact arithmetic (rounding noise here)
    t2 = "xyz"[(axis + 2) % 3]
    _parity(pb, 25, zero=("M" + t2, "B" + t2))


def test_ryu_jones():
    pb = P.ryu_jones(128)
    _parity(pb, 25)


def test_disc_outflow_source_floors():
    """Disc slab: outflow on all sides, logarithmic-potential source, floors."""
    pb = P.disc(40, 36, 20, lx=24.0, ly=21.6, lz=6.0, seed=3)
    s, o, err = _parity(pb, 4)
    assert s.diag()["n_floor"] == o.diag()["n_floor"]


def _cell_pressure(pb):
    """Gas pressure of a periodic problem's cells (face-mean B)."""
    rho, mx, my, mz, e = pb.cell5
    bcx = 0.5 * (pb.bx + np.roll(pb.bx, -1, axis=2))
    bcy = 0.5 * (pb.by + np.roll(pb.by, -1, axis=1))
    bcz = 0.5 * (pb.bz + np.roll(pb.bz, -1, axis=0))
    return (pb.gamma - 1.0) * (e - 0.5 * (mx * mx + my * my + mz * mz) / rho
                               - 0.5 * (bcx * bcx + bcy * bcy + bcz * bcz))


@pytest.mark.parametrize("which", ["rho", "p", "both"])
def test_floors_periodic(which):
    """Floors acting in about a third of a periodic box's cells (the last
    cell of each periodic axis takes its upper face from the first face)."""
    pb = P.random_smooth((20, 16, 12), seed=41, amp=0.5)
    if which in ("rho", "both"):
        pb.rho_floor = float(np.quantile(pb.cell5[0], 0.3))
    if which in ("p", "both"):
        pb.p_floor = float(np.quantile(_cell_pressure(pb), 0.3))
    s, o, err = _parity(pb, 3)
    assert o.diag()["n_floor"] > 0
    assert s.diag()["n_floor"] == o.diag()["n_floor"]


def test_uniform_gravity_source():
    pb = P.random_smooth((20, 16, 12), seed=33)
    pb.source, pb.src = P.SRC_UNIFORM, (0.3, -0.2, 0.5, 0.0)
    _parity(pb, 4)


def test_gaussian_well_inflow():
    """Supersonic flow into a Gaussian potential well: inflow ghost state on
    the low-x side, outflow on the high side."""
    pb = P.riemann_1d((1, 1, 0, 0, 1, 0, 0, 0), (1, 1, 0, 0, 1, 0, 0, 0), 80, xlo=-0.5,
                      xhi=0.5, gamma=1.4, bc_lohi=(P.INFLOW, P.OUTFLOW))
    pb.source, pb.src = P.SRC_GAUSS_X, (5.0, 0.1, 0.0, 0.0)
    pb.inflow = (1.0, 1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0)
    _parity(pb, 30)


@pytest.mark.parametrize("shape", [(1, 9, 7), (9, 1, 7), (9, 7, 1), (1, 1, 5), (3, 2, 2)])
def test_degenerate_extents(shape):
    pb = P.random_smooth(shape, seed=34)
    _parity(pb, 3)


@pytest.mark.parametrize("full", [True, False])
def test_intermediate_arrays_match(full):
    """Corrector fluxes, mass-flux-upwinded edge EMFs and primitives of the
    last stage agree with the oracle's.  Without full fluxes the fused sweep
    keeps only the field components (for the EMFs) in memory."""
    pb = P.random_smooth((24, 20, 16), seed=35)
    o = oracle_of(pb)
    s = gpu_sim(pb)
    s.set_full_fluxes(full)
    dt = o.dt()
    o.step(dt)
    s.step(1, dt=dt)
    nz, ny, nx = pb.shape
    sl = lambda extra: (slice(2, 2 + nz + extra[2]), slice(2, 2 + ny + extra[1]),
                        slice(2, 2 + nx + extra[0]))
    for a in range(3):
        ex = [0, 0, 0]
        ex[a] = 1
        t1, t2 = (a + 1) % 3, (a + 2) % 3
        # frame comps -> oracle global comps
        gmap = {0: 0, 1: 1 + a, 2: 1 + t1, 3: 1 + t2, 4: 4, 5: 5 + t1, 6: 5 + t2}
        for m, gm in gmap.items():
            if not full and m < 5:
                continue
            g = s.debug_array(7 * a + m).cpu().numpy()[sl(ex)]
            r = o.debug_array(8 * a + gm)[sl(ex)]
            assert rel_err(g, r) <= 1e-12, (a, m)
    for c in range(3):
        ex = [1, 1, 1]
        ex[c] = 0
        g = s.debug_array(21 + c).cpu().numpy()[sl(ex)]
        r = o.debug_array(24 + c)[sl(ex)]
        assert rel_err(g, r) <= 1e-12, c


def test_determinism_and_checkpoint_resume():
    """Two runs are bitwise identical; stopping, reading the state out and
    re-initialising from it continues bit for bit."""
    pb = P.random_smooth((33, 17, 9), seed=36)
    a = gpu_sim(pb)
    a.step(6)
    sa = host_state(a)
    b = gpu_sim(pb)
    b.step(3)
    d3 = b.diag()
    st = [t.clone() for t in b.get_state()]
    c = gpu_sim(pb, state=st)
    c.step(3)
    sc = host_state(c)
    b.step(3)
    sb = host_state(b)
    for x, y, z in zip(sa, sb, sc):
        np.testing.assert_array_equal(x, y)
        np.testing.assert_array_equal(x, z)
    assert d3["step"] == 3


def test_ghost_fill_modes_agree():
    """On a fully periodic box the fused path's stage ghost fills leave out
    the x ghost layers (every reader takes the interior images instead);
    a step on another path (here: all fluxes kept) refills them first.
    Switching between the two mid-run gives bitwise the runs that never
    switch, and both match the oracle."""
    pb = P.random_smooth((9, 7, 70), seed=38)
    runs = []
    for plan in ((False,) * 6, (True,) * 6, (False, False, True, True, False, False)):
        s = gpu_sim(pb)
        for full in plan:
            s.set_full_fluxes(full)
            s.step(1)
        runs.append(host_state(s))
    for a, b, c in zip(*runs):
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(a, c)
    o = oracle_of(pb)
    s = gpu_sim(pb)
    for _ in range(6):
        dt = o.dt()
        o.step(dt)
        s.step(1, dt=dt)
    err = field_errors(host_state(s), o.get_state())
    assert max(err.values()) <= TOL, err


def test_bad_state_rejected():
    from paper_1502_02935_amd import MHDError
    pb = P.random_smooth((8, 8, 8), seed=37)
    c5 = pb.cell5.copy()
    c5[0, 3, 4, 5] = -1.0
    with pytest.raises(MHDError) as e:
        gpu_sim(pb, state=(c5, pb.bx, pb.by, pb.bz))
    assert e.value.code == -3
    c5 = pb.cell5.copy()
    c5[4, 1, 1, 1] = np.nan
    with pytest.raises(MHDError):
        gpu_sim(pb, state=(c5, pb.bx, pb.by, pb.bz))


@pytest.mark.parametrize("precision", [0, 1])
def test_unstable_run_sets_sticky_state(precision):
    """Steps far above the CFL limit drive the state to rho <= 0, P <= 0 or
    non-finite values inside the run: the device status word, set by the
    stage update's checks, makes mhd_dt and mhd_diag return MHD_E_STATE
    (with the diagnostics filled), and every later step is refused with it
    (sticky), on the same context."""
    from paper_1502_02935_amd import MHDError
    pb = P.random_smooth((16, 16, 16), seed=38)
    s = gpu_sim(pb, precision=precision)
    dt = s.dt()
    s.step(20, dt=30.0 * dt)
    d = s.diag(check=False)
    print("UNSTABLE", precision, d["rc"], d["status"], d["rho_min"], d["p_min"], flush=True)
    assert d["rc"] == -3 and d["status"] != 0
    with pytest.raises(MHDError) as e:
        s.dt()
    assert e.value.code == -3
    with pytest.raises(MHDError) as e:
        s.step(1, dt=dt)
    assert e.value.code == -3
    s.close()


def test_conservation_and_divb_on_device():
    """Periodic box on the GPU alone (any size): FP64 sums of mass, momentum,
    energy and face B are constant; div B stays at rounding level."""
    pb = P.turbulent_ism(96, seed=5)
    s = gpu_sim(pb)
    d0 = s.diag()
    s.step(10)
    d1 = s.diag()
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * d0["mass"]
    for a in range(3):
        assert abs(d1["mom"][a] - d0["mom"][a]) <= 1e-12 * (abs(d0["mom"][a]) + d0["mass"])
        assert abs(d1["bsum"][a] - d0["bsum"][a]) <= 1e-13 * (abs(d0["bsum"][a]) + 1.0)
    assert abs(d1["energy"] - d0["energy"]) <= 1e-13 * d0["energy"]
    assert d1["divb_max"] < 1e-12
    assert d1["n_hll_fallback"] == 0
