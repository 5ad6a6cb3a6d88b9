"""Host-side logic that needs no GPU: workload construction for the
learned-correction driver and the disc runs, coarse-grid configuration, and
the workspace the disc's largest box asks for."""
import numpy as np
import pytest

from mhd_inputs import problems as P
from paper_1502_02935_amd import _lib as L
from paper_1502_02935_amd import learned
from paper_1502_02935_amd.sim import config_from_problem, workspace_bytes


def test_disc_problem_keeps_cell_size_and_outflow():
    pb = learned.make_problem("disc", 64, seed=3)
    assert (pb.nx, pb.ny, pb.nz) == (64, 64, 16)
    # 24 x 24 x 6 kpc at 512: the box scales with n, the cell stays 46.875 pc
    assert pb.dx == pb.dy == pb.dz == 24.0 / 512
    assert pb.bc == (P.OUTFLOW,) * 6
    assert pb.source == P.SRC_LOGPOT and pb.rho_floor > 0
    # rounded to FP32 and back
    assert np.array_equal(pb.cell5, pb.cell5.astype(np.float32).astype(np.float64))


def test_coarse_config_halves_the_grid():
    pb = learned.make_problem("disc", 64, seed=3)
    f = config_from_problem(pb, precision=L.MHD_FP32)
    c = learned.coarse_config(f)
    assert (c.nx, c.ny, c.nz) == (32, 32, 8)
    assert (c.dx, c.dy, c.dz) == (2 * f.dx, 2 * f.dy, 2 * f.dz)
    assert (c.x0, c.y0, c.z0) == (f.x0, f.y0, f.z0)
    assert c.bc == f.bc and c.source == f.source and c.src == f.src
    assert (c.rho_floor, c.p_floor) == (f.rho_floor, f.p_floor)


def test_turbulent_problem_is_periodic_fp32():
    pb = learned.make_problem("turbulent", 16, seed=4)
    assert pb.bc == (P.PERIODIC,) * 6 and (pb.nx, pb.ny, pb.nz) == (16, 16, 16)
    assert abs(pb.cell5[0].mean() - 1.0) < 1e-6


def test_unknown_problem_rejected():
    with pytest.raises(ValueError):
        learned.make_problem("sedov", 16, seed=1)


def test_largest_disc_fits_one_gpu():
    """The 1024 x 1024 x 256 FP32 disc asks for ~68 GB of workspace (60
    padded arrays of 1029 x 1029 x 261 floats plus scratch), far inside
    288 GB of HBM."""
    from paper_1502_02935_amd.sim import MHDConfig
    cfg = MHDConfig(nx=1024, ny=1024, nz=256, dx=0.046875, dy=0.046875, dz=0.046875,
                    precision=L.MHD_FP32, bc=(L.BC_OUTFLOW,) * 6, source=1,
                    src=(200.0, 0.5, 1.0, 0.0), rho_floor=1e-5, p_floor=1e-3)
    b = workspace_bytes(cfg)
    assert 60 * 1029 * 1029 * 261 * 4 < b < 70e9
