"""The C-ABI library loads and exports every symbol include/mhd.h declares;
host-side argument checking (no GPU needed: these calls never touch HIP)."""
import ctypes as C

import pytest

from paper_1502_02935_amd import _lib as L
from paper_1502_02935_amd.sim import MHDConfig, workspace_bytes


def test_library_exports_header_symbols():
    lib = L.load()
    syms = L.declared_symbols()
    assert len(syms) >= 10
    for s in syms:
        assert hasattr(lib, s), s
    assert lib.mhd_abi_version() == 1
    for code in (0, -1, -2, -3, -4, -5, 7):
        assert isinstance(L.strerror(code), str) and L.strerror(code)


def _cfg(**kw):
    c = MHDConfig(nx=16, ny=8, nz=4, dx=0.1, dy=0.1, dz=0.1)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_workspace_bytes_valid():
    n64 = workspace_bytes(_cfg())
    n32 = workspace_bytes(_cfg(precision=1))
    assert n64 > n32 > 0
    assert n64 % 256 == 0
    # 60 padded arrays of 21 x 13 x 9 points at least
    assert n64 >= 60 * 21 * 13 * 9 * 8


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-3), dict(dx=0.0), dict(dz=-1.0), dict(gamma=1.0), dict(cfl=0.0),
    dict(cfl=1.5), dict(precision=3), dict(recon=5), dict(kappa=1.0), dict(source=9),
    dict(rho_floor=-1.0), dict(bc=(0, 1, 0, 0, 0, 0)), dict(bc=(7, 7, 0, 0, 0, 0)),
    dict(nx=1 << 21), dict(nx=2048, ny=2048, nz=1024), dict(nscalar=-1), dict(nscalar=9),
    dict(npart=-1), dict(npart=10),
])
def test_workspace_bytes_rejects(bad):
    c = _cfg(**bad).to_c()
    n = C.c_size_t(12345)
    assert L.load().mhd_workspace_bytes(C.byref(c), C.byref(n)) == L.MHD_E_ARG


def test_null_arguments_rejected():
    lib = L.load()
    c = _cfg().to_c()
    assert lib.mhd_workspace_bytes(C.byref(c), None) == L.MHD_E_ARG
    assert lib.mhd_workspace_bytes(None, None) == L.MHD_E_ARG
    assert lib.mhd_step(None, None, 1) == L.MHD_E_ARG
    assert lib.mhd_dt(None, None) == L.MHD_E_ARG
    assert lib.mhd_diag(None, None) == L.MHD_E_ARG
    assert lib.mhd_destroy(None) == L.MHD_E_ARG
    assert lib.mhd_get_state(None, None, None, None, None) == L.MHD_E_ARG
    assert lib.mhd_set_scalars(None, None) == L.MHD_E_ARG
    assert lib.mhd_set_particles(None, None, None, None) == L.MHD_E_ARG
    assert lib.mhd_get_particles(None, None, None) == L.MHD_E_ARG
    assert lib.mhd_get_scalars(None, None) == L.MHD_E_ARG
    ctx = C.c_void_p()
    assert lib.mhd_init(C.byref(c), None, 0, None, None, None, None, None,
                        C.byref(ctx)) == L.MHD_E_ARG
    assert lib.mhd_hlld_batch(0, -1, None, None, None, 1.4, None, None, None) == L.MHD_E_ARG
    assert lib.mhd_hlld_batch(3, 1, None, None, None, 1.4, None, None, None) == L.MHD_E_ARG
    assert lib.mhd_recon_batch(0, 1, None, 0, 0.3, None, None, None) == L.MHD_E_ARG
    # zero-length batches are valid no-ops
    assert lib.mhd_hlld_batch(0, 0, None, None, None, 1.4, None, None, None) == L.MHD_OK
    assert lib.mhd_recon_batch(1, 0, None, 0, 0.3, None, None, None) == L.MHD_OK


def test_workspace_rejects_arrays_beyond_32bit_offsets():
    """An FP64 padded array above 4 GiB cannot be addressed by the flux
    kernel's 32-bit byte offsets: rejected; the same grid in FP32 fits."""
    big = dict(nx=1000, ny=1000, nz=600, dx=1.0, dy=1.0, dz=1.0)
    assert workspace_bytes(MHDConfig(precision=L.MHD_FP32, **big)) > 0
    with pytest.raises(Exception):
        workspace_bytes(MHDConfig(precision=L.MHD_FP64, **big))


def test_self_gravity_needs_periodic_power_of_two_box():
    base = dict(dx=0.1, dy=0.1, dz=0.1, source=L.SRC_SELF_GRAVITY, src=(1.0, 0.0, 0.0, 0.0))
    assert workspace_bytes(MHDConfig(nx=32, ny=16, nz=8, **base)) > 0
    with pytest.raises(Exception):
        workspace_bytes(MHDConfig(nx=24, ny=16, nz=8, **base))
    with pytest.raises(Exception):
        workspace_bytes(MHDConfig(nx=32, ny=16, nz=8, bc=(L.BC_OUTFLOW,) * 6, **base))
    # the gravity buffers come on top of the plain step's
    plain = workspace_bytes(MHDConfig(nx=32, ny=16, nz=8, dx=0.1, dy=0.1, dz=0.1))
    assert workspace_bytes(MHDConfig(nx=32, ny=16, nz=8, **base)) > plain


def test_scalars_add_two_padded_arrays_each():
    """Each passive scalar takes two padded arrays (t^n and t^{n+1/2})."""
    base = workspace_bytes(_cfg())
    arr = (16 + 5) * (8 + 5) * (4 + 5) * 8
    arr = (arr + 255) // 256 * 256
    for ns in (1, 3, 8):
        assert workspace_bytes(_cfg(nscalar=ns)) == base + 2 * ns * arr


def test_particles_need_self_gravity_and_add_their_buffers():
    """Per particle: two buffers of 7 values (x, v, m; the sort's target)
    and two ids; per 8^3-cell tile: counter, offset, cursor, chunk offset;
    the chunk list (tile, first, end) of at most n / 2048 + tiles chunks."""
    base = dict(nx=16, ny=8, nz=4, dx=0.1, dy=0.1, dz=0.1, source=L.SRC_SELF_GRAVITY,
                src=(1.0, 0.0, 0.0, 0.0))
    a = lambda b: (b + 255) // 256 * 256
    nt = 2 * 1 * 1
    for n, es, prec in ((1000, 8, 0), (1000, 4, 1), (12345, 4, 1)):
        w = workspace_bytes(MHDConfig(npart=n, precision=prec, **base))
        w0 = workspace_bytes(MHDConfig(precision=prec, **base))
        mc = n // 2048 + nt
        assert w - w0 == 2 * a(7 * n * es) + 2 * a(4 * n) + a(4 * (4 * nt + 3 + 3 * mc))
    with pytest.raises(L.MHDError):
        workspace_bytes(MHDConfig(npart=1 << 31, **base))


def test_grad_noalloc_checks_arguments_on_the_host():
    """The gradient entry point without allocation refuses bad sizes and
    NULL pointers before any HIP call (so this runs without a GPU): n <= 0
    or a NULL pointer -> MHD_E_ARG; n above MHD_MLP_NOALLOC_MAX -> MHD_E_WS."""
    lib = L.load()
    fake = C.c_void_p(256)  # never dereferenced: the call returns first
    assert lib.mhd_mlp_grad_noalloc(L.MLP_NOALLOC_MAX + 1, fake, fake, fake, fake, None,
                                    None) == L.MHD_E_WS
    assert lib.mhd_mlp_grad_noalloc(0, fake, fake, fake, fake, None, None) == L.MHD_E_ARG
    assert lib.mhd_mlp_grad_noalloc(10, None, fake, fake, fake, None, None) == L.MHD_E_ARG
    assert lib.mhd_mlp_grad_noalloc(10, fake, fake, fake, None, None, None) == L.MHD_E_ARG


def test_compensated_precision_configuration():
    """MHD_FP32_COMP: 15 FP32 arrays more than MHD_FP32 (the low parts of the
    two state sets' cells, the stage increments); the recovery switch is an
    MHD_FP32 option only."""
    base = workspace_bytes(_cfg(precision=L.MHD_FP32))
    comp = workspace_bytes(_cfg(precision=L.MHD_FP32_COMP))
    arr = (16 + 5) * (8 + 5) * (4 + 5) * 4
    arr = (arr + 255) // 256 * 256
    assert comp == base + 15 * arr
    lib = L.load()
    n = C.c_size_t()
    for prec in (L.MHD_FP64, L.MHD_FP32_COMP):
        c = _cfg(precision=prec, recovery=L.RECOVERY_OFF).to_c()
        assert lib.mhd_workspace_bytes(C.byref(c), C.byref(n)) == L.MHD_E_ARG
    c = _cfg(precision=L.MHD_FP32, recovery=L.RECOVERY_OFF).to_c()
    assert lib.mhd_workspace_bytes(C.byref(c), C.byref(n)) == L.MHD_OK
    c = _cfg(precision=3).to_c()
    assert lib.mhd_workspace_bytes(C.byref(c), C.byref(n)) == L.MHD_E_ARG


def test_library_links_roctx_for_stage_ranges():
    """The step marks its enqueueing with roctx ranges (mhd_step,
    mhd_predictor, mhd_corrector) for rocprofv3 --marker-trace: the library
    needs the roctx runtime and imports its range calls."""
    import shutil
    import subprocess
    if shutil.which("readelf") is None:
        pytest.skip("readelf not available")
    dyn = subprocess.run(["readelf", "-d", L.LIB_PATH], capture_output=True, text=True).stdout
    assert "librocprofiler-sdk-roctx" in dyn
    syms = subprocess.run(["readelf", "--dyn-syms", "-W", L.LIB_PATH], capture_output=True,
                          text=True).stdout
    assert "roctxRangePushA" in syms and "roctxRangePop" in syms
