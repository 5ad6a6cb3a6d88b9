"""Python face of the C ABI: a simulation object holding the device state
(torch tensors) and the context, plus the batch kernel entry points."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L


@dataclass
class MHDConfig:
    """Mirror of the C struct mhd_config."""
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    x0: float = 0.0
    y0: float = 0.0
    z0: float = 0.0
    precision: int = L.MHD_FP64
    gamma: float = 5.0 / 3.0
    cfl: float = 0.4
    bc: tuple = (0, 0, 0, 0, 0, 0)
    recon: int = L.RECON_PAPER
    kappa: float = 1.0 / 3.0
    source: int = L.SRC_NONE
    src: tuple = (0.0, 0.0, 0.0, 0.0)
    rho_floor: float = 0.0
    p_floor: float = 0.0
    inflow: tuple = field(default_factory=lambda: (0.0,) * 8)
    riemann: int = L.RIEMANN_HLLD
    nscalar: int = 0
    npart: int = 0
    recovery: int = L.RECOVERY_FP64

    def to_c(self) -> L.mhd_config:
        c = L.mhd_config()
        c.nx, c.ny, c.nz = self.nx, self.ny, self.nz
        c.precision = int(self.precision)
        for i in range(6):
            c.bc[i] = int(self.bc[i])
        c.x0, c.y0, c.z0 = self.x0, self.y0, self.z0
        c.dx, c.dy, c.dz = self.dx, self.dy, self.dz
        c.gamma, c.cfl = self.gamma, self.cfl
        c.recon, c.source, c.kappa = int(self.recon), int(self.source), self.kappa
        for i in range(4):
            c.src[i] = float(self.src[i]) if i < len(self.src) else 0.0
        c.rho_floor, c.p_floor = self.rho_floor, self.p_floor
        for i in range(8):
            c.inflow[i] = float(self.inflow[i])
        c.riemann = int(self.riemann)
        c.nscalar = int(self.nscalar)
        c.npart = int(self.npart)
        c.recovery = int(self.recovery)
        return c

    @property
    def dtype(self):
        """Element type of the state arrays handed across the ABI (FP64 for
        MHD_FP64 and the compensated MHD_FP32_COMP, FP32 for MHD_FP32)."""
        return torch.float32 if self.precision == L.MHD_FP32 else torch.float64

    @property
    def work_dtype(self):
        """Element type of the working arrays (scalars, particles, debug
        arrays, flux accumulator): FP32 in both FP32 forms."""
        return torch.float64 if self.precision == L.MHD_FP64 else torch.float32

    def face_shapes(self):
        ox = 0 if self.bc[0] == L.BC_PERIODIC else 1
        oy = 0 if self.bc[2] == L.BC_PERIODIC else 1
        oz = 0 if self.bc[4] == L.BC_PERIODIC else 1
        return ((self.nz, self.ny, self.nx + ox), (self.nz, self.ny + oy, self.nx),
                (self.nz + oz, self.ny, self.nx))


def config_from_problem(pb, precision=L.MHD_FP64, recon=L.RECON_PAPER, kappa=1.0 / 3.0,
                        cfl=None, riemann=L.RIEMANN_HLLD, nscalar=0, npart=0) -> MHDConfig:
    return MHDConfig(nx=pb.nx, ny=pb.ny, nz=pb.nz, dx=pb.dx, dy=pb.dy, dz=pb.dz, x0=pb.x0,
                     y0=pb.y0, z0=pb.z0, precision=precision, gamma=pb.gamma,
                     cfl=pb.cfl if cfl is None else cfl, bc=tuple(pb.bc), recon=recon,
                     kappa=kappa, source=pb.source, src=tuple(pb.src), rho_floor=pb.rho_floor,
                     p_floor=pb.p_floor, inflow=tuple(pb.inflow), riemann=riemann,
                     nscalar=nscalar, npart=npart)


def workspace_bytes(cfg: MHDConfig) -> int:
    n = C.c_size_t()
    c = cfg.to_c()
    L.check(L.load().mhd_workspace_bytes(C.byref(c), C.byref(n)), "mhd_workspace_bytes")
    return n.value


def _dev(a, dtype, device):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device).contiguous()


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


class Sim:
    """One grid on one GPU.  State arrays may be numpy or torch; they are
    converted to the configured precision on `device`."""

    def __init__(self, cfg: MHDConfig, cell5, bx, by, bz, device="cuda", stream=None):
        self.L = L.load()
        self.cfg = cfg
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        dt = cfg.dtype
        fs = cfg.face_shapes()
        c5 = _dev(cell5, dt, self.device)
        b = [_dev(x, dt, self.device) for x in (bx, by, bz)]
        assert tuple(c5.shape) == (5, cfg.nz, cfg.ny, cfg.nx), c5.shape
        for x, s in zip(b, fs):
            assert tuple(x.shape) == s, (x.shape, s)
        nbytes = workspace_bytes(cfg)
        self._ws_raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws_raw.data_ptr()) % 256
        self.ws = self._ws_raw[off:off + nbytes]
        self._c = cfg.to_c()
        self.ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            rc = self.L.mhd_init(C.byref(self._c), _ptr(self.ws), nbytes, _ptr(c5), _ptr(b[0]),
                                 _ptr(b[1]), _ptr(b[2]), C.c_void_p(self.stream.cuda_stream),
                                 C.byref(self.ctx))
        L.check(rc, "mhd_init")

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            self.L.mhd_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1, dt=None):
        """n steps; dt None = device CFL dt, a float or a sequence of n floats."""
        if dt is None:
            rc = self.L.mhd_step(self.ctx, None, n)
        else:
            arr = np.broadcast_to(np.asarray(dt, dtype=np.float64), (n,)).copy()
            rc = self.L.mhd_step(self.ctx, arr.ctypes.data_as(C.POINTER(C.c_double)), n)
        L.check(rc, "mhd_step")

    def dt(self) -> float:
        out = C.c_double()
        L.check(self.L.mhd_dt(self.ctx, C.byref(out)), "mhd_dt")
        return out.value

    def diag(self, check: bool = True) -> dict:
        d = L.mhd_diag_t()
        rc = self.L.mhd_diag(self.ctx, C.byref(d))
        if check:
            L.check(rc, "mhd_diag")
        return {
            "t": d.t, "step": d.step, "dt": d.dt, "mass": d.mass, "mom": tuple(d.mom),
            "energy": d.energy, "bsum": tuple(d.bsum), "divb_max": d.divb_max,
            "rho_min": d.rho_min, "p_min": d.p_min, "n_floor": d.n_floor,
            "n_hll_fallback": d.n_hll_fallback, "n_degenerate": d.n_degenerate,
            "n_fp64_recovery": d.n_fp64_recovery, "n_mlp_faces": d.n_mlp_faces,
            "n_mlp_gated": d.n_mlp_gated, "status": d.status, "rc": rc,
        }

    # ---- learned correction ------------------------------------------------

    def set_mlp(self, params=None, tau: float = 0.5, jump: float = 0.5, tau_flux: float = 0.0):
        """Enable the fused correction with FP32 device params [6792] (kept
        referenced here), or disable it with None.  Each correction component
        is clipped to tau_flux |F| + tau a_max |U_R - U_L|."""
        if params is None:
            L.check(self.L.mhd_set_mlp(self.ctx, None, None), "mhd_set_mlp")
            self._mlp = None
            return
        assert params.dtype == torch.float32 and params.is_contiguous()
        assert params.numel() == L.MLP_NPARAM and params.device == self.device
        self._mlp = params
        gate = L.mhd_gate(tau, jump, tau_flux)
        L.check(self.L.mhd_set_mlp(self.ctx, _ptr(params), C.byref(gate)), "mhd_set_mlp")

    def flux_accumulator(self, enable: bool = True):
        """Start (zeroed) or stop accumulating dt-weighted corrector fluxes on
        the 2x-coarsened faces; returns the accumulator tensor
        [3][7][nz/2][ny/2][nx/2]."""
        if not enable:
            L.check(self.L.mhd_flux_accumulate(self.ctx, None), "mhd_flux_accumulate")
            return getattr(self, "_acc", None)
        cfg = self.cfg
        self._acc = torch.zeros((3, 7, cfg.nz // 2, cfg.ny // 2, cfg.nx // 2), dtype=cfg.work_dtype,
                                device=self.device)
        L.check(self.L.mhd_flux_accumulate(self.ctx, _ptr(self._acc)), "mhd_flux_accumulate")
        return self._acc

    def coarsen(self):
        cfg = self.cfg
        dt = cfg.dtype
        nx, ny, nz = cfg.nx // 2, cfg.ny // 2, cfg.nz // 2
        c5 = torch.empty((5, nz, ny, nx), dtype=dt, device=self.device)
        ox, oy, oz = (0 if cfg.bc[2 * a] == L.BC_PERIODIC else 1 for a in range(3))
        shapes = ((nz, ny, nx + ox), (nz, ny + oy, nx), (nz + oz, ny, nx))
        b = [torch.empty(sh, dtype=dt, device=self.device) for sh in shapes]
        L.check(self.L.mhd_coarsen(self.ctx, _ptr(c5), _ptr(b[0]), _ptr(b[1]), _ptr(b[2])),
                "mhd_coarsen")
        return c5, b[0], b[1], b[2]

    def set_full_fluxes(self, enable: bool = True):
        """Keep every face's full flux of each stage in memory from the next
        step on (for mlp_samples and the flux entries of debug_array)."""
        L.check(self.L.mhd_set_full_fluxes(self.ctx, 1 if enable else 0), "mhd_set_full_fluxes")

    def mlp_samples(self, acc: torch.Tensor, dt_coarse: float, faces: torch.Tensor):
        """Features, targets and masks of faces [n][4] (axis, i, j, k) from
        this context's last step (taken with set_full_fluxes on, or with the
        learned correction)."""
        n = faces.shape[0]
        assert faces.dtype == torch.int32 and faces.is_contiguous() and faces.shape == (n, 4)
        assert acc.dtype == self.cfg.work_dtype and acc.is_contiguous()
        x = torch.empty((n, 32), dtype=torch.float32, device=self.device)
        t = torch.empty((n, 8), dtype=torch.float32, device=self.device)
        m = torch.empty(n, dtype=torch.uint8, device=self.device)
        L.check(self.L.mhd_mlp_samples(self.ctx, _ptr(acc), dt_coarse, n, _ptr(faces), _ptr(x),
                                       _ptr(t), _ptr(m)), "mhd_mlp_samples")
        return x, t, m

    # ---- N-body particles -----------------------------------------------------

    def set_particles(self, x, v, m):
        """Replace the particles: positions and velocities [3][npart], masses
        [npart] (positions wrap into the box)."""
        cfg = self.cfg
        n = cfg.npart
        xs = _dev(x, cfg.work_dtype, self.device)
        vs = _dev(v, cfg.work_dtype, self.device)
        ms = _dev(m, cfg.work_dtype, self.device)
        assert tuple(xs.shape) == (3, n) and tuple(vs.shape) == (3, n) and tuple(ms.shape) == (n,)
        L.check(self.L.mhd_set_particles(self.ctx, _ptr(xs), _ptr(vs), _ptr(ms)),
                "mhd_set_particles")

    def get_particles(self):
        """(positions, velocities), each [3][npart] on the device."""
        cfg = self.cfg
        x = torch.empty((3, cfg.npart), dtype=cfg.work_dtype, device=self.device)
        v = torch.empty_like(x)
        L.check(self.L.mhd_get_particles(self.ctx, _ptr(x), _ptr(v)), "mhd_get_particles")
        return x, v

    # ---- passive scalars ------------------------------------------------------

    def set_scalars(self, rho_x):
        """Replace the passive scalars rho X_s ([nscalar][nz][ny][nx])."""
        cfg = self.cfg
        a = _dev(rho_x, cfg.work_dtype, self.device)
        assert tuple(a.shape) == (cfg.nscalar, cfg.nz, cfg.ny, cfg.nx), a.shape
        L.check(self.L.mhd_set_scalars(self.ctx, _ptr(a)), "mhd_set_scalars")

    def get_scalars(self) -> torch.Tensor:
        cfg = self.cfg
        a = torch.empty((cfg.nscalar, cfg.nz, cfg.ny, cfg.nx), dtype=cfg.work_dtype,
                        device=self.device)
        L.check(self.L.mhd_get_scalars(self.ctx, _ptr(a)), "mhd_get_scalars")
        return a

    def get_state(self):
        cfg = self.cfg
        dt = cfg.dtype
        c5 = torch.empty((5, cfg.nz, cfg.ny, cfg.nx), dtype=dt, device=self.device)
        b = [torch.empty(s, dtype=dt, device=self.device) for s in cfg.face_shapes()]
        L.check(self.L.mhd_get_state(self.ctx, _ptr(c5), _ptr(b[0]), _ptr(b[1]), _ptr(b[2])),
                "mhd_get_state")
        return c5, b[0], b[1], b[2]

    def profile(self, enable: bool = True):
        """Start (clearing earlier records) or stop per-kernel event timing."""
        L.check(self.L.mhd_profile(self.ctx, 1 if enable else 0), "mhd_profile")

    def profile_get(self) -> dict:
        """{kernel class: (total ms, launches)} since profiling was enabled."""
        p = L.mhd_profile_t()
        L.check(self.L.mhd_profile_get(self.ctx, C.byref(p)), "mhd_profile_get")
        return {k: (p.ms[i], p.launches[i]) for i, k in enumerate(L.KERNEL_KINDS)}

    def debug_array(self, what: int) -> torch.Tensor:
        cfg = self.cfg
        out = torch.empty((cfg.nz + 5, cfg.ny + 5, cfg.nx + 5), dtype=cfg.work_dtype,
                          device=self.device)
        n = C.c_size_t()
        L.check(self.L.mhd_debug_array(self.ctx, what, _ptr(out), C.byref(n)), "mhd_debug_array")
        assert n.value == out.numel()
        return out


def hlld_batch(wl: torch.Tensor, wr: torch.Tensor, bn: torch.Tensor, gamma: float,
               stream=None):
    """HLLD fluxes of n face-frame states on the device ([n][7], [n][7], [n])."""
    lib = L.load()
    prec = L.MHD_FP64 if wl.dtype == torch.float64 else L.MHD_FP32
    n = wl.shape[0]
    assert wl.is_contiguous() and wr.is_contiguous() and bn.is_contiguous()
    assert wl.shape == (n, 7) and wr.shape == (n, 7) and bn.shape == (n,)
    assert wl.dtype == wr.dtype == bn.dtype and wl.device == wr.device == bn.device
    flux = torch.empty_like(wl)
    code = torch.empty(n, dtype=torch.int8, device=wl.device)
    st = stream if stream is not None else torch.cuda.current_stream(wl.device)
    L.check(lib.mhd_hlld_batch(prec, n, _ptr(wl), _ptr(wr), _ptr(bn), gamma, _ptr(flux),
                               _ptr(code), C.c_void_p(st.cuda_stream)), "mhd_hlld_batch")
    return flux, code


def recon_batch(w4: torch.Tensor, recon: int = L.RECON_PAPER, kappa: float = 1.0 / 3.0,
                stream=None):
    lib = L.load()
    prec = L.MHD_FP64 if w4.dtype == torch.float64 else L.MHD_FP32
    n = w4.shape[0]
    assert w4.is_contiguous() and w4.shape == (n, 4)
    wl = torch.empty(n, dtype=w4.dtype, device=w4.device)
    wr = torch.empty_like(wl)
    st = stream if stream is not None else torch.cuda.current_stream(w4.device)
    L.check(lib.mhd_recon_batch(prec, n, _ptr(w4), recon, kappa, _ptr(wl), _ptr(wr),
                                C.c_void_p(st.cuda_stream)), "mhd_recon_batch")
    return wl, wr


# ---- learned correction: training kernels ----------------------------------

def _stream(dev, stream=None):
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    return C.c_void_p(st.cuda_stream)


def mlp_forward(x: torch.Tensor, params: torch.Tensor, stream=None) -> torch.Tensor:
    lib = L.load()
    assert x.dtype == torch.float32 and x.is_contiguous() and x.shape[1] == 32
    assert params.dtype == torch.float32 and params.numel() == L.MLP_NPARAM
    y = torch.empty((x.shape[0], 8), dtype=torch.float32, device=x.device)
    L.check(lib.mhd_mlp_forward(x.shape[0], _ptr(x), _ptr(params), _ptr(y),
                                _stream(x.device, stream)), "mhd_mlp_forward")
    return y


class MlpTrainer:
    """Adam on the MSE loss, every pass in the library's MFMA kernels."""

    def __init__(self, params: torch.Tensor, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        assert params.dtype == torch.float32 and params.numel() == L.MLP_NPARAM
        self.lib = L.load()
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.grad = torch.zeros_like(params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.step_count = 0
        self._ws = None

    def gradient(self, x: torch.Tensor, t: torch.Tensor):
        n = x.shape[0]
        assert x.shape == (n, 32) and t.shape == (n, 8)
        assert x.is_contiguous() and t.is_contiguous()
        nb = C.c_size_t()
        L.check(self.lib.mhd_mlp_grad_workspace_bytes(n, C.byref(nb)), "mhd_mlp_grad_workspace_bytes")
        if self._ws is None or self._ws.numel() < nb.value:
            self._ws = torch.empty(nb.value, dtype=torch.uint8, device=x.device)
        L.check(self.lib.mhd_mlp_grad(n, _ptr(x), _ptr(t), _ptr(self.params), _ptr(self.grad),
                                      _ptr(self.loss), _ptr(self._ws), self._ws.numel(),
                                      _stream(x.device)), "mhd_mlp_grad")
        return self.grad, self.loss

    def step(self, x: torch.Tensor, t: torch.Tensor):
        self.gradient(x, t)
        self.step_count += 1
        L.check(self.lib.mhd_mlp_adam(_ptr(self.params), _ptr(self.m), _ptr(self.v),
                                      _ptr(self.grad), self.step_count, self.lr, self.b1, self.b2,
                                      self.eps, _stream(self.params.device)), "mhd_mlp_adam")
        return self.loss
