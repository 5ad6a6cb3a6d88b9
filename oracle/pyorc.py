"""ctypes binding of the FP64 CPU oracle (oracle/orc.c).

Test infrastructure only.  The C library follows section 2.1 of the paper
(Eq. 1-14, HLLD of Miyoshi & Kusano); this module only marshals arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

BC_PERIODIC, BC_OUTFLOW, BC_INFLOW = 0, 1, 2
RECON_PAPER, RECON_KAPPA, RECON_FIRST = 0, 1, 2
RIEMANN_HLLD, RIEMANN_HLL, RIEMANN_HLLC = 0, 1, 2
MLP_NPARAM = 6792
SRC_NONE, SRC_LOGPOT, SRC_UNIFORM, SRC_GAUSS_X, SRC_SELF_GRAVITY = 0, 1, 2, 3, 4


class _Cfg(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("bc", C.c_int32 * 6),
        ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
        ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
        ("gamma", C.c_double), ("cfl", C.c_double),
        ("recon", C.c_int32), ("kappa", C.c_double),
        ("source", C.c_int32), ("src", C.c_double * 4),
        ("rho_floor", C.c_double), ("p_floor", C.c_double),
        ("inflow", C.c_double * 8),
        ("riemann", C.c_int32),
        ("nscalar", C.c_int32),
        ("npart", C.c_int64),
    ]


class _Diag(C.Structure):
    _fields_ = [
        ("t", C.c_double), ("step", C.c_int64),
        ("mass", C.c_double), ("mom", C.c_double * 3), ("energy", C.c_double),
        ("bsum", C.c_double * 3), ("divb_max", C.c_double),
        ("rho_min", C.c_double), ("p_min", C.c_double),
        ("n_floor", C.c_int64), ("n_hll_fallback", C.c_int64),
        ("n_degenerate", C.c_int64),
        ("n_mlp_faces", C.c_int64), ("n_mlp_gated", C.c_int64),
    ]


@dataclass
class OrcConfig:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    x0: float = 0.0
    y0: float = 0.0
    z0: float = 0.0
    gamma: float = 5.0 / 3.0
    cfl: float = 0.4
    bc: tuple = (0, 0, 0, 0, 0, 0)
    recon: int = RECON_PAPER
    kappa: float = 1.0 / 3.0
    source: int = SRC_NONE
    src: tuple = (0.0, 0.0, 0.0, 0.0)
    rho_floor: float = 0.0
    p_floor: float = 0.0
    inflow: tuple = field(default_factory=lambda: (0.0,) * 8)
    riemann: int = RIEMANN_HLLD
    nscalar: int = 0
    npart: int = 0

    def to_c(self) -> _Cfg:
        c = _Cfg()
        c.nx, c.ny, c.nz = self.nx, self.ny, self.nz
        for i in range(6):
            c.bc[i] = int(self.bc[i])
        c.x0, c.y0, c.z0 = self.x0, self.y0, self.z0
        c.dx, c.dy, c.dz = self.dx, self.dy, self.dz
        c.gamma, c.cfl = self.gamma, self.cfl
        c.recon, c.kappa = int(self.recon), self.kappa
        c.source = int(self.source)
        for i in range(4):
            c.src[i] = float(self.src[i]) if i < len(self.src) else 0.0
        c.rho_floor, c.p_floor = self.rho_floor, self.p_floor
        for i in range(8):
            c.inflow[i] = float(self.inflow[i])
        c.riemann = int(self.riemann)
        c.nscalar = int(self.nscalar)
        c.npart = int(self.npart)
        return c


def build_oracle(force: bool = False) -> str:
    """Compile liborc.so with gcc (plain C11, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_OPC_SRC = os.path.join(_HERE, "opcount.cpp")
_OPC_LIB = os.path.join(_HERE, "libopcount.so")


def build_opcount(force: bool = False) -> str:
    """Compile the operation-counting build of the oracle (libopcount.so)."""
    import re
    import tempfile
    if not force and os.path.exists(_OPC_LIB) and os.path.getmtime(_OPC_LIB) >= max(
            os.path.getmtime(_SRC), os.path.getmtime(_OPC_SRC)):
        return _OPC_LIB
    with open(_SRC) as f:
        src = f.read()
    with open(os.path.join(_HERE, "orc.h")) as f:
        hdr = f.read()
    with tempfile.TemporaryDirectory() as d:
        with open(os.path.join(d, "orc.h"), "w") as f:
            f.write(re.sub(r"\bdouble\b", "orc_real", hdr))
        gen = os.path.join(d, "orc_real.c")
        with open(gen, "w") as f:
            f.write(re.sub(r"\bdouble\b", "orc_real", src))
        tmp = _OPC_LIB + ".tmp%d" % os.getpid()
        subprocess.run(["g++", "-std=c++17", "-O1", "-fPIC", "-shared", "-w",
                        "-DORC_REAL_SOURCE=\"%s\"" % gen, "-I", d, "-o", tmp, _OPC_SRC],
                       check=True)
        os.replace(tmp, _OPC_LIB)
    return _OPC_LIB


_lib = None


def load_oracle():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build_oracle()
    L = C.CDLL(_LIB)
    dp = C.POINTER(C.c_double)
    L.orc_create.restype = C.c_void_p
    L.orc_create.argtypes = [C.POINTER(_Cfg)]
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_set_state.restype = C.c_int
    L.orc_set_state.argtypes = [C.c_void_p, dp, dp, dp, dp]
    L.orc_get_state.argtypes = [C.c_void_p, dp, dp, dp, dp]
    L.orc_set_time.argtypes = [C.c_void_p, C.c_double, C.c_int64]
    L.orc_set_scalars.argtypes = [C.c_void_p, dp]
    L.orc_set_particles.argtypes = [C.c_void_p, dp, dp, dp]
    L.orc_get_particles.argtypes = [C.c_void_p, dp, dp]
    L.orc_particle_deposit.argtypes = [C.c_void_p, dp, dp]
    L.orc_particle_interp.argtypes = [C.c_void_p, dp, dp, C.c_long, dp]
    L.orc_get_scalars.argtypes = [C.c_void_p, dp]
    L.orc_dt.restype = C.c_double
    L.orc_dt.argtypes = [C.c_void_p]
    L.orc_step.restype = C.c_double
    L.orc_step.argtypes = [C.c_void_p, C.c_double]
    L.orc_diag_get.argtypes = [C.c_void_p, C.POINTER(_Diag)]
    L.orc_threads.restype = C.c_int
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_debug_array.restype = C.c_long
    L.orc_debug_array.argtypes = [C.c_void_p, C.c_int, dp]
    L.orc_padded_size.restype = C.c_long
    L.orc_padded_size.argtypes = [C.c_void_p]
    L.orc_fast_speed.restype = C.c_double
    L.orc_fast_speed.argtypes = [dp, C.c_double, C.c_double]
    L.orc_poisson_periodic.restype = None
    L.orc_poisson_periodic.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                       C.c_double, C.c_double, dp, dp]
    for nm in ("orc_hlld", "orc_hll", "orc_hllc"):
        getattr(L, nm).restype = C.c_int
        getattr(L, nm).argtypes = [dp, dp, C.c_double, C.c_double, dp]
    L.orc_phys_flux.argtypes = [dp, C.c_double, C.c_double, dp]
    L.orc_prim_to_cons.argtypes = [dp, C.c_double, C.c_double, dp]
    L.orc_minmod.restype = C.c_double
    L.orc_minmod.argtypes = [C.c_double, C.c_double]
    L.orc_recon.argtypes = [dp, C.c_int, C.c_double, dp, dp]
    L.orc_hlld_batch.argtypes = [C.c_long, dp, dp, dp, C.c_double, dp, C.POINTER(C.c_int32)]
    L.orc_bf16.restype = C.c_double
    L.orc_bf16.argtypes = [C.c_double]
    L.orc_mlp_forward.argtypes = [dp, C.c_int, C.c_long, dp, dp]
    L.orc_mlp_backward.argtypes = [dp, C.c_int, C.c_long, dp, dp, dp]
    L.orc_mlp_features.argtypes = [dp, C.c_double, dp]
    L.orc_mlp_out_to_flux.argtypes = [dp, C.c_double, dp, dp]
    L.orc_mlp_flux_to_out.argtypes = [dp, C.c_double, dp, dp]
    L.orc_set_mlp.restype = C.c_int
    L.orc_set_mlp.argtypes = [C.c_void_p, dp, C.c_double, C.c_double, C.c_double]
    L.orc_recon_batch.argtypes = [C.c_long, dp, C.c_int, C.c_double, dp, dp]
    _lib = L
    return L


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def face_shapes(cfg: OrcConfig):
    """Interior array shapes (z, y, x) of bx, by, bz; faces on a non-periodic
    axis have one extra entry along their normal."""
    ox = 0 if cfg.bc[0] == BC_PERIODIC else 1
    oy = 0 if cfg.bc[2] == BC_PERIODIC else 1
    oz = 0 if cfg.bc[4] == BC_PERIODIC else 1
    return ((cfg.nz, cfg.ny, cfg.nx + ox), (cfg.nz, cfg.ny + oy, cfg.nx),
            (cfg.nz + oz, cfg.ny, cfg.nx))


class Oracle:
    """One FP64 CPU grid.  State arrays are numpy FP64, interior only."""

    def __init__(self, cfg: OrcConfig):
        self.L = load_oracle()
        self.cfg = cfg
        self._c = cfg.to_c()
        self.h = self.L.orc_create(C.byref(self._c))
        if not self.h:
            raise ValueError("orc_create rejected the configuration")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.L.orc_destroy(h)
            self.h = None

    def set_state(self, cell5, bx, by, bz) -> int:
        c5, bx, by, bz = _f64(cell5), _f64(bx), _f64(by), _f64(bz)
        fs = face_shapes(self.cfg)
        assert c5.shape == (5, self.cfg.nz, self.cfg.ny, self.cfg.nx), c5.shape
        assert bx.shape == fs[0] and by.shape == fs[1] and bz.shape == fs[2]
        return self.L.orc_set_state(self.h, _ptr(c5), _ptr(bx), _ptr(by), _ptr(bz))

    def get_state(self):
        fs = face_shapes(self.cfg)
        c5 = np.empty((5, self.cfg.nz, self.cfg.ny, self.cfg.nx))
        bx, by, bz = (np.empty(s) for s in fs)
        self.L.orc_get_state(self.h, _ptr(c5), _ptr(bx), _ptr(by), _ptr(bz))
        return c5, bx, by, bz

    def set_particles(self, x, v, m):
        """Particles: x, v [3][npart], m [npart] (positions wrap into the box)."""
        n = self.cfg.npart
        x, v, m = _f64(x), _f64(v), _f64(m)
        assert x.shape == (3, n) and v.shape == (3, n) and m.shape == (n,)
        self.L.orc_set_particles(self.h, _ptr(x), _ptr(v), _ptr(m))

    def get_particles(self):
        n = self.cfg.npart
        x, v = np.empty((3, n)), np.empty((3, n))
        self.L.orc_get_particles(self.h, _ptr(x), _ptr(v))
        return x, v

    def particle_deposit(self, x):
        """Cloud-in-cell density [nz][ny][nx] of the particle masses at x [3][npart]."""
        x = _f64(x)
        assert x.shape == (3, self.cfg.npart)
        rho = np.empty((self.cfg.nz, self.cfg.ny, self.cfg.nx))
        self.L.orc_particle_deposit(self.h, _ptr(x), _ptr(rho))
        return rho

    def particle_interp(self, f, x):
        """Cloud-in-cell interpolation of the cell field f at positions x [3][n]."""
        f, x = _f64(f), _f64(x)
        assert f.shape == (self.cfg.nz, self.cfg.ny, self.cfg.nx) and x.shape[0] == 3
        out = np.empty(x.shape[1])
        self.L.orc_particle_interp(self.h, _ptr(f), _ptr(x), x.shape[1], _ptr(out))
        return out

    def set_scalars(self, rho_x):
        """Passive scalars rho X_s, shape (nscalar, nz, ny, nx)."""
        a = _f64(rho_x)
        assert a.shape == (self.cfg.nscalar, self.cfg.nz, self.cfg.ny, self.cfg.nx), a.shape
        self.L.orc_set_scalars(self.h, _ptr(a))

    def get_scalars(self):
        a = np.empty((self.cfg.nscalar, self.cfg.nz, self.cfg.ny, self.cfg.nx))
        self.L.orc_get_scalars(self.h, _ptr(a))
        return a

    def set_time(self, t: float, step: int = 0):
        self.L.orc_set_time(self.h, t, step)

    def dt(self) -> float:
        return self.L.orc_dt(self.h)

    def step(self, dt: float = 0.0) -> float:
        return self.L.orc_step(self.h, dt)

    def diag(self) -> dict:
        d = _Diag()
        self.L.orc_diag_get(self.h, C.byref(d))
        return {
            "t": d.t, "step": d.step, "mass": d.mass, "mom": tuple(d.mom),
            "energy": d.energy, "bsum": tuple(d.bsum), "divb_max": d.divb_max,
            "rho_min": d.rho_min, "p_min": d.p_min, "n_floor": d.n_floor,
            "n_hll_fallback": d.n_hll_fallback, "n_degenerate": d.n_degenerate,
            "n_mlp_faces": d.n_mlp_faces, "n_mlp_gated": d.n_mlp_gated,
        }

    def set_mlp(self, params, tau: float = 0.5, jump: float = 0.5, tau_flux: float = 0.0):
        """Enable (params: 6792 values) or disable (None) the learned
        correction of the corrector fluxes; clip tau_flux |F| +
        tau a_max |U_R - U_L| per component."""
        if params is None:
            self.L.orc_set_mlp(self.h, None, tau, jump, tau_flux)
            return
        p = _f64(params)
        assert p.shape == (MLP_NPARAM,)
        self.L.orc_set_mlp(self.h, _ptr(p), tau, jump, tau_flux)

    def debug_array(self, what: int) -> np.ndarray:
        """Padded array [nz+5][ny+5][nx+5] of the last corrector stage."""
        n = self.L.orc_padded_size(self.h)
        out = np.empty(n)
        r = self.L.orc_debug_array(self.h, what, _ptr(out))
        if r < 0:
            raise ValueError(what)
        c = self.cfg
        return out.reshape(c.nz + 5, c.ny + 5, c.nx + 5)


# ---- unit entry points ----------------------------------------------------

def hlld(wl, wr, bn: float, gamma: float):
    L = load_oracle()
    wl, wr = _f64(wl), _f64(wr)
    f = np.empty(7)
    code = L.orc_hlld(_ptr(wl), _ptr(wr), bn, gamma, _ptr(f))
    return f, code


def hll(wl, wr, bn: float, gamma: float):
    L = load_oracle()
    wl, wr = _f64(wl), _f64(wr)
    f = np.empty(7)
    L.orc_hll(_ptr(wl), _ptr(wr), bn, gamma, _ptr(f))
    return f


def hllc(wl, wr, bn: float, gamma: float):
    L = load_oracle()
    wl, wr = _f64(wl), _f64(wr)
    f = np.empty(7)
    L.orc_hllc(_ptr(wl), _ptr(wr), bn, gamma, _ptr(f))
    return f


def poisson_periodic(rho, d, G: float):
    """Psi of Lap Psi = 4 pi G (rho - <rho>) on the periodic box rho [nz][ny][nx]
    with the 7-point Laplacian (oracle)."""
    L = load_oracle()
    rho = _f64(rho)
    nz, ny, nx = rho.shape
    psi = np.empty_like(rho)
    L.orc_poisson_periodic(nx, ny, nz, float(d[0]), float(d[1]), float(d[2]), float(G), _ptr(rho),
                           _ptr(psi))
    return psi


def phys_flux(w, bn: float, gamma: float):
    L = load_oracle()
    w = _f64(w)
    f = np.empty(7)
    L.orc_phys_flux(_ptr(w), bn, gamma, _ptr(f))
    return f


def prim_to_cons(w, bn: float, gamma: float):
    L = load_oracle()
    w = _f64(w)
    u = np.empty(7)
    L.orc_prim_to_cons(_ptr(w), bn, gamma, _ptr(u))
    return u


def fast_speed(w, bn: float, gamma: float) -> float:
    L = load_oracle()
    return L.orc_fast_speed(_ptr(_f64(w)), bn, gamma)


def minmod(a: float, b: float) -> float:
    return load_oracle().orc_minmod(a, b)


def recon(w4, recon: int = RECON_PAPER, kappa: float = 1.0 / 3.0):
    L = load_oracle()
    w4 = _f64(w4)
    wl, wr = C.c_double(), C.c_double()
    L.orc_recon(_ptr(w4), recon, kappa, C.byref(wl), C.byref(wr))
    return wl.value, wr.value


def hlld_batch(wl, wr, bn, gamma: float):
    """Oracle HLLD over n faces: returns flux [n][7] and codes [n]."""
    L = load_oracle()
    wl, wr, bn = _f64(wl), _f64(wr), _f64(bn)
    n = bn.shape[0]
    f = np.empty((n, 7))
    code = np.empty(n, dtype=np.int32)
    L.orc_hlld_batch(n, _ptr(wl), _ptr(wr), _ptr(bn), gamma, _ptr(f),
                     code.ctypes.data_as(C.POINTER(C.c_int32)))
    return f, code


def recon_batch(w4, recon: int = RECON_PAPER, kappa: float = 1.0 / 3.0):
    L = load_oracle()
    w4 = _f64(w4)
    n = w4.shape[0]
    wl, wr = np.empty(n), np.empty(n)
    L.orc_recon_batch(n, _ptr(w4), recon, kappa, _ptr(wl), _ptr(wr))
    return wl, wr


# ---- learned correction -----------------------------------------------------

def bf16(x: float) -> float:
    return load_oracle().orc_bf16(float(x))


def mlp_forward(params, x, bf16_round: bool = False):
    L = load_oracle()
    p, x = _f64(params), _f64(x)
    n = x.shape[0]
    y = np.empty((n, 8))
    L.orc_mlp_forward(_ptr(p), 1 if bf16_round else 0, n, _ptr(x), _ptr(y))
    return y


def mlp_backward(params, x, dy, bf16_round: bool = False):
    L = load_oracle()
    p, x, dy = _f64(params), _f64(x), _f64(dy)
    g = np.empty(MLP_NPARAM)
    L.orc_mlp_backward(_ptr(p), 1 if bf16_round else 0, x.shape[0], _ptr(x), _ptr(dy), _ptr(g))
    return g


def mlp_features(w8, gamma):
    L = load_oracle()
    w8 = _f64(w8).reshape(32)
    x = np.empty(32)
    L.orc_mlp_features(_ptr(w8), gamma, _ptr(x))
    return x


def mlp_out_to_flux(w8, gamma, y):
    L = load_oracle()
    w8, y = _f64(w8).reshape(32), _f64(y)
    f = np.empty(7)
    L.orc_mlp_out_to_flux(_ptr(w8), gamma, _ptr(y), _ptr(f))
    return f


def mlp_flux_to_out(w8, gamma, df):
    L = load_oracle()
    w8, df = _f64(w8).reshape(32), _f64(df)
    y = np.empty(8)
    L.orc_mlp_flux_to_out(_ptr(w8), gamma, _ptr(df), _ptr(y))
    return y


def coarsen(cell5, bx, by, bz):
    """2x coarse-graining of a state: volume means of the cell fields over
    2^3 fine cells, area means of each face field over the 2^2 fine faces
    that tile a coarse face (plain definition, numpy).  A face array with n+1
    faces along its normal (non-periodic axis) keeps its boundary face."""
    c5 = np.asarray(cell5, dtype=np.float64)
    nz, ny, nx = c5.shape[1:]
    cc = c5.reshape(5, nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(2, 4, 6))
    bx = np.asarray(bx, dtype=np.float64)[:, :, 0::2]
    by = np.asarray(by, dtype=np.float64)[:, 0::2, :]
    bz = np.asarray(bz, dtype=np.float64)[0::2, :, :]
    bx = bx.reshape(nz // 2, 2, ny // 2, 2, bx.shape[2])
    by = by.reshape(nz // 2, 2, by.shape[1], nx // 2, 2)
    bz = bz.reshape(bz.shape[0], ny // 2, 2, nx // 2, 2)
    return cc, bx.mean(axis=(1, 3)), by.mean(axis=(1, 4)), bz.mean(axis=(2, 4))
