"""ctypes binding of libmhd.so (C ABI in include/mhd.h).

Argument marshalling only: every step of the method runs in the HIP kernels.
PyTorch provides device memory and the stream.  There is no fallback: if the
library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmhd.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "mhd.h")

MHD_OK, MHD_E_ARG, MHD_E_HIP, MHD_E_STATE, MHD_E_UNSUPPORTED, MHD_E_WS = 0, -1, -2, -3, -4, -5
MHD_FP64, MHD_FP32, MHD_FP32_COMP = 0, 1, 2
RECOVERY_FP64, RECOVERY_OFF = 0, 1
BC_PERIODIC, BC_OUTFLOW, BC_INFLOW = 0, 1, 2
RECON_PAPER, RECON_KAPPA, RECON_FIRST = 0, 1, 2
RIEMANN_HLLD, RIEMANN_HLL, RIEMANN_HLLC = 0, 1, 2
SRC_NONE, SRC_LOGPOT, SRC_UNIFORM, SRC_GAUSS_X, SRC_SELF_GRAVITY = 0, 1, 2, 3, 4


class mhd_config(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("precision", C.c_int32),
        ("bc", C.c_int32 * 6),
        ("x0", C.c_double), ("y0", C.c_double), ("z0", C.c_double),
        ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
        ("gamma", C.c_double), ("cfl", C.c_double),
        ("recon", C.c_int32), ("source", C.c_int32),
        ("kappa", C.c_double),
        ("src", C.c_double * 4),
        ("rho_floor", C.c_double), ("p_floor", C.c_double),
        ("inflow", C.c_double * 8),
        ("riemann", C.c_int32),
        ("nscalar", C.c_int32),
        ("recovery", C.c_int32),
        ("reserved", C.c_int32),
        ("npart", C.c_int64),
    ]


class mhd_diag_t(C.Structure):
    _fields_ = [
        ("t", C.c_double), ("step", C.c_int64), ("dt", C.c_double),
        ("mass", C.c_double), ("mom", C.c_double * 3), ("energy", C.c_double),
        ("bsum", C.c_double * 3), ("divb_max", C.c_double),
        ("rho_min", C.c_double), ("p_min", C.c_double),
        ("n_floor", C.c_int64), ("n_hll_fallback", C.c_int64),
        ("n_degenerate", C.c_int64), ("n_fp64_recovery", C.c_int64),
        ("n_mlp_faces", C.c_int64), ("n_mlp_gated", C.c_int64),
        ("status", C.c_uint32), ("pad", C.c_uint32),
    ]


MLP_NPARAM = 6792
MLP_NOALLOC_MAX = 32768


class mhd_gate(C.Structure):
    _fields_ = [("tau", C.c_double), ("jump", C.c_double), ("tau_flux", C.c_double)]


class mhd_profile_t(C.Structure):
    _fields_ = [("ms", C.c_double * 16), ("launches", C.c_int64 * 16),
                ("n_kinds", C.c_int32), ("pad", C.c_int32)]


KERNEL_KINDS = ("ghosts", "prim", "flux", "flux_mlp", "shock", "emf", "update", "cfl", "other",
                "gravity", "scalars", "nbody", "flux_outer")
MAX_SCALARS = 8


class MHDError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (where, strerror(code), code))


_lib = None


def load() -> C.CDLL:
    """Load libmhd.so (built by paper_1502_02935_amd.build).  Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmhd.so is not built (%s); run __graft_entry__.build() or "
                          "python paper_1502_02935_amd/build.py" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    vp, i64, sz = C.c_void_p, C.c_int64, C.c_size_t
    L.mhd_abi_version.restype = C.c_int
    L.mhd_abi_version.argtypes = []
    L.mhd_strerror.restype = C.c_char_p
    L.mhd_strerror.argtypes = [C.c_int]
    L.mhd_workspace_bytes.restype = C.c_int
    L.mhd_workspace_bytes.argtypes = [C.POINTER(mhd_config), C.POINTER(sz)]
    L.mhd_init.restype = C.c_int
    L.mhd_init.argtypes = [C.POINTER(mhd_config), vp, sz, vp, vp, vp, vp, vp, C.POINTER(vp)]
    L.mhd_step.restype = C.c_int
    L.mhd_step.argtypes = [vp, C.POINTER(C.c_double), C.c_int]
    L.mhd_dt.restype = C.c_int
    L.mhd_dt.argtypes = [vp, C.POINTER(C.c_double)]
    L.mhd_diag.restype = C.c_int
    L.mhd_diag.argtypes = [vp, C.POINTER(mhd_diag_t)]
    L.mhd_get_state.restype = C.c_int
    L.mhd_get_state.argtypes = [vp, vp, vp, vp, vp]
    L.mhd_set_particles.restype = C.c_int
    L.mhd_set_particles.argtypes = [vp, vp, vp, vp]
    L.mhd_get_particles.restype = C.c_int
    L.mhd_get_particles.argtypes = [vp, vp, vp]
    L.mhd_set_scalars.restype = C.c_int
    L.mhd_set_scalars.argtypes = [vp, vp]
    L.mhd_get_scalars.restype = C.c_int
    L.mhd_get_scalars.argtypes = [vp, vp]
    L.mhd_debug_array.restype = C.c_int
    L.mhd_debug_array.argtypes = [vp, C.c_int, vp, C.POINTER(sz)]
    L.mhd_profile.restype = C.c_int
    L.mhd_profile.argtypes = [vp, C.c_int]
    L.mhd_profile_get.restype = C.c_int
    L.mhd_profile_get.argtypes = [vp, C.POINTER(mhd_profile_t)]
    L.mhd_set_mlp.restype = C.c_int
    L.mhd_set_mlp.argtypes = [vp, vp, C.POINTER(mhd_gate)]
    L.mhd_flux_accumulate.restype = C.c_int
    L.mhd_flux_accumulate.argtypes = [vp, vp]
    L.mhd_coarsen.restype = C.c_int
    L.mhd_coarsen.argtypes = [vp, vp, vp, vp, vp]
    L.mhd_set_full_fluxes.restype = C.c_int
    L.mhd_set_full_fluxes.argtypes = [vp, C.c_int]
    L.mhd_mlp_samples.restype = C.c_int
    L.mhd_mlp_samples.argtypes = [vp, vp, C.c_double, i64, vp, vp, vp, vp]
    L.mhd_mlp_forward.restype = C.c_int
    L.mhd_mlp_forward.argtypes = [i64, vp, vp, vp, vp]
    L.mhd_mlp_grad_workspace_bytes.restype = C.c_int
    L.mhd_mlp_grad_workspace_bytes.argtypes = [i64, C.POINTER(sz)]
    L.mhd_mlp_grad.restype = C.c_int
    L.mhd_mlp_grad.argtypes = [i64, vp, vp, vp, vp, vp, vp, sz, vp]
    L.mhd_mlp_grad_noalloc.restype = C.c_int
    L.mhd_mlp_grad_noalloc.argtypes = [i64, vp, vp, vp, vp, vp, vp]
    L.mhd_mlp_adam.restype = C.c_int
    L.mhd_mlp_adam.argtypes = [vp, vp, vp, vp, i64, C.c_double, C.c_double, C.c_double,
                               C.c_double, vp]
    L.mhd_destroy.restype = C.c_int
    L.mhd_destroy.argtypes = [vp]
    L.mhd_hlld_batch.restype = C.c_int
    L.mhd_hlld_batch.argtypes = [C.c_int, i64, vp, vp, vp, C.c_double, vp, vp, vp]
    L.mhd_recon_batch.restype = C.c_int
    L.mhd_recon_batch.argtypes = [C.c_int, i64, vp, C.c_int, C.c_double, vp, vp, vp]
    _lib = L
    return L


def strerror(code: int) -> str:
    return load().mhd_strerror(code).decode()


def declared_symbols() -> list:
    """Function names declared in include/mhd.h."""
    with open(HEADER) as f:
        txt = f.read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mhd_[a-z_0-9]+)\s*\(", txt)))


def check(code: int, where: str) -> None:
    if code != MHD_OK:
        raise MHDError(code, where)
