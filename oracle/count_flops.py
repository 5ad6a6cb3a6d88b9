"""Algorithmic flop counts of the step, measured on the oracle (test
infrastructure): every +, -, *, /, sqrt, exp the FP64 oracle executes is
tallied by libopcount.so (oracle/opcount.cpp).

Per face: MUSCL reconstruction of the 7 face variables (Eq. 12-14) plus the
HLLD solve, on the corrector face states of the turbulent-ISM box.
Per cell-update: one full step (both stages, all parts) divided by the cell
count, on n = 32 and n = 64 boxes, extrapolated as a + b/n to remove the
ghost-row overhead of a finite grid.

    python oracle/count_flops.py   -> prints a JSON object
"""
from __future__ import annotations

import ctypes as C
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle.pyorc import OrcConfig, _Cfg, build_opcount  # noqa: E402
from mhd_inputs import problems as P  # noqa: E402


def _lib():
    L = C.CDLL(build_opcount())
    dp = C.POINTER(C.c_double)
    L.opc_reset.argtypes = []
    L.opc_get.argtypes = [C.POINTER(C.c_longlong)]
    L.orc_create.restype = C.c_void_p
    L.orc_create.argtypes = [C.POINTER(_Cfg)]
    L.orc_set_state.argtypes = [C.c_void_p, dp, dp, dp, dp]
    L.orc_step.restype = C.c_double
    L.orc_step.argtypes = [C.c_void_p, C.c_double]
    L.orc_dt.restype = C.c_double
    L.orc_dt.argtypes = [C.c_void_p]
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_hlld_batch.argtypes = [C.c_long, dp, dp, dp, C.c_double, dp, C.POINTER(C.c_int32)]
    L.orc_recon_batch.argtypes = [C.c_long, dp, C.c_int, C.c_double, dp, dp]
    return L


def _tally(L):
    out = (C.c_longlong * 5)()
    L.opc_get(out)
    return dict(zip(("add", "mul", "div", "sqrt", "exp"), [int(x) for x in out]))


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def per_step(L, n, steps=2):
    pb = P.turbulent_ism(n, seed=1)
    cfg = OrcConfig(nx=n, ny=n, nz=n, dx=pb.dx, dy=pb.dy, dz=pb.dz, gamma=pb.gamma, cfl=pb.cfl,
                    bc=pb.bc).to_c()
    h = L.orc_create(C.byref(cfg))
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (pb.cell5, pb.bx, pb.by, pb.bz)]
    L.orc_set_state(h, *[_p(a) for a in arrs])
    dts = [L.orc_dt(h)]
    L.opc_reset()
    for _ in range(steps):
        L.orc_step(h, dts[0])
    t = _tally(L)
    L.orc_destroy(h)
    tot = sum(t.values())
    return tot / (steps * n ** 3), t


def face_states(n=32, seed=1):
    """Corrector-like face states (x-faces) of the turbulent box: primitives
    of the initial state, 4-cell stencils along x."""
    pb = P.turbulent_ism(n, seed=seed)
    rho = pb.cell5[0]
    v = pb.cell5[1:4] / rho
    bc = [0.5 * (pb.bx + np.roll(pb.bx, -1, 2)), 0.5 * (pb.by + np.roll(pb.by, -1, 1)),
          0.5 * (pb.bz + np.roll(pb.bz, -1, 0))]
    Pr = (pb.gamma - 1) * (pb.cell5[4] - 0.5 * rho * (v ** 2).sum(0) - 0.5 * sum(b * b for b in bc))
    w = [rho, v[0], v[1], v[2], Pr, bc[1], bc[2]]
    st = np.stack([np.stack([np.roll(q, s, 2) for s in (2, 1, 0, -1)], -1).reshape(-1, 4)
                   for q in w])  # [7][faces][4]
    bn = pb.bx.reshape(-1)
    return st, bn, pb.gamma


def per_face(L):
    st, bn, g = face_states()
    m = bn.shape[0]
    wl = np.empty((7, m))
    wr = np.empty((7, m))
    L.opc_reset()
    for v in range(7):
        s = np.ascontiguousarray(st[v])
        L.orc_recon_batch(m, _p(s), 0, 1.0 / 3.0, _p(wl[v]), _p(wr[v]))
    rec = _tally(L)
    wlT = np.ascontiguousarray(wl.T)
    wrT = np.ascontiguousarray(wr.T)
    f = np.empty((m, 7))
    code = np.empty(m, dtype=np.int32)
    L.opc_reset()
    L.orc_hlld_batch(m, _p(wlT), _p(wrT), _p(np.ascontiguousarray(bn)), g, _p(f),
                     code.ctypes.data_as(C.POINTER(C.c_int32)))
    hl = _tally(L)
    return sum(rec.values()) / m, sum(hl.values()) / m, rec, hl


def main():
    L = _lib()
    rec, hl, rect, hlt = per_face(L)
    f32, t32 = per_step(L, 32)
    f64, t64 = per_step(L, 64)
    a = 2.0 * f64 - f32  # a + b/n through n = 32, 64
    out = {
        "flops_per_face_muscl7": rec,
        "flops_per_face_hlld": hl,
        "flops_per_face_first_order": hl,
        "flops_per_face_corrector": rec + hl,
        "flops_per_cell_update_n32": f32,
        "flops_per_cell_update_n64": f64,
        "flops_per_cell_update": a,
        "hlld_op_mix_per_face": {k: v / 32 ** 3 for k, v in hlt.items()},
        "step_op_mix_n64": t64,
    }
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
