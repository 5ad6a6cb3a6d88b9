"""Test glue: build oracle grids from the shared input generators."""
from __future__ import annotations

import numpy as np

from oracle.pyorc import Oracle, OrcConfig


def orc_config(pb, recon=0, kappa=1.0 / 3.0, cfl=None, riemann=0) -> OrcConfig:
    return OrcConfig(nx=pb.nx, ny=pb.ny, nz=pb.nz, dx=pb.dx, dy=pb.dy, dz=pb.dz,
                     x0=pb.x0, y0=pb.y0, z0=pb.z0, gamma=pb.gamma,
                     cfl=pb.cfl if cfl is None else cfl, bc=pb.bc, recon=recon, kappa=kappa,
                     source=pb.source, src=pb.src, rho_floor=pb.rho_floor, p_floor=pb.p_floor,
                     inflow=pb.inflow, riemann=riemann)


def oracle_of(pb, **kw) -> Oracle:
    o = Oracle(orc_config(pb, **kw))
    rc = o.set_state(pb.cell5, pb.bx, pb.by, pb.bz)
    assert rc == 0, rc
    return o


def run_to(o: Oracle, t_end: float, max_steps: int = 100000):
    """Advance with CFL steps, shortening the last one to land on t_end."""
    t = o.diag()["t"]
    n = 0
    while t < t_end * (1 - 1e-14) and n < max_steps:
        dt = o.dt()
        if t + dt > t_end:
            dt = t_end - t
        o.step(dt)
        t += dt
        n += 1
    return n


def prim_1d(o: Oracle, axis: int = 0):
    """rho, vn, vt1, vt2, P, Bn(cell), Bt1, Bt2 along the problem axis of a
    one-dimensional problem (cell centres), in the axis' cyclic frame."""
    c5, bx, by, bz = o.get_state()
    g = o.cfg.gamma
    rho = c5[0].reshape(-1)
    M = [c5[1 + d].reshape(-1) for d in range(3)]
    E = c5[4].reshape(-1)
    faces = [bx, by, bz]
    bcc = []
    for d in range(3):
        f = faces[d]
        if d == axis:
            f1 = f.reshape(-1)
            bcc.append(0.5 * (f1[:-1] + f1[1:]))
        else:
            bcc.append(f.reshape(-1))
    v = [m / rho for m in M]
    P = (g - 1.0) * (E - 0.5 * (M[0] ** 2 + M[1] ** 2 + M[2] ** 2) / rho
                     - 0.5 * (bcc[0] ** 2 + bcc[1] ** 2 + bcc[2] ** 2))
    t1, t2 = (axis + 1) % 3, (axis + 2) % 3
    return dict(rho=rho, vn=v[axis], vt1=v[t1], vt2=v[t2], P=P, bn=bcc[axis], bt1=bcc[t1],
                bt2=bcc[t2])
