"""Sub-boxes of a periodic problem, for sampled parity at full size: the
oracle advances a small box cut out around a sample point (outflow sides),
and only cells and faces far enough from its sides to be untouched by the
wrong ghost data are compared.  Host-side index work only."""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from mhd_inputs import problems as P


def cut(pb, lo, m):
    """The m^3 box of cells lo .. lo + m - 1 (periodic wrap) of a periodic
    problem, with m + 1 faces along each face array's normal, outflow on
    every side."""
    iz, iy, ix = (np.arange(lo[a], lo[a] + m) % n for a, n in ((2, pb.nz), (1, pb.ny), (0, pb.nx)))
    fz, fy, fx = (np.arange(lo[a], lo[a] + m + 1) % n
                  for a, n in ((2, pb.nz), (1, pb.ny), (0, pb.nx)))
    c5 = pb.cell5[:, iz][:, :, iy][:, :, :, ix]
    bx = pb.bx[iz][:, iy][:, :, fx]
    by = pb.by[iz][:, fy][:, :, ix]
    bz = pb.bz[fz][:, iy][:, :, ix]
    return replace(pb, name=pb.name + "_cut", nx=m, ny=m, nz=m, bc=(P.OUTFLOW,) * 6,
                   cell5=np.ascontiguousarray(c5), bx=np.ascontiguousarray(bx),
                   by=np.ascontiguousarray(by), bz=np.ascontiguousarray(bz))


def core(state, lo, m, margin, full=None):
    """Cells and faces of the box core (margin cells in from every side):
    from a sub-box state (full=None) or, at the same global positions, from
    a periodic full-size state (full = (nx, ny, nz))."""
    c5, bx, by, bz = state
    k = np.arange(margin, m - margin)
    if full is None:
        ix = iy = iz = k
    else:
        ix, iy, iz = ((lo[a] + k) % full[a] for a in range(3))
    return (c5[:, iz][:, :, iy][:, :, :, ix], bx[iz][:, iy][:, :, ix],
            by[iz][:, iy][:, :, ix], bz[iz][:, iy][:, :, ix])
