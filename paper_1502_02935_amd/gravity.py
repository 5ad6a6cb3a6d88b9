"""Self-gravity workloads (the paper's Poisson equation with the FFT solver,
section 2.1; spherical-collapse test, section 3).

    python -m paper_1502_02935_amd.gravity collapse   [--n 128 --t-end 1.0]
    python -m paper_1502_02935_amd.gravity throughput [--n 256 --steps 20]

collapse: the 1/r gas sphere on [-1, 1]^3 collapsing under its own gravity
(FP32 bulk, HLLC gas solver); reports the central density, the kinetic and
gravitational energies along the run, and radial profiles of density,
pressure and radial velocity at the start and the end.  throughput: the
turbulent-ISM box with self-gravity switched on: step time, the Poisson
solve's share and its FFT passes' algorithmic bytes against HBM peak.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import _lib as L
from .sim import Sim, config_from_problem

PEAK_HBM_GBS = 8000.0


def _log(*m):
    print(*m, file=sys.stderr, flush=True)


def _profiles(pb, state, nbins=32):
    """Radial profiles (cell-count means in shells) of rho, P and v_r."""
    c5 = state[0].double().cpu().numpy()
    n = pb.nx
    c = pb.x0 + (np.arange(n) + 0.5) * pb.dx
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    rho = c5[0]
    v = [c5[1 + a] / rho for a in range(3)]
    vr = (v[0] * X + v[1] * Y + v[2] * Z) / np.maximum(r, 1e-300)
    ke = 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    P = (pb.gamma - 1.0) * (c5[4] - ke)  # B = 0
    edges = np.linspace(0.0, 1.2, nbins + 1)
    idx = np.digitize(r.ravel(), edges) - 1
    out = {"r": (0.5 * (edges[1:] + edges[:-1])).tolist()}
    for nm, f in (("rho", rho), ("P", P), ("v_r", vr)):
        s = np.bincount(idx, weights=f.ravel(), minlength=nbins + 2)[:nbins]
        cnt = np.bincount(idx, minlength=nbins + 2)[:nbins]
        out[nm] = (s / np.maximum(cnt, 1)).tolist()
    return out


def _energies(pb, sim):
    """Kinetic, thermal and gravitational (1/2 sum rho Psi dV) energies."""
    c5 = sim.get_state()[0].double()
    dv = pb.dx * pb.dy * pb.dz
    rho = c5[0]
    ke = 0.5 * (c5[1] ** 2 + c5[2] ** 2 + c5[3] ** 2) / rho
    th = c5[4] - ke
    psi = sim.debug_array(35).double()[2:2 + pb.nz, 2:2 + pb.ny, 2:2 + pb.nx]
    return {"kinetic": float(ke.sum() * dv), "thermal": float(th.sum() * dv),
            "gravitational": float(0.5 * (rho * psi).sum() * dv)}


def collapse(n, t_end, precision=L.MHD_FP32):
    from mhd_inputs import problems as P
    pb = P.collapse(n)
    cfg = config_from_problem(pb, precision=precision, riemann=L.RIEMANN_HLLC)
    sim = Sim(cfg, pb.cell5, pb.bx, pb.by, pb.bz)
    res = {"workload": "collapse of a 1/r gas sphere (M = R = G = 1, u = 0.05, gamma 5/3), "
                       "periodic [-1,1]^3 at %d^3, self-gravity by FFT, HLLC" % n,
           "profile_t0": _profiles(pb, sim.get_state())}
    sim.step(1)  # one step so the potential of the initial state exists
    hist = []
    t, steps = float(sim.diag()["t"]), 1
    mark = 0.1
    t0 = time.perf_counter()
    while t < t_end * (1 - 1e-12):
        dt = min(sim.dt(), t_end - t)
        sim.step(1, dt=dt)
        t += dt
        steps += 1
        if t >= mark - 1e-12 or t >= t_end * (1 - 1e-12):
            d = sim.diag(check=False)
            e = _energies(pb, sim)
            hist.append({"t": t, "steps": steps, "rho_max": float(sim.get_state()[0][0].max()),
                         "status": d["status"], "mass": d["mass"], **e})
            _log("t %.2f  steps %d  rho_max %.3g  E_kin %.4f  W %.4f" % (
                t, steps, hist[-1]["rho_max"], e["kinetic"], e["gravitational"]))
            mark += 0.1
    el = time.perf_counter() - t0
    res["history"] = hist
    res["profile_t_end"] = _profiles(pb, sim.get_state())
    res["steps"] = steps
    res["wall_seconds"] = el
    res["cell_updates_per_s_incl_host_dt"] = n ** 3 * steps / el
    sim.close()
    return res


def throughput(n, steps, warmup=2, G=1.0, precision=L.MHD_FP32):
    from mhd_inputs import problems as P
    pb = P.turbulent_ism(n, seed=1).astype("float32")
    out = {}
    for name, src in (("plain", None), ("self_gravity", (G, 0.0, 0.0, 0.0))):
        if src is not None:
            pb.source, pb.src = P.SRC_SELF_GRAVITY, src
        sim = Sim(config_from_problem(pb, precision=precision), pb.cell5, pb.bx, pb.by, pb.bz)
        sim.step(warmup)
        torch.cuda.synchronize()
        sim.profile(True)
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = sim.profile_get()
        sim.profile(False)
        d = sim.diag(check=False)
        out[name] = {"ms_per_step": 1e3 * el / steps, "cell_updates_per_s": pb.ncell * steps / el,
                     "status": d["status"],
                     "kernel_ms_per_launch": {k: v[0] / v[1] for k, v in prof.items() if v[1]}}
        sim.close()
    es = 4 if precision == L.MHD_FP32 else 8
    N = n ** 3
    # algorithmic bytes of one Poisson solve: density in, complex array out;
    # six FFT passes and the k-space division each read and write the
    # complex array; the gradient reads it and writes Psi and 3 components
    byts = N * es + 2 * N * es + 6 * 2 * (2 * N * es) + 2 * (2 * N * es) + 2 * N * es + 4 * N * es
    ms = out["self_gravity"]["kernel_ms_per_launch"]["gravity"]
    out["poisson_solve"] = {"ms": ms, "algorithmic_bytes": byts,
                            "achieved_GBps": byts / (ms * 1e-3) / 1e9,
                            "frac_of_hbm_peak": byts / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    out["workload"] = "turbulent-ISM box %d^3 (seed 1), FP32, self-gravity G = %g vs none" % (n, G)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("mode", choices=("collapse", "throughput"))
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--t-end", type=float, default=1.0)
    ap.add_argument("--steps", type=int, default=20)
    a = ap.parse_args(argv)
    if a.mode == "collapse":
        r = collapse(a.n or 128, a.t_end)
    else:
        r = throughput(a.n or 256, a.steps)
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
