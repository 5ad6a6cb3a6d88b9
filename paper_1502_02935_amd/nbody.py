"""N-body workloads of the step (the paper's particle-in-cell dynamics with
the flip-flop integrator, section 2.1), sharing the FFT potential with the
gas.

    python -m paper_1502_02935_amd.nbody throughput [--n 256 --steps 20 --counts 0 4194304 16777216]
    python -m paper_1502_02935_amd.nbody plummer    [--n 128 --npart 1048576 --t-end 2.0]

throughput: the turbulent-ISM box (FP32, self-gravity G = 1, gas coupled)
with a Plummer sphere of N particles: step time, the kernel classes'
shares, particle-updates/s and the particle passes' algorithmic bytes.
plummer: an isolated Plummer sphere (gas decoupled, FP32) run for a few
crossing times: total energy (kinetic plus the mesh potential energy) and
the radii holding 10, 50 and 90 % of the mass.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import _lib as L
from .sim import Sim, config_from_problem

PEAK_HBM_GBS = 8000.0


def _log(*m):
    print(*m, file=sys.stderr, flush=True)


def particle_bytes(npart: int, es: int) -> int:
    """Algorithmic bytes of the particle passes of one step: the predictor's
    deposit reads x and m, the corrector's x, v and m; the kick-drift reads
    and writes x and v; the CFL pass reads v.  (The 8 cells a particle
    touches are counted with the Poisson solve's complex array.)"""
    return npart * es * (4 + 7 + 12 + 3)


def throughput(n, steps, counts, warmup=2, precision=L.MHD_FP32):
    from mhd_inputs import problems as P
    pb = P.turbulent_ism(n, seed=1).astype("float32")
    pb.source, pb.src = P.SRC_SELF_GRAVITY, (1.0, 0.0, 0.0, 0.0)
    es = 4 if precision == L.MHD_FP32 else 8
    out = {"workload": "turbulent-ISM box %d^3 (seed 1), FP32, self-gravity G = 1 (gas "
                       "coupled), Plummer sphere (scale 0.1, mass 1) of N particles" % n}
    for npart in counts:
        sim = Sim(config_from_problem(pb, precision=precision, npart=npart), pb.cell5, pb.bx,
                  pb.by, pb.bz)
        if npart:
            x, v, m = P.particles_plummer(pb, npart, seed=2, scale=0.1, mass_total=1.0, G=1.0)
            sim.set_particles(x, v, m)
            del x, v, m
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
        r = {"ms_per_step": 1e3 * el / steps, "cell_updates_per_s": pb.ncell * steps / el,
             "status": d["status"],
             "kernel_ms_per_step": {k: v[0] / steps for k, v in prof.items() if v[1]}}
        if npart:
            ms_nb = prof["nbody"][0] / steps
            r["particle_updates_per_s"] = npart * steps / el
            r["kick_drift_ms"] = ms_nb
            r["particle_algorithmic_bytes_per_step"] = particle_bytes(npart, es)
        out["npart_%d" % npart] = r
        _log("N %d: %.3f ms/step" % (npart, r["ms_per_step"]))
        sim.close()
        torch.cuda.empty_cache()
    return out


def _energy_and_radii(sim, pb, m, G):
    """Kinetic energy, the mesh potential energy and the 10/50/90 % mass
    radii about the centre of mass.  The potential energy 1/2 sum rho Psi dV
    is taken in its field form, -1/(8 pi G) sum |D+ Psi|^2 dV (summation by
    parts with the 7-point Laplacian of the solve; Psi of the last corrector
    stage, i.e. of the half-step positions)."""
    x, v = (t.double() for t in sim.get_particles())
    mm = torch.as_tensor(m, dtype=torch.float64, device=x.device)
    kin = float(0.5 * (mm * (v * v).sum(dim=0)).sum())
    n = pb.nx
    psi = sim.debug_array(35).double()[2:2 + n, 2:2 + n, 2:2 + n]
    grad2 = sum(((torch.roll(psi, -1, dims=ax) - psi) / h) ** 2
                for ax, h in ((2, pb.dx), (1, pb.dy), (0, pb.dz)))
    w = -float(grad2.sum()) * pb.dx * pb.dy * pb.dz / (8.0 * math.pi * G)
    xs = x.cpu().numpy()
    c = xs.mean(axis=1, keepdims=True)
    r = np.sqrt(((xs - c) ** 2).sum(axis=0))
    q = np.quantile(r, [0.1, 0.5, 0.9])
    return kin, w, q.tolist()


def plummer(n, npart, t_end, G=1.0, precision=L.MHD_FP32):
    from mhd_inputs import problems as P
    pb = P.gravity_box((n, n, n), G=G)
    x, v, m = P.particles_plummer(pb, npart, seed=3, scale=0.08, mass_total=1.0, G=G)
    sim = Sim(config_from_problem(pb, precision=precision, npart=npart), pb.cell5, pb.bx, pb.by,
              pb.bz)
    sim.set_particles(x, v, m)
    hist = []
    t, steps, mark = 0.0, 0, 0.0
    t0 = time.perf_counter()
    while t < t_end * (1 - 1e-12):
        dt = min(sim.dt(), t_end - t)
        sim.step(1, dt=dt)
        t += dt
        steps += 1
        if t >= mark - 1e-12 or t >= t_end * (1 - 1e-12):
            k, w, q = _energy_and_radii(sim, pb, m, G)
            hist.append({"t": t, "steps": steps, "kinetic": k, "potential": w, "total": k + w,
                         "r10_r50_r90": q})
            _log("t %.2f steps %d  E %.5f  r50 %.4f" % (t, steps, k + w, q[1]))
            mark += 0.25
    el = time.perf_counter() - t0
    sim.close()
    e0 = hist[0]["total"]
    return {"workload": "isolated Plummer sphere (scale 0.08, mass 1, G = 1, %d particles) in a "
                        "%d^3 periodic box, gas decoupled, FP32" % (npart, n),
            "history": hist, "steps": steps, "wall_seconds": el,
            "energy_drift_rel": (hist[-1]["total"] - e0) / abs(e0)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("mode", choices=("throughput", "plummer"))
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--counts", type=int, nargs="+", default=[0, 1 << 22, 1 << 24])
    ap.add_argument("--npart", type=int, default=1 << 20)
    ap.add_argument("--t-end", type=float, default=2.0)
    a = ap.parse_args(argv)
    if a.mode == "throughput":
        r = throughput(a.n or 256, a.steps, a.counts)
    else:
        r = plummer(a.n or 128, a.npart, a.t_end)
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
