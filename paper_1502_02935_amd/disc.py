"""Galactic-disc slab workloads of the step (the paper's section 4 disc, as a
synthetic Cartesian slab: exponential, sech^2 gas disc in a logarithmic
potential, toroidal field, outflow sides).

    python -m paper_1502_02935_amd.disc precision [--nx 512 --ny 512 --nz 128 --steps 200]
    python -m paper_1502_02935_amd.disc large     [--nx 1024 --ny 1024 --nz 256 --steps 100]

precision: FP32 bulk against the FP64 path from one FP32-rounded state with
the FP64 run's time steps (L1 and Linf per field), plus the throughput of
both precisions with their own device CFL steps.  large: throughput of the
FP32 path on the largest one-GPU machine (same profiles on a 48 x 48 x 12 kpc
box, so the cell size is that of the 512 x 512 x 128 slab).
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


def _log(*m):
    print(*m, file=sys.stderr, flush=True)


def _problem(nx, ny, nz, seed):
    from mhd_inputs import problems as P
    scale = nx / 512.0
    t0 = time.perf_counter()
    pb = P.disc(nx, ny, nz, lx=24.0 * scale, ly=24.0 * scale, lz=6.0 * scale, seed=seed)
    pb = pb.astype("float32")
    _log("disc %dx%dx%d generated in %.1f s" % (nx, ny, nz, time.perf_counter() - t0))
    return pb


def throughput(pb, precision, steps, warmup=2):
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
    sim.close()
    return {"cell_updates_per_s": pb.ncell * steps / el, "ms_per_step": 1e3 * el / steps,
            "steps": steps, "status": d["status"], "n_floor": d["n_floor"],
            "n_fp64_recovery": d["n_fp64_recovery"], "n_hll_fallback": d["n_hll_fallback"],
            "n_degenerate": d["n_degenerate"],
            "kernel_ms_per_launch": {k: v[0] / v[1] for k, v in prof.items() if v[1]}}


def _errors(a, b):
    """L1 and Linf of state b against state a per field (momentum and face-B
    components relative to their own mean / max magnitude)."""
    names = ("rho", "Mx", "My", "Mz", "E")
    out = {}
    for m in range(5):
        r = a[0][m]
        e = b[0][m].double() - r
        out[names[m]] = {"L1_rel": float(e.abs().mean() / r.abs().mean()),
                         "Linf_rel": float(e.abs().max() / r.abs().max())}
    for q, nm in enumerate(("Bx", "By", "Bz")):
        r = a[1 + q]
        e = b[1 + q].double() - r
        out[nm] = {"L1_rel": float(e.abs().mean() / max(float(r.abs().mean()), 1e-300)),
                   "Linf_rel": float(e.abs().max() / max(float(r.abs().max()), 1e-300))}
    return out


def precision(nx, ny, nz, steps, seed=1):
    pb = _problem(nx, ny, nz, seed)
    res = {"workload": "disc slab %dx%dx%d, %g x %g x %g kpc, outflow, log-potential source, "
                       "floors on; FP32-rounded initial state" % (
                           nx, ny, nz, pb.nx * pb.dx, pb.ny * pb.dy, pb.nz * pb.dz),
           "cells": pb.ncell, "steps": steps}
    _log("FP32 throughput")
    res["fp32"] = throughput(pb, L.MHD_FP32, steps)
    _log("  %.3f ms/step" % res["fp32"]["ms_per_step"])
    _log("FP64 throughput")
    res["fp64"] = throughput(pb, L.MHD_FP64, steps)
    _log("  %.3f ms/step" % res["fp64"]["ms_per_step"])
    _log("error run: FP64 with its CFL steps, FP32 forced to them")
    s64 = Sim(config_from_problem(pb, precision=L.MHD_FP64), pb.cell5, pb.bx, pb.by, pb.bz)
    dts = []
    for i in range(steps):
        dts.append(s64.dt())
        s64.step(1, dt=dts[-1])
        if (i + 1) % 50 == 0:
            _log("  FP64 step %d" % (i + 1))
    a = s64.get_state()
    d64 = s64.diag(check=False)
    s64.close()
    del s64
    s32 = Sim(config_from_problem(pb, precision=L.MHD_FP32), pb.cell5, pb.bx, pb.by, pb.bz)
    s32.step(steps, dt=dts)
    b = s32.get_state()
    d32 = s32.diag(check=False)
    s32.close()
    res["error_fp32_vs_fp64"] = _errors(a, b)
    res["error_run"] = {"t_end_kpc_per_kms": float(np.sum(dts)),
                        "t_end_myr": float(np.sum(dts)) * 977.8,
                        "status_fp64": d64["status"], "status_fp32": d32["status"],
                        "floor_hits_fp64": d64["n_floor"], "floor_hits_fp32": d32["n_floor"],
                        "fp64_recovery_cell_evals": d32["n_fp64_recovery"],
                        "mass_fp64": d64["mass"], "mass_fp32": d32["mass"]}
    return res


def large(nx, ny, nz, steps, seed=1):
    pb = _problem(nx, ny, nz, seed)
    res = {"workload": "disc slab %dx%dx%d, %g x %g x %g kpc, FP32" % (
        nx, ny, nz, pb.nx * pb.dx, pb.ny * pb.dy, pb.nz * pb.dz), "cells": pb.ncell}
    _log("FP32 throughput, %d steps" % steps)
    res["fp32"] = throughput(pb, L.MHD_FP32, steps)
    _log("  %.3f ms/step" % res["fp32"]["ms_per_step"])
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("mode", choices=("precision", "large"))
    ap.add_argument("--nx", type=int, default=None)
    ap.add_argument("--ny", type=int, default=None)
    ap.add_argument("--nz", type=int, default=None)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--seed", type=int, default=1)
    a = ap.parse_args(argv)
    if a.mode == "precision":
        r = precision(a.nx or 512, a.ny or 512, a.nz or 128, a.steps or 200, a.seed)
    else:
        r = large(a.nx or 1024, a.ny or 1024, a.nz or 256, a.steps or 100, a.seed)
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
