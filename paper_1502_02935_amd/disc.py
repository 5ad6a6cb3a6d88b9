"""Galactic-disc slab workloads of the step (the paper's section 4 disc, as a
synthetic Cartesian slab: exponential, sech^2 gas disc in a logarithmic
potential, toroidal field, outflow sides).

    python -m paper_1502_02935_amd.disc precision [--nx 512 --ny 512 --nz 128 --steps 200]
    python -m paper_1502_02935_amd.disc large     [--nx 1024 --ny 1024 --nz 256 --steps 100]
    python -m paper_1502_02935_amd.disc attribution [--nx 512 --ny 512 --nz 128 --steps 200]

precision: FP32 bulk against the FP64 path from one FP32-rounded state with
the FP64 run's time steps (L1 and Linf per field), plus the throughput of
both precisions with their own device CFL steps.  large: throughput of the
FP32 path on the largest one-GPU machine (same profiles on a 48 x 48 x 12 kpc
box, so the cell size is that of the 512 x 512 x 128 slab).  attribution:
where the FP32 error comes from -- the FP64 path with chosen conserved
fields rounded to FP32 after every step (storage alone, per field), the
FP32 path, and the FP64 path from a state whose E is perturbed by 1e-12
(how much the flow amplifies a small difference), each against the plain
FP64 run with the same steps, with the share of the density error in
bands of density.
Prints one JSON line (attribution: one per run).
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


def _banded(a, b, tag):
    """L1 per field of state b against a, plus the density error by density
    band (share of the summed |d rho| and mean relative error per band)."""
    out = {"run": tag, "L1": {k: v["L1_rel"] for k, v in _errors(a, b).items()}}
    rho = a[0][0]
    e = (b[0][0].double() - rho).abs()
    tot = float(e.sum())
    bands = {}
    for lo, hi in ((0.1, 1e30), (1e-2, 0.1), (1e-3, 1e-2), (0.0, 1e-3)):
        m = (rho >= lo) & (rho < hi)
        n = int(m.sum())
        bands["rho>=%g" % lo] = {"cells": n, "share": float(e[m].sum()) / tot if tot > 0 else 0.0,
                                 "rel": float((e[m] / rho[m]).mean()) if n else 0.0}
    out["rho_bands"] = bands
    return out


def _fp64_run(pb, dts, round_fields=(), perturb=0.0):
    """FP64 run with the given steps; round_fields: conserved fields (0-4
    cells rho, Mx, My, Mz, E; 5-7 faces) rounded to FP32 after every step
    (a restart from the rounded state, bitwise what continuing would give);
    perturb: relative Gaussian perturbation of E at the start."""
    c5 = torch.as_tensor(pb.cell5, device="cuda")
    b = [torch.as_tensor(x, device="cuda") for x in (pb.bx, pb.by, pb.bz)]
    if perturb:
        g = torch.Generator(device="cuda")
        g.manual_seed(7)
        c5 = c5.clone()
        c5[4] *= 1.0 + perturb * torch.randn(c5[4].shape, device="cuda", generator=g,
                                             dtype=torch.float64)
    cfg = config_from_problem(pb, precision=L.MHD_FP64)
    s = Sim(cfg, c5, *b)
    if not round_fields:
        s.step(len(dts), dt=dts)
    else:
        for dt in dts:
            s.step(1, dt=dt)
            c5, bx, by, bz = s.get_state()
            s.close()
            del s
            for m in round_fields:
                t = c5[m] if m < 5 else (bx, by, bz)[m - 5]
                t.copy_(t.float().double())
            s = Sim(cfg, c5, bx, by, bz)
    out = s.get_state()
    s.close()
    return out


def attribution(nx, ny, nz, steps, seed=1):
    pb = _problem(nx, ny, nz, seed)
    s64 = Sim(config_from_problem(pb, precision=L.MHD_FP64), pb.cell5, pb.bx, pb.by, pb.bz)
    dts = []
    for _ in range(steps):
        dts.append(s64.dt())
        s64.step(1, dt=dts[-1])
    ref = s64.get_state()
    s64.close()
    del s64
    rows = []
    s32 = Sim(config_from_problem(pb, precision=L.MHD_FP32), pb.cell5, pb.bx, pb.by, pb.bz)
    s32.step(steps, dt=dts)
    rows.append(_banded(ref, s32.get_state(), "fp32"))
    s32.close()
    del s32
    sc = Sim(config_from_problem(pb, precision=L.MHD_FP32_COMP), pb.cell5, pb.bx, pb.by, pb.bz)
    sc.step(steps, dt=dts)
    rows.append(_banded(ref, sc.get_state(), "fp32_comp"))
    sc.close()
    del sc
    for tag, rf in (("fp64_rounded_all", (0, 1, 2, 3, 4, 5, 6, 7)), ("fp64_rounded_E", (4,)),
                    ("fp64_rounded_M", (1, 2, 3)), ("fp64_rounded_rho", (0,)),
                    ("fp64_rounded_B", (5, 6, 7))):
        _log(tag)
        rows.append(_banded(ref, _fp64_run(pb, dts, rf), tag))
    rows.append(_banded(ref, _fp64_run(pb, dts, perturb=1e-12), "fp64_E_perturbed_1e-12"))
    for r in rows:
        r.update({"cells": pb.ncell, "steps": steps})
    return rows


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
    ap.add_argument("mode", choices=("precision", "large", "attribution"))
    ap.add_argument("--nx", type=int, default=None)
    ap.add_argument("--ny", type=int, default=None)
    ap.add_argument("--nz", type=int, default=None)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--seed", type=int, default=1)
    a = ap.parse_args(argv)
    if a.mode == "precision":
        r = precision(a.nx or 512, a.ny or 512, a.nz or 128, a.steps or 200, a.seed)
    elif a.mode == "attribution":
        for row in attribution(a.nx or 512, a.ny or 512, a.nz or 128, a.steps or 200, a.seed):
            print(json.dumps(row), flush=True)
        return
    else:
        r = large(a.nx or 1024, a.ny or 1024, a.nz or 256, a.steps or 100, a.seed)
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
