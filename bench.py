"""Throughput benchmark of the ideal-MHD TVD-MUSCL step on one MI355X.

Workload: periodic turbulent-ISM box (256^3 cells, ideal MHD gamma 5/3,
lognormal density sigma_lnrho = 1, k^-4 Gaussian random velocity on
1 <= |k| <= 16 at rms Mach 3, isothermal start P = 0.1 rho, uniform B_x at
plasma beta 1, seed 1, CFL 0.4).  One step = one full predictor-corrector
step of the whole box (every kernel of the path, device CFL dt).

Prints one JSON line: FP32-bulk throughput (the headline value), the FP64
throughput, the FP32-vs-FP64 L1/Linf error per field after 100 steps from the
same FP32-rounded state with the same time steps, the roofline position of
the dominant kernel (HIP events around each launch inside the timed region)
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="cells per axis")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--err-steps", type=int, default=100)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_run(pb, precision, steps, warmup):
    import torch
    from paper_1502_02935_amd import Sim, config_from_problem
    cfg = config_from_problem(pb, precision=precision)
    sim = Sim(cfg, pb.cell5, pb.bx, pb.by, pb.bz)
    sim.step(warmup)
    torch.cuda.synchronize()
    sim.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile_get()
    sim.profile(False)
    d = sim.diag()
    return (t1 - t0), prof, d, sim


def error_run(pb, nsteps):
    """FP64 run recording its CFL dts, then FP32 with the same dts, both from
    the same FP32-rounded initial state; L1 and Linf per field."""
    import numpy as np
    import torch
    from paper_1502_02935_amd import Sim, config_from_problem
    s64 = Sim(config_from_problem(pb, precision=0), pb.cell5, pb.bx, pb.by, pb.bz)
    dts = []
    for _ in range(nsteps):
        dts.append(s64.dt())
        s64.step(1, dt=dts[-1])
    s32 = Sim(config_from_problem(pb, precision=1), pb.cell5, pb.bx, pb.by, pb.bz)
    s32.step(nsteps, dt=dts)
    a = s64.get_state()
    b = s32.get_state()
    names = ("rho", "Mx", "My", "Mz", "E")
    out = {}
    for m in range(5):
        r = a[0][m]
        e = (b[0][m].double() - r)
        out[names[m]] = {"L1_rel": float(e.abs().mean() / r.abs().mean()),
                         "Linf_rel": float(e.abs().max() / r.abs().max())}
    for q, nm in enumerate(("Bx", "By", "Bz")):
        r = a[1 + q]
        e = b[1 + q].double() - r
        den_mean = float(r.abs().mean())
        den_max = float(r.abs().max())
        out[nm] = {"L1_rel": float(e.abs().mean()) / den_mean if den_mean > 0 else float(e.abs().mean()),
                   "Linf_rel": float(e.abs().max()) / den_max if den_max > 0 else float(e.abs().max())}
    d32 = s32.diag()
    torch.cuda.synchronize()
    return out, {"steps": nsteps, "t_end": float(np.sum(dts)),
                 "fp64_recovery_cell_evals": d32["n_fp64_recovery"]}


# Algorithmic work of one launch of the fused flux sweep (the dominant
# kernel: fluxes of the three lower faces of every interior cell and the
# stage's conservative update).  Bytes per cell, FP32: read the primitive
# arrays, the 3 face-normal B and the 5 conserved cell values once (64 B in
# the corrector; 60 B in the predictor, whose primitive density is the
# conserved density array it also reads; 62 B as the mean of the two
# launches); write the 5 updated cell values, the 6 field components of the 3 fluxes
# and the 3 mass-flux sign bytes (47 B), and the 5 hydrodynamic components
# of the faces on tile seams, which the stage update adds (1/64 of the x,
# 1/8 of the y and 1/16 of the z faces: 4.06 B).  Flops per face, counted on
# the FP64 oracle over the turbulent-box face states (oracle/count_flops.py):
# HLLD 400.6, MUSCL of 7 variables 154.0; the update adds 30 per cell.
SWEEP_BYTES_PER_CELL_FP32 = (7.5 * 4 + 3 * 4 + 5 * 4 + 5 * 4 + 6 * 4 + 3
                             + 5 * 4 * (1 / 64 + 1 / 8 + 1 / 16))
HLLD_FLOPS_PER_FACE = 400.6
MUSCL_FLOPS_PER_FACE = 154.0
UPDATE_FLOPS_PER_CELL = 30.0
# Whole step per cell-update (both stages, every part), same count.
STEP_FLOPS_PER_CELL_UPDATE = 3162.0
STEP_BYTES_PER_CELL_UPDATE_FP32 = 64.0  # read and write the 8 state fields
# Measured HBM traffic of one sweep launch at n = 256 (2 x TCC FETCH_SIZE +
# WRITE_SIZE: a plain 1 GiB copy reads as 512 MiB of FETCH_SIZE and 1 GiB of
# WRITE_SIZE), valid only for the kernel sources with this hash.
PROFILED_SWEEP = {"sources_sha256_16": "22087e2bbb30120c", "n": 256,
                  "bytes_per_launch": 2.331e9}
# The sources that define the sweep's code (kernel, tile sizes and interfaces,
# geometry, solver, source).
KERNEL_SOURCES = ("paper_1502_02935_amd/csrc/mhd_flux.hip",
                  "paper_1502_02935_amd/csrc/mhd_kernels.hpp",
                  "paper_1502_02935_amd/csrc/mhd_span.hpp",
                  "paper_1502_02935_amd/csrc/mhd_physics.hpp",
                  "paper_1502_02935_amd/csrc/mhd_source.hpp")


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def sweep_roofline(n, prof):
    """Roofline of the fused flux sweep (the dominant kernel): its mean
    launch time from HIP events over the timed region, algorithmic bytes and
    flops per launch.  Arithmetic intensity about 10.5 (first order) to 14.4
    (MUSCL) flop/byte, below the FP32 ridge of 157.3/8 = 19.7: HBM bound by
    the published peaks (the measured limiter is the vector ALUs' issue)."""
    ms_tot, nl = prof["flux"]
    ms = ms_tot / nl
    cells = n ** 3
    faces = 3 * cells
    byts = cells * SWEEP_BYTES_PER_CELL_FP32
    flops = faces * (HLLD_FLOPS_PER_FACE + 0.5 * MUSCL_FLOPS_PER_FACE) + cells * UPDATE_FLOPS_PER_CELL
    ach = byts / (ms * 1e-3) / 1e9
    traffic = None
    if kernel_sources_hash() == PROFILED_SWEEP["sources_sha256_16"] and n == PROFILED_SWEEP["n"]:
        traffic = PROFILED_SWEEP["bytes_per_launch"]
    return {"kernel": "k_sweep (fused flux sweep and stage update: three face families, "
                      "first-order and MUSCL + HLLD)",
            "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS, "traffic": traffic, "ms_per_launch": ms,
            "bytes_per_launch": byts, "faces_per_launch": faces,
            "alu_view": {"flops_per_launch": flops,
                         "achieved_tflops": flops / (ms * 1e-3) / 1e12,
                         "peak_tflops": PEAK_FP32_TFLOPS,
                         "frac": flops / (ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS}}


def cpu_baseline(pb, seconds):
    """The FP64 oracle on the first steps of the same workload, on this host's
    cores, stopping after about `seconds` of work."""
    from oracle.pyorc import Oracle, OrcConfig, load_oracle
    L = load_oracle()
    o = Oracle(OrcConfig(nx=pb.nx, ny=pb.ny, nz=pb.nz, dx=pb.dx, dy=pb.dy, dz=pb.dz,
                         gamma=pb.gamma, cfl=pb.cfl, bc=pb.bc))
    assert o.set_state(pb.cell5, pb.bx, pb.by, pb.bz) == 0
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.step()
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 50:
            break
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": pb.ncell * steps / el, "unit": "cell-updates/s", "cores": L.orc_threads(),
            "kind": "oracle",
            "sample": "first %d FP64 steps of the same %dx%dx%d box (CPU: %s)" % (
                steps, pb.nx, pb.ny, pb.nz, model),
            "seconds": el}


def main():
    args = _args()
    if args.gpus != 1:
        print("bench.py runs one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if "cpu_baseline_threads" not in os.environ:
        try:
            os.environ.setdefault("OMP_NUM_THREADS", str(len(os.sched_getaffinity(0))))
        except AttributeError:
            pass
    import torch

    from mhd_inputs import problems as P
    n = args.n
    log("generating turbulent ISM box %d^3 seed %d" % (n, args.seed))
    pb = P.turbulent_ism(n, seed=args.seed).astype("float32")
    cells = pb.ncell

    if args.calib_copy:
        # a plain copy of known size: 2^28 floats read and written once
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    log("FP32 timed run: %d warmup + %d steps" % (args.warmup, args.steps))
    el32, prof32, d32, _ = timed_run(pb, 1, args.steps, args.warmup)
    rate32 = cells * args.steps / el32
    log("  %.3f ms/step, %.3e cell-updates/s" % (1e3 * el32 / args.steps, rate32))
    result = {
        "metric": "MHD cell-updates/s",
        "value": rate32,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "turbulent-ISM periodic box %d^3, ideal MHD gamma 5/3, lognormal rho "
                        "(sigma 1), k^-4 velocity rms Mach 3, beta 1, seed %d, CFL 0.4; "
                        "FP32 bulk with FP64 pressure recovery, dt and sums" % (n, args.seed),
            "cells": cells,
            "kernels_per_step": {k: v[1] / args.steps for k, v in prof32.items() if v[1]},
        },
    }
    kern = {k: {"ms_per_launch": v[0] / v[1], "launches": v[1], "share": v[0] / sum(
        x[0] for x in prof32.values())} for k, v in prof32.items() if v[1]}
    result["kernel_profile_fp32"] = kern
    result["roofline"] = sweep_roofline(n, prof32)
    # the whole path: arithmetic intensity 3162 flop / 64 B = 49 flop/byte
    result["path_roofline"] = {
        "bound": "alu", "flops_per_cell_update": STEP_FLOPS_PER_CELL_UPDATE,
        "achieved_tflops": rate32 * STEP_FLOPS_PER_CELL_UPDATE / 1e12,
        "peak_tflops": PEAK_FP32_TFLOPS,
        "frac": rate32 * STEP_FLOPS_PER_CELL_UPDATE / 1e12 / PEAK_FP32_TFLOPS,
        "bound_cell_updates_per_s": PEAK_FP32_TFLOPS * 1e12 / STEP_FLOPS_PER_CELL_UPDATE,
        "hbm_bound_cell_updates_per_s": PEAK_HBM_GBS * 1e9 / STEP_BYTES_PER_CELL_UPDATE_FP32}

    if not args.no_fp64:
        log("FP64 timed run")
        el64, prof64, d64, _ = timed_run(pb, 0, args.steps, args.warmup)
        result["fp64"] = {"value": cells * args.steps / el64, "ms_per_step": 1e3 * el64 / args.steps,
                          "kernel_ms": {k: v[0] / v[1] for k, v in prof64.items() if v[1]}}
        log("  %.3f ms/step" % (1e3 * el64 / args.steps))
    if not args.no_error:
        log("FP32 vs FP64 error run, %d steps" % args.err_steps)
        err, info = error_run(pb, args.err_steps)
        result["error_fp32_vs_fp64"] = err
        result["error_run"] = info
    torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        log("CPU oracle baseline (~%.0f s)" % args.cpu_seconds)
        result["cpu_baseline"] = cpu_baseline(pb, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
