"""Throughput benchmark of the ideal-MHD TVD-MUSCL step on one MI355X.

Workload (the headline value): periodic turbulent-ISM box (256^3 cells,
ideal MHD gamma 5/3, lognormal density sigma_lnrho = 1, k^-4 Gaussian random
velocity on 1 <= |k| <= 16 at rms Mach 3, isothermal start P = 0.1 rho,
uniform B_x at plasma beta 1, seed 1, CFL 0.4).  One step = one full
predictor-corrector step of the whole box (every kernel of the path, device
CFL dt).

Prints one JSON line: FP32-bulk throughput (the headline value), the FP64
throughput, the FP32-vs-FP64 L1/Linf error per field after 100 steps from the
same FP32-rounded state with the same time steps (plain and compensated
FP32), the disc slab's (512 x 512 x 128, 200 steps) FP32 errors and
throughput, the production-size disc's (1024 x 1024 x 256) plain and
compensated FP32 throughput, the compensated FP32 throughput, the roofline position of the
dominant kernel (HIP events around each launch inside the timed region) and
of the whole path, and the FP64 CPU oracle timed on a bounded sample of the
same workload (all host threads, and one).
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

# MI355X published peaks.  FP32 vector: 256 CUs x 4 SIMDs x 16 lanes x 2
# (FMA) x 2 (packed FP32) x 2.4 GHz = 157.3 TFLOP/s; without packed FP32
# (not used by this build) the FMA rate is half of it.
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_FP64_TFLOPS = 78.6


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="cells per axis")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--err-steps", type=int, default=100)
    ap.add_argument("--disc-steps", type=int, default=200)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-comp", action="store_true", help="skip the compensated FP32 run")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--no-disc", action="store_true")
    ap.add_argument("--no-disc-large", action="store_true",
                    help="skip the 1024x1024x256 disc throughput")
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
    sim.close()
    return (t1 - t0), prof, d


def _field_errors(a, b):
    """L1 (mean |b - a| / mean |a|) and Linf (max |b - a| / max |a|) of state
    b against state a, per field, each relative to its own magnitude."""
    names = ("rho", "Mx", "My", "Mz", "E")
    out = {}
    for m in range(5):
        r = a[0][m]
        e = (b[0][m].double() - r).abs()
        out[names[m]] = {"L1_rel": float(e.mean() / r.abs().mean()),
                         "Linf_rel": float(e.max() / r.abs().max())}
    for q, nm in enumerate(("Bx", "By", "Bz")):
        r = a[1 + q]
        e = (b[1 + q].double() - r).abs()
        den_mean = float(r.abs().mean())
        den_max = float(r.abs().max())
        out[nm] = {"L1_rel": float(e.mean()) / den_mean if den_mean > 0 else float(e.mean()),
                   "Linf_rel": float(e.max()) / den_max if den_max > 0 else float(e.max())}
    return out


def error_run(pb, nsteps, precisions=(1,)):
    """FP64 run recording its CFL dts, then each FP32 form with the same dts,
    all from the same FP32-rounded initial state; L1 and Linf per field
    against the FP64 run."""
    import numpy as np
    import torch
    from paper_1502_02935_amd import Sim, config_from_problem
    s64 = Sim(config_from_problem(pb, precision=0), pb.cell5, pb.bx, pb.by, pb.bz)
    dts = []
    for _ in range(nsteps):
        dts.append(s64.dt())
        s64.step(1, dt=dts[-1])
    a = s64.get_state()
    d64 = s64.diag(check=False)
    s64.close()
    del s64
    errs, info = {}, {"steps": nsteps, "t_end": float(np.sum(dts)),
                      "status_fp64": d64["status"], "floor_hits_fp64": d64["n_floor"]}
    for prec in precisions:
        s = Sim(config_from_problem(pb, precision=prec), pb.cell5, pb.bx, pb.by, pb.bz)
        s.step(nsteps, dt=dts)
        b = s.get_state()
        d = s.diag(check=False)
        s.close()
        del s
        key = {1: "fp32", 2: "fp32_comp"}.get(prec, "precision_%d" % prec)
        errs[key] = _field_errors(a, b)
        info[key] = {"fp64_recovery_cell_evals": d["n_fp64_recovery"], "status": d["status"],
                     "floor_hits": d["n_floor"], "n_degenerate": d["n_degenerate"],
                     "n_hll_fallback": d["n_hll_fallback"]}
        del b
    torch.cuda.synchronize()
    return errs, info


# ---- roofline ---------------------------------------------------------------
# Algorithmic work, counted on the FP64 oracle (oracle/count_flops.py; every
# +, -, *, /, sqrt one flop) over the turbulent box's face states: HLLD 400.6
# flops per face, MUSCL of the 7 face variables 154.0, the stage update 30
# per cell; the whole step 3162 flops per cell-update.  Algorithmic bytes:
# the step reads and writes the 8 state fields once per cell-update, 64 B in
# FP32; one launch of the fused sweep is one stage pass over every cell, so
# its share is the same 64 B per cell.
HLLD_FLOPS_PER_FACE = 400.6
MUSCL_FLOPS_PER_FACE = 154.0
UPDATE_FLOPS_PER_CELL = 30.0
STEP_FLOPS_PER_CELL_UPDATE = 3162.0
STATE_BYTES_PER_CELL_FP32 = 64.0
# What the fused sweep itself must move given its design (the staged step):
# read the primitives, the 3 face-normal B and the 5 conserved cell values
# (62 B per cell as the mean of the predictor, whose primitive density is the
# conserved density it also reads, and the corrector), write the 5 updated
# cell values, the 6 field components of the 3 fluxes and the 3 mass-flux
# sign bytes (47 B), and the 5 hydrodynamic components of the faces on tile
# seams (1/64 of the x, 1/8 of the y and 1/16 of the z faces: 4.06 B).
SWEEP_KERNEL_BYTES_PER_CELL_FP32 = (7.5 * 4 + 3 * 4 + 5 * 4 + 5 * 4 + 6 * 4 + 3
                                    + 5 * 4 * (1 / 64 + 1 / 8 + 1 / 16))
# Counter figures of the sweep at n = 256 (rocprofv3: 2 x TCC FETCH_SIZE +
# WRITE_SIZE, a plain 1 GiB copy reading as 512 MiB of FETCH_SIZE and 1 GiB of
# WRITE_SIZE; VALUBusy), and the whole step's counter traffic, valid only
# for the kernel sources with this hash (else reported as null).
PROFILED = {"sources_sha256_16": "99e5dcaaa6ccf43f", "n": 256,
            "sweep_bytes_per_launch": 2.2960e9, "sweep_valu_busy": 0.695,
            "step_bytes": 10.443e9}
# The sources that define the step's kernels.
KERNEL_SOURCES = ("paper_1502_02935_amd/csrc/mhd_flux.hip",
                  "paper_1502_02935_amd/csrc/mhd_kernels.hip",
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


def _profiled(n):
    return kernel_sources_hash() == PROFILED["sources_sha256_16"] and n == PROFILED["n"]


def sweep_roofline(n, prof):
    """Roofline of the fused flux sweep (the dominant kernel): mean launch
    time from HIP events over the timed region.  Its arithmetic intensity,
    3 faces x (HLLD + MUSCL/2) + update = 1461 flops per 64 algorithmic bytes
    = 22.8 flop/B, is above the FP32 ridge of 157.3/8 = 19.7 flop/B: ALU bound
    (the measured limiter is vector-ALU issue, VALUBusy)."""
    ms_tot, nl = prof["flux"]
    ms = ms_tot / nl
    cells = n ** 3
    faces = 3 * cells
    flops = faces * (HLLD_FLOPS_PER_FACE + 0.5 * MUSCL_FLOPS_PER_FACE) + cells * UPDATE_FLOPS_PER_CELL
    alg_bytes = cells * STATE_BYTES_PER_CELL_FP32
    kern_bytes = cells * SWEEP_KERNEL_BYTES_PER_CELL_FP32
    tflops = flops / (ms * 1e-3) / 1e12
    prof_ok = _profiled(n)
    traffic = PROFILED["sweep_bytes_per_launch"] if prof_ok else None
    return {"kernel": "k_sweep (fused flux sweep and stage update: three face families, "
                      "first-order and MUSCL + HLLD)",
            "bound": "alu", "achieved": tflops, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": tflops / PEAK_FP32_TFLOPS, "traffic": traffic,
            "frac_of_unpacked_fma_peak": tflops / PEAK_FP32_UNPACKED_TFLOPS,
            "ms_per_launch": ms, "flops_per_launch": flops, "faces_per_launch": faces,
            "bytes_per_launch": alg_bytes,
            "hbm_frac": alg_bytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "kernel_bytes_per_launch": kern_bytes,
            "traffic_over_algorithmic": traffic / alg_bytes if traffic else None,
            "valu_busy": PROFILED["sweep_valu_busy"] if prof_ok else None}


def path_roofline(n, rate):
    """The whole step: 3162 flops per 64 B = 49 flop/B, ALU bound; its HBM
    position by the algorithmic bytes and by the counters' traffic."""
    prof_ok = _profiled(n)
    step_traffic = PROFILED["step_bytes"] if prof_ok else None
    alg_step = STATE_BYTES_PER_CELL_FP32 * n ** 3
    return {"bound": "alu", "flops_per_cell_update": STEP_FLOPS_PER_CELL_UPDATE,
            "achieved_tflops": rate * STEP_FLOPS_PER_CELL_UPDATE / 1e12,
            "peak_tflops": PEAK_FP32_TFLOPS,
            "frac": rate * STEP_FLOPS_PER_CELL_UPDATE / 1e12 / PEAK_FP32_TFLOPS,
            "alu_bound_cell_updates_per_s": PEAK_FP32_TFLOPS * 1e12 / STEP_FLOPS_PER_CELL_UPDATE,
            "bytes_per_cell_update": STATE_BYTES_PER_CELL_FP32,
            "hbm_achieved_gbs": rate * STATE_BYTES_PER_CELL_FP32 / 1e9,
            "hbm_frac": rate * STATE_BYTES_PER_CELL_FP32 / 1e9 / PEAK_HBM_GBS,
            "hbm_bound_cell_updates_per_s": PEAK_HBM_GBS * 1e9 / STATE_BYTES_PER_CELL_FP32,
            "traffic_per_step": step_traffic,
            "traffic_over_algorithmic": step_traffic / alg_step if step_traffic else None}


def cpu_baseline(pb, seconds, threads=None, max_steps=50):
    """The FP64 oracle on the first steps of the same workload, on this host's
    cores (or `threads` of them), stopping after about `seconds` of work."""
    from oracle.pyorc import Oracle, OrcConfig, load_oracle
    L = load_oracle()
    nthr0 = L.orc_threads()
    if threads:
        L.orc_set_threads(threads)
    try:
        o = Oracle(OrcConfig(nx=pb.nx, ny=pb.ny, nz=pb.nz, dx=pb.dx, dy=pb.dy, dz=pb.dz,
                             gamma=pb.gamma, cfl=pb.cfl, bc=pb.bc))
        assert o.set_state(pb.cell5, pb.bx, pb.by, pb.bz) == 0
        steps = 0
        t0 = time.perf_counter()
        while True:
            o.step()
            steps += 1
            el = time.perf_counter() - t0
            if el >= seconds or steps >= max_steps:
                break
        cores = L.orc_threads()
    finally:
        L.orc_set_threads(nthr0)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": pb.ncell * steps / el, "unit": "cell-updates/s", "cores": cores,
            "kind": "oracle",
            "sample": "first %d FP64 steps of the same %dx%dx%d box (CPU: %s)" % (
                steps, pb.nx, pb.ny, pb.nz, model),
            "seconds": el}


def disc_leg(steps):
    """Disc slab 512 x 512 x 128 (24 x 24 x 6 kpc, outflow, logarithmic
    potential, floors): FP32 throughput with its own CFL steps, and the FP32
    error against the FP64 run after `steps` steps from the same FP32-rounded
    state with the FP64 run's steps."""
    from mhd_inputs import problems as P
    t0 = time.perf_counter()
    pb = P.disc(512, 512, 128).astype("float32")
    log("  disc generated in %.1f s" % (time.perf_counter() - t0))
    el, prof, d = timed_run(pb, 1, 20, 2)
    out = {"workload": "disc slab 512x512x128, 24x24x6 kpc, rotation 200 km/s (Mach 20), "
                       "toroidal B beta 10, outflow, log-potential source, floors",
           "cells": pb.ncell, "fp32_cell_updates_per_s": pb.ncell * 20 / el,
           "fp32_ms_per_step": 1e3 * el / 20}
    log("  FP32 %.3f ms/step" % out["fp32_ms_per_step"])
    errs, info = error_run(pb, steps, precisions=(1, 2))
    out["error_vs_fp64"] = errs
    out["error_run"] = info
    return out


def disc_large_leg(steps=10, warmup=2):
    """The production-size disc slab 1024 x 1024 x 256 (48 x 48 x 12 kpc,
    the same cell size): plain and compensated FP32 throughput with their own
    CFL steps."""
    import gc
    from mhd_inputs import problems as P
    t0 = time.perf_counter()
    pb = P.disc(1024, 1024, 256, lx=48.0, ly=48.0, lz=12.0).astype("float32")
    log("  large disc generated in %.1f s" % (time.perf_counter() - t0))
    out = {"workload": "disc slab 1024x1024x256, 48x48x12 kpc, rotation 200 km/s (Mach 20), "
                       "toroidal B beta 10, outflow, log-potential source, floors",
           "cells": pb.ncell, "steps": steps}
    for prec, key in ((1, "fp32"), (2, "fp32_comp")):
        el, _, d = timed_run(pb, prec, steps, warmup)
        out[key] = {"cell_updates_per_s": pb.ncell * steps / el, "ms_per_step": 1e3 * el / steps,
                    "status": d["status"]}
        log("  %s %.3f ms/step" % (key, 1e3 * el / steps))
        gc.collect()
    return out


def main():
    args = _args()
    if args.gpus != 1:
        print("bench.py runs one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
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
    el32, prof32, d32 = timed_run(pb, 1, args.steps, args.warmup)
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
        "counters_fp32": {k: d32[k] for k in ("n_hll_fallback", "n_degenerate", "n_floor",
                                                "n_fp64_recovery")},
    }
    kern = {k: {"ms_per_launch": v[0] / v[1], "launches": v[1], "share": v[0] / sum(
        x[0] for x in prof32.values())} for k, v in prof32.items() if v[1]}
    result["kernel_profile_fp32"] = kern
    result["roofline"] = sweep_roofline(n, prof32)
    result["path_roofline"] = path_roofline(n, rate32)

    if not args.no_comp:
        log("compensated FP32 timed run")
        elc, profc, _ = timed_run(pb, 2, args.steps, args.warmup)
        result["fp32_comp"] = {"value": cells * args.steps / elc,
                               "ms_per_step": 1e3 * elc / args.steps,
                               "kernel_ms": {k: v[0] / v[1] for k, v in profc.items() if v[1]}}
        log("  %.3f ms/step" % (1e3 * elc / args.steps))
    if not args.no_fp64:
        log("FP64 timed run")
        el64, prof64, d64 = timed_run(pb, 0, args.steps, args.warmup)
        result["fp64"] = {"value": cells * args.steps / el64, "ms_per_step": 1e3 * el64 / args.steps,
                          "kernel_ms": {k: v[0] / v[1] for k, v in prof64.items() if v[1]}}
        log("  %.3f ms/step" % (1e3 * el64 / args.steps))
    if not args.no_error:
        log("FP32 vs FP64 error run, %d steps" % args.err_steps)
        errs, info = error_run(pb, args.err_steps, precisions=(1, 2))
        result["error_fp32_vs_fp64"] = errs["fp32"]
        result["error_fp32_comp_vs_fp64"] = errs["fp32_comp"]
        info["reference"] = ("FP64 GPU path from the same FP32-rounded state with the same "
                             "steps (its parity with the FP64 oracle: <= 1e-11 per field)")
        result["error_run"] = info
    if not args.no_disc:
        log("disc slab 512x512x128: FP32 throughput and %d-step error" % args.disc_steps)
        result["disc"] = disc_leg(args.disc_steps)
    if not args.no_disc_large:
        log("disc slab 1024x1024x256: FP32 and compensated FP32 throughput")
        result["disc_large"] = disc_large_leg()
    torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        log("CPU oracle baseline (~%.0f s)" % args.cpu_seconds)
        result["cpu_baseline"] = cpu_baseline(pb, args.cpu_seconds)
        log("CPU oracle baseline, one thread (one step)")
        result["cpu_baseline_1thread"] = cpu_baseline(pb, 0.0, threads=1, max_steps=1)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
