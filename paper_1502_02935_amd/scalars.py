"""Passive-scalar workloads of the step (mass fractions carried by the flow,
the code's multi-species advection of section 2.1).

    python -m paper_1502_02935_amd.scalars throughput [--n 256 --steps 20]

throughput: the turbulent-ISM box (FP32) with 0, 1, 4 and 8 random mass
fractions: step time, the scalar kernels' share, their algorithmic bytes
per launch against HBM peak, and the drift of the scalar totals (periodic
box: constant to rounding).  Prints one JSON line.
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


def scalar_bytes(ncell: int, ns: int, es: int) -> int:
    """Algorithmic HBM bytes of the two scalar passes of one step: each reads
    the stage density and the three mass-flux arrays once; the predictor
    reads rho X^n and writes rho X^{n+1/2}; the corrector reads rho X^n and
    rho X^{n+1/2} and writes rho X^{n+1}."""
    return ncell * es * ((4 + 2 * ns) + (4 + 3 * ns))


def throughput(n, steps, warmup=2, counts=(0, 1, 4, 8), precision=L.MHD_FP32):
    from mhd_inputs import problems as P
    pb = P.turbulent_ism(n, seed=1).astype("float32")
    es = 4 if precision == L.MHD_FP32 else 8
    out = {"workload": "turbulent-ISM box %d^3 (seed 1), FP32, random mass fractions" % n}
    for ns in counts:
        sim = Sim(config_from_problem(pb, precision=precision, nscalar=ns), pb.cell5, pb.bx,
                  pb.by, pb.bz)
        if ns:
            rx = P.mass_fractions(pb, ns, "random", seed=3)
            sim.set_scalars(rx)
            t0_tot = sim.get_scalars().double().sum(dim=(1, 2, 3)).cpu().numpy()
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
             "kernel_ms_per_launch": {k: v[0] / v[1] for k, v in prof.items() if v[1]}}
        if ns:
            tot = sim.get_scalars().double().sum(dim=(1, 2, 3)).cpu().numpy()
            r["scalar_total_rel_drift_max"] = float(np.max(np.abs(tot - t0_tot) / np.abs(t0_tot)))
            ms = prof["scalars"][0] / steps  # both stages and their ghost fills
            byts = scalar_bytes(pb.ncell, ns, es)
            r["scalar_pass_ms_per_step"] = ms
            r["scalar_algorithmic_bytes_per_step"] = byts
            r["scalar_achieved_GBps"] = byts / (ms * 1e-3) / 1e9
            r["scalar_frac_of_hbm_peak"] = r["scalar_achieved_GBps"] / PEAK_HBM_GBS
        out["ns_%d" % ns] = r
        _log("ns %d: %.3f ms/step" % (ns, r["ms_per_step"]))
        sim.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("mode", choices=("throughput",))
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--counts", type=int, nargs="+", default=[0, 1, 4, 8],
                    help="scalar counts to run")
    a = ap.parse_args(argv)
    print(json.dumps(throughput(a.n, a.steps, counts=tuple(a.counts))), flush=True)


if __name__ == "__main__":
    main()
