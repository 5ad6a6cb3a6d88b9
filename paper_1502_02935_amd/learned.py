"""Learned flux correction on a 2x-coarsened grid: data generation from fine
runs, training with the library's MFMA kernels, and evaluation against the
coarse-grained fine run.

Data: a fine periodic run advances two steps (dt1, dt2) while the library
accumulates dt-weighted corrector fluxes on the coarse faces; the coarse
state at the start of the pair is the 2x coarse-graining of the fine state.
A coarse context started from it takes one step of dt1 + dt2; its corrector
state gives the features, and the target is the MLP output that would turn
its corrector flux into the fine time-and-area average.  Faces touching a
shock cell are left out (the gate keeps the plain flux there).

Training: Adam on the mean squared error of standardised targets; the
standardisation is folded into the output layer afterwards.

Evaluation: the fine run and two coarse runs (plain, learned) from the
coarse-grained initial state, the coarse runs forced to the fine run's
pair-summed time steps; L1 per field of each coarse run against the
coarse-graining of the fine one.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import _lib as L
from .sim import MHDConfig, MlpTrainer, Sim, config_from_problem


def coarse_config(fine: MHDConfig) -> MHDConfig:
    return MHDConfig(nx=fine.nx // 2, ny=fine.ny // 2, nz=fine.nz // 2, dx=2 * fine.dx,
                     dy=2 * fine.dy, dz=2 * fine.dz, x0=fine.x0, y0=fine.y0, z0=fine.z0,
                     precision=fine.precision, gamma=fine.gamma, cfl=fine.cfl, bc=fine.bc,
                     recon=fine.recon, kappa=fine.kappa, source=fine.source, src=fine.src,
                     rho_floor=fine.rho_floor, p_floor=fine.p_floor, inflow=fine.inflow,
                     riemann=fine.riemann)


def random_faces(cfg: MHDConfig, n: int, gen: torch.Generator, device) -> torch.Tensor:
    a = torch.randint(0, 3, (n,), generator=gen, device="cpu")
    i = torch.randint(0, cfg.nx, (n,), generator=gen, device="cpu")
    j = torch.randint(0, cfg.ny, (n,), generator=gen, device="cpu")
    k = torch.randint(0, cfg.nz, (n,), generator=gen, device="cpu")
    return torch.stack([a, i, j, k], dim=1).to(torch.int32).contiguous().to(device)


def generate(problem, pairs: int, faces_per_pair: int, seed: int = 0, precision=L.MHD_FP32,
             device="cuda", log=None):
    """Samples (x [m][32], t [m][8]) from `pairs` fine step pairs of
    `problem` (even extents; per axis periodic on both sides or on neither)."""
    fcfg = config_from_problem(problem, precision=precision)
    ccfg = coarse_config(fcfg)
    fine = Sim(fcfg, problem.cell5, problem.bx, problem.by, problem.bz, device=device)
    gen = torch.Generator().manual_seed(seed)
    xs, ts = [], []
    kept = 0
    for p in range(pairs):
        cstate = fine.coarsen()
        acc = fine.flux_accumulator(True)
        dt1 = fine.dt()
        fine.step(1, dt=dt1)
        dt2 = fine.dt()
        fine.step(1, dt=dt2)
        fine.flux_accumulator(False)
        coarse = Sim(ccfg, *cstate, device=device)
        coarse.set_full_fluxes(True)
        coarse.step(1, dt=dt1 + dt2)
        faces = random_faces(ccfg, faces_per_pair, gen, device)
        x, t, m = coarse.mlp_samples(acc, dt1 + dt2, faces)
        keep = m == 0
        xs.append(x[keep])
        ts.append(t[keep])
        kept += int(keep.sum())
        del coarse
        if log and (p + 1) % 20 == 0:
            log("  pair %d/%d: %d samples" % (p + 1, pairs, kept))
    fine.close()
    return torch.cat(xs), torch.cat(ts)


def standardise(t: torch.Tensor, clip: float = 8.0):
    """Per-output mean and std (over the training targets) and the clipped,
    standardised targets."""
    mu = t.mean(dim=0)
    sd = t.std(dim=0).clamp_min(1e-12)
    z = ((t - mu) / sd).clamp(-clip, clip)
    return z.contiguous(), mu, sd


def fold_output_scaling(params: torch.Tensor, mu: torch.Tensor, sd: torch.Tensor):
    """y = sd * (W3 h + b3) + mu, folded into W3, b3 in place."""
    p = params
    w3 = p[6208:6208 + 512].view(8, 64)
    b3 = p[6784:6792]
    w3.mul_(sd.view(8, 1))
    b3.mul_(sd).add_(mu)
    p[6784 + 5] = 0.0  # normal-B output unused
    p[6208 + 5 * 64:6208 + 6 * 64] = 0.0


def init_params(seed: int, device) -> torch.Tensor:
    """He-style initialisation of W1, W2, small W3, zero biases."""
    g = torch.Generator().manual_seed(seed)
    p = torch.zeros(L.MLP_NPARAM, dtype=torch.float32)
    p[0:2048] = torch.randn(2048, generator=g) * math.sqrt(2.0 / 32)
    p[2112:6208] = torch.randn(4096, generator=g) * math.sqrt(2.0 / 64)
    p[6272:6784] = torch.randn(512, generator=g) * 0.01
    return p.to(device).contiguous()


def train(x: torch.Tensor, t: torch.Tensor, steps: int = 4000, batch: int = 16384,
          lr: float = 2e-3, seed: int = 0, log=None):
    """Adam on standardised targets with cosine learning-rate decay; returns
    folded params, history of (step, loss) and the standardisation."""
    z, mu, sd = standardise(t)
    params = init_params(seed, x.device)
    tr = MlpTrainer(params, lr=lr)
    g = torch.Generator(device=x.device).manual_seed(seed)
    n = x.shape[0]
    hist = []
    for s in range(steps):
        tr.lr = lr * 0.5 * (1.0 + math.cos(math.pi * s / steps))
        idx = torch.randint(0, n, (batch,), generator=g, device=x.device)
        loss = tr.step(x[idx].contiguous(), z[idx].contiguous())
        if s % 200 == 0 or s == steps - 1:
            hist.append((s, float(loss.item())))
            if log:
                log("  step %d loss %.4e" % (s, hist[-1][1]))
    fold_output_scaling(tr.params, mu, sd)
    return tr.params, hist, (mu, sd)


def _l1(a, b):
    return float((a - b).abs().mean() / b.abs().mean())


def evaluate(problem, params, pairs: int, precision=L.MHD_FP32, tau=0.5, jump=0.5,
             tau_flux=0.0, device="cuda"):
    """Fine run for 2*pairs steps vs plain and learned coarse runs forced to
    the pair-summed time steps: L1 per field against the coarse-grained fine
    state (B components relative to the mean |B| of the reference), and
    throughput: the fine run with device time steps, the coarse runs in
    fine-equivalent cell-updates/s (fine cells x fine steps / coarse time)."""
    fcfg = config_from_problem(problem, precision=precision)
    ccfg = coarse_config(fcfg)
    fine = Sim(fcfg, problem.cell5, problem.bx, problem.by, problem.bz, device=device)
    c0 = fine.coarsen()
    dts = []
    for _ in range(pairs):
        d1 = fine.dt()
        fine.step(1, dt=d1)
        d2 = fine.dt()
        fine.step(1, dt=d2)
        dts.append(d1 + d2)
    ref = fine.coarsen()
    fine.close()
    del fine
    # fine throughput: same run, device CFL steps, no host synchronisation
    fine2 = Sim(fcfg, problem.cell5, problem.bx, problem.by, problem.bz, device=device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fine2.step(2 * pairs)
    torch.cuda.synchronize()
    t_fine = time.perf_counter() - t0
    fine2.close()
    del fine2
    fine_cells = fcfg.nx * fcfg.ny * fcfg.nz
    out = {"t_end": float(sum(dts)), "coarse_steps": pairs, "fine_steps": 2 * pairs,
           "fine_seconds": t_fine, "fine_cell_updates_per_s": fine_cells * 2 * pairs / t_fine}
    bref = (ref[1].double().abs().mean() + ref[2].double().abs().mean() +
            ref[3].double().abs().mean()) / 3.0
    for name, mlp in (("plain", None), ("learned", params)):
        c = Sim(ccfg, *[x.clone() for x in c0], device=device)
        if mlp is not None:
            c.set_mlp(mlp, tau=tau, jump=jump, tau_flux=tau_flux)
        c.step(2, dt=dts[:2])  # warm-up on a copy of the start: rebuilt below
        c.close()
        c = Sim(ccfg, *[x.clone() for x in c0], device=device)
        if mlp is not None:
            c.set_mlp(mlp, tau=tau, jump=jump, tau_flux=tau_flux)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.step(pairs, dt=dts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = c.get_state()
        d = c.diag(check=False)
        errs = {nm: _l1(st[0][m].double(), ref[0][m].double())
                for m, nm in enumerate(("rho", "Mx", "My", "Mz", "E"))}
        for q, nm in enumerate(("Bx", "By", "Bz")):
            errs[nm] = float((st[1 + q].double() - ref[1 + q].double()).abs().mean() / bref)
        out[name] = {"L1": errs, "seconds": el, "status": d["status"],
                     "mlp_faces": d["n_mlp_faces"], "mlp_gated": d["n_mlp_gated"],
                     "fine_equivalent_cell_updates_per_s": fine_cells * 2 * pairs / el}
        c.close()
    return out


def default_weights() -> str:
    """The network trained on the 256^3 turbulent boxes (seeds 100-109)."""
    import os
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                        "mlp_turbulent256.npy")


def time_coarse(problem, params, steps: int, tau=0.1, jump=0.5, dt=1e-4, warmup=5,
                device="cuda"):
    """Step time of the plain and the learned coarse run (2x coarse-graining
    of `problem`), same fixed dt, with the per-kernel-class profile."""
    fcfg = config_from_problem(problem, precision=L.MHD_FP32)
    fine = Sim(fcfg, problem.cell5, problem.bx, problem.by, problem.bz, device=device)
    c0 = fine.coarsen()
    fine.close()
    ccfg = coarse_config(fcfg)
    out = {"coarse_cells": ccfg.nx * ccfg.ny * ccfg.nz, "steps": steps, "dt": dt}
    for name, mlp in (("plain", None), ("learned", params)):
        c = Sim(ccfg, *[x.clone() for x in c0], device=device)
        if mlp is not None:
            c.set_mlp(mlp, tau=tau, jump=jump)
        c.step(warmup, dt=dt)
        torch.cuda.synchronize()
        c.profile(True)
        t0 = time.perf_counter()
        c.step(steps, dt=dt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = c.profile_get()
        c.profile(False)
        d = c.diag(check=False)
        out[name] = {"ms_per_step": 1e3 * el / steps, "status": d["status"],
                     "kernel_ms_per_launch": {k: v[0] / v[1] for k, v in prof.items() if v[1]},
                     "launches_per_step": {k: v[1] / steps for k, v in prof.items() if v[1]}}
        c.close()
    out["learned_over_plain"] = out["learned"]["ms_per_step"] / out["plain"]["ms_per_step"]
    return out


def make_problem(kind: str, n: int, seed: int):
    """A fine-grid workload, rounded to FP32: the periodic turbulent-ISM box
    n^3, or the disc slab n x n x n/4 (24 x 24 x 6 kpc at n = 512, the box
    growing with n so the cell size stays 46.875 pc)."""
    from mhd_inputs import problems as P
    if kind == "turbulent":
        return P.turbulent_ism(n, seed=seed).astype("float32")
    if kind == "disc":
        sc = n / 512.0
        return P.disc(n, n, n // 4, lx=24.0 * sc, ly=24.0 * sc, lz=6.0 * sc,
                      seed=seed).astype("float32")
    raise ValueError(kind)


def _seeds(s: str):
    if "-" in s:
        a, b = s.split("-")
        return list(range(int(a), int(b) + 1))
    return [int(v) for v in s.split(",")]


def main(argv=None):
    import argparse
    import json
    import os
    import sys


    ap = argparse.ArgumentParser(description="train and evaluate the learned flux correction")
    ap.add_argument("--problem", choices=("turbulent", "disc"), default="turbulent")
    ap.add_argument("--n", type=int, default=256, help="fine cells per axis (disc: along x, y)")
    ap.add_argument("--eval-n", type=int, default=None,
                    help="fine cells per axis of the evaluation runs (default --n)")
    ap.add_argument("--train-seeds", default="100-109")
    ap.add_argument("--eval-seeds", default="200-204")
    ap.add_argument("--pairs", type=int, default=100, help="fine step pairs per seed (= coarse steps)")
    ap.add_argument("--eval-pairs", type=int, default=None,
                    help="fine step pairs of the evaluation runs (default --pairs)")
    ap.add_argument("--faces", type=int, default=16384, help="sampled coarse faces per pair")
    ap.add_argument("--steps", type=int, default=4000, help="Adam steps")
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--tau", type=float, default=0.1)
    ap.add_argument("--params-out", default=None)
    ap.add_argument("--params-in", default=None, help="skip training, load these weights (.npy)")
    ap.add_argument("--taus", default=None,
                    help="comma list of tau or tau:tau_flux clip settings to evaluate")
    ap.add_argument("--tau-flux", type=float, default=0.0)
    ap.add_argument("--json-out", default=None)
    ap.add_argument("--time-coarse", type=int, default=0, metavar="STEPS",
                    help="only time STEPS plain and learned coarse steps (weights: --params-in "
                         "or the shipped ones) on the first evaluation seed")
    a = ap.parse_args(argv)

    def log(*m):
        print(*m, file=sys.stderr, flush=True)

    if a.time_coarse:
        params = torch.as_tensor(np.load(a.params_in or default_weights()), dtype=torch.float32,
                                 device="cuda")
        sd = _seeds(a.eval_seeds)[0]
        r = time_coarse(make_problem(a.problem, a.eval_n or a.n, sd), params, a.time_coarse,
                        tau=a.tau)
        print(json.dumps(r))
        return
    if a.params_in:
        params = torch.as_tensor(np.load(a.params_in), dtype=torch.float32, device="cuda")
        res = {"params_in": a.params_in, "eval": {}}
        for spec in (a.taus or "%g:%g" % (a.tau, a.tau_flux)).split(","):
            tau, tauf = (float(v) for v in (spec.split(":") + ["0"])[:2])
            for sd in _seeds(a.eval_seeds):
                r = evaluate(make_problem(a.problem, a.eval_n or a.n, sd), params,
                             a.eval_pairs or a.pairs, tau=tau, tau_flux=tauf)
                res["eval"]["%g:%g/%d" % (tau, tauf, sd)] = r
                log("tau %g seed %d: L1 rho plain %.4e learned %.4e; E %.4e %.4e; status %d "
                    "faces %d gated %d" % (tau, sd, r["plain"]["L1"]["rho"],
                                           r["learned"]["L1"]["rho"], r["plain"]["L1"]["E"],
                                           r["learned"]["L1"]["E"], r["learned"]["status"],
                                           r["learned"]["mlp_faces"], r["learned"]["mlp_gated"]))
        if a.json_out:
            with open(a.json_out, "w") as f:
                f.write(json.dumps(res))
        return
    xs, ts = [], []
    t0 = time.perf_counter()
    for sd in _seeds(a.train_seeds):
        log("training data, seed %d" % sd)
        x, t = generate(make_problem(a.problem, a.n, sd), a.pairs, a.faces, seed=sd, log=log)
        xs.append(x)
        ts.append(t)
    x = torch.cat(xs)
    t = torch.cat(ts)
    t_gen = time.perf_counter() - t0
    log("samples: %d (%.1f s)" % (x.shape[0], t_gen))
    t0 = time.perf_counter()
    params, hist, (mu, sd_) = train(x, t, steps=a.steps, batch=a.batch, lr=a.lr, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    if a.params_out:
        np.save(a.params_out, params.cpu().numpy())
    res = {"samples": int(x.shape[0]), "generate_seconds": t_gen, "train_seconds": t_train,
           "adam_steps": a.steps, "batch": a.batch, "loss_history": hist,
           "target_mean": mu.tolist(), "target_std": sd_.tolist(), "eval": {}}
    del x, t, xs, ts
    for sd in _seeds(a.eval_seeds):
        log("evaluation, seed %d" % sd)
        r = evaluate(make_problem(a.problem, a.eval_n or a.n, sd), params,
                     a.eval_pairs or a.pairs, tau=a.tau, tau_flux=a.tau_flux)
        res["eval"][str(sd)] = r
        log("  L1 rho plain %.4e learned %.4e" % (r["plain"]["L1"]["rho"], r["learned"]["L1"]["rho"]))
    fields = ("rho", "Mx", "My", "Mz", "E", "Bx", "By", "Bz")
    summ = {}
    for f in fields:
        pl = [res["eval"][k]["plain"]["L1"][f] for k in res["eval"]]
        le = [res["eval"][k]["learned"]["L1"][f] for k in res["eval"]]
        summ[f] = {"plain": float(np.mean(pl)), "learned": float(np.mean(le)),
                   "gain": float(np.mean(pl) / np.mean(le))}
    res["summary_L1"] = summ
    res["summary_rates"] = {
        k: float(np.mean([res["eval"][s][k]["fine_equivalent_cell_updates_per_s"]
                          for s in res["eval"]])) for k in ("plain", "learned")}
    res["summary_rates"]["fine"] = float(np.mean([res["eval"][s]["fine_cell_updates_per_s"]
                                                  for s in res["eval"]]))
    js = json.dumps(res)
    if a.json_out:
        os.makedirs(os.path.dirname(a.json_out) or ".", exist_ok=True)
        with open(a.json_out, "w") as f:
            f.write(js)
    print(json.dumps({"summary_L1": summ, "summary_rates": res["summary_rates"]}))


if __name__ == "__main__":
    main()
