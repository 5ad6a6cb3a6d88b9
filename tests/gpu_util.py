"""Helpers of the GPU parity tests: run the HIP library and the oracle on the
same seeded input with the same time steps, and compare element by element."""
from __future__ import annotations

import numpy as np
import pytest

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    HAVE_GPU = False

needs_gpu = pytest.mark.skipif(not HAVE_GPU, reason="no GPU visible")


def gpu_sim(pb, precision=0, recon=0, kappa=1.0 / 3.0, state=None, riemann=0):
    from paper_1502_02935_amd import Sim, config_from_problem
    cfg = config_from_problem(pb, precision=precision, recon=recon, kappa=kappa, riemann=riemann)
    c5, bx, by, bz = state if state is not None else (pb.cell5, pb.bx, pb.by, pb.bz)
    return Sim(cfg, c5, bx, by, bz)


def host_state(sim):
    return [t.double().cpu().numpy() for t in sim.get_state()]


def rel_err(a, b):
    """max |a - b| / max |b| (b the reference); absolute if b is all zero."""
    s = float(np.abs(b).max())
    d = float(np.abs(a - b).max())
    return d / s if s > 0 else d


FIELDS = ("rho", "Mx", "My", "Mz", "E", "Bx", "By", "Bz")


# A component whose own largest value is below this fraction of its group's
# (the momentum components, the face-B components) is measured against that
# fraction of the group scale: a component that is zero in exact arithmetic
# carries rounding noise of either code and has no scale of its own.
DEGENERATE_FRACTION = 1e-6


def _scales(orc_state):
    c5o, *bo = orc_state
    mscale = max(float(np.abs(c5o[m]).max()) for m in (1, 2, 3))
    bscale = max(float(np.abs(b).max()) for b in bo)
    return c5o, bo, mscale, bscale


def field_errors(gpu_state, orc_state, zero=()):
    """max |gpu - oracle| per field relative to that field's own max |oracle|
    (strict per field); a momentum or face-B component below
    DEGENERATE_FRACTION of its group's largest component, or named in
    `zero` (a component the problem keeps at zero in exact arithmetic, whose
    values are rounding noise of either code), is taken relative to the
    group scale instead."""
    c5g, *bg = gpu_state
    c5o, bo, mscale, bscale = _scales(orc_state)
    out = {}
    for m in range(5):
        own = float(np.abs(c5o[m]).max())
        if m in (1, 2, 3):
            sc = mscale if FIELDS[m] in zero else max(own, DEGENERATE_FRACTION * mscale)
        else:
            sc = own
        d = float(np.abs(c5g[m] - c5o[m]).max())
        out[FIELDS[m]] = d / sc if sc > 0 else d
    for a in range(3):
        own = float(np.abs(bo[a]).max())
        sc = bscale if FIELDS[5 + a] in zero else max(own, DEGENERATE_FRACTION * bscale)
        d = float(np.abs(bg[a] - bo[a]).max())
        out[FIELDS[5 + a]] = d / sc if sc > 0 else d
    return out


def field_errors_group(gpu_state, orc_state):
    """The same maxima relative to the group scale: rho and E to their own
    max, each momentum component to the largest momentum component, each
    face-B component to the largest face-B component (the vector-scaled
    form, reported beside the strict one)."""
    c5g, *bg = gpu_state
    c5o, bo, mscale, bscale = _scales(orc_state)
    out = {}
    for m in range(5):
        sc = mscale if m in (1, 2, 3) else float(np.abs(c5o[m]).max())
        d = float(np.abs(c5g[m] - c5o[m]).max())
        out[FIELDS[m]] = d / sc if sc > 0 else d
    for a in range(3):
        d = float(np.abs(bg[a] - bo[a]).max())
        out[FIELDS[5 + a]] = d / bscale if bscale > 0 else d
    return out


def field_l1(gpu_state, orc_state):
    """mean |gpu - oracle| / mean |oracle| per field (0 where the oracle
    field is zero and the difference too)."""
    c5g, *bg = gpu_state
    c5o, *bo = orc_state
    out = {}
    for m in range(5):
        den = float(np.abs(c5o[m]).mean())
        d = float(np.abs(c5g[m] - c5o[m]).mean())
        out[FIELDS[m]] = d / den if den > 0 else d
    for a in range(3):
        den = float(np.abs(bo[a]).mean())
        d = float(np.abs(bg[a] - bo[a]).mean())
        out[FIELDS[5 + a]] = d / den if den > 0 else d
    return out


def l1_rel(a, b):
    return float(np.abs(a - b).mean() / np.abs(b).mean())
