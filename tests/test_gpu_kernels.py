"""Kernel-level parity of the HIP device functions against the oracle:
HLLD on random face states and Eq. 12-14 reconstruction on random stencils."""
import numpy as np
import pytest

from mhd_inputs.problems import random_face_states
from oracle import pyorc as O
from tests.gpu_util import needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]


def _dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("gamma", [5.0 / 3.0, 1.4, 2.0])
def test_hlld_fp64_matches_oracle(gamma):
    import torch
    from paper_1502_02935_amd import hlld_batch
    wl, wr, bn = random_face_states(400_000, seed=21)
    fo, co = O.hlld_batch(wl, wr, bn, gamma)
    fg, cg = hlld_batch(_dev(wl, torch.float64), _dev(wr, torch.float64),
                        _dev(bn, torch.float64), gamma)
    torch.cuda.synchronize()
    fg = fg.cpu().numpy()
    cg = cg.cpu().numpy().astype(np.int32)
    scale = np.abs(fo).max(axis=1) + 1.0
    err = (np.abs(fg - fo).max(axis=1) / scale)
    # the kernel contracts a*b+c into FMAs (the oracle does not): 1-ulp
    # differences per operation, amplified only where S - S_M or a star
    # denominator is small
    assert np.percentile(err, 99.99) <= 1e-14, np.percentile(err, 99.99)
    assert err.max() <= 1e-11, err.max()
    # branch decisions (HLL fallback / degenerate) agree except where a
    # rounding-level difference straddles the threshold
    assert np.mean(cg != co) < 1e-5
    assert np.isfinite(fg).all()


def test_hlld_fp32_error_bound():
    import torch
    from paper_1502_02935_amd import hlld_batch
    wl, wr, bn = random_face_states(400_000, seed=22)
    # the FP32 kernel sees FP32-rounded inputs; the oracle gets the same
    wl32, wr32, bn32 = (np.asarray(x, np.float32).astype(np.float64) for x in (wl, wr, bn))
    fo, _ = O.hlld_batch(wl32, wr32, bn32, 5.0 / 3.0)
    fg, _ = hlld_batch(_dev(wl32, torch.float32), _dev(wr32, torch.float32),
                       _dev(bn32, torch.float32), 5.0 / 3.0)
    torch.cuda.synchronize()
    fg = fg.double().cpu().numpy()
    scale = np.abs(fo).max(axis=1) + 1.0
    err = np.abs(fg - fo).max(axis=1) / scale
    # FP32 unit roundoff 6e-8; the star states divide by S - S_M
    assert np.percentile(err, 99.9) <= 1e-5, np.percentile(err, 99.9)
    assert np.isfinite(fg).all()


@pytest.mark.parametrize("recon", [O.RECON_PAPER, O.RECON_KAPPA, O.RECON_FIRST])
def test_recon_matches_oracle(recon):
    import torch
    from paper_1502_02935_amd import recon_batch
    rng = np.random.default_rng(23)
    w4 = rng.normal(size=(200_000, 4))
    w4[::7] = np.cumsum(w4[::7], axis=1)  # monotone runs
    w4[::11, 2] = w4[::11, 1]               # zero slopes
    wlo, wro = O.recon_batch(w4, recon)
    wlg, wrg = recon_batch(_dev(w4, torch.float64), recon)
    torch.cuda.synchronize()
    scale = np.abs(w4).max(axis=1) + 1e-300
    assert (np.abs(wlg.cpu().numpy() - wlo) / scale).max() <= 4e-16
    assert (np.abs(wrg.cpu().numpy() - wro) / scale).max() <= 4e-16
    w32 = w4.astype(np.float32).astype(np.float64)
    wlo, wro = O.recon_batch(w32, recon)
    wlg, wrg = recon_batch(_dev(w32, torch.float32), recon)
    torch.cuda.synchronize()
    assert (np.abs(wlg.double().cpu().numpy() - wlo) / scale).max() <= 1e-6
    assert (np.abs(wrg.double().cpu().numpy() - wro) / scale).max() <= 1e-6
