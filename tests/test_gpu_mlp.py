"""GPU parity of the learned flux correction: MFMA forward and backward
against the oracle's FP64 MLP with the same bfloat16 rounding points (and
against pure FP64), Adam, a training run, the data pipeline (coarsening,
time-weighted fine fluxes on coarse faces, features/targets) and the fused
gated correction inside the corrector step."""
import numpy as np
import pytest

from mhd_inputs import problems as P
from oracle import pyorc as O
from tests.gpu_util import field_errors, gpu_sim, host_state, needs_gpu
from tests.helpers import oracle_of

pytestmark = [pytest.mark.gpu, needs_gpu]


def _t(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype or torch.float32, device="cuda")


def _params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, O.MLP_NPARAM)


def test_mlp_forward_matches_oracle():
    from paper_1502_02935_amd import mlp_forward
    p = _params(1).astype(np.float32).astype(np.float64)
    x = np.random.default_rng(2).normal(size=(4096 + 37, 32)).astype(np.float32).astype(np.float64)
    y = mlp_forward(_t(x), _t(p)).cpu().numpy().astype(np.float64)
    yb = O.mlp_forward(p, x, bf16_round=True)
    y64 = O.mlp_forward(p, x, bf16_round=False)
    scale = np.abs(yb).max()
    # same bf16 rounding points; an activation whose FP32 and FP64 values
    # straddle a bf16 rounding boundary differs by one bf16 ulp (2^-8)
    assert np.abs(y - yb).max() <= 5e-3 * scale
    assert np.abs(y - yb).mean() <= 2e-4 * scale
    assert np.abs(y - y64).max() <= 5e-2 * scale


def test_mlp_gradient_matches_oracle():
    import torch
    from paper_1502_02935_amd import MlpTrainer
    rng = np.random.default_rng(3)
    p = _params(4).astype(np.float32).astype(np.float64)
    n = 1000
    x = rng.normal(size=(n, 32)).astype(np.float32).astype(np.float64)
    t = rng.normal(size=(n, 8)).astype(np.float32).astype(np.float64)
    tr = MlpTrainer(_t(p))
    g, loss = tr.gradient(_t(x), _t(t))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    yb = O.mlp_forward(p, x, bf16_round=True)
    dy = 2.0 * (yb - t) / (n * 8)
    gb = O.mlp_backward(p, x, dy, bf16_round=True)
    g64 = O.mlp_backward(p, x, 2.0 * (O.mlp_forward(p, x) - t) / (n * 8))
    assert abs(float(loss.item()) - np.mean((yb - t) ** 2)) <= 1e-3 * np.mean((yb - t) ** 2)
    for lo, hi in ((0, 2048), (2048, 2112), (2112, 6208), (6208, 6272), (6272, 6784), (6784, 6792)):
        sc = np.abs(gb[lo:hi]).max()
        assert np.abs(g[lo:hi] - gb[lo:hi]).max() <= 1e-2 * sc, (lo, hi)
        assert np.abs(g[lo:hi] - g64[lo:hi]).max() <= 5e-2 * np.abs(g64[lo:hi]).max(), (lo, hi)


def test_adam_update():
    import torch
    from paper_1502_02935_amd import MlpTrainer
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=O.MLP_NPARAM).astype(np.float32)
    tr = MlpTrainer(_t(p0), lr=1e-2)
    g = rng.normal(size=O.MLP_NPARAM).astype(np.float32)
    tr.grad.copy_(_t(g))
    from paper_1502_02935_amd import _lib as L
    import ctypes as C
    from paper_1502_02935_amd.sim import _ptr, _stream
    for step in (1, 2):
        L.check(tr.lib.mhd_mlp_adam(_ptr(tr.params), _ptr(tr.m), _ptr(tr.v), _ptr(tr.grad), step,
                                    1e-2, 0.9, 0.999, 1e-8, _stream(tr.params.device)), "adam")
    torch.cuda.synchronize()
    m = np.zeros(O.MLP_NPARAM)
    v = np.zeros(O.MLP_NPARAM)
    p = p0.astype(np.float64)
    for step in (1, 2):
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g * g
        p = p - 1e-2 * (m / (1 - 0.9 ** step)) / (np.sqrt(v / (1 - 0.999 ** step)) + 1e-8)
    np.testing.assert_allclose(tr.params.cpu().numpy(), p, rtol=1e-5, atol=1e-6)


def test_training_reduces_loss():
    """Fit the outputs of a random teacher network: the MFMA backward and
    Adam drive the loss down."""
    import torch
    from paper_1502_02935_amd import MlpTrainer
    rng = np.random.default_rng(6)
    teacher = _params(7, 0.2)
    x = rng.normal(size=(8192, 32))
    t = O.mlp_forward(teacher, x)
    tr = MlpTrainer(_t(_params(8, 0.1)), lr=3e-3)
    xt, tt = _t(x), _t(t)
    first = None
    for it in range(300):
        loss = float(tr.step(xt, tt).item()) if it % 50 == 0 else tr.step(xt, tt)
        if it == 0:
            first = loss
    torch.cuda.synchronize()
    last = float(tr.gradient(xt, tt)[1].item())
    assert last < 0.2 * first, (first, last)


@pytest.mark.parametrize("outflow", [False, True])
def test_coarsen_matches_definition(outflow):
    pb = P.random_smooth((16, 12, 10), seed=9, bc=(P.OUTFLOW,) * 6) if outflow else \
        P.turbulent_ism(32, seed=9)
    s = gpu_sim(pb)
    s.step(2)
    fine = host_state(s)
    got = [t.cpu().numpy() for t in s.coarsen()]
    want = O.coarsen(*fine)
    for g, w in zip(got, want):
        np.testing.assert_allclose(g, w, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("bc", [(P.PERIODIC,) * 6, (P.OUTFLOW,) * 6])
def test_flux_accumulator_matches_oracle_fluxes(bc):
    """Sum over steps of dt times the mean fine corrector flux on each
    coarse face (at the lower side of a coarse cell), against the oracle's
    corrector fluxes."""
    pb = P.random_smooth((16, 12, 8), seed=10, bc=bc)
    o = oracle_of(pb)
    s = gpu_sim(pb)
    acc = s.flux_accumulator(True)
    want = np.zeros((3, 7, 4, 6, 8))
    dts = []
    for _ in range(2):
        dt = o.dt()
        dts.append(dt)
        o.step(dt)
        for a in range(3):
            t1, t2 = (a + 1) % 3, (a + 2) % 3
            gmap = [0, 1 + a, 1 + t1, 1 + t2, 4, 5 + t1, 5 + t2]
            for m in range(7):
                F = o.debug_array(8 * a + gmap[m])[2:-3, 2:-3, 2:-3]  # interior faces [z][y][x]
                F = np.moveaxis(F, (0, 1, 2), (0, 1, 2))
                # fine face (2I, ...) along a, 2x2 transverse average
                sl = [slice(None)] * 3
                sl[2 - a] = slice(0, None, 2)
                Fa = F[tuple(sl)]
                ax_t = [2 - t1, 2 - t2]
                for ax in sorted(ax_t):
                    shp = list(Fa.shape)
                    shp[ax:ax + 1] = [shp[ax] // 2, 2]
                    Fa = Fa.reshape(shp).mean(axis=ax + 1)
                want[a, m] += dt * Fa
    s.step(2, dt=dts)
    got = acc.cpu().numpy()
    for a in range(3):
        for m in range(7):
            sc = np.abs(want[a, m]).max() + 1e-300
            assert np.abs(got[a, m] - want[a, m]).max() <= 1e-11 * sc, (a, m)


@pytest.mark.parametrize("bc", [(P.PERIODIC,) * 6, (P.OUTFLOW,) * 6])
def test_samples_match_oracle_features_and_targets(bc):
    pb = P.random_smooth((16, 12, 10), seed=11, bc=bc)
    o = oracle_of(pb)
    s = gpu_sim(pb)
    s.set_full_fluxes(True)
    dt = o.dt()
    o.step(dt)
    s.step(1, dt=dt)
    rng = np.random.default_rng(12)
    n = 300
    faces = np.stack([rng.integers(0, 3, n), rng.integers(0, 16, n), rng.integers(0, 12, n),
                      rng.integers(0, 10, n)], axis=1).astype(np.int32)
    import torch
    acc = torch.as_tensor(rng.normal(0, 1e-3, (3, 7, 10, 12, 16)), dtype=torch.float64,
                          device="cuda")
    x, t, m = s.mlp_samples(acc, dt, _t(faces, torch.int32))
    x, t, m = x.cpu().numpy(), t.cpu().numpy(), m.cpu().numpy()
    W = [o.debug_array(33 + v) for v in range(8)]
    accn = acc.cpu().numpy()
    for b in range(n):
        a, i, j, k = faces[b]
        t1, t2 = (a + 1) % 3, (a + 2) % 3
        w8 = []
        for c in range(4):
            idx = [k + 2, j + 2, i + 2]
            idx[2 - a] += c - 2
            q = tuple(idx)
            w8 += [W[0][q], W[1 + a][q], W[1 + t1][q], W[1 + t2][q], W[4][q], W[5 + a][q],
                   W[5 + t1][q], W[5 + t2][q]]
        xf = O.mlp_features(np.array(w8), pb.gamma)
        np.testing.assert_allclose(x[b], xf, rtol=1e-5, atol=1e-6)
        gmap = [0, 1 + a, 1 + t1, 1 + t2, 4, 5 + t1, 5 + t2]
        Fc = np.array([o.debug_array(8 * a + gmap[mm])[k + 2, j + 2, i + 2] for mm in range(7)])
        df = accn[a, :, k, j, i] / dt - Fc
        yt = O.mlp_flux_to_out(np.array(w8), pb.gamma, df)
        np.testing.assert_allclose(t[b], yt, rtol=1e-4, atol=1e-5 * (np.abs(yt).max() + 1))
    assert set(np.unique(m)) <= {0, 1}
    # invalid faces are flagged, not read
    bad = _t(np.array([[3, 0, 0, 0], [0, 16, 0, 0], [1, 0, -1, 0]], dtype=np.int32), torch.int32)
    _, _, mb = s.mlp_samples(acc, dt, bad)
    assert list(mb.cpu().numpy()) == [2, 2, 2]


def test_samples_refused_without_kept_fluxes():
    """mhd_mlp_samples reads every component of the last corrector fluxes:
    refused (MHD_E_ARG) before the first step and after a fused step that
    kept only what the EMFs need; accepted once a step kept them all."""
    import torch
    from paper_1502_02935_amd import MHDError
    pb = P.random_smooth((16, 12, 10), seed=13)
    s = gpu_sim(pb)
    acc = torch.zeros((3, 7, 5, 6, 8), dtype=torch.float64, device="cuda")
    faces = _t(np.array([[0, 1, 2, 3], [2, 4, 5, 6]], dtype=np.int32), torch.int32)
    with pytest.raises(MHDError) as e:
        s.mlp_samples(acc, 1e-3, faces)
    assert e.value.code == -1
    s.step(1)
    with pytest.raises(MHDError) as e:
        s.mlp_samples(acc, 1e-3, faces)
    assert e.value.code == -1
    s.set_full_fluxes(True)
    s.step(1)
    x, t, m = s.mlp_samples(acc, 1e-3, faces)
    assert torch.isfinite(x).all() and torch.isfinite(t).all()


@pytest.mark.parametrize("case,precision", [("brio_wu", 0), ("box3d", 0), ("box3d", 1),
                                            ("blast3d", 0)])
def test_fused_correction_matches_oracle(case, precision):
    """A step with the gated, clipped MLP correction in the corrector sweep
    against the oracle's (FP64, bf16-rounded MLP): a shock tube (the gate
    acts), a smooth 3-D box (all three face families corrected, FP64 and
    FP32) and a 3-D box with an over-pressured sphere (gated faces in 3-D)."""
    import torch
    if case == "brio_wu":
        pb = P.brio_wu(64)
    else:
        pb = P.random_smooth((24, 20, 16), seed=13)
        if case == "blast3d":
            X, Y, Z = P.cell_centres(pb)
            hot = (X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2 < 0.2 ** 2
            pb.cell5[4][hot] += 10.0  # P raised by 6.7 inside the sphere
    params = _params(14, 0.05).astype(np.float32).astype(np.float64)
    o = oracle_of(pb)
    o.set_mlp(params, tau=0.5, jump=0.5, tau_flux=0.1)
    s = gpu_sim(pb, precision=precision)
    pt = _t(params)
    s.set_mlp(pt, tau=0.5, jump=0.5, tau_flux=0.1)
    dts = []
    for _ in range(3):
        dts.append(o.dt())
        o.step(dts[-1])
    s.step(3, dt=dts)
    err = field_errors(host_state(s), o.get_state())
    print("MLP_PARITY", case, precision, {k: float(v) for k, v in err.items()}, flush=True)
    tol = 2e-5 if precision == 0 else 1e-4
    assert max(err.values()) <= tol, err
    dg, do = s.diag(), o.diag()
    assert dg["n_mlp_faces"] > 0
    assert abs(dg["n_mlp_faces"] - do["n_mlp_faces"]) <= 0.001 * do["n_mlp_faces"]
    assert dg["n_mlp_gated"] == do["n_mlp_gated"]
    if case != "box3d":
        assert do["n_mlp_gated"] > 0


def _corner_blast(shape, seed):
    """A periodic smooth box with an over-pressured ball centred on the box
    corner, so that its shocks cross every periodic side (gated faces and
    shock flags on the sides, read at their images)."""
    pb = P.random_smooth(shape, seed=seed)
    X, Y, Z = P.cell_centres(pb)
    r2 = 0.0
    for c, x0, n, d in ((X, pb.x0, pb.nx, pb.dx), (Y, pb.y0, pb.ny, pb.dy),
                        (Z, pb.z0, pb.nz, pb.dz)):
        u = c - x0
        r2 = r2 + np.minimum(u, n * d - u) ** 2
    hot = r2 < (0.3 * min(pb.nx * pb.dx, pb.ny * pb.dy, pb.nz * pb.dz)) ** 2
    pb.cell5[4][hot] += 10.0
    return pb


COUNTERS = ("n_hll_fallback", "n_degenerate", "n_mlp_faces", "n_mlp_gated", "n_floor")


@pytest.mark.parametrize("shape", [(9, 7, 70), (10, 3, 2)])
def test_learned_step_reads_periodic_images(shape):
    """On a fully periodic box the learned step solves only the interior
    faces and reads every ghost at its interior image (no ghost layer, shell
    primitives or outer flux layer), counting each event as often as the
    full range holds copies of its face.  Bitwise the same state and event
    counts as the step that fills the ghost layers and solves the full range
    (full fluxes kept), whether the plain steps before it kept the ghosts or
    left them stale (then it refills them).  Also with periodic axes of 3
    and 2 cells, where the stencils wrap more than once."""
    pb = _corner_blast(shape, seed=15)
    params = _t(_params(14, 0.05).astype(np.float32))
    out, cnt = [], []
    # (full fluxes in the plain steps, in the learned step)
    for full_plain, full_mlp in ((False, False), (True, True), (False, True)):
        s = gpu_sim(pb, precision=1)
        s.set_full_fluxes(full_plain)
        s.step(2)
        s.set_full_fluxes(full_mlp)
        s.set_mlp(params, tau=0.5, jump=0.5, tau_flux=0.1)
        s.step(1)
        d = s.diag()
        assert d["n_mlp_faces"] > 0
        out.append(host_state(s))
        cnt.append({k: d[k] for k in COUNTERS})
    if min(shape) > 3:
        assert cnt[0]["n_mlp_gated"] > 0
    for o in out[1:]:
        for a, b in zip(out[0], o):
            np.testing.assert_array_equal(a, b)
    assert cnt[0] == cnt[1] == cnt[2], cnt


def test_samples_after_periodic_learned_step():
    """Training samples after a learned step on a fully periodic box that
    left the ghost layers stale (features, targets and shock masks read at
    the interior images) equal those after the same step with every ghost
    layer filled, on every face of the box's sides and a random set inside."""
    import torch
    pb = _corner_blast((16, 12, 10), seed=11)
    params = _t(_params(14, 0.05).astype(np.float32))
    rng = np.random.default_rng(12)
    side = [(a, i, j, k) for a in range(3) for i in (0, 1, 15) for j in (0, 11) for k in (0, 9)]
    inner = np.stack([rng.integers(0, 3, 200), rng.integers(0, 16, 200),
                      rng.integers(0, 12, 200), rng.integers(0, 10, 200)], axis=1)
    faces = _t(np.concatenate([np.array(side), inner]).astype(np.int32), torch.int32)
    acc = torch.as_tensor(rng.normal(0, 1e-3, (3, 7, 10, 12, 16)), dtype=torch.float32,
                          device="cuda")
    res = []
    for full in (False, True):
        s = gpu_sim(pb, precision=1)
        s.set_full_fluxes(full)
        s.set_mlp(params, tau=0.5, jump=0.5, tau_flux=0.1)
        s.step(1, dt=1e-3)
        res.append([v.cpu().numpy() for v in s.mlp_samples(acc, 1e-3, faces)])
    assert (res[0][2] == 1).any()
    for a, b in zip(*res):
        np.testing.assert_array_equal(a, b)


def test_trained_network_beats_plain_coarse():
    """What the trained network gains: on a held-out turbulent box (seed 205,
    not used in training), 40 fine 256^3 steps against 20 coarse 128^3 steps
    from the coarse-grained start, forced to the fine pair-summed steps.  The
    learned coarse run is closer to the coarse-grained fine run than the
    plain coarse run (L1 of rho and E at least 5 % lower), stays physical,
    and runs faster than the fine run in fine-equivalent cell-updates/s."""
    import os

    import torch

    from paper_1502_02935_amd import learned

    w = os.path.join(os.path.dirname(learned.__file__), "weights", "mlp_turbulent256.npy")
    params = torch.as_tensor(np.load(w), dtype=torch.float32, device="cuda")
    r = learned.evaluate(P.turbulent_ism(256, seed=205), params, pairs=20, tau=0.1, jump=0.5)
    pl, le = r["plain"], r["learned"]
    assert pl["status"] == 0 and le["status"] == 0
    assert le["mlp_faces"] > 0
    for f in ("rho", "E"):
        assert le["L1"][f] <= 0.95 * pl["L1"][f], (f, le["L1"], pl["L1"])
    assert le["fine_equivalent_cell_updates_per_s"] > r["fine_cell_updates_per_s"]
