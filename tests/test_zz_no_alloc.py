"""The gradient entry point without allocation (mhd_mlp_grad_noalloc) against
the workspace one (mhd_mlp_grad), through the C ABI: same kernels and the
same fixed reduction order, so the two must agree bit for bit.  Two calls in
a row, the second with fewer samples (its blocks read only rows of the
static array that it has just written), and the size limit."""
import ctypes as C

import numpy as np
import pytest

from tests.gpu_util import needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]


def _grad_with_workspace(lib, x, t, p, stream):
    import torch
    n = x.shape[0]
    nb = C.c_size_t()
    assert lib.mhd_mlp_grad_workspace_bytes(n, C.byref(nb)) == 0
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    g = torch.full((p.numel(),), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    rc = lib.mhd_mlp_grad(n, x.data_ptr(), t.data_ptr(), p.data_ptr(), g.data_ptr(),
                          loss.data_ptr(), ws.data_ptr(), ws.numel(), stream)
    assert rc == 0, rc
    return g, loss


def _grad_noalloc(lib, x, t, p, stream):
    import torch
    n = x.shape[0]
    g = torch.full((p.numel(),), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    rc = lib.mhd_mlp_grad_noalloc(n, x.data_ptr(), t.data_ptr(), p.data_ptr(), g.data_ptr(),
                                  loss.data_ptr(), stream)
    assert rc == 0, rc
    return g, loss


def test_grad_noalloc_equals_workspace_grad():
    import torch
    from paper_1502_02935_amd import _lib as L
    lib = L.load()
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(11)
    p = torch.as_tensor(rng.normal(0, 0.3, L.MLP_NPARAM), dtype=torch.float32, device="cuda")
    # first call: many blocks and a ragged last block; second: fewer samples
    for n in (20000 + 37, 700):
        x = torch.as_tensor(rng.normal(size=(n, 32)), dtype=torch.float32, device="cuda")
        t = torch.as_tensor(rng.normal(size=(n, 8)), dtype=torch.float32, device="cuda")
        g0, l0 = _grad_with_workspace(lib, x, t, p, stream)
        g1, l1 = _grad_noalloc(lib, x, t, p, stream)
        torch.cuda.synchronize()
        assert torch.isfinite(g0).all() and torch.isfinite(l0).all()
        assert torch.equal(g0, g1), (n, float((g0 - g1).abs().max()))
        assert torch.equal(l0, l1), (n, float(l0), float(l1))


def test_grad_noalloc_at_the_limit_and_beyond():
    import torch
    from paper_1502_02935_amd import _lib as L
    lib = L.load()
    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(12)
    p = torch.as_tensor(rng.normal(0, 0.3, L.MLP_NPARAM), dtype=torch.float32, device="cuda")
    n = L.MLP_NOALLOC_MAX
    x = torch.as_tensor(rng.normal(size=(n, 32)), dtype=torch.float32, device="cuda")
    t = torch.as_tensor(rng.normal(size=(n, 8)), dtype=torch.float32, device="cuda")
    g0, l0 = _grad_with_workspace(lib, x, t, p, stream)
    g1, l1 = _grad_noalloc(lib, x, t, p, stream)
    torch.cuda.synchronize()
    assert torch.equal(g0, g1) and torch.equal(l0, l1)
    # one sample above the limit: refused on the host before any launch
    g = torch.zeros(L.MLP_NPARAM, dtype=torch.float32, device="cuda")
    rc = lib.mhd_mlp_grad_noalloc(n + 1, x.data_ptr(), t.data_ptr(), p.data_ptr(),
                                  g.data_ptr(), None, stream)
    assert rc == L.MHD_E_WS
    assert lib.mhd_mlp_grad_noalloc(0, x.data_ptr(), t.data_ptr(), p.data_ptr(), g.data_ptr(),
                                    None, stream) == L.MHD_E_ARG
