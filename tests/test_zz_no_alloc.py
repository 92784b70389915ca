"""The allocation-free loss/gradient call (bc_mlp_loss_grad_noalloc) against
the allocating one (bc_mlp_loss_grad), through the C ABI: same kernels on the
same inputs, so the same bits; two calls in a row, the second with fewer
samples (the fixed scratch keeps the first call's contents, which must not
leak into the second); sizes beyond the limit are refused."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2008_05718_amd import binding as b

pytestmark = pytest.mark.gpu


def _samples(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.random((n, b.BC_MLP_IN), dtype=np.float32)
    Y = (rng.standard_normal((n, b.BC_MLP_OUT)) * 3).astype(np.float32)
    mask = (rng.random((n, b.BC_MLP_OUT)) < 0.8).astype(np.uint8)
    mask[0] = 1
    return X, Y, mask


def test_noalloc_matches_allocating_call():
    import torch
    torch.cuda.set_device(0)
    rng = np.random.default_rng(3)
    w = (rng.standard_normal(b.BC_MLP_PARAMS) * 0.3).astype(np.float32)
    wt = torch.from_numpy(w).cuda()
    stream = torch.cuda.current_stream()
    for n, seed in ((16384, 1), (1000, 2)):
        X, Y, mask = _samples(n, seed)
        ref_loss, ref_grad = b.bc_mlp_loss_grad(w, X, Y, mask)
        Xt, Yt, Mt = (torch.from_numpy(a).cuda() for a in (X, Y, mask))
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        grad = torch.full((b.BC_MLP_PARAMS,), float("nan"), dtype=torch.float32, device="cuda")
        b.bc_mlp_loss_grad_noalloc(wt, Xt, Yt, Mt, loss, grad, stream=stream)
        torch.cuda.synchronize()
        got_loss = float(loss.cpu()[0])
        got_grad = grad.cpu().numpy()
        print(f"[noalloc] n={n} loss {got_loss:.6g} vs {ref_loss:.6g}", flush=True)
        assert np.float32(got_loss).view(np.uint32) == np.float32(ref_loss).view(np.uint32)
        assert np.array_equal(got_grad.view(np.uint32), ref_grad.view(np.uint32))


def test_noalloc_refuses_sizes_beyond_its_scratch():
    import torch
    n = 16385
    X, Y, mask = (torch.zeros((n, k), dtype=dt, device="cuda")
                  for k, dt in ((5, torch.float32), (3, torch.float32), (3, torch.uint8)))
    w = torch.zeros(b.BC_MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros(b.BC_MLP_PARAMS, dtype=torch.float32, device="cuda")
    with pytest.raises(b.BCError) as ei:
        b.bc_mlp_loss_grad_noalloc(w, X, Y, mask, loss, grad)
    assert ei.value.status == 1 and "16384" in ei.value.message
