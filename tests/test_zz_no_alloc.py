"""The allocation-free gradient entry point (pibm_mlp_grads_noalloc) against
pibm_mlp_grads: the same kernels on the same inputs, with the partial
gradients in the library's fixed device array instead of the network's
workspace, so the results must agree bit for bit.  Two calls in a row, the
second with a smaller batch (the array keeps the first call's contents);
a network created for small batches still takes a full batch; sizes beyond the
fixed maximum are refused."""
import numpy as np
import pytest

from paper_1502_01159_amd import pibm

pytestmark = pytest.mark.gpu


def _batch(torch, n, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.randn((n, pibm.MLP_IN), generator=g).to(torch.bfloat16).cuda()
    t = torch.randn((n, pibm.MLP_OUT), generator=g).cuda()
    return x, t


def test_noalloc_grads_match_workspace_grads():
    torch = pytest.importorskip("torch")
    assert torch.cuda.is_available()
    ref = pibm.Mlp(seed=11, max_batch=pibm.MLP_NOALLOC_MAX_BATCH)
    small = pibm.Mlp(seed=11, max_batch=64)            # same parameters, one gradient slot
    for n, seed in ((3001, 1), (130, 2)):              # ragged: not whole workgroups of 64
        x, t = _batch(torch, n, seed)
        print(f"noalloc grads: n = {n}", flush=True)
        loss_ref, g_ref = ref.grads(x, t)
        loss_na, g_na = ref.grads_noalloc(x, t)
        assert np.isfinite(g_ref).all() and np.abs(g_ref).max() > 0
        assert np.array_equal(g_na, g_ref)
        assert loss_na == loss_ref
        loss_sm, g_sm = small.grads_noalloc(x, t)      # beyond that network's max_batch
        assert np.array_equal(g_sm, g_ref)
        assert loss_sm == loss_ref
    with pytest.raises(pibm.PibmError):
        small.grads(*_batch(torch, 65, 3))             # the workspace entry point is bounded by max_batch
    x, t = _batch(torch, pibm.MLP_NOALLOC_MAX_BATCH + 1, 4)
    with pytest.raises(pibm.PibmError):
        ref.grads_noalloc(x, t)                        # beyond the fixed array: refused
    # the full maximum batch still works after a refused call
    x, t = _batch(torch, pibm.MLP_NOALLOC_MAX_BATCH, 5)
    loss_ref, g_ref = ref.grads(x, t)
    loss_na, g_na = ref.grads_noalloc(x, t)
    assert np.array_equal(g_na, g_ref) and loss_na == loss_ref
