"""mlp_backward_noalloc (no caller workspace, the library's per-GPU array)
against mlp_backward (caller workspace), through the C ABI: two calls in a
row, the second with a smaller batch (the array keeps the first call's
entries, which must not leak into the second), a call at the largest
allowed batch, and the size limit.  Both run the same kernels in a fixed
summation order, so gradients and losses agree bit for bit."""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _data(rng, rows):
    import torch
    x = torch.as_tensor(rng.standard_normal((rows, 16)).astype(np.float32)).cuda()
    y = torch.as_tensor(rng.integers(0, 3, rows).astype(np.int8)).cuda()
    return x, y


def _both(P, X, Y, idx):
    import torch
    from paper_2410_21607_amd import api
    n = X.shape[0] if idx is None else idx.numel()
    work = torch.full((n * api.MLP_WORK,), float("nan"), dtype=torch.float32, device="cuda")
    g_ref = torch.zeros(api.MLP_NPARAM, dtype=torch.float32, device="cuda")
    l_ref = torch.zeros(1, dtype=torch.float32, device="cuda")
    api.mlp_backward(P, X, Y, idx, work, g_ref, l_ref)
    g = torch.full_like(g_ref, float("nan"))
    l = torch.full_like(l_ref, float("nan"))
    api.mlp_backward_noalloc(P, X, Y, idx, g, l)
    torch.cuda.synchronize()
    return g_ref, l_ref, g, l


def test_noalloc_backward_matches_workspace_backward():
    import torch
    from paper_2410_21607_amd import api, native
    rng = np.random.default_rng(21)
    P = torch.as_tensor((rng.standard_normal(api.MLP_NPARAM) * 0.3).astype(np.float32)).cuda()
    # first call: 1500 rows, all of them
    X, Y = _data(rng, 1500)
    say("noalloc call 1: 1500 samples")
    g_ref, l_ref, g, l = _both(P, X, Y, None)
    assert torch.isfinite(g_ref).all() and torch.equal(g, g_ref) and torch.equal(l, l_ref)
    # second call: a smaller batch drawn through an index list
    X2, Y2 = _data(rng, 700)
    idx = torch.as_tensor(rng.permutation(700)[:333].astype(np.int32)).cuda()
    say("noalloc call 2: 333 of 700 samples")
    g_ref, l_ref, g, l = _both(P, X2, Y2, idx)
    assert torch.isfinite(g_ref).all() and torch.equal(g, g_ref) and torch.equal(l, l_ref)
    # the largest batch the array holds
    X3, Y3 = _data(rng, native.SEM_MLP_NOALLOC_MAX)
    say("noalloc call 3:", native.SEM_MLP_NOALLOC_MAX, "samples")
    g_ref, l_ref, g, l = _both(P, X3, Y3, None)
    assert torch.equal(g, g_ref) and torch.equal(l, l_ref)
    # one sample more is refused before any launch
    X4, Y4 = _data(rng, native.SEM_MLP_NOALLOC_MAX + 1)
    with pytest.raises(native.SemError):
        api.mlp_backward_noalloc(P, X4, Y4, None, torch.zeros_like(g), torch.zeros_like(l))
