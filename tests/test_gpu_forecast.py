"""GPU tests of the refinement forecaster kernels against the oracle:
element features and criterion levels, the flag combination (bit-exact),
the network's forward pass, its back-propagated gradient (FP32 kernels vs the
FP64 oracle) and Adam, and a short training run that must lower the loss."""

import sys

import numpy as np
import pytest

from harness import match, oracle_mesh
from oracle import amr, assembly, forecast, mlp
from synth import cases

pytestmark = pytest.mark.gpu

SCALE = np.array([1.0, 1e3, 1e3, 0.05, 1.0, 1.0, 1.0, 20.0, 1e3, 1e4, 1e3, 1e3, 0.05, 0.5,
                  1e4, 1.0])


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name,kw,criterion", [("small_amr3", {}, 1), ("small_amr3", {"N": 7}, 0),
                                               ("vortex_8x8x4_n4", {}, 1),
                                               ("small_amr2", {"periodic": False}, 1)])
def test_features_match_oracle(name, kw, criterion):
    import torch
    from paper_2410_21607_amd import api
    c = cases.get(name, **kw)
    say("features", name, kw, criterion)
    gm = api.Mesh.from_case(c)
    _, _, z = gm.coords()
    bg = cases.reference_state(c, z)
    gm.set_reference(bg["rho0"], bg["theta0"], bg["dtheta0dz"])
    om = oracle_mesh(c)
    perm = match(om.node_xyz, gm.node_xyz(), c)
    q = cases.initial_state(c, om.node_xyz)
    rng = np.random.default_rng(1)
    qp = q * (1.0 + 0.05 * rng.standard_normal(q.shape))
    ne = gm.info["n_elem"]
    ref = cases.reference_state(c, om.zl)
    ref_local = dict(rho0=ref["rho0"], theta0=ref["theta0"])
    qL, qLp = assembly.scatter(om, q), assembly.scatter(om, qp)
    crit = amr.criterion_speed(qL) if criterion == 0 else amr.criterion_vorticity(om, qL)
    cmax = crit.reshape(ne, -1).max(1)
    # thresholds in gaps between element maxima (so round-off cannot flip dem)
    srt = np.unique(cmax)
    gaps = np.argsort(np.diff(srt))[::-1][:2]
    thr = np.sort(0.5 * (srt[gaps] + srt[gaps + 1]))
    plain = rng.integers(-1, 2, size=ne).astype(np.int8)
    want, dem_o = forecast.features(om, qL, qLp, plain, ref_local, c["phys"], criterion, thr, 2, SCALE)
    feat = torch.zeros(ne * 16, dtype=torch.float32, device="cuda")
    dem = torch.zeros(ne, dtype=torch.int8, device="cuda")
    api.amr_features(gm, gm.unpack(q[:, perm]), gm.unpack(qp[:, perm]),
                     torch.as_tensor(plain).cuda(), criterion, thr, 2, SCALE, feat, dem)
    torch.cuda.synchronize()
    got = feat.cpu().numpy().reshape(ne, 16).astype(np.float64)
    err = np.abs(got - want) / (np.abs(want) + 1e-3)
    say("  worst relative error per feature", err.max(0))
    assert np.all(np.abs(got - want) <= 2e-6 * np.abs(want) + 1e-6)
    np.testing.assert_array_equal(dem.cpu().numpy(), dem_o)


@pytest.mark.parametrize("seed", range(3))
def test_forecast_flags_match_oracle(seed):
    import torch
    from paper_2410_21607_amd import api
    c = cases.get("small_amr3", N=3)
    gm = api.Mesh.from_case(c)
    ne, nc = gm.info["n_elem"], gm.info["n_col"]
    rng = np.random.default_rng(seed)
    logits = rng.standard_normal((ne, 3)).astype(np.float32)
    logits[::7, 1] = logits[::7, 0]         # ties
    plain = rng.integers(-1, 2, size=ne).astype(np.int8)
    if seed == 2:
        plain[:] = -1
        logits[:, 0] = 5.0                  # whole families coarsen
    ae = torch.zeros(ne, dtype=torch.int8, device="cuda")
    ac = torch.zeros(nc, dtype=torch.int8, device="cuda")
    api.amr_forecast_flags(gm, torch.as_tensor(logits).cuda(), torch.as_tensor(plain).cuda(), 2, ae, ac)
    torch.cuda.synchronize()
    lv = np.repeat(np.asarray(c["columns"])[:, 0], c["z_edges"].size - 1)
    we, wc = forecast.forecast_flags(logits, plain, lv, 2, c["columns"], c["z_edges"].size - 1)
    np.testing.assert_array_equal(ae.cpu().numpy(), we)
    np.testing.assert_array_equal(ac.cpu().numpy(), wc)
    if seed == 2:
        assert (wc == -1).any()


def _mlp_case(seed, n=1000):
    rng = np.random.default_rng(seed)
    p = (rng.standard_normal(mlp.N_PARAM) * 0.3).astype(np.float32)
    x = rng.standard_normal((n, 16)).astype(np.float32)
    y = rng.integers(0, 3, size=n).astype(np.int8)
    return p, x, y


@pytest.mark.parametrize("seed,n,use_idx", [(0, 1000, False), (1, 4096, True), (2, 1, False),
                                            (3, 257, True)])
def test_mlp_forward_and_gradient_match_oracle(seed, n, use_idx):
    import torch
    from paper_2410_21607_amd import api
    p, x, y = _mlp_case(seed, n)
    say("mlp", seed, n, use_idx)
    P, X, Y = (torch.as_tensor(a).cuda() for a in (p, x, y))
    logits = torch.zeros(n * 3, dtype=torch.float32, device="cuda")
    api.mlp_forward(P, X, logits)
    z, _, _ = mlp.forward(p.astype(np.float64), x.astype(np.float64))
    got = logits.cpu().numpy().reshape(n, 3)
    assert np.max(np.abs(got - z)) <= 1e-5 * max(1.0, np.max(np.abs(z)))
    rng = np.random.default_rng(seed + 10)
    if use_idx:
        idx = rng.permutation(n)[: max(1, n // 3)].astype(np.int32)
        I = torch.as_tensor(idx).cuda()
        xs, ys = x[idx], y[idx]
    else:
        I, xs, ys = None, x, y
    nb = len(ys)
    work = torch.zeros(nb * api.MLP_WORK, dtype=torch.float32, device="cuda")
    grad = torch.zeros(mlp.N_PARAM, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    api.mlp_backward(P, X, Y, I, work, grad, loss)
    grad2 = torch.zeros_like(grad)
    api.mlp_backward(P, X, Y, I, work, grad2, loss)
    torch.cuda.synchronize()
    assert torch.equal(grad, grad2)          # fixed summation order
    L, g = mlp.gradient(p.astype(np.float64), xs.astype(np.float64), ys.astype(np.int64))
    gg = grad.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(gg - g) / np.linalg.norm(g)
    say("  loss", float(loss.item()), L, "grad rel", rel)
    assert abs(float(loss.item()) - L) <= 1e-5 * max(1.0, L)
    assert rel <= 1e-5
    for name, s in mlp.SHAPES:          # every block, not only the largest
        a, b = mlp.unflatten(gg)[name], mlp.unflatten(g)[name]
        assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b) + 1e-9, name


def test_adam_matches_oracle():
    import torch
    from paper_2410_21607_amd import api
    rng = np.random.default_rng(4)
    p = (rng.standard_normal(mlp.N_PARAM) * 0.3).astype(np.float32)
    P = torch.as_tensor(p).cuda()
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    po, mo, vo = p.astype(np.float64), np.zeros(mlp.N_PARAM), np.zeros(mlp.N_PARAM)
    for t in range(1, 6):
        g = (rng.standard_normal(mlp.N_PARAM) * 10.0 ** rng.uniform(-4, 0)).astype(np.float32)
        api.mlp_adam_step(P, torch.as_tensor(g).cuda(), M, V, t, lr=1e-2)
        po, mo, vo = mlp.adam(po, g.astype(np.float64), mo, vo, t, lr=1e-2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(P.cpu().numpy(), po, rtol=1e-5, atol=1e-6)


def test_gpu_training_lowers_the_loss():
    import torch
    from paper_2410_21607_amd import api
    rng = np.random.default_rng(5)
    x = rng.standard_normal((4096, 16)).astype(np.float32)
    y = np.digitize(x[:, 0] + 0.5 * x[:, 1], [-0.5, 0.5]).astype(np.int8)
    p = (rng.standard_normal(mlp.N_PARAM) * 0.1).astype(np.float32)
    P, X, Y = (torch.as_tensor(a).cuda() for a in (p, x, y))
    M, V = torch.zeros_like(P), torch.zeros_like(P)
    B = 512
    work = torch.zeros(B * api.MLP_WORK, dtype=torch.float32, device="cuda")
    grad = torch.zeros_like(P)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    losses = []
    t = 0
    for epoch in range(6):
        perm = torch.randperm(4096, device="cuda", generator=g).to(torch.int32)
        for b0 in range(0, 4096, B):
            t += 1
            api.mlp_backward(P, X, Y, perm[b0:b0 + B].contiguous(), work, grad, loss)
            api.mlp_adam_step(P, grad, M, V, t, lr=1e-2)
        losses.append(float(loss.item()))
    say("  losses", losses)
    assert losses[-1] < 0.25 * mlp.loss(p.astype(np.float64), x.astype(np.float64), y.astype(np.int64))
