"""Learned refinement forecaster: training data, training, inference.

The paper's refinement criterion (Section 4.1) decides from the current
state only, so a moving feature forces a rebuild at nearly every adaptation
interval.  The forecaster predicts, per element, the refinement decision
``horizon`` intervals ahead; a run driven by it rebuilds only every
``horizon`` intervals, with the forecast merged into the criterion's flags
(the criterion overrides every refinement the forecaster misses, and no
column is merged against the criterion).

Everything numerical runs in the HIP library: ``amr_features`` (16 features
per element), ``mlp_forward`` / ``mlp_backward`` / ``mlp_adam_step`` (the
16 -> 64 -> 64 -> 3 network), ``amr_forecast_flags`` (merge), and
``sem_forecast_labels`` (training classes from a later layout).  This module
only moves arrays between those calls.
"""

import numpy as np
import torch

from . import api

# scale of each raw feature (see amr_features): brings the workloads'
# typical magnitudes to order one
DEFAULT_SCALE = np.array([1.0, 1e3, 1e3, 0.05, 1.0, 1.0, 1.0, 20.0, 1e3, 1e4, 1e3, 1e3, 0.05,
                          0.5, 1e4, 1.0], dtype=np.float32)


def features(run, plain_elem, scale=DEFAULT_SCALE):
    """(feat (n_elem*16,) float32, dem (n_elem,) int8) for the run's state."""
    m = run.mesh
    ne = m.info["n_elem"]
    feat = torch.empty(ne * api.NFEAT, dtype=torch.float32, device="cuda")
    dem = torch.empty(ne, dtype=torch.int8, device="cuda")
    api.amr_features(m, run.q, run.q_prev, plain_elem, run.criterion, run.thresholds,
                     run.lvl_max, scale, feat, dem)
    return feat, dem


class Recorder:
    """``on_boundary`` hook of a plain-criterion run: keeps, at every
    boundary, the layout, the features and the criterion's levels."""

    def __init__(self, scale=DEFAULT_SCALE):
        self.scale = scale
        self.frames = []

    def __call__(self, run, plain_elem):
        feat, dem = features(run, plain_elem, self.scale)
        self.frames.append(dict(columns=run.mesh.columns.copy(), params=run.mesh.params,
                                feat=feat.cpu().numpy().reshape(-1, api.NFEAT),
                                dem=dem.cpu().numpy()))

    def samples(self, horizon):
        """(X (n, 16) float32, y (n,) int8): features at boundary t with the
        class the criterion asks for at boundary t + horizon."""
        X, Y = [], []
        for t in range(len(self.frames) - horizon):
            a, b = self.frames[t], self.frames[t + horizon]
            y = api.sem_forecast_labels(a["params"], a["columns"], b["columns"], b["dem"])
            X.append(a["feat"])
            Y.append(y)
        if not X:
            return np.zeros((0, api.NFEAT), np.float32), np.zeros(0, np.int8)
        return np.concatenate(X), np.concatenate(Y)


def balanced_subset(X, Y, n, seed=0):
    """n samples, a third of each class present; a class with fewer samples
    than its share is drawn with replacement (the refine class is rare)."""
    rng = np.random.default_rng(seed)
    present = [c for c in range(3) if np.any(Y == c)]
    idx = []
    for k, c in enumerate(present):
        cand = np.nonzero(Y == c)[0]
        share = n // len(present) + (1 if k < n % len(present) else 0)
        idx.append(rng.choice(cand, size=share, replace=cand.size < share))
    idx = rng.permutation(np.concatenate(idx)) if idx else np.zeros(0, np.int64)
    return X[idx], Y[idx]


def class_scores(pred, Y):
    """Per-class recall and precision of predictions against labels."""
    out = {}
    for c, name in enumerate(("coarsen", "keep", "refine")):
        t, p = (Y == c), (pred == c)
        out[name] = {"support": int(t.sum()),
                     "recall": float((t & p).sum() / t.sum()) if t.any() else None,
                     "precision": float((t & p).sum() / p.sum()) if p.any() else None}
    return out


class Forecaster:
    """Owns the network's parameters and Adam moments on the device."""

    def __init__(self, seed=0, scale=DEFAULT_SCALE, horizon=5):
        self.scale = np.asarray(scale, dtype=np.float32)
        self.horizon = int(horizon)
        g = torch.Generator().manual_seed(int(seed))
        parts = []
        for fan_out, fan_in in ((64, 16), (64, 64), (3, 64)):
            parts.append(torch.randn(fan_out * fan_in, generator=g) / np.sqrt(fan_in))
            parts.append(torch.zeros(fan_out))
        self.params = torch.cat(parts).to(torch.float32).cuda()
        assert self.params.numel() == api.MLP_NPARAM
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.losses = []

    def train(self, X, Y, epochs=20, batch=1024, lr=1e-3, seed=0):
        """Adam on the mean cross-entropy, shuffled mini-batches."""
        X = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32)).cuda()
        Y = torch.as_tensor(np.ascontiguousarray(Y, dtype=np.int8)).cuda()
        n = X.shape[0]
        B = min(batch, n)
        work = torch.empty(B * api.MLP_WORK, dtype=torch.float32, device="cuda")
        grad = torch.empty_like(self.params)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        g = torch.Generator(device="cuda")
        g.manual_seed(int(seed))
        for _ in range(epochs):
            perm = torch.randperm(n, device="cuda", generator=g).to(torch.int32)
            tot, cnt = 0.0, 0
            for b0 in range(0, n - B + 1, B):
                self.t += 1
                api.mlp_backward(self.params, X, Y, perm[b0:b0 + B].contiguous(), work, grad, loss)
                api.mlp_adam_step(self.params, grad, self.m, self.v, self.t, lr=lr)
                tot += float(loss.item())
                cnt += 1
            self.losses.append(tot / max(cnt, 1))
        return self.losses

    def predict(self, X):
        """Classes (argmax of the logits) for rows of X (numpy)."""
        Xd = torch.as_tensor(np.ascontiguousarray(X, dtype=np.float32)).cuda()
        logits = torch.empty(Xd.shape[0] * 3, dtype=torch.float32, device="cuda")
        api.mlp_forward(self.params, Xd, logits)
        return logits.cpu().numpy().reshape(-1, 3).argmax(axis=1)

    def __call__(self, run, plain_elem, plain_col):
        """Combined column flags for ``AdaptiveRun``."""
        feat, _ = features(run, plain_elem, self.scale)
        ne = run.mesh.info["n_elem"]
        logits = torch.empty(ne * 3, dtype=torch.float32, device="cuda")
        api.mlp_forward(self.params, feat.view(ne, api.NFEAT), logits)
        ae = torch.empty(ne, dtype=torch.int8, device="cuda")
        ac = torch.empty_like(plain_col)
        api.amr_forecast_flags(run.mesh, logits, plain_elem, run.lvl_max, ae, ac)
        return ac
