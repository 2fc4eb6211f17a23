"""Pins of the oracle MLP (back-propagation and Adam) by what the mathematics
fixes: central finite differences of the loss (the network is smooth), the
zero-sum property of the softmax cross-entropy gradient, a one-layer special
case with a closed form, and Adam's first step."""

import numpy as np

from oracle import mlp


def params(seed, scale=0.5):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(mlp.N_PARAM) * scale


def test_parameter_count():
    assert mlp.N_PARAM == 64 * 16 + 64 + 64 * 64 + 64 + 3 * 64 + 3 == 5443
    p = params(0)
    np.testing.assert_array_equal(mlp.flatten(mlp.unflatten(p)), p)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = params(1, 0.3)
    x = rng.standard_normal((7, 16))
    lab = rng.integers(0, 3, size=7)
    L0, g = mlp.gradient(p, x, lab)
    assert abs(L0 - mlp.loss(p, x, lab)) < 1e-15
    idx = rng.choice(mlp.N_PARAM, size=120, replace=False)
    # include every bias block and the last layer
    idx = np.unique(np.concatenate([idx, np.arange(1024, 1088), np.arange(5440, 5443),
                                    np.arange(5248, 5260)]))
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, x, lab) - mlp.loss(p - e, x, lab)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-8 + 1e-6 * abs(fd), (i, fd, g[i])


def test_logit_gradient_sums_to_zero():
    """d loss / d b3 = mean(softmax - onehot): its components sum to zero."""
    rng = np.random.default_rng(2)
    p = params(2)
    x = rng.standard_normal((33, 16))
    lab = rng.integers(0, 3, size=33)
    _, g = mlp.gradient(p, x, lab)
    assert abs(g[-3:].sum()) < 1e-15


def test_closed_form_with_zero_hidden_weights():
    """With W1 = W2 = 0 and b1 = b2 = 0 the hidden layers are zero, so the
    logits are b3 and d loss / d b3 = softmax(b3) - mean onehot exactly."""
    P = {k: np.zeros(s) for k, s in mlp.SHAPES}
    P["b3"] = np.array([0.3, -1.1, 2.0])
    p = mlp.flatten(P)
    lab = np.array([0, 2, 2, 1, 0])
    x = np.random.default_rng(3).standard_normal((5, 16))
    L, g = mlp.gradient(p, x, lab)
    s = np.exp(P["b3"]) / np.exp(P["b3"]).sum()
    want = s - np.bincount(lab, minlength=3) / 5.0
    np.testing.assert_allclose(g[-3:], want, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(L, -np.mean(np.log(s[lab])), rtol=1e-14)
    assert not g[:-3].any()


def test_adam_first_step():
    """At t = 1 the bias-corrected moments are g and g^2, so every parameter
    moves by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(4)
    p = params(4)
    g = rng.standard_normal(mlp.N_PARAM)
    p1, m, v = mlp.adam(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr=1e-2)
    np.testing.assert_allclose(p1, p - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_training_lowers_the_loss():
    """A separable three-class problem is learned by a few hundred steps."""
    rng = np.random.default_rng(5)
    x = rng.standard_normal((256, 16))
    lab = np.digitize(x[:, 0] + 0.5 * x[:, 1], [-0.5, 0.5])
    p = params(5, 0.1)
    m, v = np.zeros_like(p), np.zeros_like(p)
    L0 = mlp.loss(p, x, lab)
    for t in range(1, 301):
        _, g = mlp.gradient(p, x, lab)
        p, m, v = mlp.adam(p, g, m, v, t, lr=1e-2)
    assert mlp.loss(p, x, lab) < 0.2 * L0
