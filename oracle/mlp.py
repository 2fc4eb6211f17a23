"""Small multilayer perceptron of the refinement forecaster (oracle, FP64 by
default; test infrastructure only).

The paper motivates better refinement criteria without specifying a learned
one; the forecaster here is a three-layer perceptron 16 -> 64 -> 64 -> 3
with tanh activations, trained with the softmax cross-entropy on three
classes (coarsen, keep, refine) by Adam.  This module writes the textbook
definitions out:

  z1 = W1 x + b1,  h1 = tanh(z1)
  z2 = W2 h1 + b2, h2 = tanh(z2)
  z3 = W3 h2 + b3  (logits)
  loss = mean over the batch of -log softmax(z3)[label]

Back-propagation is the chain rule with d tanh(z)/dz = 1 - tanh(z)^2 and
d loss / d z3 = (softmax(z3) - onehot(label)) / B.  Adam (Kingma & Ba) with
bias-corrected moments:
  m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2
  p <- p - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)

Parameters travel as one flat vector in the order W1 (64x16, row-major),
b1, W2 (64x64), b2, W3 (3x64), b3.
"""

import numpy as np

N_IN, N_HID, N_OUT = 16, 64, 3
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(p):
    out, o = {}, 0
    for name, s in SHAPES:
        n = int(np.prod(s))
        out[name] = p[o:o + n].reshape(s)
        o += n
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[name]).reshape(-1) for name, _ in SHAPES])


def forward(p, x):
    """Logits (B, 3) and the hidden activations."""
    P = unflatten(p)
    h1 = np.tanh(x @ P["W1"].T + P["b1"])
    h2 = np.tanh(h1 @ P["W2"].T + P["b2"])
    z3 = h2 @ P["W3"].T + P["b3"]
    return z3, h1, h2


def softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def loss(p, x, label):
    """Mean cross-entropy; label in {0, 1, 2} (coarsen, keep, refine)."""
    z3, _, _ = forward(p, x)
    zs = z3 - z3.max(axis=1, keepdims=True)
    logp = zs - np.log(np.exp(zs).sum(axis=1, keepdims=True))
    return -np.mean(logp[np.arange(len(label)), label])


def gradient(p, x, label):
    """(loss, d loss / d p) by back-propagation."""
    P = unflatten(p)
    z3, h1, h2 = forward(p, x)
    B = x.shape[0]
    d3 = softmax(z3)
    d3[np.arange(B), label] -= 1.0
    d3 /= B
    g = {"W3": d3.T @ h2, "b3": d3.sum(axis=0)}
    d2 = (d3 @ P["W3"]) * (1.0 - h2 * h2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ P["W2"]) * (1.0 - h1 * h1)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(axis=0)
    return loss(p, x, label), flatten(g)


def adam(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1**t)
    vh = v / (1.0 - beta2**t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
