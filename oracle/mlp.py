"""Oracle (test infrastructure only): plain binary64 multilayer perceptron
alpha(x) ~ N_theta(x) (Sec. 3.2, eq:nn_apprx), its hand-written backward
pass and the Adam update used to train it.

Parameter layout (shared convention with the solver's C-ABI, not code): for
each layer l, the weight W_l (out x in, row-major) then the bias b_l (out),
all layers concatenated.  Hidden layers use `hidden_act` ('tanh', or
'relu' as in the velocity-profile network of Sec. 5.2); the output layer
applies `out_act` ('none' or 'sigmoid') and then y = shift + scale * act(z).
"""
from __future__ import annotations

import numpy as np


class Spec:
    def __init__(self, widths, out_act="none", out_scale=1.0, out_shift=0.0, hidden_act="tanh"):
        self.widths = list(widths)
        self.out_act = out_act
        self.hidden_act = hidden_act
        self.out_scale = float(out_scale)
        self.out_shift = float(out_shift)

    @property
    def n_params(self):
        return sum(o * i + o for i, o in zip(self.widths[:-1], self.widths[1:]))

    def unpack(self, params):
        p = np.asarray(params, dtype=np.float64)
        out, off = [], 0
        for i, o in zip(self.widths[:-1], self.widths[1:]):
            W = p[off:off + o * i].reshape(o, i)
            off += o * i
            b = p[off:off + o]
            off += o
            out.append((W, b))
        return out


def init_params(spec, seed):
    """Uniform(-1/sqrt(in), 1/sqrt(in)) weights and biases (seeded)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in zip(spec.widths[:-1], spec.widths[1:]):
        r = 1.0 / np.sqrt(i)
        parts.append(rng.uniform(-r, r, size=o * i))
        parts.append(rng.uniform(-r, r, size=o))
    return np.concatenate(parts)


def forward(spec, params, x):
    """x: (n, d_in).  Returns y (n, d_out) and the per-layer activations."""
    layers = spec.unpack(params)
    h = np.asarray(x, dtype=np.float64)
    acts = [h]
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        if li < len(layers) - 1:
            h = np.tanh(z) if spec.hidden_act == "tanh" else np.maximum(z, 0.0)
        elif spec.out_act == "sigmoid":
            h = 1.0 / (1.0 + np.exp(-z))
        else:
            h = z
        acts.append(h)
    y = spec.out_shift + spec.out_scale * acts[-1]
    return y, acts


def backward(spec, params, acts, dy):
    """Gradient of sum(dy * y) with respect to the parameters (same layout)."""
    layers = spec.unpack(params)
    L = len(layers)
    h_out = acts[-1]
    dz = np.asarray(dy, dtype=np.float64) * spec.out_scale
    if spec.out_act == "sigmoid":
        dz = dz * h_out * (1.0 - h_out)
    grads = [None] * L
    for li in range(L - 1, -1, -1):
        W, _ = layers[li]
        h_in = acts[li]
        gW = dz.T @ h_in
        gb = dz.sum(axis=0)
        grads[li] = (gW, gb)
        if li > 0:
            dh = dz @ W
            if spec.hidden_act == "tanh":
                dz = dh * (1.0 - h_in * h_in)     # tanh'(z) = 1 - tanh(z)^2
            else:
                dz = dh * (h_in > 0.0)            # relu'(z) = 1 for z > 0, else 0
    return np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in grads])


def adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba); step counts from 1.  In place."""
    m *= beta1
    m += (1.0 - beta1) * grad
    v *= beta2
    v += (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    params -= lr * mh / (np.sqrt(vh) + eps)
    return params
