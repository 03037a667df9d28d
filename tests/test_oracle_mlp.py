"""Pins of the oracle network against finite differences and closed forms."""
import numpy as np
import pytest

from oracle import mlp as M


@pytest.mark.parametrize("widths,act,hidden", [([2, 64, 64, 2], "none", "tanh"), ([2, 128, 128, 1], "sigmoid", "tanh"),
                                               ([3, 16, 5], "none", "tanh"), ([1, 30, 30, 30, 1], "none", "relu")])
def test_backward_matches_finite_differences(widths, act, hidden):
    spec = M.Spec(widths, out_act=act, out_scale=0.8 if act == "sigmoid" else 1.0,
                  out_shift=0.1 if act == "sigmoid" else 0.0, hidden_act=hidden)
    p = M.init_params(spec, 1)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, size=(37, widths[0]))
    dy = rng.normal(size=(37, widths[-1]))
    y, acts = M.forward(spec, p, x)
    g = M.backward(spec, p, acts, dy)
    assert g.shape == p.shape
    h = 1e-6
    for _ in range(3):
        d = rng.normal(size=p.shape)
        fp = (M.forward(spec, p + h * d, x)[0] * dy).sum()
        fm = (M.forward(spec, p - h * d, x)[0] * dy).sum()
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g @ d) <= 1e-7 * max(1.0, abs(fd))
    # every individual parameter of the first layer
    for k in range(0, widths[0] * widths[1], 7):
        e = np.zeros_like(p)
        e[k] = h
        fd = ((M.forward(spec, p + e, x)[0] - M.forward(spec, p - e, x)[0]) * dy).sum() / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(fd))


def test_single_linear_layer_is_affine():
    spec = M.Spec([3, 4])
    rng = np.random.default_rng(3)
    W = rng.normal(size=(4, 3))
    b = rng.normal(size=4)
    p = np.concatenate([W.reshape(-1), b])
    x = rng.normal(size=(10, 3))
    y, _ = M.forward(spec, p, x)
    assert np.allclose(y, x @ W.T + b, atol=1e-14)
    # gradient of sum(y) wrt W is the column sums of x, per output row
    g = M.backward(spec, p, M.forward(spec, p, x)[1], np.ones((10, 4)))
    assert np.allclose(g[:12].reshape(4, 3), np.tile(x.sum(axis=0), (4, 1)))
    assert np.allclose(g[12:], 10.0)


def test_sigmoid_output_range():
    spec = M.Spec([2, 8, 1], out_act="sigmoid", out_scale=1.0, out_shift=0.0)
    p = M.init_params(spec, 4) * 50
    y, _ = M.forward(spec, p, np.random.default_rng(5).uniform(-1, 1, (100, 2)))
    assert np.all((y >= 0) & (y <= 1))


def test_adam_first_step_is_sign_step():
    # with m, v starting at 0 the bias-corrected first step is lr * sign(g)
    rng = np.random.default_rng(6)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    q = p.copy()
    M.adam(q, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=0.0)
    assert np.allclose(q, p - 0.01 * np.sign(g), atol=1e-15)
    # a constant gradient keeps the step at lr * sign(g)
    m, v = np.zeros(50), np.zeros(50)
    q = p.copy()
    for t in range(1, 6):
        M.adam(q, g, m, v, t, lr=0.01, eps=0.0)
    assert np.allclose(q, p - 5 * 0.01 * np.sign(g), atol=1e-12)


def test_relu_layer_closed_form():
    """A ReLU hidden layer is max(Wx + b, 0) (the velocity-profile network
    of Sec. 5.2): checked against the definition with weights that make half
    of the units inactive; the gradient through an inactive unit is zero."""
    rng = np.random.default_rng(7)
    W1 = rng.normal(size=(6, 1))
    b1 = np.array([-5.0, -5.0, -5.0, 5.0, 5.0, 5.0])      # units 0-2 off, 3-5 on for |x| < 1 / max|W|
    W1 *= 0.1
    W2 = rng.normal(size=(1, 6))
    b2 = rng.normal(size=1)
    p = np.concatenate([W1.reshape(-1), b1, W2.reshape(-1), b2])
    spec = M.Spec([1, 6, 1], hidden_act="relu")
    x = rng.uniform(-1, 1, size=(20, 1))
    y, acts = M.forward(spec, p, x)
    h = np.maximum(x @ W1.T + b1, 0.0)
    assert np.allclose(y, h @ W2.T + b2, atol=1e-14)
    assert not h[:, :3].any() and (h[:, 3:] > 0).all()
    g = M.backward(spec, p, acts, np.ones((20, 1)))
    gW1 = g[:6].reshape(6, 1)
    assert not gW1[:3].any()
    assert np.allclose(gW1[3:, 0], W2[0, 3:] * x.sum())
