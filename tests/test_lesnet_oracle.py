"""Pins of the FP64 network oracle (oracle/lesnet.py).

conv3 against scipy's correlation (a library routine realizing the same
definition channel pair by channel pair), pooling and the transposed
convolution against closed forms, the whole backward pass against central
finite differences, Adam against its closed form for a constant gradient.
"""
import numpy as np
import pytest
from scipy import ndimage

from oracle import lesnet as N


def test_conv3_matches_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((4, 5, 6, 3))
    W = rng.standard_normal((27, 3, 2))
    b = rng.standard_normal(2)
    y = N.conv3(x, W, b)
    for co in range(2):
        want = np.full(x.shape[:3], b[co])
        for ci in range(3):
            k = W[:, ci, co].reshape(3, 3, 3)   # t = 9(dz+1) + 3(dy+1) + (dx+1)
            want += ndimage.correlate(x[..., ci], k, mode="constant", cval=0.0)
        assert np.allclose(y[..., co], want, rtol=1e-12, atol=1e-12)


def test_pool_and_up_closed_forms():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 4, 8, 2))
    y, idx = N.pool(x)
    want = x.reshape(2, 2, 2, 2, 4, 2, 2).max(axis=(1, 3, 5))
    assert np.array_equal(y, want)
    # transposed conv of a one-hot input places U[s] at 2v + s
    U = rng.standard_normal((8, 2, 3))
    z = np.zeros((2, 2, 2, 2))
    z[1, 0, 1, 1] = 1.0
    u = N.up(z, U, np.zeros(3))
    for s, (dz, dy, dx) in enumerate(N.SUB):
        assert np.array_equal(u[2 + dz, 0 + dy, 2 + dx], U[s, 1])
    assert np.count_nonzero(np.abs(u).sum(-1)) == 8


def _tiny():
    p = N.init_params(seed=3, c1=2, c2=3, c3=4)
    for k in p:                      # non-zero biases so their gradients are tested
        if k.endswith(".b"):
            p[k] = np.random.default_rng(len(k)).standard_normal(p[k].shape) * 0.1
    x = np.random.default_rng(5).standard_normal((4, 8, 8, 3))
    t = np.random.default_rng(6).standard_normal((4, 8, 8, 1))
    return p, x, t


def test_backward_matches_finite_differences():
    """P16: every weight tensor's gradient against central differences."""
    p, x, t = _tiny()
    y, c = N.forward(p, x)
    loss, dy = N.mse(y, t)
    g = N.backward(p, c, dy)
    rng = np.random.default_rng(9)
    h = 1e-6
    for name in p:
        flat = p[name].reshape(-1)
        for q in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[q]
            flat[q] = old + h
            lp, _ = N.mse(N.forward(p, x)[0], t)
            flat[q] = old - h
            lm, _ = N.mse(N.forward(p, x)[0], t)
            flat[q] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[q]
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-9), (name, q)


def test_adam_constant_gradient_closed_form():
    p = {"w": np.array([1.0, -2.0])}
    opt = N.Adam(p, lr=0.01)
    g = {"w": np.array([0.5, -3.0])}
    for _ in range(7):
        opt.step(p, g)
    want = np.array([1.0, -2.0]) - 0.01 * 7 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(p["w"], want, rtol=1e-12)


def test_training_reduces_loss():
    """A few Adam steps on a fixed sample lower the loss (sanity)."""
    p, x, t = _tiny()
    opt = N.Adam(p, lr=1e-2)
    losses = []
    for _ in range(15):
        y, c = N.forward(p, x)
        loss, dy = N.mse(y, t)
        losses.append(loss)
        opt.step(p, N.backward(p, c, dy))
    assert losses[-1] < losses[0]
