"""FP64 oracle of the learned SOR warm start -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this module.  It shares no code with the GPU network
(``paper_1504_02264_amd/csrc/lesnet.hip``).

A small 3-D U-Net in plain numpy float64, written from the definitions of
its layers:

* conv3   y[v, co] = b[co] + sum_t sum_ci x[v + o_t, ci] W[t, ci, co], the 27
          offsets o_t = (dz, dy, dx) in {-1, 0, 1}^3, t = 9(dz+1) + 3(dy+1) +
          (dx+1), zero outside the grid ("same" padding)
* relu    max(x, 0)
* pool    2x2x2 max pooling (argmax kept for the backward pass; ties go to
          the first index in t = 4 dz + 2 dy + dx order)
* up      2x2x2 stride-2 transposed convolution:
          y[2v + s, co] = b[co] + sum_ci x[v, ci] U[s, ci, co], s = 4 dz + 2 dy + dx
* cat     channel concatenation [upsampled, skip]
* head    1x1x1 convolution to one channel

Network (channels c1, c2, c3 = 16, 32, 64 by default), input 3 channels:
  e1 = relu(conv3(relu(conv3(x))))                 level 1 (skip)
  e2 = relu(conv3(relu(conv3(pool(e1)))))          level 2 (skip)
  b  = relu(conv3(relu(conv3(pool(e2)))))          level 3
  d2 = relu(conv3(relu(conv3(cat(up(b), e2)))))
  d1 = relu(conv3(relu(conv3(cat(up(d2), e1)))))
  y  = head(d1)
Tensors are [D, H, W, C] (channels last).  D, H, W must be multiples of 4.

Loss: mean squared error over the voxels.  Optimiser: Adam (Kingma & Ba
2015) on float64 copies of the weights.
"""
from __future__ import annotations

import numpy as np

OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
SUB = [(dz, dy, dx) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]


def shift(x, off):
    """z[v] = x[v + off], zero outside (x is [D, H, W, C])."""
    dz, dy, dx = off
    D, H, W = x.shape[:3]
    z = np.zeros_like(x)
    zs = slice(max(0, -dz), D - max(0, dz))
    ys = slice(max(0, -dy), H - max(0, dy))
    xs = slice(max(0, -dx), W - max(0, dx))
    zs2 = slice(max(0, dz), D - max(0, -dz))
    ys2 = slice(max(0, dy), H - max(0, -dy))
    xs2 = slice(max(0, dx), W - max(0, -dx))
    z[zs, ys, xs] = x[zs2, ys2, xs2]
    return z


def conv3(x, W, b):
    y = np.zeros(x.shape[:3] + (W.shape[2],))
    for t, off in enumerate(OFFSETS):
        y += shift(x, off) @ W[t]
    return y + b


def conv3_backward(x, W, dy):
    """Gradients (dx, dW, db) of conv3 for the output gradient dy."""
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for t, off in enumerate(OFFSETS):
        xs = shift(x, off)
        dW[t] = xs.reshape(-1, x.shape[3]).T @ dy.reshape(-1, dy.shape[3])
        neg = (-off[0], -off[1], -off[2])
        dx += shift(dy @ W[t].T, neg)
    db = dy.reshape(-1, dy.shape[3]).sum(0)
    return dx, dW, db


def pool(x):
    D, H, W, C = x.shape
    blocks = np.stack([x[dz::2, dy::2, dx::2] for dz, dy, dx in SUB], axis=0)
    idx = np.argmax(blocks, axis=0)
    return np.take_along_axis(blocks, idx[None], 0)[0], idx


def pool_backward(dy, idx, shape):
    dx = np.zeros(shape)
    for s, (dz, dyy, dxx) in enumerate(SUB):
        dx[dz::2, dyy::2, dxx::2] = np.where(idx == s, dy, 0.0)
    return dx


def up(x, U, b):
    D, H, W, C = x.shape
    y = np.zeros((2 * D, 2 * H, 2 * W, U.shape[2]))
    for s, (dz, dy, dx) in enumerate(SUB):
        y[dz::2, dy::2, dx::2] = x @ U[s]
    return y + b


def up_backward(x, U, dy):
    dx = np.zeros_like(x)
    dU = np.zeros_like(U)
    for s, (dz, dyy, dxx) in enumerate(SUB):
        g = dy[dz::2, dyy::2, dxx::2]
        dx += g @ U[s].T
        dU[s] = x.reshape(-1, x.shape[3]).T @ g.reshape(-1, g.shape[3])
    db = dy.reshape(-1, dy.shape[3]).sum(0)
    return dx, dU, db


LAYERS = ("e1a", "e1b", "e2a", "e2b", "b1", "b2", "u2", "d2a", "d2b", "u1", "d1a", "d1b", "head")


def shapes(c1=16, c2=32, c3=64, cin=3):
    """Weight shapes: conv3 [27, Cin, Cout], up [8, Cin, Cout], head [Cin, 1]."""
    return {
        "e1a": (27, cin, c1), "e1b": (27, c1, c1),
        "e2a": (27, c1, c2), "e2b": (27, c2, c2),
        "b1": (27, c2, c3), "b2": (27, c3, c3),
        "u2": (8, c3, c2), "d2a": (27, 2 * c2, c2), "d2b": (27, c2, c2),
        "u1": (8, c2, c1), "d1a": (27, 2 * c1, c1), "d1b": (27, c1, c1),
        "head": (c1, 1),
    }


def init_params(seed=0, c1=16, c2=32, c3=64, cin=3):
    """He-normal weights from numpy PCG64(seed), zero biases (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {}
    for name, shp in shapes(c1, c2, c3, cin).items():
        fan_in = int(np.prod(shp[:-1]))
        p[name] = rng.standard_normal(shp) * np.sqrt(2.0 / fan_in)
        p[name + ".b"] = np.zeros(shp[-1])
    return p


def forward(p, x):
    """y [D, H, W, 1] and the cache of activations for backward."""
    c = {"x": x}
    c["e1a"] = np.maximum(conv3(x, p["e1a"], p["e1a.b"]), 0)
    c["e1b"] = np.maximum(conv3(c["e1a"], p["e1b"], p["e1b.b"]), 0)
    c["p1"], c["i1"] = pool(c["e1b"])
    c["e2a"] = np.maximum(conv3(c["p1"], p["e2a"], p["e2a.b"]), 0)
    c["e2b"] = np.maximum(conv3(c["e2a"], p["e2b"], p["e2b.b"]), 0)
    c["p2"], c["i2"] = pool(c["e2b"])
    c["b1"] = np.maximum(conv3(c["p2"], p["b1"], p["b1.b"]), 0)
    c["b2"] = np.maximum(conv3(c["b1"], p["b2"], p["b2.b"]), 0)
    c["u2"] = up(c["b2"], p["u2"], p["u2.b"])
    c["c2"] = np.concatenate([c["u2"], c["e2b"]], axis=3)
    c["d2a"] = np.maximum(conv3(c["c2"], p["d2a"], p["d2a.b"]), 0)
    c["d2b"] = np.maximum(conv3(c["d2a"], p["d2b"], p["d2b.b"]), 0)
    c["u1"] = up(c["d2b"], p["u1"], p["u1.b"])
    c["c1"] = np.concatenate([c["u1"], c["e1b"]], axis=3)
    c["d1a"] = np.maximum(conv3(c["c1"], p["d1a"], p["d1a.b"]), 0)
    c["d1b"] = np.maximum(conv3(c["d1a"], p["d1b"], p["d1b.b"]), 0)
    y = c["d1b"] @ p["head"] + p["head.b"]
    return y, c


def backward(p, c, dy):
    """Gradients of every weight and bias for the output gradient dy."""
    g = {}
    g["head"] = c["d1b"].reshape(-1, c["d1b"].shape[3]).T @ dy.reshape(-1, 1)
    g["head.b"] = dy.reshape(-1, 1).sum(0)
    d = dy @ p["head"].T

    def conv_relu_back(name, xin, d_out):
        dz = d_out * (c[name] > 0)
        dx, g[name], g[name + ".b"] = conv3_backward(xin, p[name], dz)
        return dx

    d = conv_relu_back("d1b", c["d1a"], d)
    d = conv_relu_back("d1a", c["c1"], d)
    c1 = p["u1"].shape[2]
    d_u1, d_skip1 = d[..., :c1], d[..., c1:]
    d, g["u1"], g["u1.b"] = up_backward(c["d2b"], p["u1"], d_u1)
    d = conv_relu_back("d2b", c["d2a"], d)
    d = conv_relu_back("d2a", c["c2"], d)
    c2 = p["u2"].shape[2]
    d_u2, d_skip2 = d[..., :c2], d[..., c2:]
    d, g["u2"], g["u2.b"] = up_backward(c["b2"], p["u2"], d_u2)
    d = conv_relu_back("b2", c["b1"], d)
    d = conv_relu_back("b1", c["p2"], d)
    d = pool_backward(d, c["i2"], c["e2b"].shape) + d_skip2
    d = conv_relu_back("e2b", c["e2a"], d)
    d = conv_relu_back("e2a", c["p1"], d)
    d = pool_backward(d, c["i1"], c["e1b"].shape) + d_skip1
    d = conv_relu_back("e1b", c["e1a"], d)
    conv_relu_back("e1a", c["x"], d)
    return g


def mse(y, target):
    n = y.size
    r = y - target
    return float((r * r).sum() / n), 2.0 * r / n


class Adam:
    """Adam (Kingma & Ba 2015) on float64 parameters."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = {k: np.zeros_like(v) for k, v in params.items()}
        self.v = {k: np.zeros_like(v) for k, v in params.items()}
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        for k in params:
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * grads[k]
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * grads[k] ** 2
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            params[k] = params[k] - self.lr * mh / (np.sqrt(vh) + self.eps)
