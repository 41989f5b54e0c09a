"""GPU parity of the warm-start network (matrix-core kernels through the C
ABI) against the FP64 oracle of oracle/lesnet.py.

Both sides get the same bfloat16-representable weights and inputs.  The
GPU rounds every activation and activation gradient to bfloat16 (unit
roundoff u = 2^-8) and accumulates in float32; the oracle keeps float64
throughout.  Each rounding perturbs a tensor by at most u relative per
element; independent perturbations through L rounding stages of unit gain
add in quadrature, so the relative L2 error of the output is about
u sqrt(L).  The forward pass has L = 13 rounded tensors on its longest
path (u sqrt(13) = 1.4e-2), the backward pass another 13 plus the
forward's (u sqrt(26) = 2.0e-2).  The bars below are those figures.

Whole-network gradients are compared in the linear regime only (every
ReLU on its linear branch): with random weights some ReLU signs and
pooling argmaxes sit within the forward's rounding band of their
threshold and may fall the other way on the GPU, which moves whole terms
of a gradient sum, so no rounding bar holds there.  The kernels of the
backward pass (input and weight gradients of each layer) are checked one
by one at 1e-5 on identical bfloat16 operands,
which covers their decisions exactly (test_op_conv3_forward_dgrad_wgrad,
test_op_up_forward_dgrad_wgrad).
"""
import numpy as np
import pytest
import torch

import paper_1504_02264_amd as les
from oracle import lesnet as N

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -8
TOL_FWD = U_BF16 * np.sqrt(13)
TOL_GRAD = U_BF16 * np.sqrt(26)


def bf16(a):
    return torch.from_numpy(np.asarray(a, np.float64)).to(torch.bfloat16).to(torch.float64).numpy()


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def make_params(seed, c=(16, 32, 64)):
    p = N.init_params(seed=seed, c1=c[0], c2=c[1], c3=c[2])
    rng = np.random.default_rng(seed + 100)
    for k in list(p):
        if k.endswith(".b"):
            p[k] = (rng.standard_normal(p[k].shape) * 0.05).astype(np.float32).astype(np.float64)
        elif k == "head":
            p[k] = p[k].astype(np.float32).astype(np.float64)
        else:
            p[k] = bf16(p[k])
    return p


def flat(p):
    return np.concatenate([np.concatenate([p[n].ravel(), p[n + ".b"].ravel()]) for n in N.LAYERS])


def unflat(v, c=(16, 32, 64)):
    out, o = {}, 0
    for n, shp in N.shapes(*c).items():
        k = int(np.prod(shp))
        out[n] = v[o:o + k].reshape(shp)
        o += k
        out[n + ".b"] = v[o:o + shp[-1]]
        o += shp[-1]
    assert o == v.size
    return out


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.fixture(scope="module")
def net():
    n = les.Net(seed=1)
    yield n
    n.close()


def test_param_count_matches_oracle(net):
    assert net.num_params == sum(int(np.prod(s)) + s[-1] for s in N.shapes().values())


@pytest.mark.parametrize("B,D,H,W", [(1, 8, 12, 16), (2, 4, 8, 4), (1, 16, 8, 12)])
def test_forward_parity(net, B, D, H, W):
    print(f"[lesnet_forward] B={B} D={D} H={H} W={W}", flush=True)
    p = make_params(7)
    net.set_params(flat(p))
    x = bf16(np.random.default_rng(B * 100 + D).standard_normal((B, D, H, W, 3)))
    y = net.forward(dev(x)).cpu().numpy()
    torch.cuda.synchronize()
    for b in range(B):
        yo, _ = N.forward(p, x[b])
        e = rel(y[b], yo[..., 0])
        print(f"  sample {b}: rel L2 {e:.3e} (bar {TOL_FWD:.3e})", flush=True)
        assert e <= TOL_FWD


def ambiguous_fraction(p, x):
    """Fraction of the network's discrete decisions (ReLU signs, pooling
    argmaxes) whose margin is within the forward error band of the GPU."""
    band = 2 * TOL_FWD
    tot = amb = 0
    for b in range(x.shape[0]):
        _, c = N.forward(p, x[b])
        ins = {"e1a": c["x"], "e1b": c["e1a"], "e2a": c["p1"], "e2b": c["e2a"], "b1": c["p2"],
               "b2": c["b1"], "d2a": c["c2"], "d2b": c["d2a"], "d1a": c["c1"], "d1b": c["d1a"]}
        for k, xin in ins.items():
            pre = N.conv3(xin, p[k], p[k + ".b"])
            amb += np.count_nonzero(np.abs(pre) < band * np.sqrt(np.mean(pre ** 2)))
            tot += pre.size
        for k in ("e1b", "e2b"):
            a = c[k]
            blocks = np.sort(np.stack([a[dz::2, dy::2, dx::2] for dz, dy, dx in N.SUB]), axis=0)
            amb += np.count_nonzero(blocks[-1] - blocks[-2] < band * np.sqrt(np.mean(a ** 2)))
            tot += blocks[-1].size
    return amb / tot


def test_gradient_parity_linear_regime(net):
    """Non-negative weights, inputs and positive biases keep every ReLU in
    its linear branch on both sides, so only rounding separates them (and
    the rare pooling near-tie)."""
    B, D, H, W = 1, 8, 8, 12
    rng = np.random.default_rng(17)
    p = {}
    for k, shp in N.shapes().items():
        fan = int(np.prod(shp[:-1]))
        w = rng.uniform(0, 2.0 / fan, shp)
        p[k] = w.astype(np.float32).astype(np.float64) if k == "head" else bf16(w)
        p[k + ".b"] = rng.uniform(0.01, 0.1, shp[-1]).astype(np.float32).astype(np.float64)
    net.set_params(flat(p))
    x = bf16(np.abs(rng.standard_normal((B, D, H, W, 3))))
    dy = rng.standard_normal((B, D, H, W)).astype(np.float32)
    g = unflat(net.gradients(dev(x), dev(dy)).astype(np.float64))
    _, c = N.forward(p, x[0])
    go = N.backward(p, c, dy[0][..., None].astype(np.float64))
    errs = {k: rel(g[k], go[k]) for k in go}
    for k, e in errs.items():
        print(f"  {k:7s} rel L2 {e:.3e}", flush=True)
    print(f"  ambiguous fraction {ambiguous_fraction(p, x):.3e}", flush=True)
    for k, e in errs.items():
        assert e <= TOL_GRAD, k


def test_gradients_deterministic(net):
    p = make_params(3)
    net.set_params(flat(p))
    rng = np.random.default_rng(9)
    x = dev(bf16(rng.standard_normal((1, 8, 8, 8, 3))))
    dy = dev(rng.standard_normal((1, 8, 8, 8)))
    g1 = net.gradients(x, dy)
    g2 = net.gradients(x, dy)
    assert np.array_equal(g1, g2)


def test_train_step_loss_and_adam_direction():
    """The reported loss is the oracle's MSE of the forward pass; the first
    Adam step moves every weight by lr * sign(g) (bias correction makes
    m/sqrt(v) = g/|g|), checked where the oracle's gradient is clearly
    away from zero."""
    lr = 1e-3
    n = les.Net(seed=2, lr=lr)
    try:
        p = make_params(13)
        w0 = flat(p)
        n.set_params(w0)
        rng = np.random.default_rng(21)
        x = bf16(rng.standard_normal((1, 8, 8, 8, 3)))
        t = rng.standard_normal((1, 8, 8, 8)).astype(np.float32)
        loss = n.train_step(dev(x), dev(t))
        yo, c = N.forward(p, x[0])
        lo, dyo = N.mse(yo, t[0][..., None].astype(np.float64))
        assert abs(loss - lo) <= 2 * TOL_FWD * lo
        go = flat(N.backward(p, c, dyo))
        step = n.get_params().astype(np.float64) - w0.astype(np.float32).astype(np.float64)
        big = np.abs(go) > 0.2 * np.abs(go).max()
        assert big.sum() > 20
        assert np.allclose(step[big], -lr * np.sign(go[big]), rtol=1e-3, atol=1e-7)
    finally:
        n.close()


def test_training_lowers_loss():
    n = les.Net(seed=4, lr=3e-3)
    try:
        rng = np.random.default_rng(8)
        x = dev(rng.standard_normal((2, 8, 8, 8, 3)))
        t = dev(np.tanh(rng.standard_normal((2, 8, 8, 8))))
        losses = [n.train_step(x, t) for _ in range(30)]
        print(f"  loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
        assert losses[-1] < 0.5 * losses[0]
    finally:
        n.close()


def test_bad_arguments(net):
    L = les.lib()
    x = torch.zeros((1, 6, 8, 8, 3), device="cuda")
    y = torch.zeros((1, 6, 8, 8), device="cuda")
    # D not a multiple of 4
    assert L.lesnet_forward(net.h, 1, 6, 8, 8, x.data_ptr(), y.data_ptr(), None) == les.LES_EINVAL
    assert L.lesnet_forward(net.h, 0, 8, 8, 8, x.data_ptr(), y.data_ptr(), None) == les.LES_EINVAL
    w = np.zeros(net.num_params - 1, np.float32)
    assert L.lesnet_set_params(net.h, w.ctypes.data, w.size) == les.LES_EINVAL
    cfg = les.NetConfig()
    L.lesnet_default_config(cfg)
    cfg.c1 = 24
    import ctypes as C
    h = C.c_void_p()
    assert L.lesnet_create(cfg, C.byref(h)) == les.LES_EINVAL and not h.value


# ------------------------------------------------------------ single ops
# Each kernel on its own: bfloat16 operands, float32 accumulation and
# float32 output.  The sums have at most K = 27 * 64 = 1728 products (conv)
# or one per voxel (weight gradients, split over blocks); float32 rounding
# of a K-term sum of random-sign products leaves a relative L2 error near
# sqrt(K) 2^-24 = 2.5e-6, so 1e-5 is the bar.
TOL_OP = 1e-5
OP_CASES = [  # (B, D, H, W, cin, cout)
    (1, 6, 5, 7, 3, 16), (2, 4, 6, 8, 16, 32), (1, 5, 4, 6, 32, 64), (1, 4, 4, 4, 64, 16),
    (1, 3, 5, 4, 64, 64),
]


def _rnd(shape, seed):
    return bf16(np.random.default_rng(seed).standard_normal(shape))


@pytest.mark.parametrize("B,D,H,W,cin,cout", OP_CASES)
def test_op_conv3_forward_dgrad_wgrad(B, D, H, W, cin, cout):
    print(f"[lesnet_op conv3] B={B} D={D} H={H} W={W} cin={cin} cout={cout}", flush=True)
    x = _rnd((B, D, H, W, cin), 1)
    Wt = _rnd((27, cin, cout), 2) / np.sqrt(27 * cin)
    Wt = bf16(Wt)
    bias = np.random.default_rng(3).standard_normal(cout).astype(np.float32)
    dy = _rnd((B, D, H, W, cout), 4)
    y = les.net_op("conv3", dev(x), dev(Wt), dev(bias)).cpu().numpy()
    yo = np.stack([N.conv3(x[b], Wt, bias.astype(np.float64)) for b in range(B)])
    assert rel(y, yo) <= TOL_OP
    wg = les.net_op("conv3_wgrad", dev(x), dev(dy)).cpu().numpy()
    dxo, dWo = np.zeros_like(x), np.zeros_like(Wt)
    for b in range(B):
        dx_b, dW_b, _ = N.conv3_backward(x[b], Wt, dy[b])
        dxo[b] = dx_b
        dWo += dW_b
    assert rel(wg, dWo) <= TOL_OP
    if cin in (16, 32, 64):
        dx = les.net_op("conv3_dgrad", dev(dy), dev(Wt)).cpu().numpy()
        assert rel(dx, dxo) <= TOL_OP


@pytest.mark.parametrize("B,D,H,W,cin,cout", OP_CASES)
def test_op_up_forward_dgrad_wgrad(B, D, H, W, cin, cout):
    print(f"[lesnet_op up] B={B} D={D} H={H} W={W} cin={cin} cout={cout}", flush=True)
    x = _rnd((B, D, H, W, cin), 5)
    U = bf16(_rnd((8, cin, cout), 6) / np.sqrt(cin))
    bias = np.random.default_rng(7).standard_normal(cout).astype(np.float32)
    dy = _rnd((B, 2 * D, 2 * H, 2 * W, cout), 8)
    y = les.net_op("up", dev(x), dev(U), dev(bias)).cpu().numpy()
    yo = np.stack([N.up(x[b], U, bias.astype(np.float64)) for b in range(B)])
    assert rel(y, yo) <= TOL_OP
    dxo, dUo = np.zeros_like(x), np.zeros_like(U)
    for b in range(B):
        dx_b, dU_b, _ = N.up_backward(x[b], U, dy[b])
        dxo[b] = dx_b
        dUo += dU_b
    wg = les.net_op("up_wgrad", dev(x), dev(dy)).cpu().numpy()
    assert rel(wg, dUo) <= TOL_OP
    if cin in (16, 32, 64):
        dx = les.net_op("up_dgrad", dev(dy), dev(U)).cpu().numpy()
        assert rel(dx, dxo) <= TOL_OP


def test_op_rejects_bad_sizes():
    a = torch.zeros((1, 4, 4, 4, 16), device="cuda")
    w = torch.zeros((27, 16, 24), device="cuda")
    with pytest.raises(les.LesError):
        les.net_op("conv3", a, w)              # cout 24 is not a tile size
    L = les.lib()
    assert L.lesnet_op(9, 1, 4, 4, 4, 16, 16, a.data_ptr(), w.data_ptr(), None, a.data_ptr(),
                       None) == les.LES_EINVAL
