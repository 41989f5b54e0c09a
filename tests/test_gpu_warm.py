"""GPU tests of the warm-start coupling (les_set_capture, les_set_warm_start).

The capture checks compare the device's input channels and targets with
what they are defined from (the handle's own fields, and the oracle's
operator A applied to them); the hand-off checks that a start is only
taken when its residual is smaller, so a network that cannot help leaves
the run bit for bit unchanged; the last test trains the network on LES
runs and measures the iterations it saves on held-out cases.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1504_02264_amd as les
from les_inputs import building_heights, building_mask, log_law_profile

pytestmark = pytest.mark.gpu

NX, NY, NZ = 24, 20, 10          # network grid 12 x 20 x 24 (nz padded 10 -> 12)
DX, DY, DZ, DT = 4.0, 4.0, 2.0, 0.05


def case():
    h = building_heights(NX, NY, NZ, 0.15, 2, 4, 2, 6, seed=5, margin_x=4, margin_y=2)
    mask = building_mask(h, NZ)
    g = les.LES(NX, NY, NZ, DX, DY, DZ, DT, mask)
    g.set_inflow(log_law_profile(NZ, DZ), 0.01, 5)
    return g, mask


def test_warm_grid_pads_to_multiples_of_four():
    g, _ = case()
    try:
        assert les.warm_grid(g) == (12, 20, 24)
    finally:
        g.close()


def test_capture_channels_and_target():
    print(f"[capture] {NX}x{NY}x{NZ}", flush=True)
    g, mask = case()
    o = oracle.Oracle(NX, NY, NZ, DX, DY, DZ, DT, mask)
    try:
        g.step(3)
        p_prev = g.get_fields()[3].astype(np.float64)
        D, H, W = les.warm_grid(g)
        X = torch.full((D, H, W, 3), 7.0, device="cuda")
        T = torch.full((D, H, W), 7.0, device="cuda")
        les.set_capture(g, X, T)
        g.step(1)
        les.set_capture(g, None, None)
        x = X.cpu().numpy().astype(np.float64)
        t = T.cpu().numpy().astype(np.float64)
        p_new = g.get_fields()[3].astype(np.float64)
        rhs = g.get_rhs().astype(np.float64)
        # padding is zero
        assert np.all(x[NZ:] == 0) and np.all(t[NZ:] == 0)
        xc, tc = x[:NZ, :NY, :NX], t[:NZ, :NY, :NX]
        # mask channel: the building mask, exactly
        assert np.array_equal(xc[..., 1], mask.astype(np.float64))
        # residual channel: (rhs - A p_prev) / RMS, A applied by the oracle
        # in float64; the device forms A from the float32 pair (ph, pd)
        # whose rounded sum is p_prev, a difference bounded by
        # ||A|| ||p|| 2^-24 with ||A|| <= 2 dbar (Gershgorin)
        r = rhs - o.apply_A(p_prev)
        dbar = 2 * (1 / DX ** 2 + 1 / DY ** 2 + 1 / DZ ** 2)
        bound = (2 * dbar * np.linalg.norm(p_prev) * 2.0 ** -24) / np.linalg.norm(r) + 2.0 ** -23
        rn = r / np.sqrt(np.mean(r ** 2))
        err = np.linalg.norm(xc[..., 0] - rn) / np.linalg.norm(rn)
        print(f"  residual channel rel err {err:.2e} (bound {bound:.2e})", flush=True)
        assert err <= bound
        # previous-pressure channel: p_prev / RMS(p_prev)
        pn = p_prev / np.sqrt(np.mean(p_prev ** 2))
        assert np.linalg.norm(xc[..., 2] - pn) / np.linalg.norm(pn) <= 1e-6
        # target: (p* - p_prev) dbar / RMS(r)
        want = (p_new - p_prev) * dbar / np.sqrt(np.mean(r ** 2))
        terr = np.linalg.norm(tc - want) / np.linalg.norm(want)
        print(f"  target rel err {terr:.2e}", flush=True)
        assert terr <= 1e-5 + bound
    finally:
        g.close()


def _run(net_params, scale, steps=4, zero=False, rule=les.WARM_RESIDUAL, param=0):
    g, _ = case()
    net = None
    try:
        if net_params is not None:
            net = les.Net(seed=3)
            w = net.get_params()
            if zero:
                w[:] = 0
            else:
                w *= net_params
            net.set_params(w)
            les.set_warm_start(g, net, scale, rule, param)
        stats = []
        for _ in range(steps):
            _, st, _ = g.step(1)
            stats.append(st)
        return g.get_fields(), stats
    finally:
        g.close()
        if net is not None:
            net.close()


def test_unhelpful_network_is_never_taken():
    """A zero network proposes p_prev itself (equal residual: not taken);
    a wildly scaled one proposes a far worse start.  Either way the run is
    the plain run, bit for bit."""
    base, _ = _run(None, 1.0)
    for mult, scale, zero, rule, param in ((1.0, 1.0, True, les.WARM_RESIDUAL, 0),
                                           (1.0, 1.0, True, les.WARM_SMOOTH, 8),
                                           (1.0, 1.0, True, les.WARM_TRIAL, 8),
                                           (1.0, 1e4, False, les.WARM_RESIDUAL, 0),
                                           (1.0, 1e4, False, les.WARM_SMOOTH, 8)):
        print(f"  rule {rule} param {param} zero={zero}", flush=True)
        f, stats = _run(mult, scale, zero=zero, rule=rule, param=param)
        assert all(s["warm_taken"] == 0 for s in stats)
        for a, b in zip(f, base):
            assert np.array_equal(a, b)
        if not zero:
            assert all(s["warm_r_net_last"] > s["warm_r_prev_last"] for s in stats)


def test_choice_follows_the_residuals():
    """taken == (R(p0) < R(p_prev)), and R(p_prev) is the residual of the
    previous pressure as the oracle's operator gives it."""
    g, mask = case()
    o = oracle.Oracle(NX, NY, NZ, DX, DY, DZ, DT, mask)
    net = les.Net(seed=9)
    try:
        les.set_warm_start(g, net, 0.05)
        for _ in range(5):
            p_prev = g.get_fields()[3].astype(np.float64)
            _, st, _ = g.step(1)
            rhs = g.get_rhs().astype(np.float64)
            r_prev = o.residual(rhs, p_prev)
            assert st["warm_taken"] == int(st["warm_r_net_last"] < st["warm_r_prev_last"])
            if np.linalg.norm(p_prev) > 0:
                dbar = 2 * (1 / DX ** 2 + 1 / DY ** 2 + 1 / DZ ** 2)
                slack = 2 * dbar * np.linalg.norm(p_prev) * 2.0 ** -24 / np.linalg.norm(rhs)
                assert abs(st["warm_r_prev_last"] - r_prev) <= 1e-9 + slack + 1e-6 * r_prev
            assert st["resid_last"] <= 1e-5
    finally:
        g.close()
        net.close()


def test_learned_start_saves_iterations_on_held_out_cases():
    """Train on pairs captured from C1-size runs with building seeds 11-14
    (and their mirror images in y), then run held-out seeds 21 and 22:
    starting each solve from the network's (smoothed) proposal lowers the
    mean SOR iteration count at the same tolerance.  Training and the runs
    are deterministic."""
    from paper_1504_02264_amd import warmstart as ws

    smooth = 16
    Xs, Ts = [], []
    for seed in (11, 12, 13, 14):
        X, T, _ = ws.collect("C1", seed, steps=24, skip=2, smooth=smooth)
        Xs.append(X)
        Ts.append(T)
    X, T = ws.mirror_y(torch.cat(Xs), torch.cat(Ts))
    print(f"  {X.shape[0]} training pairs", flush=True)
    net = les.Net(seed=0, lr=1e-3)
    try:
        scale, losses = ws.train(net, X, T, iters=6000, batch=8, lr=1e-3, lr_final=5e-5)
        print(f"  loss {losses[0][1]:.3f} -> {losses[-1][1]:.4f}", flush=True)
        del X, T
        base, warm = [], []
        for seed in (21, 22):
            b = ws.evaluate("C1", seed, steps=8, net=None, skip=2)
            w = ws.evaluate("C1", seed, steps=8, net=net, scale=scale, skip=2,
                            rule=les.WARM_ALWAYS, smooth=smooth)
            print(f"  seed {seed}: plain {b['iters'].mean():.0f} it {b['ms_per_step']:.1f} ms/step; "
                  f"learned {w['iters'].mean():.0f} it {w['ms_per_step']:.1f} ms/step", flush=True)
            base.append(b["iters"].mean())
            warm.append(w["iters"].mean())
        assert np.mean(warm) <= 0.95 * np.mean(base)
    finally:
        net.close()


def test_initial_guess_dev_starts_the_next_solve():
    """A solve started (les_set_initial_guess_dev) from the converged
    pressure of the same step needs at most a couple of check intervals and
    lands on the same solution."""
    a, _ = case()
    b, _ = case()
    try:
        _, _, it_a = a.step(1)
        pa = a.get_fields()[3]
        b.set_initial_guess_dev(torch.from_numpy(pa).cuda())
        torch.cuda.synchronize()
        _, st, it_b = b.step(1)
        pb = b.get_fields()[3]
        print(f"  iterations from p_prev {it_a[0]}, from the converged p {it_b[0]}", flush=True)
        assert it_a[0] > 8 and it_b[0] <= 8
        assert np.linalg.norm(pb - pa) / np.linalg.norm(pa) <= 1e-4
        assert st["resid_last"] <= 1e-5
    finally:
        a.close()
        b.close()
