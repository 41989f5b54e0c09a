"""Training and evaluation of the learned SOR warm start on LES runs.

Pairs come from the LES itself: with capture on (``les_set_capture``) each
step leaves its network input (residual of the previous pressure, building
mask, previous pressure, normalised) and its target (the converged change
of pressure, scaled by dbar / RMS(residual)) on the device.  Training runs
the network's own kernels (``lesnet_train_step``); evaluation runs the
same cases with and without the warm start and compares the SOR iteration
counts, which stop at the same tolerance either way.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

import paper_1504_02264_amd as les


def make_case(base: str, seed: int, tune: bool = False, **params):
    """An LES handle for workload `base` with buildings and inflow noise
    drawn from `seed`; with tune, its SOR sweep variant autotuned."""
    from les_inputs import WORKLOADS, make_workload_inputs

    w = dataclasses.replace(WORKLOADS[base], seed=seed)
    mask, prof = make_workload_inputs(w)
    g = les.LES(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.dt, mask, **params)
    g.set_inflow(prof, w.noise_amp, seed)
    if tune:
        g.autotune(reps=10)
    return g


def collect(base: str, seed: int, steps: int, skip: int = 0, smooth: int = 0):
    """Run `skip` + `steps` steps; return the (inputs [n, D, H, W, 3],
    targets [n, D, H, W]) of the last `steps` as device tensors, with the
    per-step SOR iterations."""
    import torch

    g = make_case(base, seed)
    try:
        if skip:
            g.step(skip)
        D, H, W = les.warm_grid(g)
        X = torch.empty((steps, D, H, W, 3), device="cuda")
        T = torch.empty((steps, D, H, W), device="cuda")
        its = []
        for s in range(steps):
            les.set_capture(g, X[s], T[s], smooth)
            _, _, it = g.step(1)
            its.append(int(it[0]))
        les.set_capture(g, None, None)
        torch.cuda.synchronize()
        return X, T, np.array(its)
    finally:
        g.close()


def collect_crops(base: str, seed: int, steps: int, skip: int = 0, smooth: int = 0, crops: int = 8,
                  crop=(64, 128, 128), rng_seed: int = 0, tune: bool = True, **params):
    """Like collect, for grids larger than the training crop: after each of
    the last `steps` steps, `crops` random D x H x W windows (aligned to 4,
    drawn from numpy PCG64(rng_seed)) of the step's input and target;
    params (e.g. max_iter) go to the handle's les_params."""
    import torch

    g = make_case(base, seed, tune=tune, **params)
    try:
        if skip:
            g.step(skip)
        D, H, W = les.warm_grid(g)
        cd, ch, cw = crop
        Xf = torch.empty((D, H, W, 3), device="cuda")
        Tf = torch.empty((D, H, W), device="cuda")
        X = torch.empty((steps * crops, cd, ch, cw, 3), device="cuda")
        T = torch.empty((steps * crops, cd, ch, cw), device="cuda")
        rng = np.random.default_rng(rng_seed)
        n = 0
        for _ in range(steps):
            les.set_capture(g, Xf, Tf, smooth)
            g.step(1)
            for _ in range(crops):
                z = 4 * int(rng.integers(0, (D - cd) // 4 + 1))
                y = 4 * int(rng.integers(0, (H - ch) // 4 + 1))
                x = 4 * int(rng.integers(0, (W - cw) // 4 + 1))
                les.crop(Xf, (z, y, x, cd, ch, cw), out=X[n])
                les.crop(Tf, (z, y, x, cd, ch, cw), out=T[n])
                n += 1
        les.set_capture(g, None, None)
        torch.cuda.synchronize()
        return X, T
    finally:
        g.close()


def mirror_y(X, T):
    """The pairs and their mirror images in y.  The y walls carry the same
    boundary condition on both sides, so the pressure operator commutes
    with the reflection j -> ny-1-j and a mirrored pair (input and target
    reflected alike) is as valid a training pair as the original."""
    import torch

    n = X.shape[0]
    Xm = torch.empty((2 * n,) + tuple(X.shape[1:]), device=X.device)
    Tm = torch.empty((2 * n,) + tuple(T.shape[1:]), device=T.device)
    D, H, W = T.shape[1:4]
    for i in range(n):
        for m in (0, 1):
            les.crop(X[i], (0, 0, 0, D, H, W), out=Xm[i + m * n], mirror_y=bool(m))
            les.crop(T[i], (0, 0, 0, D, H, W), out=Tm[i + m * n], mirror_y=bool(m))
    return Xm, Tm


def train(net: les.Net, X, T, iters: int, batch: int = 4, seed: int = 0, log=None,
          lr: float | None = None, lr_final: float | None = None):
    """Adam on random mini-batches of the pairs; targets are divided by
    their RMS over the set, which is returned as the warm start's
    target_scale, with the loss history.  With lr given, the step size
    decays geometrically from lr to lr_final (default lr / 10)."""
    import torch

    scale = float(np.sqrt(les.sum_squares(T) / T.numel()))
    Tn = les.scale_div(T, scale)
    rng = np.random.default_rng(seed)
    losses = []
    n = X.shape[0]
    nb = min(batch, n)
    xb = torch.empty((nb,) + tuple(X.shape[1:]), device=X.device)
    tb = torch.empty((nb,) + tuple(T.shape[1:]), device=T.device)
    for it in range(iters):
        if lr is not None:
            lf = lr / 10 if lr_final is None else lr_final
            net.set_lr(lr * (lf / lr) ** (it / max(iters - 1, 1)))
        idx = rng.choice(n, size=nb, replace=False)
        les.gather(X, idx, out=xb)
        les.gather(Tn, idx, out=tb)
        want = (it % 50 == 0) or it == iters - 1
        loss = net.train_step(xb, tb, want_loss=want)
        if want:
            losses.append((it, loss))
            if log:
                log(f"train iter {it}: loss {loss:.4f}")
    return scale, losses


def evaluate(base: str, seed: int, steps: int, net: les.Net | None, scale: float = 1.0,
             skip: int = 0, rule: int = les.WARM_RESIDUAL, param: int = 0, smooth: int = 0,
             tune: bool = False, **params):
    """Iterations per step and wall ms per step of `steps` steps (after
    `skip` plain steps), warm-started by `net` if given (choice `rule`,
    `param`, see les_set_warm_start); with tune, on the autotuned sweep;
    params (e.g. tol) go to the handle's les_params."""
    import torch

    g = make_case(base, seed, tune=tune, **params)
    try:
        if skip:
            g.step(skip)
        if net is not None:
            les.set_warm_start(g, net, scale, rule, param, smooth)
        torch.cuda.synchronize()
        its, taken, rnet, rprev, res = [], 0, [], [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st, it = g.step(1)
            its.append(int(it[0]))
            res.append(st["resid_last"])
            taken += st["warm_taken"]
            rnet.append(st["warm_r_net_last"])
            rprev.append(st["warm_r_prev_last"])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        if net is not None:
            les.set_warm_start(g, None)
        return {"iters": np.array(its), "ms_per_step": ms, "taken": taken,
                "r_net": np.array(rnet), "r_prev": np.array(rprev), "resid": np.array(res)}
    finally:
        g.close()
