#!/usr/bin/env python3
"""Benchmark of the MI355X urban-LES time step.

One benchmark step is one full LES time step (nu_t, tendency + feedback +
AB2, inflow, rhs, red-black SOR to relative residual 1e-5, projection,
ghost refresh) on the 300 x 300 x 90 urban workload (30% building cover,
power-law inflow), inputs resident in HBM before the timed region.  Every
step iterates SOR (omega 1.8, from the previous step's pressure) until the
tolerance is met: about 1.5e5 iterations per step on this grid; the cap
of 2e6 is only a guard (--max-iter lowers it for profiling runs, and the
line then says how many steps stopped at the cap).

Prints ONE JSON line:
  value      LES cell-updates/s = cells * steps / wall time of les_step(steps)
  roofline   the dominant kernel, the SOR sweep: algorithmic bytes per launch
             over its mean HIP-event duration on the library's stream.  A
             fused red-black iteration (k_sor_rb) moves 12 B per cell: the
             correction p read and the new one written (4 + 4 B) and r0 read
             (4 B); a half-sweep (k_sor) 8 B per cell of the grid: the other
             colour read (4 B per cell of that colour), own p read and
             written and own r0 read (12 B per cell of this colour).
             `traffic` is the measured HBM bytes (rocprofv3 FETCH_SIZE +
             WRITE_SIZE, copy-calibrated) from the summaries in profiles/.
  cpu_baseline  the FP64 oracle on the host cores, on a bounded sample

Other modes print their own JSON line: --ensemble N, --warm-start,
--twinned (twinned double buffering against red-black SOR).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor figure
BENCH_MAX_ITER = 2000000   # SOR cap of the benchmark's steps: a guard, not a budget


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_sample(workload, sample_iters):
    """The oracle's two timed pieces on this host: one step without its SOR
    iterations, and `sample_iters` SOR iterations (seconds each)."""
    import oracle
    from les_inputs import WORKLOADS, make_workload_inputs
    w = WORKLOADS[workload]
    mask, prof = make_workload_inputs(w)
    o = oracle.Oracle(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.dt, mask)
    o.set_inflow(prof, w.noise_amp, w.seed)
    t0 = time.perf_counter()
    o.step(1, forced=[0])          # all of the step except the SOR iterations
    t_fixed = time.perf_counter() - t0
    rhs = o.get_rhs()
    p0 = o.get_fields()[3]
    t0 = time.perf_counter()
    o.sor_iterations(rhs, p0, sample_iters)
    t_iter = (time.perf_counter() - t0) / sample_iters
    return t_fixed, t_iter


def cpu_baseline(w, gpu_iters_per_step, sample_iters):
    """Time the FP64 oracle on this host: one step's non-SOR work plus a
    bounded number of SOR iterations, combined at the GPU's mean iteration
    count into a per-step time; on all host threads (OpenMP within a colour
    or stencil pass) and, in a child process, on one thread."""
    import subprocess
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t_fixed, t_iter = oracle_sample(w.name, sample_iters)
    t_step = t_fixed + gpu_iters_per_step * t_iter
    cells = w.nx * w.ny * w.nz
    one = None
    n1 = max(1, sample_iters // 10)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-sample", w.name,
                        "--cpu-sample-iters", str(n1)], capture_output=True, text=True, env=env)
    if r.returncode == 0 and r.stdout.strip():
        f1, i1 = json.loads(r.stdout.strip().splitlines()[-1])
        s1 = f1 + gpu_iters_per_step * i1
        one = {"value": cells / s1, "s_per_step": s1, "cores": 1,
               "sample": f"1 step without SOR ({f1:.2f} s) + {n1} SOR iterations ({i1 * 1e3:.1f} ms each)"}
    return {
        "value": cells / t_step,
        "unit": "cell-updates/s",
        "cores": threads,
        "kind": "oracle",
        "cpu": cpu_model(),
        "sample": (f"{w.name} {w.nx}x{w.ny}x{w.nz}: 1 step without SOR ({t_fixed:.2f} s) + "
                   f"{sample_iters} SOR iterations ({t_iter * 1e3:.1f} ms each), combined at the "
                   f"GPU's mean {gpu_iters_per_step:.0f} iterations/step -> {t_step:.2f} s/step "
                   f"(extrapolated)"),
        "s_per_step": t_step,
        "single_thread": one,
    }


def young_omega(w):
    """Young's optimal relaxation factor 2 / (1 + sqrt(1 - rho_J^2)) for the
    urban operator of workload w, with the Jacobi radius estimated as
    1 - lambda_min / d from the smoothest mode (a quarter cosine in x
    between the Neumann inflow face and the Dirichlet outflow face:
    lambda_min = 4 / dx^2 sin^2(pi / (4 nx))) and the interior diagonal d."""
    import math
    lam = 4.0 / w.dx ** 2 * math.sin(math.pi / (4 * w.nx)) ** 2
    d = 2.0 * (1.0 / w.dx ** 2 + 1.0 / w.dy ** 2 + 1.0 / w.dz ** 2)
    rho = 1.0 - lam / d
    return 2.0 / (1.0 + math.sqrt(1.0 - rho * rho))


def omega_study(les, torch, w, mask, g, variant, omega, K, steps=2):
    """The state after the timed steps (checkpoint) continued for `steps`
    steps with another relaxation factor, each solved to 1e-5: SOR
    iterations and wall ms per step (timing off: graph replay)."""
    blob = g.get_state()
    t = les.LES(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.dt, mask, timing=0, max_iter=BENCH_MAX_ITER,
                omega=omega, check_every=K, rebase_every=max(1, 128 // K))
    rows = []
    try:
        t.set_state(blob)
        t.set_sor_variant(variant)
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st, it = t.step(1)
            torch.cuda.synchronize()
            rows.append({"sor_iters": int(it[0]), "ms": (time.perf_counter() - t0) * 1e3,
                         "resid": st["resid_last"], "converged": bool(rc == les.LES_OK)})
            log(f"omega {omega:.5f}: {rows[-1]}")
    finally:
        t.close()
    return {"omega": omega, "note": "study, not the configured step: Young's factor for this operator",
            "steps": rows,
            "sor_iters_per_step": sum(r["sor_iters"] for r in rows) / len(rows),
            "ms_per_step": sum(r["ms"] for r in rows) / len(rows)}


MFMA_BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix peak, vendor figure


def net_flops(D, H, W, c=(16, 32, 64), cin=3):
    """Algorithmic FLOPs (multiply-add = 2) of one forward pass and one
    backward pass (input and weight gradients) of the warm-start U-Net on
    a D x H x W grid, with the unpadded channel counts."""
    c1, c2, c3 = c
    m1, m2, m3 = D * H * W, D * H * W // 8, D * H * W // 64
    convs = [(m1, cin, c1), (m1, c1, c1), (m2, c1, c2), (m2, c2, c2), (m3, c2, c3), (m3, c3, c3),
             (m2, 2 * c2, c2), (m2, c2, c2), (m1, 2 * c1, c1), (m1, c1, c1)]
    ups = [(m3, c3, c2), (m2, c2, c1)]
    fwd = sum(2 * 27 * ci * co * m for m, ci, co in convs) + sum(2 * 8 * ci * co * m for m, ci, co in ups)
    fwd += 2 * c1 * m1
    # backward: weight gradients for every layer, input gradients for all but the first
    bwd = 2 * fwd - 2 * 27 * cin * c1 * m1
    return fwd, bwd


def bench_net(les, torch, D=64, H=128, W=128, reps=10):
    """Forward and training-step time of the warm-start network on one
    D x H x W crop (HIP events on torch's stream, which the network's
    kernels run on), against the dense BF16 matrix peak."""
    net = les.Net(seed=0)
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((1, D, H, W, 3), device="cuda", generator=g)
    t = torch.randn((1, D, H, W), device="cuda", generator=g)
    for _ in range(2):
        net.forward(x)
        net.train_step(x, t, want_loss=False)
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    for _ in range(reps):
        net.forward(x)
    e1.record()
    for _ in range(reps):
        net.train_step(x, t, want_loss=False)
    e2.record()
    torch.cuda.synchronize()
    f_ms = e0.elapsed_time(e1) / reps
    t_ms = e1.elapsed_time(e2) / reps
    fwd, bwd = net_flops(D, H, W)
    nparams = net.num_params
    net.close()
    f_tf = fwd / (f_ms * 1e-3) / 1e12
    t_tf = (fwd + bwd) / (t_ms * 1e-3) / 1e12
    return {
        "grid": [D, H, W],
        "voxels": D * H * W,
        "params": int(nparams),
        "forward_ms": f_ms,
        "train_step_ms": t_ms,
        "forward_gflop": fwd / 1e9,
        "train_step_gflop": (fwd + bwd) / 1e9,
        "roofline": {"bound": "mfma", "achieved": f_tf, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": f_tf / MFMA_BF16_PEAK_TFLOPS, "scope": "whole forward pass"},
        "train_step_tflops": t_tf,
        "train_step_frac": t_tf / MFMA_BF16_PEAK_TFLOPS,
    }


def bench_warm_start_c2(args, les, torch):
    """The learned start at 300x300x90 with every solve run to 1e-5: trained
    on 8 random 64x128x128 crops per step of runs with building seeds 11-14
    (converged targets), evaluated on whole held-out runs (seeds 21, 22):
    SOR iterations and wall ms per step to the tolerance, plain SOR from the
    previous step's pressure against the network's start (inference and
    the smoothing of its proposal inside the time)."""
    import numpy as np
    from paper_1504_02264_amd import warmstart as ws
    smooth = 16
    conv = {"max_iter": BENCH_MAX_ITER, "check_every": args.check_every,
            "rebase_every": max(1, 128 // args.check_every)}
    Xs, Ts = [], []
    t0 = time.perf_counter()
    for seed in (11, 12, 13, 14):
        log(f"C2 crops from seed {seed}")
        X, T = ws.collect_crops("C2", seed, steps=2, skip=1, smooth=smooth, crops=8, rng_seed=seed, **conv)
        Xs.append(X)
        Ts.append(T)
    X, T = ws.mirror_y(torch.cat(Xs), torch.cat(Ts))
    collect_s = time.perf_counter() - t0
    net = les.Net(seed=0, lr=1e-3)
    t0 = time.perf_counter()
    scale, losses = ws.train(net, X, T, iters=3000, batch=4, lr=1e-3, lr_final=5e-5)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del X, T, Xs, Ts
    rows = {}
    for seed in (21, 22):
        log(f"C2 evaluation, seed {seed}")
        b = ws.evaluate("C2", seed, steps=args.steps, net=None, skip=1, tune=True, **conv)
        w = ws.evaluate("C2", seed, steps=args.steps, net=net, scale=scale, skip=1, rule=les.WARM_ALWAYS,
                        smooth=smooth, tune=True, **conv)
        for name, r in (("plain", b), ("always", w)):
            d = rows.setdefault(name, {"iters": [], "ms": [], "resid": []})
            d["iters"] += [int(x) for x in r["iters"]]
            d["ms"].append(r["ms_per_step"])
            d["resid"] += [float(x) for x in r["resid"]]
    base = float(np.mean(rows["plain"]["ms"]))
    out = {
        "metric": "time to relative Poisson residual 1e-5 per step, learned start vs plain SOR (300x300x90)",
        "value": float(np.mean(rows["always"]["ms"])),
        "unit": "ms/step",
        "higher_is_better": False,
        "n_gpus": 1,
        "steps": args.steps,
        "dtype": "f32 LES, bf16 network",
        "data": "synthetic",
        "config": {"workload": f"C2 300x300x90 urban LES, every solve to relative residual 1e-5 (checked every "
                               f"{args.check_every} iterations); network "
                               "trained on 8 random 64x128x128 crops per step of building seeds 11-14 (converged "
                               "targets, 64 crops and their mirror images in y, 3000 Adam steps), evaluated on "
                               "seeds 21-22 after one plain step", "collect_s": collect_s, "train_s": train_s,
                   "final_loss": losses[-1][1], "smooth_passes": smooth},
        "rules": {k: {"sor_iters_per_step": v["iters"], "mean_sor_iters": float(np.mean(v["iters"])),
                      "ms_per_step": float(np.mean(v["ms"])), "ms_vs_plain": float(np.mean(v["ms"])) / base,
                      "resid_per_step": v["resid"]}
                  for k, v in rows.items()},
    }
    net.close()
    print(json.dumps(out), flush=True)


def bench_warm_start_c3(args, les, torch):
    """The learned start at 1024x1024x96: trained on 8 random 64x128x128
    crops per step of runs with building seeds 11-14, evaluated on whole
    held-out runs (seeds 21, 22).  The solve stops at max_iter there either
    way, so the comparison is the residual reached and the time per step."""
    import numpy as np
    from paper_1504_02264_amd import warmstart as ws
    smooth = 32
    Xs, Ts = [], []
    t0 = time.perf_counter()
    for seed in (11, 12, 13, 14):
        log(f"C3 crops from seed {seed}")
        X, T = ws.collect_crops("C3", seed, steps=2, skip=1, smooth=smooth, crops=8, rng_seed=seed)
        Xs.append(X)
        Ts.append(T)
    X, T = ws.mirror_y(torch.cat(Xs), torch.cat(Ts))
    collect_s = time.perf_counter() - t0
    net = les.Net(seed=0, lr=1e-3)
    t0 = time.perf_counter()
    scale, losses = ws.train(net, X, T, iters=3000, batch=4, lr=1e-3, lr_final=5e-5)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del X, T, Xs, Ts
    rows = {}
    for seed in (21, 22):
        log(f"C3 evaluation, seed {seed}")
        b = ws.evaluate("C3", seed, steps=args.steps, net=None, skip=1, tune=True)
        w = ws.evaluate("C3", seed, steps=args.steps, net=net, scale=scale, skip=1, rule=les.WARM_ALWAYS,
                        smooth=smooth, tune=True)
        # time to the residual plain SOR reaches in max_iter iterations: the
        # first evaluated step (the same state for both runs) again, from
        # the learned start, to the residual plain SOR ended that step on
        tol_plain = float(b["resid"][0])
        log(f"C3 learned start to the plain run's residual {tol_plain:.4f}, seed {seed}")
        w2 = ws.evaluate("C3", seed, steps=1, net=net, scale=scale, skip=1, rule=les.WARM_ALWAYS,
                         smooth=smooth, tune=True, tol=tol_plain)
        for name, r in (("plain", b), ("always", w), ("always, to the plain residual", w2)):
            d = rows.setdefault(name, {"resid": [], "iters": [], "ms": []})
            d["resid"] += [float(x) for x in r["resid"]]
            d["iters"].append(float(r["iters"].mean()))
            d["ms"].append(r["ms_per_step"])
    out = {
        "metric": "relative Poisson residual at the end of each step (learned start, 1024x1024x96)",
        # plain SOR stops at max_iter here; the third rule measures the time
        # the learned start needs, on the first evaluated step, to reach the
        # residual plain SOR ends that step on
        "value": float(np.mean(rows["always"]["resid"])),
        "unit": "relative residual",
        "higher_is_better": False,
        "n_gpus": 1,
        "steps": args.steps,
        "dtype": "f32 LES, bf16 network",
        "data": "synthetic",
        "config": {"workload": "C3 1024x1024x96 urban LES; network trained on 8 random 64x128x128 crops per "
                               "step of building seeds 11-14 (64 crops and their mirror images in y, 3000 Adam steps), evaluated on seeds "
                               "21-22 after one plain step", "collect_s": collect_s, "train_s": train_s,
                   "final_loss": losses[-1][1], "smooth_passes": smooth},
        "rules": {k: {"resid_per_step": v["resid"], "mean_resid": float(np.mean(v["resid"])),
                      "sor_iters_per_step": float(np.mean(v["iters"])), "ms_per_step": float(np.mean(v["ms"]))}
                  for k, v in rows.items()},
    }
    net.close()
    print(json.dumps(out), flush=True)


def bench_warm_start(args, les, torch):
    """Plain SOR from p_prev against the learned start on held-out C1
    cases (train on seeds 11-14, evaluate on 21-22); network inference is
    inside the timed steps."""
    import numpy as np
    from paper_1504_02264_amd import warmstart as ws
    if args.workload == "C3":
        return bench_warm_start_c3(args, les, torch)
    if args.workload == "C2":
        return bench_warm_start_c2(args, les, torch)
    smooth = 16
    Xs, Ts = [], []
    for seed in (11, 12, 13, 14):
        X, T, _ = ws.collect("C1", seed, steps=24, skip=2, smooth=smooth)
        Xs.append(X)
        Ts.append(T)
    X, T = ws.mirror_y(torch.cat(Xs), torch.cat(Ts))
    net = les.Net(seed=0, lr=1e-3)
    t0 = time.perf_counter()
    scale, losses = ws.train(net, X, T, iters=12000, batch=8, lr=1e-3, lr_final=5e-5)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del X, T
    rows = []
    for seed in (21, 22):
        b = ws.evaluate("C1", seed, steps=args.steps, net=None, skip=2)
        rows.append(("plain", seed, b))
        for name, rule, param in (("residual rule", les.WARM_RESIDUAL, 0), ("trial rule 64", les.WARM_TRIAL, 64),
                                  ("always", les.WARM_ALWAYS, 0)):
            w = ws.evaluate("C1", seed, steps=args.steps, net=net, scale=scale, skip=2, rule=rule, param=param,
                            smooth=smooth)
            rows.append((name, seed, w))
    res = {}
    for name, seed, r in rows:
        d = res.setdefault(name, {"iters": [], "ms": [], "taken": 0})
        d["iters"].append(float(r["iters"].mean()))
        d["ms"].append(r["ms_per_step"])
        d["taken"] += int(r.get("taken", 0))
    base_ms = float(np.mean(res["plain"]["ms"]))
    out = {
        "metric": "time to relative residual 1e-5 per step (learned start)",
        "value": float(np.mean(res["always"]["ms"])),
        "unit": "ms/step",
        "higher_is_better": False,
        "n_gpus": 1,
        "steps": args.steps,
        "dtype": "f32 LES, bf16 network",
        "data": "synthetic",
        "config": {"workload": "C1 64x64x32 urban LES; network trained on building seeds 11-14 "
                               "(96 captured pairs and their mirror images in y, 12000 Adam steps), evaluated on seeds 21-22",
                   "train_s": train_s, "final_loss": losses[-1][1], "smooth_passes": smooth},
        "rules": {k: {"sor_iters_per_step": float(np.mean(v["iters"])), "ms_per_step": float(np.mean(v["ms"])),
                      "steps_from_network": v["taken"], "ms_vs_plain": float(np.mean(v["ms"])) / base_ms}
                  for k, v in res.items()},
    }
    net.close()
    print(json.dumps(out), flush=True)


def bench_twinned(args, les, torch):
    """Twinned double buffering (section 2.6) against red-black SOR at the
    same iteration counts (the paper's default setup runs 50), from p = 0
    on the Poisson rhs of the workload's first step.  Twinned: device time
    of its sweeps (events); red-black: host wall time of the stand-alone
    solve with the residual checks (tol unreachable, so it runs max_iter)."""
    import numpy as np
    from les_inputs import WORKLOADS, make_workload_inputs
    w = WORKLOADS[args.workload]
    cells = w.nx * w.ny * w.nz
    mask, prof = make_workload_inputs(w)
    g = les.LES(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.dt, mask)
    g.set_inflow(prof, w.noise_amp, w.seed)
    variant, _ = g.autotune(reps=20)
    g.step(1)
    rhs = torch.from_numpy(np.ascontiguousarray(g.get_rhs(), dtype=np.float32)).cuda()
    p = torch.zeros_like(rhs)
    rows = []
    for n in (50, 500):
        best_tw, best_rb = None, None
        for _ in range(3):
            p.zero_()
            st_tw, ms_tw = g.pressure_solve_twinned(rhs, p, 1.0, n)
            best_tw = ms_tw if best_tw is None else min(best_tw, ms_tw)
            p.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st_rb, _ = g.pressure_solve_dev(rhs, p, tol=1e-30, max_iter=n)
            torch.cuda.synchronize()
            ms_rb = (time.perf_counter() - t0) * 1e3
            best_rb = ms_rb if best_rb is None else min(best_rb, ms_rb)
        tw_bytes = 32.0 * cells * n            # per half: pair 8 B + rhs 4 B + one component 4 B
        rows.append({"iters": n,
                     "twinned": {"resid": st_tw["resid"], "ms": best_tw, "us_per_iter": 1e3 * best_tw / n,
                                 "GB_per_s": tw_bytes / (best_tw * 1e-3) / 1e9,
                                 "hbm_frac": tw_bytes / (best_tw * 1e-3) / 8e12},
                     "red_black": {"resid": st_rb["resid"], "ms": best_rb, "us_per_iter": 1e3 * best_rb / n,
                                   "sor_variant": int(variant)}})
        log(f"{n} iterations: twinned {1e3 * best_tw / n:.1f} us/it resid {st_tw['resid']:.3e}; "
            f"red-black {1e3 * best_rb / n:.1f} us/it resid {st_rb['resid']:.3e}")
    out = {"metric": "twinned double buffering vs red-black SOR at fixed iteration counts",
           "unit": "us per iteration, relative residual", "n_gpus": 1, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"{args.workload} {w.nx}x{w.ny}x{w.nz} urban LES, Poisson rhs of the first step, "
                                  "from p = 0; twinned omega 1, red-black omega 1.8"},
           "rows": rows}
    g.close()
    print(json.dumps(out), flush=True)


def bench_ensemble(args, les, torch):
    """Aggregate cell-updates/s of an uneven ensemble (batched solves by default)."""
    import numpy as np
    from les_inputs import ensemble_members, make_workload_inputs
    ws = ensemble_members(args.ensemble)
    members = []
    for w in ws:
        mask, prof = make_workload_inputs(w)
        extra = {} if args.max_iter is None else {"max_iter": args.max_iter}
        # the members check their residuals at the benchmark's interval (fold
        # and rebase every 128 iterations), as the single-grid benchmark does
        K = args.check_every
        g = les.LES(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.dt, mask, check_every=K,
                    rebase_every=max(1, 128 // K), **extra)
        g.set_inflow(prof, w.noise_amp, w.seed)
        members.append(g)
    ens = les.Ensemble(members)
    ens.set_mode(les.ENSEMBLE_BATCHED if args.ensemble_mode == "batched" else les.ENSEMBLE_PERSISTENT)
    variant, us = ens.autotune(reps=3)
    log(f"ensemble autotune: variant {variant}, us per half-sweep {[round(float(x), 1) for x in us]}")
    if args.sor_variant is not None:
        variant = args.sor_variant
        ens.set_variant(variant)
        log(f"ensemble sweep variant {variant} as asked")
    cells = sum(w.nx * w.ny * w.nz for w in ws)
    log(f"ensemble of {len(ws)} members, {cells} cells; warmup {args.warmup}")
    for k in range(args.warmup):
        ens.step(1)
        log(f"warmup step {k + 1} done")
    torch.cuda.synchronize()
    # one call per step (each returns after its solves), a line after each
    t0 = time.perf_counter()
    its, n_capped = [], 0
    for k in range(args.steps):
        rc, st, it = ens.step(1)
        its.append(it)
        n_capped += int(st["not_converged"])
        log(f"timed step {k + 1}: {time.perf_counter() - t0:.3f} s so far")
    torch.cuda.synchronize()
    dt_s = time.perf_counter() - t0
    iters = np.concatenate(its, axis=0)
    log(f"timed {args.steps} steps in {dt_s:.3f} s; mean SOR iterations {iters.mean():.0f}")
    out = {
        "metric": "LES cell-updates/s (ensemble aggregate)",
        "value": cells * args.steps / dt_s,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt_s * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"ensemble of {len(ws)} urban LES members, nx, ny in 96-256, nz in 64-90, "
                         "power-law inflow (alpha 0.1-0.35, 2-12 m/s), 15-35% building cover, "
                         f"{args.ensemble_mode} solve of all members to relative residual 1e-5, "
                         f"checked every {args.check_every} iterations"),
            "cells_total": cells,
            "sor_iters_mean": float(iters.mean()),
            "sor_iters_min": int(iters.min()),
            "sor_iters_max": int(iters.max()),
            "not_converged_member_steps": n_capped,
            "sor_variant": int(variant),
            "autotune_us_per_sweep": [round(float(x), 2) for x in us],
        },
    }
    ens.close()
    for g in members:
        g.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C2", choices=["C1", "C2", "C3"])
    ap.add_argument("--ensemble-mode", choices=["batched", "persistent"], default="batched")
    ap.add_argument("--ensemble", type=int, default=0, metavar="N",
                    help="instead: an ensemble of N uneven members (sizes 96-256 x 96-256 x "
                         "64-90, seeds 1000+i) advanced together; aggregate cell-updates/s")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-net", action="store_true",
                    help="skip the warm-start network timing (forward / train step on a 64x128x128 crop)")
    ap.add_argument("--warm-start", action="store_true",
                    help="instead of the LES line: plain SOR vs the learned start on held-out cases "
                         "(C1 size; with --workload C3, trained on crops of 1024x1024x96 runs)")
    ap.add_argument("--twinned", action="store_true",
                    help="compare twinned double buffering with red-black SOR (JSON line of its own)")
    ap.add_argument("--check-every", type=int, default=64, metavar="K",
                    help="residual check interval of the timed solves (fused sweeps need an even K, "
                         "the two-iteration form a multiple of 4)")
    ap.add_argument("--omega", type=float, default=1.8,
                    help="SOR relaxation factor (the workloads' 1.8 by default; other values are a study, "
                         "not the configured benchmark)")
    ap.add_argument("--no-omega-study", action="store_true",
                    help="skip the study that continues the timed state for 2 steps with Young's "
                         "relaxation factor for the operator (reported beside the configured line)")
    ap.add_argument("--cpu-sample-iters", type=int, default=200)
    ap.add_argument("--oracle-sample", default=None, metavar="WORKLOAD",
                    help=argparse.SUPPRESS)   # child process of the single-thread CPU baseline
    ap.add_argument("--no-timing", action="store_true",
                    help="do not bracket kernels with HIP events (no roofline object)")
    ap.add_argument("--max-iter", type=int, default=None,
                    help="cap SOR iterations per step (profiling runs only; not the benchmark)")
    ap.add_argument("--sor-variant", type=int, default=None, metavar="V",
                    help="run SOR sweep variant V instead of the autotuner's choice (profiling "
                         "runs: a profiler's per-dispatch overhead can change that choice)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="also run 5 plain torch copies of MB megabytes (the known-size kernel "
                         "that scales rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.oracle_sample:
        print(json.dumps(oracle_sample(args.oracle_sample, args.cpu_sample_iters)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "slab decomposition is a design note, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1504_02264_amd as les
    from les_inputs import WORKLOADS, make_workload_inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.warm_start:
        return bench_warm_start(args, les, torch)
    if args.twinned:
        return bench_twinned(args, les, torch)
    if args.ensemble:
        return bench_ensemble(args, les, torch)
    w = WORKLOADS[args.workload]
    cells = w.nx * w.ny * w.nz
    mask, prof = make_workload_inputs(w)
    # the configured step solves to the tolerance: the cap is only a guard
    # (a converged 300x300x90 step takes about 1.5e5 iterations at omega 1.8)
    max_iter = args.max_iter if args.max_iter is not None else BENCH_MAX_ITER
    # residual checked every K iterations; the fold-and-rebase cadence kept
    # at 128 iterations whatever K
    K = args.check_every
    g = les.LES(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.dt, mask,
                timing=0 if args.no_timing else 1, max_iter=max_iter, omega=args.omega,
                check_every=K, rebase_every=max(1, 128 // K))
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    g.set_inflow(prof, w.noise_amp, w.seed)
    variant, us = g.autotune(reps=50)
    log(f"autotune: SOR sweep variant {variant}; us per half-sweep {[round(x, 2) for x in us]}")
    if args.sor_variant is not None:
        variant = args.sor_variant
        g.set_sor_variant(variant)
        log(f"SOR sweep variant {variant} as asked")
    log(f"workload {w.name} {w.nx}x{w.ny}x{w.nz} ({cells} cells); warmup {args.warmup} steps")
    if args.warmup:
        g.step(args.warmup)
    g.get_timing(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st, iters = g.step(args.steps)
    torch.cuda.synchronize()
    dt_s = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {dt_s:.3f} s; SOR iterations/step mean {iters.mean():.0f}")
    timing = g.get_timing(reset=True)

    value = cells * args.steps / dt_s
    n_capped = int(st["not_converged"])
    solve = (f"red-black SOR omega={args.omega:g} to relative residual 1e-5, checked every {K} iterations "
             f"(all {args.steps} timed steps converged)"
             if n_capped == 0 else
             f"red-black SOR omega={args.omega:g} toward relative residual 1e-5, checked every {K} iterations, "
             f"capped at max_iter={max_iter} per step: "
             f"{n_capped} of {args.steps} timed steps stopped at the cap, last relative residual "
             f"{st['resid_last']:.2e}")
    out = {
        "metric": "LES cell-updates/s",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt_s * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{w.name}: urban LES {w.nx}x{w.ny}x{w.nz}, dx=dy={w.dx} m dz={w.dz} m, "
                         f"dt={w.dt} s, {int(w.coverage * 100)}% building cover (heights "
                         f"{w.h_min}-{w.h_max} cells), {w.profile}-law inflow + {w.noise_amp:.0%} "
                         f"noise, {solve}"),
            "cells": cells,
            "max_iter": int(max_iter),
            "sor_iters_per_step": float(iters.mean()),
            "steps_per_s": args.steps / dt_s,
            "not_converged_steps": n_capped,
            "resid_last": st["resid_last"],
            # per timed step: SOR iterations and wall time from the previous
            # step's pressure to relative residual 1e-5 (plain SOR)
            "time_to_tol": {"tol": 1e-5, "converged_steps": args.steps - n_capped,
                            "sor_iters_per_step": float(iters.mean()),
                            "sor_iters_min": int(iters.min()), "sor_iters_max": int(iters.max()),
                            "ms_per_step": dt_s * 1e3 / args.steps},
            "sor_variant": int(variant),
            "autotune_us_per_sweep": [round(float(x), 3) for x in us],
        },
    }
    sor_ms, sor_n = timing["sor"]
    if sor_n > 0:
        t_launch = sor_ms / sor_n * 1e-3
        fused = variant >= les.NUM_SPLIT_SOR_VARIANTS
        two = variant >= les.FIRST_TWO_ITER_SOR_VARIANT
        iters_per_launch = 2 if two else (1 if fused else 0.5)
        # algorithmic bytes per launch = the per-cell-iteration figure of the
        # sweep's form (16 B for two half-sweeps, 12 B for a fused
        # iteration) x the cell-iterations one launch performs: 8 B/cell for
        # a half-sweep, 12 for a fused iteration, 24 for two fused
        # iterations.  The two-iteration form moves only the 12 B/cell of
        # one iteration (its minimum bytes): its measured traffic can sit
        # below the algorithmic bytes.
        per_unit = 12.0 if fused else 16.0
        bytes_per_launch = per_unit * iters_per_launch * cells
        min_bytes_per_launch = (12.0 if fused else 8.0) * cells
        achieved = bytes_per_launch / t_launch / 1e9
        from paper_1504_02264_amd import profsum
        # kernel names as the profiler prints them (uniform-grid instantiations)
        if two:
            kname, what = "k_sor_rb2<false>", "two fused red-black SOR iterations"
        elif fused:
            tx, kt, nw = les.SOR_VARIANTS[variant]
            kname, what = f"k_sor_rb<{tx}, {nw}, {kt}, false>", "fused red-black SOR iteration"
        else:
            tx, kt = les.SOR_VARIANTS[variant]
            kname, what = f"k_sor<{tx}, {kt}, false>", "red-black SOR half-sweep"
        pmc_file = os.path.join(ROOT, "profiles", f"k_sor_traffic_{w.nx}x{w.ny}x{w.nz}.txt")
        tr = profsum.read_traffic(pmc_file, kname)
        out["roofline"] = {
            "bound": "hbm",
            "kernel": f"{kname} ({what})",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            # measured HBM bytes of the same launch (rocprofv3 FETCH_SIZE +
            # WRITE_SIZE, copy-calibrated) over the same launch time; null if
            # the kernel changed since the counters were taken
            "traffic": None if tr is None else (tr[0] + tr[1]) / t_launch / 1e9,
            "traffic_bytes_per_launch": None if tr is None else tr[0] + tr[1],
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "launch_us": t_launch * 1e6,
            "iterations_per_launch": iters_per_launch,
            "us_per_iteration": t_launch * 1e6 / iters_per_launch,
            "bytes_per_cell_iteration": per_unit,
            # the bytes a launch must move at least (p and r0 read once, p
            # written once) and that rate as a fraction of the peak
            "min_bytes_per_launch": min_bytes_per_launch,
            "min_bytes_frac": min_bytes_per_launch / t_launch / 1e9 / HBM_PEAK_GBS,
            "timed_launches": int(sor_n),
        }
        out["kernel_ms_per_step"] = {k: v[0] / args.steps for k, v in timing.items()
                                     if v[1] > 0 and k not in ("sor", "check")}
        # the residual checks are sampled with the sweeps (one interval in 8):
        # mean check time (skipped ones included) times the intervals per step
        chk_ms, chk_n = timing["check"]
        if chk_n > 0:
            out["kernel_ms_per_step"]["check"] = chk_ms / chk_n * float(iters.mean()) / K
        # the SOR sweeps are sampled (one check interval in 8): scale to all
        out["kernel_ms_per_step"]["sor"] = (sor_ms / sor_n) / iters_per_launch * float(iters.mean())
        # device time of the pressure solve per timed step (sweeps, stopping
        # tests, fold and rebase), whether or not the steps converged
        out["solve_kernel_ms_per_step"] = (out["kernel_ms_per_step"]["sor"]
                                           + out["kernel_ms_per_step"].get("check", 0.0)
                                           + out["kernel_ms_per_step"].get("rebase", 0.0))
    if not args.no_omega_study:
        log("omega study: Young's relaxation factor from the timed state")
        out["omega_study"] = omega_study(les, torch, w, mask, g, variant, young_omega(w), K)
    if not args.no_net:
        log("warm-start network: forward and train step on a 64x128x128 crop")
        out["warm_start_net"] = bench_net(les, torch)
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle, bounded sample)")
        out["cpu_baseline"] = cpu_baseline(w, float(iters.mean()), args.cpu_sample_iters)
    g.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
