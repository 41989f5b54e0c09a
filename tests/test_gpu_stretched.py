"""GPU parity on stretched grids (the paper's 1-D spacing arrays dx1, dy1,
dzn of section 2.5.3 and the per-axis SOR coefficients of section 2.6):
les_create_stretched through the C ABI against the FP64 oracle built on
the same cell widths.

As for uniform grids, the oracle replays the GPU's per-step SOR iteration
counts, so the two differ by float32 rounding only; bar: relative L2 per
field <= 1e-5 after one step, <= 1e-4 after ten.
"""
import numpy as np
import pytest

import oracle
import paper_1504_02264_amd as les
from les_inputs import (building_heights, building_mask, log_law_profile, random_rhs,
                        smooth_widths, stretched_widths)

pytestmark = pytest.mark.gpu


def rel(a, b):
    nb = np.linalg.norm(np.asarray(b, np.float64))
    return np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64)) / max(nb, 1e-300)


def widths(case, nx, ny, nz):
    """Cell widths per axis: 'z' stretches only the vertical (finer near the
    ground, growing 12% per cell above the first 3), 'xyz' all three axes
    (smooth mappings with different amplitudes)."""
    if case == "z":
        return 4.0, 4.0, stretched_widths(nz, 1.0, 1.12, n_uniform=3)
    return (smooth_widths(nx, 4.0 * nx, 0.45), smooth_widths(ny, 4.0 * ny, -0.35),
            stretched_widths(nz, 1.0, 1.08, n_uniform=2))


def urban_inputs(nx, ny, nz, hz, seed, hmax):
    h = building_heights(nx, ny, nz, 0.15, 2, 4, 2, hmax, seed=seed, margin_x=4, margin_y=2)
    return building_mask(h, nz), log_law_profile(nz, hz)


def pair(nx, ny, nz, hx, hy, hz, mask=None, dt=0.05, **kw):
    g = les.LES(nx, ny, nz, hx, hy, hz, dt, mask, **kw)
    o = oracle.Oracle(nx, ny, nz, hx, hy, hz, dt, mask, **kw)
    return g, o


@pytest.mark.parametrize("shape,case", [((33, 17, 9), "z"), ((24, 20, 12), "xyz"),
                                        ((64, 64, 32), "z"), ((45, 38, 20), "xyz")])
def test_stretched_one_step_parity(shape, case):
    nx, ny, nz = shape
    print(f"[stretched one step] {shape} {case}", flush=True)
    hx, hy, hz = widths(case, nx, ny, nz)
    mask, prof = urban_inputs(nx, ny, nz, hz, seed=nx + nz, hmax=max(3, nz // 3))
    g, o = pair(nx, ny, nz, hx, hy, hz, mask)
    try:
        g.set_inflow(prof, 0.01, 7)
        o.set_inflow(prof, 0.01, 7)
        rc, st, iters = g.step(1)
        assert rc == les.LES_OK
        o.step(1, forced=iters)
        for name, a, b in zip("uvwp", g.get_fields(), o.get_fields()):
            e = rel(a, b)
            print(f"  {name}: rel L2 {e:.3e}", flush=True)
            assert e <= 1e-5, name
        assert rel(g.get_nut(), o.get_nut()) <= 1e-5
        assert rel(g.get_rhs(), o.get_rhs()) <= 1e-5
        for a, b in zip(g.get_force(), o.get_force()):
            assert rel(a, b) <= 1e-5
        for a, b in zip(g.get_usum(), o.get_usum()):
            if np.linalg.norm(b) > 0:
                assert rel(a, b) <= 1e-5
        # projection identity (P5) holds on a stretched grid too
        assert st["div_new_last"] / st["div_star_last"] == pytest.approx(st["resid_last"], rel=0.05)
    finally:
        g.close()


def test_stretched_ten_step_parity():
    nx, ny, nz = 64, 64, 32
    hx, hy, hz = widths("xyz", nx, ny, nz)
    mask, prof = urban_inputs(nx, ny, nz, hz, seed=1, hmax=10)
    print("[stretched ten steps] 64x64x32 xyz", flush=True)
    g, o = pair(nx, ny, nz, hx, hy, hz, mask)
    try:
        g.set_inflow(prof, 0.01, 1)
        o.set_inflow(prof, 0.01, 1)
        rc, st, iters = g.step(10)
        assert rc == les.LES_OK and st["not_converged"] == 0
        o.step(10, forced=iters)
        for name, a, b in zip("uvwp", g.get_fields(), o.get_fields()):
            e = rel(a, b)
            print(f"  {name}: rel L2 {e:.3e} iters {list(iters)}", flush=True)
            assert e <= 1e-4, name
    finally:
        g.close()


@pytest.mark.parametrize("shape,case", [((5, 7, 4), "z"), ((33, 17, 9), "xyz"), ((64, 48, 16), "xyz")])
def test_stretched_pressure_solve_parity(shape, case):
    nx, ny, nz = shape
    hx, hy, hz = widths(case, max(nx, 4), max(ny, 4), max(nz, 4))
    g, o = pair(nx, ny, nz, hx, hy, hz)
    try:
        rhs = random_rhs(nx, ny, nz, seed=nx * 3 + nz, smooth=2)
        p0 = random_rhs(nx, ny, nz, seed=5, smooth=1) * 0.1
        p, st, rc = g.pressure_solve(rhs, p0, tol=1e-5, max_iter=50000)
        assert rc == les.LES_OK and st["converged"] == 1
        po, _, _ = o.pressure_solve(rhs, p0, tol=1e-5, max_iter=50000, forced=st["iters"])
        assert rel(p, po) <= 1e-5
        _, stf, _ = o.pressure_solve(rhs, p0, tol=1e-5, max_iter=50000)
        assert abs(stf["iters"] - st["iters"]) <= 4
    finally:
        g.close()


def test_stretched_sor_variants_bitwise_identical():
    """Every sweep variant (half-sweeps and fused iterations) runs the same
    per-cell update on a stretched grid: same answer, same count."""
    nx, ny, nz = 45, 37, 19
    hx, hy, hz = widths("xyz", nx, ny, nz)
    g = les.LES(nx, ny, nz, hx, hy, hz, 0.05)
    try:
        rhs = random_rhs(nx, ny, nz, seed=8, smooth=2)
        ref = None
        for v in range(les.NUM_SOR_VARIANTS):
            g.set_sor_variant(v)
            p, st, rc = g.pressure_solve(rhs, None, tol=1e-5)
            if ref is None:
                ref = (p, st["iters"])
            else:
                assert st["iters"] == ref[1], v
                assert np.array_equal(p, ref[0]), v
    finally:
        g.close()


def test_equal_widths_match_the_uniform_grid():
    """A stretched handle with equal widths runs the stretched kernels on a
    uniform table: the same fields as the uniform handle up to rounding."""
    nx, ny, nz = 33, 17, 9
    h = building_heights(nx, ny, nz, 0.15, 2, 4, 2, 4, seed=4, margin_x=4, margin_y=2)
    mask, prof = building_mask(h, nz), log_law_profile(nz, 2.0)
    a = les.LES(nx, ny, nz, 4.0, 4.0, 2.0, 0.05, mask)
    b = les.LES(nx, ny, nz, np.full(nx, 4.0), np.full(ny, 4.0), np.full(nz, 2.0), 0.05, mask)
    try:
        for x in (a, b):
            x.set_inflow(prof, 0.01, 4)
        _, _, ia = a.step(1)
        _, _, ib = b.step(1)
        assert abs(int(ia[0]) - int(ib[0])) <= 4
        for x, y in zip(a.get_fields(), b.get_fields()):
            assert rel(y, x) <= 1e-5
        assert rel(b.get_nut(), a.get_nut()) <= 1e-6
        for x, y in zip(a.get_force(), b.get_force()):
            assert rel(y, x) <= 1e-6
    finally:
        a.close()
        b.close()


def test_stretched_full_size_step():
    """300 x 300 x 90 with the vertical stretched (1 m at the ground growing
    3% per cell): one step with the solve capped at 400 iterations, every
    field against the oracle replaying the same count."""
    nx, ny, nz = 300, 300, 90
    hz = stretched_widths(nz, 1.0, 1.03, n_uniform=4)
    h = building_heights(nx, ny, nz, 0.30, 2, 16, 5, 40, seed=2, margin_x=8, margin_y=4)
    mask, prof = building_mask(h, nz), log_law_profile(nz, hz)
    print("[stretched full size] 300x300x90, 400 iterations", flush=True)
    g, o = pair(nx, ny, nz, 4.0, 4.0, hz, mask, max_iter=400)
    try:
        g.autotune(reps=5)
        g.set_inflow(prof, 0.01, 2)
        o.set_inflow(prof, 0.01, 2)
        rc, st, iters = g.step(1)
        assert iters[0] == 400
        o.step(1, forced=iters)
        for name, a, b in zip("uvwp", g.get_fields(), o.get_fields()):
            e = rel(a, b)
            print(f"  {name}: rel L2 {e:.3e}", flush=True)
            assert e <= 1e-5, name
    finally:
        g.close()


def test_stretched_refusals():
    nx, ny, nz = 16, 12, 8
    hz = stretched_widths(nz, 1.0, 1.1)
    with pytest.raises(les.LesError) as e:
        les.LES(nx, ny, nz, 2.0, 2.0, hz, 0.05, bc=(les.FREESLIP,) * 6)
    assert e.value.code == les.LES_EINVAL
    bad = hz.copy()
    bad[3] = 0.0
    with pytest.raises(les.LesError):
        les.LES(nx, ny, nz, 2.0, 2.0, bad, 0.05)
    g = les.LES(nx, ny, nz, 2.0, 2.0, hz, 0.05)
    u = les.LES(nx, ny, nz, 2.0, 2.0, 1.0, 0.05)
    try:
        with pytest.raises(les.LesError):
            les.Ensemble([u, g])
        import torch
        d = torch.zeros((nz, ny, nx), device="cuda")
        with pytest.raises(les.LesError) as e:
            g.pressure_solve_twinned(d, d.clone(), 1.0, 5)
        assert e.value.code == les.LES_EINVAL
        net = les.Net(seed=0)
        try:
            with pytest.raises(les.LesError):
                les.set_warm_start(g, net)
        finally:
            net.close()
    finally:
        g.close()
        u.close()
