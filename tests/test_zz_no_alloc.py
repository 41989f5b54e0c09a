"""The allocation-free stand-alone solve (les_pressure_solve_noalloc)
against les_pressure_solve_dev through the C ABI: same kernels and
iterates on a static workspace, so the answers are identical; two calls in
a row, the second on a smaller grid (the workspace keeps the first call's
contents in another layout and must be cleared), and a grid beyond the
workspace refused."""
import numpy as np
import pytest

import paper_1504_02264_amd as les
from les_inputs import random_rhs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("bc", [les.URBAN_BC, (les.FREESLIP,) * 6])
def test_noalloc_equals_dev_solve_two_calls(bc):
    import torch
    prev = None
    for shape, seed in (((150, 150, 90), 3), ((40, 33, 21), 4)):
        nx, ny, nz = shape
        print(f"[noalloc] {shape} bc={'urban' if bc == les.URBAN_BC else 'walls'}", flush=True)
        g = les.LES(nx, ny, nz, 2.0, 2.0, 1.0, 0.05, bc=bc)
        try:
            rhs = torch.from_numpy(random_rhs(nx, ny, nz, seed=seed, smooth=2)).cuda()
            p0 = torch.from_numpy(random_rhs(nx, ny, nz, seed=seed + 1, smooth=1) * 0.1).cuda()
            p_dev = p0.clone()
            p_na = p0.clone()
            st_d, rc_d = g.pressure_solve_dev(rhs, p_dev, tol=1e-5, max_iter=3000)
            st_n, rc_n = g.pressure_solve_noalloc(rhs, p_na, tol=1e-5, max_iter=3000)
            torch.cuda.synchronize()
            assert rc_n == rc_d
            assert st_n["iters"] == st_d["iters"] and st_n["resid"] == st_d["resid"]
            assert torch.equal(p_na, p_dev)
            assert st_n["iters"] > 0
            prev = shape
        finally:
            g.close()
    assert prev == (40, 33, 21)


def test_noalloc_refuses_a_grid_beyond_its_workspace():
    import torch
    nx, ny, nz = 256, 256, 128
    g = les.LES(nx, ny, nz, 2.0, 2.0, 1.0, 0.05)
    try:
        rhs = torch.zeros((nz, ny, nx), device="cuda")
        p = torch.zeros_like(rhs)
        with pytest.raises(les.LesError) as e:
            g.pressure_solve_noalloc(rhs, p, tol=1e-5, max_iter=10)
        assert e.value.code == les.LES_EINVAL
        assert "64 MiB" in str(e.value)
        # the handle still solves through the allocating entry point
        st, rc = g.pressure_solve_dev(rhs, p, tol=1e-5, max_iter=10)
        assert rc == les.LES_OK and st["iters"] == 0
    finally:
        g.close()
