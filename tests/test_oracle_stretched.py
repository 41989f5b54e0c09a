"""Pins of the FP64 oracle on stretched (non-uniform) grids.

The paper's velfg assembly carries 1-D spacing arrays (dx1, dy1, dzn;
section 2.5.3) and its SOR per-axis neighbour weights with a 3-D diagonal
(section 2.6), i.e. the method runs on axes with varying cell widths.  These
tests fix the oracle's stretched-grid arithmetic against facts outside it:
the operator identity and its symmetry in the volume-weighted inner
product, a dense solve, second-order convergence to an analytic solution,
and closed forms that linear interpolation and central differences must
reproduce exactly on any grid (linear fields, quadratic diffusion).
"""
import math

import numpy as np
import pytest

import oracle
from les_inputs import (building_heights, building_mask, cell_centres, log_law_profile,
                        smooth_widths, stretched_widths)
from oracle import FREESLIP, INFLOW, OUTFLOW, URBAN_BC

ALL_WALLS = (FREESLIP,) * 6


def widths(n, h0, ratio, seed=None):
    """Geometric stretching, optionally jittered so that no two widths agree."""
    h = stretched_widths(n, h0, ratio)
    if seed is not None:
        h = h * np.random.default_rng(seed).uniform(0.8, 1.25, n)
    return h


def make(nx, ny, nz, hx, hy, hz, dt=0.05, mask=None, **kw):
    return oracle.Oracle(nx, ny, nz, hx, hy, hz, dt, mask, **kw)


def faces_of(h):
    return np.concatenate(([0.0], np.cumsum(h)))


def assemble(o, fn):
    n = o.nx * o.ny * o.nz
    M = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        M[:, c] = fn(e.reshape(o.shapes[3])).ravel()
    return M


def assemble_DG(o):
    su, sv, sw, _ = o.shapes
    z = (np.zeros(su), np.zeros(sv), np.zeros(sw))

    def dg(p):
        u, v, w = o.project(*z, p)          # u = -dt G p
        return -o.divergence(u, v, w) / o.dt
    return assemble(o, dg)


def volumes(o):
    return (o.hz[:, None, None] * o.hy[None, :, None] * o.hx[None, None, :]).ravel()


# ------------------------------------------------------------- operator
@pytest.mark.parametrize("bc", [URBAN_BC, ALL_WALLS])
def test_stretched_operator_is_div_grad_and_volume_symmetric(bc):
    """A = D G on a grid stretched along every axis, and V A is symmetric
    (V the cell volumes): the discrete Laplacian of a finite-volume MAC
    grid is self-adjoint in the volume-weighted inner product."""
    nx, ny, nz = 6, 5, 4
    o = make(nx, ny, nz, widths(nx, 1.1, 1.3, 1), widths(ny, 0.7, 0.8, 2), widths(nz, 0.4, 1.5, 3),
             bc=bc)
    A = assemble(o, o.apply_A)
    DG = assemble_DG(o)
    scale = np.abs(A).max()
    assert np.abs(A - DG).max() <= 1e-13 * scale
    VA = volumes(o)[:, None] * A
    assert np.allclose(VA, VA.T, rtol=0, atol=1e-14 * np.abs(VA).max())
    assert not np.allclose(A, A.T, rtol=0, atol=1e-6 * scale)   # plain A is not symmetric
    # negative semi-definite, with the constants as null space only without an outflow face
    ev = np.linalg.eigvals(VA)
    assert ev.real.max() <= 1e-12 * scale * volumes(o).max()
    n_zero = int(np.sum(np.abs(ev) <= 1e-10 * np.abs(ev).max()))
    assert n_zero == (0 if bc[1] == OUTFLOW else 1)


@pytest.mark.parametrize("bc", [URBAN_BC, ALL_WALLS])
def test_stretched_sor_matches_dense_solve(bc):
    """P1 on a stretched grid: SOR to 1e-13 equals LAPACK on D G."""
    nx, ny, nz = 8, 6, 5
    o = make(nx, ny, nz, widths(nx, 2.0, 1.2, 4), widths(ny, 1.5, 1.0, 5), widths(nz, 0.5, 1.4),
             bc=bc)
    rhs = np.random.default_rng(7).standard_normal(o.shapes[3])
    DG = assemble_DG(o)
    if bc[1] == OUTFLOW:
        want = np.linalg.solve(DG, rhs.ravel())
    else:
        # solvable part: the volume-weighted mean removed (V A symmetric, so
        # the null space of A^T is V); the gauge is the weighted mean too
        V = volumes(o)
        r = rhs.ravel() - np.dot(V, rhs.ravel()) / V.sum()
        want = np.linalg.lstsq(DG, r, rcond=None)[0]
        want -= np.dot(V, want) / V.sum()
    p, st, rc = o.pressure_solve(rhs, tol=1e-13, max_iter=400000)
    assert rc == 0 and st["converged"] == 1
    assert np.linalg.norm(p.ravel() - want) <= 1e-9 * np.linalg.norm(want)


def test_stretched_poisson_converges_at_second_order():
    """Grid convergence to an analytic solution on a smoothly stretched grid.

    p = cos(pi x / (2 Lx)) cos(pi z / Lz) is flat at the inflow face and
    the walls and zero on the outflow face, so it satisfies the urban
    operator's boundary conditions; its Laplacian is -(pi^2/(4 Lx^2) +
    pi^2/Lz^2) p.  Solving with that right-hand side at the cell centres on
    x and z axes mapped smoothly (the same mapping at every resolution),
    the error at the centres must fall by about 4 per halving of the
    widths.
    """
    Lx, Ly, Lz = 3.0, 1.0, 2.0
    errs = []
    for n in (8, 16, 32):
        nx, ny, nz = n, 4, n
        hx, hz = smooth_widths(nx, Lx, 0.6), smooth_widths(nz, Lz, -0.5)
        o = make(nx, ny, nz, hx, Ly / ny, hz, bc=URBAN_BC, omega=1.9)
        xc, zc = cell_centres(nx, hx), cell_centres(nz, hz)
        pe = (np.cos(np.pi * xc / (2 * Lx))[None, None, :] * np.cos(np.pi * zc / Lz)[:, None, None]
              * np.ones((1, ny, 1)))
        lam = -(np.pi**2 / (4 * Lx**2) + np.pi**2 / Lz**2)
        p, st, rc = o.pressure_solve(lam * pe, tol=1e-12, max_iter=500000)
        assert rc == 0
        errs.append(np.abs(p - pe).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 <= r1 <= 5.0 and 3.5 <= r2 <= 4.6, errs


# --------------------------------------------------------- closed forms
def _faces_linear(o, G, a0=(0.0, 0.0, 0.0)):
    """u_i = a0_i + G_ij x_j on the MAC faces of a stretched grid."""
    xf, yf, zf = faces_of(o.hx), faces_of(o.hy), faces_of(o.hz)
    xc, yc, zc = cell_centres(o.nx, o.hx), cell_centres(o.ny, o.hy), cell_centres(o.nz, o.hz)

    def lin(c, X, Y, Z):
        return a0[c] + G[c][0] * X[None, None, :] + G[c][1] * Y[None, :, None] + G[c][2] * Z[:, None, None]

    return lin(0, xf, yc, zc), lin(1, xc, yf, zc), lin(2, xc, yc, zf)


def _stretched_case(cs=0.0, nu=0.0, bc=ALL_WALLS, n=(8, 7, 9)):
    nx, ny, nz = n
    return make(nx, ny, nz, widths(nx, 0.6, 1.15, 11), widths(ny, 0.9, 0.9, 12),
                widths(nz, 0.3, 1.2, 13), cs=cs, nu=nu, bc=bc)


def test_stretched_divergence_of_linear_field():
    """P11 on a stretched grid: u = a x, v = b y, w = c z gives a + b + c."""
    o = _stretched_case()
    G = np.diag([0.3, -1.7, 2.5])
    div = o.divergence(*_faces_linear(o, G))
    assert np.allclose(div, 0.3 - 1.7 + 2.5, rtol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_stretched_smagorinsky_linear_field(seed):
    """P8 on a stretched grid: a linear field has constant strain, so
    nu_t = (Cs Delta)^2 sqrt(2 S:S) with Delta the cube root of each
    cell's own volume."""
    cs = 0.17
    o = _stretched_case(cs=cs)
    G = np.random.default_rng(50 + seed).uniform(-1, 1, (3, 3))
    nut = o.nut_of(*_faces_linear(o, G, (0.2, -0.1, 0.3)))
    S = 0.5 * (G + G.T)
    vol = o.hz[:, None, None] * o.hy[None, :, None] * o.hx[None, None, :]
    want = (cs * np.cbrt(vol)) ** 2 * math.sqrt(2 * np.sum(S * S))
    sl = (slice(1, -1),) * 3
    assert np.allclose(nut[sl], want[sl], rtol=1e-12)


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_stretched_self_advection_of_linear_component(comp):
    """u = a + b x alone gives -u du/dx = -b u on every interior u-face of a
    stretched x axis.  The centre products b u_c are interpolated onto the
    face with the paper's width weights (covx1, section 2.5.3); a plain
    mean of the two centres would miss by a term in the width ratio."""
    o = _stretched_case()
    G = np.zeros((3, 3))
    G[comp, comp] = -0.35
    a0 = [0.0, 0.0, 0.0]
    a0[comp] = 0.8
    faces = _faces_linear(o, G, a0)
    F = o.force_of(*faces)[comp]
    want = -G[comp, comp] * faces[comp]
    inner = [slice(1, -1)] * 3
    assert np.allclose(F[tuple(inner)], want[tuple(inner)], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("comp,adv", [(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)])
def test_stretched_cross_advection(comp, adv):
    """Component c = g x_d carried by a general linear velocity component d:
    -(vel_d g), with vel_d interpolated linearly onto the c-face across
    unequal cells (exact for a linear field on any grid)."""
    o = _stretched_case()
    g = 0.45
    G = np.zeros((3, 3))
    G[comp, adv] = g
    G[adv, :] = [0.3, -0.2, 0.25]
    a0 = [0.0, 0.0, 0.0]
    a0[adv] = 0.4
    faces = _faces_linear(o, G, a0)
    F = o.force_of(*faces)[comp]
    # the advecting component evaluated at the c-face positions
    pos = []
    for e, (n, h) in enumerate(((o.nx, o.hx), (o.ny, o.hy), (o.nz, o.hz))):
        pos.append(faces_of(h) if e == comp else cell_centres(n, h))
    vel = a0[adv] + G[adv][0] * pos[0][None, None, :] + G[adv][1] * pos[1][None, :, None] + \
        G[adv][2] * pos[2][:, None, None]
    want = -g * np.broadcast_to(vel, F.shape)
    inner = (slice(2, -2),) * 3
    assert np.allclose(F[inner], want[inner], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_stretched_diffusion_along_own_axis_is_exact(comp):
    """nu times the Laplacian of a quadratic along the component's own axis
    is exact on a stretched grid: the one-sided differences (diu) at the
    centres are exact derivatives at the centres (the midpoints of the
    faces), and the centre distance is the face's control-volume width
    (section 2.5.3, dfu1).  The tendency with nu minus the tendency without
    it leaves nu q''."""
    nu, c2 = 0.013, 0.7
    o1, o0 = _stretched_case(nu=nu), _stretched_case(nu=0.0)
    faces = [np.zeros(s) for s in o1.shapes[:3]]
    h = (o1.hx, o1.hy, o1.hz)[comp]
    coord = faces_of(h)
    shape = [1, 1, 1]
    shape[2 - comp] = coord.size
    faces[comp][:] = (0.3 - 0.2 * coord + c2 * coord**2).reshape(shape)
    diff = o1.force_of(*faces)[comp] - o0.force_of(*faces)[comp]
    inner = (slice(2, -2),) * 3
    assert np.allclose(diff[inner], nu * 2 * c2, rtol=1e-9)


@pytest.mark.parametrize("comp,along", [(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)])
def test_stretched_cross_diffusion_converges_at_second_order(comp, along):
    """Across the component's axis the fluxes sit between two centres and
    are differenced over the cell width (section 2.5.3: diu2 over dy1,
    diu3 over dzn), which on a stretched axis is exact only to second
    order.  On a smoothly mapped axis (the same mapping at every
    resolution) the pointwise error of nu lap(q) against nu q'' at the
    faces must fall by about 4 per halving of the widths."""
    nu, L, kq = 0.02, 2.0, 1.3
    errs = []
    for n in (12, 24, 48):
        dims = [6, 6, 6]
        dims[along] = n
        hs = [0.5, 0.5, 0.5]
        hs[along] = smooth_widths(n, L, 0.5)
        kw = dict(bc=ALL_WALLS, cs=0.0)
        o1 = make(*dims, *hs, nu=nu, **kw)
        o0 = make(*dims, *hs, nu=0.0, **kw)
        faces = [np.zeros(s) for s in o1.shapes[:3]]
        xc = cell_centres(n, hs[along])
        shape = [1, 1, 1]
        shape[2 - along] = n
        faces[comp][:] = np.sin(kq * xc).reshape(shape)
        diff = (o1.force_of(*faces)[comp] - o0.force_of(*faces)[comp]) / nu
        want = (-kq * kq * np.sin(kq * xc)).reshape(shape)
        sl = [slice(2, -2)] * 3
        sl[2 - along] = slice(1, -1)         # one cell from the walls along the axis
        errs.append(np.abs(diff - want)[tuple(sl)].max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.2 <= r1 <= 5.0 and 3.5 <= r2 <= 4.6, errs


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_stretched_sgs_normal_stress(comp):
    """div(2 nu_t S) along a stretched axis for u_c = a x_c^2 alone: S_cc =
    2 a x at each centre (exact), nu_t = (Cs Delta_cell)^2 sqrt(2) 2 a x
    with each cell's own Delta, and the force on a face is the difference
    of the two centre fluxes over the centre distance (the model's part:
    the tendency with Cs minus the tendency without)."""
    cs, a = 0.2, 0.5
    o1, o0 = _stretched_case(cs=cs), _stretched_case(cs=0.0)
    n = (o1.nx, o1.ny, o1.nz)[comp]
    h = (o1.hx, o1.hy, o1.hz)[comp]
    xf = 1.0 + faces_of(h)
    xc = 1.0 + cell_centres(n, h)
    shape = [1, 1, 1]
    shape[2 - comp] = n + 1
    faces = [np.zeros(s) for s in o1.shapes[:3]]
    faces[comp][:] = (a * xf**2).reshape(shape)
    sgs = o1.force_of(*faces)[comp] - o0.force_of(*faces)[comp]
    vol = o1.hz[:, None, None] * o1.hy[None, :, None] * o1.hx[None, None, :]
    C = (cs * np.cbrt(vol)) ** 2
    S = 2 * a * xc
    xcs = [1, 1, 1]
    xcs[2 - comp] = n
    flux = 2 * C * math.sqrt(2) * S.reshape(xcs) * S.reshape(xcs)   # 2 nu_t S at the centres
    sl_hi, sl_lo = [slice(None)] * 3, [slice(None)] * 3
    sl_hi[2 - comp], sl_lo[2 - comp] = slice(1, None), slice(None, -1)
    dist = (xc[1:] - xc[:-1]).reshape([n - 1 if s != 1 else 1 for s in xcs])
    want = (flux[tuple(sl_hi)] - flux[tuple(sl_lo)]) / dist    # on the interior faces 1..n-1
    got_sl = [slice(None)] * 3
    got_sl[2 - comp] = slice(1, n)
    got = sgs[tuple(got_sl)]
    inner = [slice(1, -1)] * 3
    inner[2 - comp] = slice(None)
    assert np.allclose(got[tuple(inner)], want[tuple(inner)], rtol=1e-10)


# ------------------------------------------------------------ whole steps
def _stretched_urban(seed):
    nx, ny, nz = 24, 20, 14
    hz = stretched_widths(nz, 1.0, 1.12, n_uniform=2)
    hgt = building_heights(nx, ny, nz, 0.15, 2, 4, 2, 5, seed=seed, margin_x=4, margin_y=2)
    o = make(nx, ny, nz, 4.0, widths(ny, 3.0, 1.0, seed), hz, mask=building_mask(hgt, nz))
    o.set_inflow(log_law_profile(nz, hz), 0.01, seed)
    return o, hz


def test_stretched_projection_identity_and_mass_balance():
    """P5 and P14 on a stretched grid: ||div u^{n+1}|| / ||div u*|| = R,
    and the outflow flux (face areas hy hz) equals the inflow flux."""
    o, hz = _stretched_urban(5)
    for _ in range(2):
        rc, st = o.step(1)
        assert rc == 0
        assert st["div_new"] / st["div_star"] == pytest.approx(st["resid"], rel=1e-8)
    u = o.get_fields()[0]
    area = hz[:, None] * o.hy[None, :]
    fin = (u[:, :, 0] * area).sum()
    fout = (u[:, :, o.nx] * area).sum()
    assert abs(fout - fin) <= 1e-5 * abs(fin)


def test_stretched_uniform_flow_preserved():
    """P6 on a stretched grid: no buildings, free-slip ground, constant
    inflow, no noise: u = U everywhere, nothing else moves."""
    nx, ny, nz = 12, 10, 8
    bc = (INFLOW, OUTFLOW, FREESLIP, FREESLIP, FREESLIP, FREESLIP)
    o = make(nx, ny, nz, widths(nx, 1.0, 1.1, 21), widths(ny, 1.0, 1.0, 22),
             stretched_widths(nz, 0.5, 1.25), bc=bc)
    U = 2.5
    o.set_inflow(np.full(nz, U, np.float32), 0.0, 1)
    rc, st = o.step(5)
    u, v, w, p = o.get_fields()
    assert np.abs(u - U).max() <= 1e-13 * U
    assert np.abs(v).max() <= 1e-13 and np.abs(w).max() <= 1e-13 and np.abs(p).max() <= 1e-13


def test_uniform_widths_equal_the_uniform_grid():
    """Widths that are all equal give the uniform grid's step bit for bit."""
    nx, ny, nz = 16, 12, 10
    hgt = building_heights(nx, ny, nz, 0.15, 2, 4, 2, 5, seed=8, margin_x=4, margin_y=2)
    mask = building_mask(hgt, nz)
    prof = log_law_profile(nz, 2.0)
    a = make(nx, ny, nz, 4.0, 4.0, 2.0, mask=mask)
    b = make(nx, ny, nz, np.full(nx, 4.0), np.full(ny, 4.0), np.full(nz, 2.0), mask=mask)
    assert b.stretched and not a.stretched
    for o in (a, b):
        o.set_inflow(prof, 0.01, 8)
        o.step(2)
    for x, y in zip(a.get_fields(), b.get_fields()):
        assert np.array_equal(x, y)
