"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test checks the oracle against a closed form, a textbook identity, a
library routine on an independently assembled operator, or a published
test vector, so that a dropped term, a sign or index slip, or a transposed
operand in ``oracle/les_oracle.cpp`` fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import FREESLIP, INFLOW, NOSLIP, OUTFLOW, URBAN_BC

ALL_WALLS = (FREESLIP, FREESLIP, FREESLIP, FREESLIP, FREESLIP, FREESLIP)


def make(nx, ny, nz, dx=4.0, dy=4.0, dz=2.0, dt=0.05, mask=None, **kw):
    return oracle.Oracle(nx, ny, nz, dx, dy, dz, dt, mask, **kw)


def zeros_faces(o):
    su, sv, sw, _ = o.shapes
    return np.zeros(su), np.zeros(sv), np.zeros(sw)


def assemble_DG(o):
    """Matrix of div(grad p) built from the oracle's projection and divergence."""
    n = o.nx * o.ny * o.nz
    M = np.zeros((n, n))
    zu, zv, zw = zeros_faces(o)
    for c in range(n):
        p = np.zeros(n)
        p[c] = 1.0
        u, v, w = o.project(zu, zv, zw, p.reshape(o.shapes[3]))   # u = -dt G p
        M[:, c] = -o.divergence(u, v, w).ravel() / o.dt
    return M


def assemble_A(o):
    """Matrix of the SOR operator (neighbour weights minus diagonal)."""
    n = o.nx * o.ny * o.nz
    M = np.zeros((n, n))
    for c in range(n):
        p = np.zeros(n)
        p[c] = 1.0
        M[:, c] = o.apply_A(p.reshape(o.shapes[3])).ravel()
    return M


def eig1d(n, h, dirichlet_high):
    """Closed-form eigenvalues of the 1-D cell-centred second difference.

    Neumann at both ends: -(4/h^2) sin^2(pi m / (2n)), m = 0..n-1.
    Neumann low / Dirichlet-on-the-face high: -(4/h^2) sin^2(pi (2m+1) / (4n)).
    """
    m = np.arange(n)
    if dirichlet_high:
        return -(4.0 / h**2) * np.sin(np.pi * (2 * m + 1) / (4 * n)) ** 2
    return -(4.0 / h**2) * np.sin(np.pi * m / (2 * n)) ** 2


# ---------------------------------------------------------------- P2, P2b
@pytest.mark.parametrize("bc", [URBAN_BC, ALL_WALLS])
@pytest.mark.parametrize("shape", [(6, 5, 4), (5, 4, 3)])
def test_operator_is_div_grad(bc, shape):
    """P2: the SOR operator equals D G assembled from projection + divergence."""
    o = make(*shape, dx=1.5, dy=2.0, dz=0.7, bc=bc)
    DG = assemble_DG(o)
    A = assemble_A(o)
    scale = np.abs(A).max()
    assert np.abs(DG - A).max() <= 1e-14 * scale * 10
    assert np.allclose(A, A.T, atol=1e-14 * scale)


@pytest.mark.parametrize("bc", [URBAN_BC, ALL_WALLS])
def test_operator_spectrum_closed_form(bc):
    """P2b: eigenvalues of A are sums of the closed-form 1-D eigenvalues."""
    nx, ny, nz, dx, dy, dz = 7, 5, 4, 1.3, 0.9, 0.6
    o = make(nx, ny, nz, dx=dx, dy=dy, dz=dz, bc=bc)
    A = assemble_A(o)
    ev = np.sort(np.linalg.eigvalsh(A))
    ex = eig1d(nx, dx, bc[1] == OUTFLOW)
    ey = eig1d(ny, dy, False)
    ez = eig1d(nz, dz, False)
    want = np.sort((ez[:, None, None] + ey[None, :, None] + ex[None, None, :]).ravel())
    assert np.allclose(ev, want, rtol=1e-12, atol=1e-12 * abs(want).max())


# ------------------------------------------------- reflection symmetry
def test_operator_commutes_with_y_reflection():
    """Both y faces carry the same boundary condition, so the pressure
    operator commutes with j -> ny-1-j: a pressure problem mirrored in y is
    solved by the mirrored solution (what makes mirrored warm-start
    training pairs valid).  x is not symmetric (inflow against outflow),
    and the check sees that."""
    nx, ny, nz = 7, 6, 5
    o = make(nx, ny, nz, dx=1.5, dy=2.0, dz=0.7, bc=URBAN_BC)
    p = np.random.default_rng(3).standard_normal((nz, ny, nx))
    Ap = o.apply_A(p)
    assert np.allclose(o.apply_A(p[:, ::-1, :]), Ap[:, ::-1, :], rtol=0, atol=1e-12 * np.abs(Ap).max())
    assert not np.allclose(o.apply_A(p[:, :, ::-1]), Ap[:, :, ::-1], rtol=0, atol=1e-6 * np.abs(Ap).max())


# -------------------------------------------------------------------- P1
@pytest.mark.parametrize("shape", [(6, 5, 4), (8, 6, 4), (12, 8, 6)])
@pytest.mark.parametrize("bc", [URBAN_BC, ALL_WALLS])
def test_sor_matches_dense_solve(shape, bc):
    """P1: SOR to 1e-13 equals a dense LAPACK solve of the assembled D G."""
    o = make(*shape, dx=2.0, dy=2.0, dz=1.0, bc=bc)
    rng = np.random.default_rng(7)
    rhs = rng.standard_normal(o.shapes[3])
    DG = assemble_DG(o)
    if bc[1] == OUTFLOW:
        want = np.linalg.solve(DG, rhs.ravel())
        r = rhs
    else:
        r = rhs - rhs.mean()
        want = np.linalg.lstsq(DG, r.ravel(), rcond=None)[0]
        want -= want.mean()
    p, st, rc = o.pressure_solve(rhs, tol=1e-13, max_iter=200000)
    assert rc == 0 and st["converged"] == 1
    got = p.ravel()
    assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)


# -------------------------------------------------------------------- P3
def test_sor_colour_order_delta():
    """P3: one iteration from p = 0 with a point source has a closed form.

    Colour 0 (0-based i+j+k even) is updated first, so the source cell gets
    -omega/d and its six neighbours (colour 1) then see it:
    -omega^2 c_nb / (d d_nb).  Cells two steps away stay 0.
    """
    nx, ny, nz, dx, dy, dz = 8, 8, 8, 1.0, 2.0, 0.5
    om = 1.8
    o = make(nx, ny, nz, dx=dx, dy=dy, dz=dz, omega=om)
    cx, cy, cz = 1 / dx**2, 1 / dy**2, 1 / dz**2
    d = 2 * (cx + cy + cz)
    rhs = np.zeros(o.shapes[3])
    k0, j0, i0 = 4, 3, 3          # 0-based sum 10: colour 0
    rhs[k0, j0, i0] = 1.0
    p, s = o.sor_iterations(rhs, np.zeros_like(rhs), 1)
    want = np.zeros_like(rhs)
    want[k0, j0, i0] = -om / d
    for (dk, dj, di), c in [((0, 0, 1), cx), ((0, 0, -1), cx), ((0, 1, 0), cy),
                            ((0, -1, 0), cy), ((1, 0, 0), cz), ((-1, 0, 0), cz)]:
        want[k0 + dk, j0 + dj, i0 + di] = -om * om * c / (d * d)
    assert np.allclose(p, want, rtol=1e-14, atol=1e-300)
    s_want = (om / d) ** 2 + 2 * sum((om * om * c / (d * d)) ** 2 for c in (cx, cy, cz))
    assert math.isclose(s, s_want, rel_tol=1e-13)
    # the same source on a colour-1 cell is updated in the second half-sweep
    rhs2 = np.zeros_like(rhs)
    rhs2[k0, j0, i0 + 1] = 1.0
    p2, _ = o.sor_iterations(rhs2, np.zeros_like(rhs), 1)
    assert p2[k0, j0, i0 + 1] == pytest.approx(-om / d, rel=1e-14)
    assert np.count_nonzero(p2) == 1


def test_sor_omega_one_is_gauss_seidel_fixed_point():
    """omega = 1 iterates converge to the same dense solution (P1 at omega 1)."""
    o = make(6, 5, 4, dx=1.0, dy=1.0, dz=1.0, omega=1.0)
    rng = np.random.default_rng(3)
    rhs = rng.standard_normal(o.shapes[3])
    p, st, rc = o.pressure_solve(rhs, tol=1e-13, max_iter=200000)
    want = np.linalg.solve(assemble_A(o), rhs.ravel())
    assert np.linalg.norm(p.ravel() - want) <= 1e-10 * np.linalg.norm(want)


# -------------------------------------------------------------------- P4
def test_sor_rate_matches_young():
    """P4: asymptotic SOR factor equals Young's formula from the Jacobi radius."""
    nx, ny, nz = 16, 12, 6
    om = 1.5
    o = make(nx, ny, nz, dx=1.0, dy=1.0, dz=1.0, omega=om)
    A = assemble_A(o)
    dgl = -np.diag(A)
    J = np.eye(A.shape[0]) + A / dgl[:, None]
    rho_j = np.max(np.abs(np.linalg.eigvals(J)))
    om_opt = 2 / (1 + math.sqrt(1 - rho_j**2))
    assert om < om_opt
    rho = ((om * rho_j + math.sqrt(om * om * rho_j * rho_j - 4 * (om - 1))) / 2) ** 2
    rng = np.random.default_rng(1)
    p = rng.standard_normal(o.shapes[3])
    z = np.zeros_like(p)
    p, _ = o.sor_iterations(z, p, 600)
    n0 = np.linalg.norm(p)
    p, _ = o.sor_iterations(z, p, 100)
    obs = (np.linalg.norm(p) / n0) ** (1 / 100)
    assert abs(obs - rho) <= 0.01 * rho


# -------------------------------------------------------------------- P11
def test_divergence_of_linear_field():
    """P11: u = a x, v = b y, w = c z gives div = a + b + c at every cell."""
    nx, ny, nz, dx, dy, dz = 5, 4, 3, 1.5, 0.5, 2.0
    o = make(nx, ny, nz, dx=dx, dy=dy, dz=dz)
    a, b, c = 0.3, -1.7, 2.5
    xu = np.arange(nx + 1) * dx
    yv = np.arange(ny + 1) * dy
    zw = np.arange(nz + 1) * dz
    u = np.broadcast_to(a * xu[None, None, :], (nz, ny, nx + 1))
    v = np.broadcast_to(b * yv[None, :, None], (nz, ny + 1, nx))
    w = np.broadcast_to(c * zw[:, None, None], (nz + 1, ny, nx))
    div = o.divergence(u, v, w)
    assert np.allclose(div, a + b + c, rtol=1e-13)


# -------------------------------------------------------------------- P5
def test_projection_identity():
    """P5: ||div u^{n+1}|| / ||div u*|| equals the final SOR residual."""
    from les_inputs import building_heights, building_mask, log_law_profile
    nx, ny, nz = 24, 20, 12
    h = building_heights(nx, ny, nz, 0.15, 2, 4, 2, 6, seed=5, margin_x=4, margin_y=2)
    mask = building_mask(h, nz)
    o = make(nx, ny, nz, mask=mask)
    o.set_inflow(log_law_profile(nz, 2.0), 0.01, 9)
    for _ in range(2):
        rc, st = o.step(1)
        assert rc == 0
        assert st["div_new"] / st["div_star"] == pytest.approx(st["resid"], rel=1e-8)
        assert st["resid"] <= 1e-5


# -------------------------------------------------------------------- P14
def test_mass_balance():
    """P14: after projection the outflow flux equals the inflow flux.

    Summing div over all cells telescopes to (outflow - inflow flux)/volume;
    the sum is bounded by sqrt(N) ||div||.
    """
    from les_inputs import building_heights, building_mask, log_law_profile
    nx, ny, nz, dx, dy, dz = 24, 16, 12, 4.0, 4.0, 2.0
    h = building_heights(nx, ny, nz, 0.2, 2, 4, 2, 6, seed=2, margin_x=4, margin_y=2)
    o = make(nx, ny, nz, mask=building_mask(h, nz))
    o.set_inflow(log_law_profile(nz, dz), 0.01, 3)
    rc, st = o.step(3)
    u, v, w, p = o.get_fields()
    fin = u[:, :, 0].sum() * dy * dz
    fout = u[:, :, nx].sum() * dy * dz
    bound = math.sqrt(nx * ny * nz) * st["div_new"] * dx * dy * dz
    assert abs(fout - fin) <= bound * (1 + 1e-9) + 1e-12
    assert abs(fout - fin) <= 1e-5 * abs(fin)


# -------------------------------------------------------------------- P6
def test_uniform_flow_preserved():
    """P6: no buildings, free-slip ground, constant inflow, no noise: u = U."""
    nx, ny, nz = 16, 12, 8
    bc = (INFLOW, OUTFLOW, FREESLIP, FREESLIP, FREESLIP, FREESLIP)
    o = make(nx, ny, nz, bc=bc)
    U = 3.25
    o.set_inflow(np.full(nz, U, np.float32), 0.0, 1)
    rc, st = o.step(10)
    u, v, w, p = o.get_fields()
    assert np.abs(u - U).max() <= 1e-14 * U
    assert np.abs(v).max() <= 1e-14 and np.abs(w).max() <= 1e-14
    assert np.abs(p).max() <= 1e-14
    assert st["total_iters"] == 0


# -------------------------------------------------------------------- P7
def _tgv(o, A, my, mz):
    nx, ny, nz, dy, dz = o.nx, o.ny, o.nz, o.dy, o.dz
    Ly, Lz = ny * dy, nz * dz
    ky, kz = my * math.pi / Ly, mz * math.pi / Lz
    B = A * (math.sin(ky * dy / 2) / dy) / (math.sin(kz * dz / 2) / dz)
    yf = np.arange(ny + 1) * dy
    yc = (np.arange(ny) + 0.5) * dy
    zf = np.arange(nz + 1) * dz
    zc = (np.arange(nz) + 0.5) * dz
    v = A * np.sin(ky * yf)[None, :, None] * np.cos(kz * zc)[:, None, None] * np.ones((1, 1, nx))
    w = -B * np.cos(ky * yc)[None, :, None] * np.sin(kz * zf)[:, None, None] * np.ones((1, 1, nx))
    lam = -(4 / dy**2) * math.sin(ky * dy / 2) ** 2 - (4 / dz**2) * math.sin(kz * dz / 2) ** 2
    return v, w, lam, ky, kz


def test_taylor_green_decay():
    """P7: a free-slip y-z Taylor-Green mode decays by the AB2 recursion.

    The mode is an exact eigenvector of the discrete Laplacian (eigenvalue
    lam) with zero discrete divergence.  With Cs = 0 and a tiny amplitude
    the nonlinear terms are negligible, so the amplitude follows
    a1 = (1 + mu) a0 (Euler first step), a_{n+1} = a_n + mu (1.5 a_n - 0.5 a_{n-1}),
    mu = nu lam dt; and tends to exp(nu lam_cont t) up to O((k h)^2).
    """
    nx, ny, nz, dx, dy, dz, dt, nu = 4, 16, 16, 1.0, 1.0, 1.0, 0.1, 1.0
    o = make(nx, ny, nz, dx=dx, dy=dy, dz=dz, dt=dt, bc=ALL_WALLS, cs=0.0, nu=nu)
    A = 1e-6
    v0, w0, lam, ky, kz = _tgv(o, A, 1, 1)
    su = o.shapes[0]
    o.set_fields(np.zeros(su), v0, w0, np.zeros(o.shapes[3]))
    mu = nu * lam * dt
    a = [1.0, 1.0 + mu]
    nsteps = 8
    for n in range(1, nsteps):
        a.append(a[n] + mu * (1.5 * a[n] - 0.5 * a[n - 1]))
    for n in range(1, nsteps + 1):
        rc, st = o.step(1)
        u, v, w, p = o.get_fields()
        amp_v = np.vdot(v, v0) / np.vdot(v0, v0)
        amp_w = np.vdot(w, w0) / np.vdot(w0, w0)
        assert amp_v == pytest.approx(a[n], rel=1e-6, abs=0)
        assert amp_w == pytest.approx(a[n], rel=1e-6, abs=0)
        resid_v = np.linalg.norm(v - amp_v * v0) / np.linalg.norm(v0)
        assert resid_v <= 1e-6
    lam_c = -(ky**2 + kz**2)
    t = nsteps * dt
    kh2 = (ky * dy) ** 2
    assert a[nsteps] == pytest.approx(math.exp(nu * lam_c * t), rel=2 * kh2 * abs(nu * lam_c * t))


# -------------------------------------------------------------------- P8
def test_smagorinsky_linear_shear():
    """P8: u = g z gives |S| = g, so nu_t = (Cs Delta)^2 g away from walls."""
    nx, ny, nz, dx, dy, dz = 6, 5, 8, 2.0, 3.0, 1.0
    cs = 0.17
    o = make(nx, ny, nz, dx=dx, dy=dy, dz=dz, cs=cs)
    g = 0.8
    zc = (np.arange(nz) + 0.5) * dz
    u = np.broadcast_to(g * zc[:, None, None], (nz, ny, nx + 1)).copy()
    su, sv, sw, sc = o.shapes
    nut = o.nut_of(u, np.zeros(sv), np.zeros(sw))
    want = (cs * (dx * dy * dz) ** (1 / 3)) ** 2 * g
    assert np.allclose(nut[1:-1], want, rtol=1e-13)
    # constant nu_t on a linear field: zero SGS force, zero advection,
    # zero Laplacian -> zero tendency away from the z walls
    fu, fv, fw = o.force_of(u, np.zeros(sv), np.zeros(sw))
    assert np.abs(fu[2:-2]).max() <= 1e-13 * g
    assert np.abs(fv[2:-2]).max() <= 1e-13 * g
    assert np.abs(fw[2:-2]).max() <= 1e-13 * g


def test_smagorinsky_solid_rotation():
    """P8: solid-body rotation in x-y has zero strain, hence nu_t = 0."""
    nx, ny, nz, dx, dy, dz = 8, 8, 4, 1.0, 1.0, 1.0
    o = make(nx, ny, nz, dx=dx, dy=dy, dz=dz, cs=0.2)
    Om = 0.5
    yc = (np.arange(ny) + 0.5) * dy - 4
    xc = (np.arange(nx) + 0.5) * dx - 4
    xf = np.arange(nx + 1) * dx - 4
    yf = np.arange(ny + 1) * dy - 4
    u = np.broadcast_to(-Om * yc[None, :, None], (nz, ny, nx + 1)).copy()
    v = np.broadcast_to(Om * xc[None, None, :], (nz, ny + 1, nx)).copy()
    nut = o.nut_of(u, v, np.zeros(o.shapes[2]))
    assert np.abs(nut[1:-1, 1:-1, 1:-1]).max() <= 1e-14


def _linear_faces(o, G, origin=(0.3, -0.2, 0.5)):
    """Faces of the linear field u_i = G_ij x_j on the MAC grid of ``o``.

    u sits at (x_face, y_centre, z_centre), v at (x_centre, y_face,
    z_centre), w at (x_centre, y_centre, z_face); ``origin`` shifts the
    coordinates so that no component is zero on a whole plane.
    """
    nx, ny, nz, dx, dy, dz = o.nx, o.ny, o.nz, o.dx, o.dy, o.dz
    xc = origin[0] + (np.arange(nx) + 0.5) * dx
    yc = origin[1] + (np.arange(ny) + 0.5) * dy
    zc = origin[2] + (np.arange(nz) + 0.5) * dz
    xf = origin[0] + np.arange(nx + 1) * dx
    yf = origin[1] + np.arange(ny + 1) * dy
    zf = origin[2] + np.arange(nz + 1) * dz

    def lin(row, X, Y, Z):
        return (row[0] * X[None, None, :] + row[1] * Y[None, :, None] + row[2] * Z[:, None, None])

    return lin(G[0], xf, yc, zc), lin(G[1], xc, yf, zc), lin(G[2], xc, yc, zf)


@pytest.mark.parametrize("seed", [0, 1])
def test_smagorinsky_general_linear_field(seed):
    """P8: a general linear field u_i = G_ij x_j has S = (G + G^T)/2 exactly.

    Every one of the six strain components is then constant, so at every
    cell whose stencil stays inside the domain nu_t = (Cs Delta)^2
    sqrt(2 S:S) with the closed-form S.  Distinct dx, dy, dz and a full,
    non-symmetric G reach S22, S33 and S23 as well as S11, S12 and S13,
    each with its own spacing.
    """
    nx, ny, nz, dx, dy, dz, cs = 7, 6, 5, 1.7, 0.9, 0.4, 0.13
    rng = np.random.default_rng(100 + seed)
    G = rng.uniform(-1.0, 1.0, (3, 3))
    o = make(nx, ny, nz, dx=dx, dy=dy, dz=dz, cs=cs, bc=ALL_WALLS)
    u, v, w = _linear_faces(o, G)
    nut = o.nut_of(u, v, w)
    S = 0.5 * (G + G.T)
    want = (cs * (dx * dy * dz) ** (1 / 3)) ** 2 * math.sqrt(2.0 * np.sum(S * S))
    inner = nut[1:-1, 1:-1, 1:-1]
    assert inner.size > 0
    assert np.allclose(inner, want, rtol=1e-12, atol=0)


@pytest.mark.parametrize("comp", ["u", "v", "w"])
def test_sgs_force_with_varying_viscosity(comp):
    """P8: div(2 nu_t S) where nu_t varies across the shear layer.

    A single quadratic velocity component, e.g. u = a y^2 (v = w = 0),
    has one strain pair S12 = S21 = a y, so |S| = 2 a y and
    nu_t = 2 C a y with C = (Cs Delta)^2.  Its SGS force is
    d/dy (2 nu_t S12) = d/dy (4 C a^2 y^2) = 8 C a^2 y, and advection and
    (with nu = 0) diffusion vanish.  On the MAC grid the edge strain and
    the 4-cell edge mean of nu_t are linear in y, so the flux difference
    is exact.  The analogues: v = a z^2 (force 8 C a^2 z on v-faces) and
    w = a x^2 (force 8 C a^2 x on w-faces).  Swapping the viscosity's
    edge offsets or dropping the factor 2 fails this.
    """
    nx, ny, nz, dx, dy, dz, cs, a = 10, 11, 12, 1.3, 0.7, 0.45, 0.21, 0.8
    o = make(nx, ny, nz, dx=dx, dy=dy, dz=dz, cs=cs, nu=0.0, bc=ALL_WALLS)
    C = (cs * (dx * dy * dz) ** (1 / 3)) ** 2
    su, sv, sw, _ = o.shapes
    u, v, w = np.zeros(su), np.zeros(sv), np.zeros(sw)
    off = 2.0   # coordinates start at 2 m: the quadratic is monotone inside
    if comp == "u":
        y = off + (np.arange(ny) + 0.5) * dy
        u[:] = (a * y**2)[None, :, None]
    elif comp == "v":
        z = off + (np.arange(nz) + 0.5) * dz
        v[:] = (a * z**2)[:, None, None]
    else:
        x = off + (np.arange(nx) + 0.5) * dx
        w[:] = (a * x**2)[None, None, :]
    fu, fv, fw = o.force_of(u, v, w)
    if comp == "u":
        got = fu[:, 2:ny - 2, 1:nx]
        want = np.broadcast_to((8 * C * a * a * y)[None, 2:ny - 2, None], got.shape)
        others = (fv, fw)
    elif comp == "v":
        got = fv[2:nz - 2, 1:ny, :]
        want = np.broadcast_to((8 * C * a * a * z)[2:nz - 2, None, None], got.shape)
        others = (fu, fw)
    else:
        got = fw[1:nz, :, 2:nx - 2]
        want = np.broadcast_to((8 * C * a * a * x)[None, None, 2:nx - 2], got.shape)
        others = (fu, fv)
    assert got.size > 0
    assert np.allclose(got, want, rtol=1e-12, atol=0)
    # the other components see no force from this field away from the walls
    for f in others:
        assert np.abs(f[2:-2, 2:-2, 2:-2]).max() <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("comp", ["v", "w"])
def test_advection_of_v_and_w_linear(comp):
    """Advection of v and w: v = b + c y gives -v dv/dy = -c v at every
    interior v-face (u = w = 0); w = b + c z gives -c w on w-faces.  The
    central cov pieces average the centre products back onto the face,
    which is exact for a linear component.
    """
    nx, ny, nz, dx, dy, dz = 6, 7, 8, 0.6, 0.35, 0.8
    o = make(nx, ny, nz, dx=dx, dy=dy, dz=dz, cs=0.0, nu=0.0, bc=ALL_WALLS)
    b, c = 0.9, -0.45
    su, sv, sw, _ = o.shapes
    u, v, w = np.zeros(su), np.zeros(sv), np.zeros(sw)
    if comp == "v":
        yf = np.arange(ny + 1) * dy
        v[:] = (b + c * yf)[None, :, None]
        _, fv, fw = o.force_of(u, v, w)
        want = -c * (b + c * yf)
        assert np.allclose(fv[:, 1:ny, :], np.broadcast_to(want[None, 1:ny, None], (nz, ny - 1, nx)),
                           rtol=1e-13)
        assert np.abs(fw[1:nz]).max() <= 1e-14
    else:
        zf = np.arange(nz + 1) * dz
        w[:] = (b + c * zf)[:, None, None]
        _, fv, fw = o.force_of(u, v, w)
        want = -c * (b + c * zf)
        assert np.allclose(fw[1:nz], np.broadcast_to(want[1:nz, None, None], (nz - 1, ny, nx)),
                           rtol=1e-13)
        assert np.abs(fv[:, 1:ny]).max() <= 1e-14


def test_advection_of_w_by_uniform_u():
    """w = q(x) quadratic carried by a constant u = U: the x-advection of w
    is -U q'(x) and the Laplacian nu q''(x), both exact for a quadratic on
    the MAC grid (the cov piece pairs the mean of two u-faces with the
    one-sided difference of w between neighbouring columns)."""
    nx, ny, nz, dx, dy, dz, nu = 9, 6, 7, 0.55, 0.8, 0.3, 0.02
    bc = (INFLOW, OUTFLOW, FREESLIP, FREESLIP, FREESLIP, FREESLIP)
    o = make(nx, ny, nz, dx=dx, dy=dy, dz=dz, bc=bc, cs=0.0, nu=nu)
    U = 0.7
    c0, c1, c2 = 0.2, -0.5, 0.35
    xc = (np.arange(nx) + 0.5) * dx
    q = c0 + c1 * xc + c2 * xc**2
    su, sv, sw, _ = o.shapes
    u = np.full(su, U)
    w = np.broadcast_to(q[None, None, :], sw).copy()
    fu, fv, fw = o.force_of(u, np.zeros(sv), w)
    want = -U * (c1 + 2 * c2 * xc) + nu * 2 * c2
    iin = slice(1, nx - 1)
    got = fw[1:nz, :, iin]
    assert np.allclose(got, np.broadcast_to(want[None, None, iin], got.shape), rtol=1e-12)


_AXES = {"u": 0, "v": 1, "w": 2}


@pytest.mark.parametrize("comp,adv", [("u", "v"), ("u", "w"), ("v", "u"), ("v", "w"),
                                      ("w", "u"), ("w", "v")])
def test_cross_advection_by_a_linear_velocity(comp, adv):
    """Advection of one component across the flow of another.

    The advected component is c = g x_d (d the direction of the advecting
    component, e.g. u = g y carried by v), the advecting component is a
    general linear function a + b . x on its own faces, the third is zero.
    Then c has no self-advection and -(vel_d dc/dx_d) = -g vel_d, with
    vel_d evaluated at the c-face: the cov pieces interpolate the advecting
    velocity linearly (face pair, then edge pair), which is exact for a
    linear field.  A wrong face index in that interpolation moves the
    evaluation point by half a cell and fails here.
    """
    nx, ny, nz, dx, dy, dz = 8, 9, 7, 0.7, 0.45, 0.9
    o = make(nx, ny, nz, dx=dx, dy=dy, dz=dz, cs=0.0, nu=0.0, bc=ALL_WALLS)
    c, d = _AXES[comp], _AXES[adv]
    g, a0 = 0.55, 0.4
    b = np.array([0.3, -0.25, 0.2])
    G = np.zeros((3, 3))
    G[c, d] = g
    G[d, :] = b
    faces = list(_linear_faces(o, G, origin=(0.0, 0.0, 0.0)))
    faces[d] = faces[d] + a0
    fu, fv, fw = o.force_of(*faces)
    F = (fu, fv, fw)[c]
    # coordinates of the c-faces
    nxyz = (nx, ny, nz)
    h = (dx, dy, dz)
    pos = []
    for e in range(3):
        n = nxyz[e] + (1 if e == c else 0)
        off = 0.0 if e == c else 0.5
        pos.append((np.arange(n) + off) * h[e])
    vel_d = a0 + b[0] * pos[0][None, None, :] + b[1] * pos[1][None, :, None] + b[2] * pos[2][:, None, None]
    want = -g * np.broadcast_to(vel_d, F.shape)
    inner = (slice(2, F.shape[0] - 2), slice(2, F.shape[1] - 2), slice(2, F.shape[2] - 2))
    assert F[inner].size > 0
    assert np.allclose(F[inner], want[inner], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("comp", ["u", "v", "w"])
def test_sgs_normal_stress_with_varying_viscosity(comp):
    """P8: the normal part of div(2 nu_t S) where nu_t varies along it.

    A single component quadratic along its own axis, e.g. u = a x^2, has
    S11 = 2 a x at cell centres (exact for the face difference), |S| =
    sqrt(2) 2 a x and nu_t = sqrt(2) 2 C a x, so d/dx (2 nu_t S11) =
    16 sqrt(2) C a^2 x at the u-faces, exact for the difference of the
    two centre fluxes.  Advection is the same with and without the model,
    so the SGS part is the tendency with Cs minus the tendency with
    Cs = 0.  A wrong centre index of nu_t in the normal flux fails here.
    """
    nx, ny, nz, dx, dy, dz, cs, a = 9, 8, 10, 0.8, 0.6, 0.35, 0.19, 0.5
    C = (cs * (dx * dy * dz) ** (1 / 3)) ** 2
    c = _AXES[comp]
    o1 = make(nx, ny, nz, dx=dx, dy=dy, dz=dz, cs=cs, nu=0.0, bc=ALL_WALLS)
    o0 = make(nx, ny, nz, dx=dx, dy=dy, dz=dz, cs=0.0, nu=0.0, bc=ALL_WALLS)
    shapes = o1.shapes[:3]
    faces = [np.zeros(s) for s in shapes]
    n = (nx, ny, nz)[c]
    h = (dx, dy, dz)[c]
    xf = 1.0 + np.arange(n + 1) * h       # face coordinates along the axis, offset by 1 m
    prof = a * xf**2
    if c == 0:
        faces[0][:] = prof[None, None, :]
    elif c == 1:
        faces[1][:] = prof[None, :, None]
    else:
        faces[2][:] = prof[:, None, None]
    F1 = o1.force_of(*faces)[c]
    F0 = o0.force_of(*faces)[c]
    sgs = F1 - F0
    want1d = 16.0 * math.sqrt(2.0) * C * a * a * xf
    sl = [slice(None)] * 3
    ax = 2 - c                           # numpy axis of this coordinate
    sl[ax] = slice(2, n - 1)
    got = sgs[tuple(sl)]
    shape = [1, 1, 1]
    shape[ax] = n - 3
    want = np.broadcast_to(want1d[2:n - 1].reshape(shape), got.shape)
    assert np.allclose(got, want, rtol=1e-10, atol=0)


# ------------------------------------------------------ advection closed forms
def test_advection_closed_forms():
    """Second-order central advection is exact on these polynomial fields.

    u = a + b x (v = w = 0): -(u du/dx) = -b u at every interior u-face.
    u = q(y) quadratic, v = V constant on interior faces: -V q'(y) exactly
    (and nu q'' from the Laplacian).
    """
    nx, ny, nz, dx, dy, dz = 8, 8, 6, 0.5, 0.25, 1.0
    bc = (INFLOW, OUTFLOW, FREESLIP, FREESLIP, FREESLIP, FREESLIP)
    o = make(nx, ny, nz, dx=dx, dy=dy, dz=dz, bc=bc, cs=0.0, nu=0.0)
    a, b = 1.2, 0.3
    xf = np.arange(nx + 1) * dx
    u = np.broadcast_to((a + b * xf)[None, None, :], (nz, ny, nx + 1)).copy()
    su, sv, sw, sc = o.shapes
    fu, fv, fw = o.force_of(u, np.zeros(sv), np.zeros(sw))
    want = -b * (a + b * xf)
    assert np.allclose(fu[:, :, 1:nx], want[None, None, 1:nx], rtol=1e-13)
    # shear advected by a uniform cross flow
    nu = 0.01
    o2 = make(nx, ny, nz, dx=dx, dy=dy, dz=dz, bc=bc, cs=0.0, nu=nu)
    yc = (np.arange(ny) + 0.5) * dy
    c0, c1, c2 = 0.4, -0.7, 0.9
    q = c0 + c1 * yc + c2 * yc**2
    u2 = np.broadcast_to(q[None, :, None], (nz, ny, nx + 1)).copy()
    V = 0.6
    v2 = np.full(sv, V)
    v2[:, 0, :] = 0.0
    v2[:, ny, :] = 0.0
    fu2, _, _ = o2.force_of(u2, v2, np.zeros(sw))
    dq = c1 + 2 * c2 * yc
    want2 = -V * dq + nu * 2 * c2
    jin = slice(2, ny - 2)
    assert np.allclose(fu2[:, jin, 1:nx], want2[None, jin, None], rtol=1e-12)


# -------------------------------------------------------------------- P9
def test_feedback_forcing_single_solid_cell():
    """P9: on a solid face F = adv/diff part + alpha usum + beta u, usum = dt u.

    With a uniform flow the advective and diffusive parts vanish on the
    faces around an isolated solid cell at the first step, so the stored
    tendency there is exactly (alpha dt + beta) U and usum = dt U; the
    second step accumulates usum by dt times the projected velocity.
    """
    nx, ny, nz = 12, 10, 8
    bc = (INFLOW, OUTFLOW, FREESLIP, FREESLIP, FREESLIP, FREESLIP)
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[4, 5, 6] = 1
    al, be, dt, U = -10.0, -1.0, 0.05, 2.0
    o = make(nx, ny, nz, dt=dt, mask=mask, bc=bc, alpha=al, beta=be, cs=0.0, nu=0.0)
    o.set_inflow(np.full(nz, U, np.float32), 0.0, 1)
    # initial state: the two u-faces of the solid cell start at 0 (solid)
    u0 = o.get_fields()[0]
    assert u0[4, 5, 6] == 0.0 and u0[4, 5, 7] == 0.0 and u0[4, 5, 5] == 2.0
    # impose the uniform flow everywhere, faces of the solid cell included
    su, sv, sw, sc = o.shapes
    o.set_fields(np.full(su, U), np.zeros(sv), np.zeros(sw), np.zeros(sc))
    o.step(1)
    fu, fv, fw = o.get_force()
    s_u, s_v, s_w = o.get_usum()
    # u-faces of the solid cell (0-based cell 6): face 6 (west) and 7 (east)
    for i in (6, 7):
        assert s_u[4, 5, i] == pytest.approx(dt * U, rel=1e-15)
        assert fu[4, 5, i] == pytest.approx((al * dt + be) * U, rel=1e-13)
    assert s_u[4, 5, 5] == 0.0 and s_u[4, 5, 8] == 0.0
    u1 = o.get_fields()[0]
    o.step(1)
    s_u2 = o.get_usum()[0]
    for i in (6, 7):
        assert s_u2[4, 5, i] == pytest.approx(dt * U + dt * u1[4, 5, i], rel=1e-13)


# ------------------------------------------------------------------- P12
def test_splitmix64_published_vectors():
    """P12: splitmix64 from state 0, gamma, 2 gamma (Steele-Lea-Flood 2014)."""
    g = 0x9E3779B97F4A7C15
    assert oracle.splitmix64(0) == 0xE220A8397B1DCDAF
    assert oracle.splitmix64(g) == 0x6E789E6AA1B965F4
    assert oracle.splitmix64((2 * g) % 2**64) == 0x06C45D188009454F


def test_inflow_noise_definition():
    """P12: inflow = U(k)(1 + a(2 xi - 1)), xi the top 24 bits of splitmix64."""
    nx, ny, nz = 12, 6, 5
    o = make(nx, ny, nz)
    prof = np.linspace(1, 3, nz).astype(np.float32)
    o.set_inflow(prof, 0.01, 12345)
    vals = []
    for k in range(1, nz + 1):
        for j in range(1, ny + 1):
            for s in (1, 7):
                ctr = (s << 40) + ((k - 1) << 20) + (j - 1)
                xi = (oracle.splitmix64(12345 ^ ctr) >> 40) / 2.0**24
                want = float(prof[k - 1]) * (1 + 0.01 * (2 * xi - 1))
                got = o.inflow_value(j, k, s)
                assert got == pytest.approx(want, rel=1e-15)
                vals.append(xi)
    vals = np.array(vals)
    assert vals.min() >= 0 and vals.max() < 1


def test_inflow_pair_interpolation():
    """Section 4 (coupled time loop): the inflow profile is interpolated
    linearly in time between two samples.  Pins on the oracle, with the
    noise off: the step starting exactly at t0 (resp. t1) carries U0 (resp.
    U1) bit for bit, steps before t0 / after t1 hold the end samples, the
    midpoint time gives the mean, equally spaced times give equal
    increments, and set_inflow switches the interpolation off again."""
    nx, ny, nz, dt = 12, 6, 5, 0.25
    o = make(nx, ny, nz, dt=dt)
    u0 = np.linspace(1.0, 3.0, nz).astype(np.float32)
    u1 = np.linspace(4.0, 1.5, nz).astype(np.float32)
    o.set_inflow(u0, 0.0, 1)
    t0, t1 = 3 * dt, 11 * dt          # step s starts at time (s - 1) dt
    o.set_inflow_pair(t0, u0, t1, u1)
    for k in range(1, nz + 1):
        a, b = float(u0[k - 1]), float(u1[k - 1])
        for j in (1, ny):
            assert o.inflow_value(j, k, 4) == a           # t = t0
            assert o.inflow_value(j, k, 12) == b          # t = t1
            assert o.inflow_value(j, k, 1) == a           # before t0: held
            assert o.inflow_value(j, k, 30) == b          # after t1: held
            assert o.inflow_value(j, k, 8) == pytest.approx(0.5 * (a + b), rel=1e-15)
            v = [o.inflow_value(j, k, s) for s in (5, 6, 7)]
            assert v[1] - v[0] == pytest.approx(v[2] - v[1], rel=1e-12)
            assert v[1] - v[0] == pytest.approx((b - a) / 8, rel=1e-12)
    o.set_inflow(u1, 0.0, 1)
    assert o.inflow_value(1, 2, 6) == float(u1[1])
    with pytest.raises(ValueError):
        o.set_inflow_pair(t1, u0, t0, u1)
    fresh = make(nx, ny, nz, dt=dt)
    with pytest.raises(ValueError):
        fresh.set_inflow_pair(t0, u0, t1, u1)


def test_inflow_pair_of_equal_samples_is_the_plain_inflow():
    """A pair whose two samples are the same profile leaves every step of
    the run bit for bit as with that profile alone (noise on)."""
    nx, ny, nz = 12, 6, 5
    prof = np.linspace(1.0, 2.0, nz).astype(np.float32)
    a, b = make(nx, ny, nz), make(nx, ny, nz)
    a.set_inflow(prof, 0.01, 4)
    b.set_inflow(prof, 0.01, 4)
    b.set_inflow_pair(0.0, prof, 0.1, prof)
    for s in (1, 2, 3):
        for k in range(1, nz + 1):
            assert b.inflow_value(3, k, s) == a.inflow_value(3, k, s)
    a.step(2)
    b.step(2, forced=a.last_iters)
    for x, y in zip(a.get_fields(), b.get_fields()):
        assert np.array_equal(x, y)


def test_profiles_closed_forms():
    """P12: log-law and power-law profiles at their cell-centre heights."""
    from les_inputs import log_law_profile, power_law_profile
    p = log_law_profile(32, 2.0)
    assert p[0] == pytest.approx(0.75 * math.log(1.0 / 0.1), rel=1e-7)     # z = 1 m
    assert p[31] == pytest.approx(0.75 * math.log(63.0 / 0.1), rel=1e-7)   # z = 63 m
    assert p[0] == pytest.approx(1.727, abs=1e-3) and p[31] == pytest.approx(4.834, abs=1e-3)
    q = power_law_profile(90, 2.0, 6.0, 0.2)
    assert q[-1] == pytest.approx(6.0 * (179.0 / 180.0) ** 0.2, rel=1e-7)
    assert q[0] == pytest.approx(6.0 * (1.0 / 180.0) ** 0.2, rel=1e-7)


# -------------------------------------------------------------- BC table
def test_ghost_rules_urban():
    """Ghost values follow the per-face rules, edges and corners included."""
    nx, ny, nz = 6, 5, 4
    o = make(nx, ny, nz)
    u, v, w, p = oracle_random_state(o, 11)
    o.set_fields(u, v, w, p)
    U, V, W = o.get_ghosted()      # [k][j][i] over the ghosted box
    # u: x+ outflow copies, y free slip mirrors, z- no slip anti-mirrors,
    # z+ free slip mirrors
    assert np.array_equal(U[1:-1, 1:-1, nx + 1], U[1:-1, 1:-1, nx])
    assert np.array_equal(U[:, 0, :], U[:, 1, :]) and np.array_equal(U[:, ny + 1, :], U[:, ny, :])
    assert np.array_equal(U[0], -U[1]) and np.array_equal(U[nz + 1], U[nz])
    # v: inflow anti-mirror on x-, outflow copy on x+, walls zero
    assert np.array_equal(V[1:-1, :ny + 1, 0], -V[1:-1, :ny + 1, 1])
    assert np.array_equal(V[1:-1, :ny + 1, nx + 1], V[1:-1, :ny + 1, nx])
    assert np.all(V[:, 0, :] == 0) and np.all(V[:, ny, :] == 0)
    # w: ground and top faces zero, y ghosts mirror
    assert np.all(W[0] == 0) and np.all(W[nz] == 0)
    assert np.array_equal(W[:nz + 1, 0, :], W[:nz + 1, 1, :])
    # a corner composes the three rules: u(nx+1, 0, 0) = -u(nx, 1, 1)
    assert U[0, 0, nx + 1] == -U[1, 1, nx]


def oracle_random_state(o, seed):
    from les_inputs import random_fields
    u, v, w, p = random_fields(o.nx, o.ny, o.nz, seed)
    return u.astype(np.float64), v.astype(np.float64), w.astype(np.float64), p.astype(np.float64)


# ------------------------------------------------------------- replay mode
def test_replay_mode_reproduces_free_run():
    """Replaying the iteration counts of a free run gives identical fields."""
    from les_inputs import log_law_profile
    nx, ny, nz = 16, 12, 8
    a = make(nx, ny, nz)
    b = make(nx, ny, nz)
    prof = log_law_profile(nz, 2.0)
    a.set_inflow(prof, 0.01, 4)
    b.set_inflow(prof, 0.01, 4)
    a.step(3)
    iters = a.last_iters
    b.step(3, forced=iters)
    for x, y in zip(a.get_fields(), b.get_fields()):
        assert np.array_equal(x, y)


def _dense_A(o, shape):
    n = int(np.prod(shape))
    M = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        M[:, c] = o.apply_A(e.reshape(shape)).ravel()
    return M


def test_twinned_is_relaxed_jacobi_on_the_dense_matrix():
    """Section 2.6, twinned double buffering: each half of an iteration
    updates every cell from the other buffer with the SOR point formula,
    which is the relaxed Jacobi step x <- x - omega D^-1 (A x - b), D the
    diagonal of A.  Pinned against the dense matrix of the operator (its
    columns A e_c), with D read off that matrix, for the urban face set
    (non-singular) and for all walls: three iterations are six Jacobi
    steps; the solution of the dense system is a fixed point; with omega =
    1 the iteration reaches it."""
    rng = np.random.default_rng(11)
    for bc in (URBAN_BC, (FREESLIP,) * 6):
        nx, ny, nz = 6, 5, 4
        o = make(nx, ny, nz, bc=bc)
        shape = (nz, ny, nx)
        M = _dense_A(o, shape)
        d = np.diag(M)
        b = rng.standard_normal(shape)
        if bc != URBAN_BC:
            b -= b.mean()
        x0 = rng.standard_normal(shape)
        x = x0.ravel().copy()
        for _ in range(6):
            x = x - 0.8 * (M @ x - b.ravel()) / d
        got = o.twinned_iterations(b, x0, 0.8, 3)
        assert np.allclose(got.ravel(), x, rtol=0, atol=1e-12 * np.abs(x).max())
        if bc == URBAN_BC:
            xs = np.linalg.solve(M, b.ravel()).reshape(shape)
            fixed = o.twinned_iterations(b, xs, 1.0, 1)
            assert np.linalg.norm(fixed - xs) <= 1e-12 * np.linalg.norm(xs)
            far = o.twinned_iterations(b, np.zeros(shape), 1.0, 3000)
            assert np.linalg.norm(far - xs) <= 1e-8 * np.linalg.norm(xs)
    # not the red-black iteration: one twinned iteration from zero differs
    o = make(6, 5, 4)
    b = rng.standard_normal((4, 5, 6))
    rb, _ = o.sor_iterations(b, np.zeros((4, 5, 6)), 1)
    assert np.linalg.norm(o.twinned_iterations(b, np.zeros((4, 5, 6)), 1.8, 1) - rb) > 1e-3
