"""Seeded synthetic inputs for the urban LES step.

This module builds the *inputs* of a simulation — building masks, inflow
profiles and workload tables — and nothing else.  It holds none of the
method's arithmetic (no tendency, no pressure solve, no boundary rule), so
both the GPU library and the CPU oracle can be driven from it without
sharing any computation.

The paper's default setup (150x150x90 cells, 50 SOR iterations; section 2.7)
ships neither its building geometry nor its hard-coded wind profile, so the
workloads below stand in for it with seeded random building blocks and
closed-form log-law / power-law profiles.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "Workload",
    "WORKLOADS",
    "building_heights",
    "building_mask",
    "log_law_profile",
    "power_law_profile",
    "make_workload_inputs",
    "ensemble_members",
    "stretched_widths",
    "smooth_widths",
    "cell_centres",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic LES configuration."""

    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    dt: float
    steps: int
    seed: int
    coverage: float          # target fraction of ground columns covered
    foot_min: int            # building footprint side range, in cells
    foot_max: int
    h_min: int               # building height range, in cells
    h_max: int
    profile: str             # "log" or "power"
    u_top: float = 6.0       # power law: speed at the domain top [m/s]
    alpha: float = 0.2       # power law exponent
    noise_amp: float = 0.01  # relative inflow noise amplitude

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz


# C1..C3: the plain-LES workloads.  Spacing and dt of the larger grids are
# not given with them; they reuse the small case's dx=dy=4 m, dz=2 m,
# dt=0.05 s.
WORKLOADS = {
    "C1": Workload("C1", 64, 64, 32, 4.0, 4.0, 2.0, 0.05, 10, 1,
                   0.15, 2, 8, 4, 16, "log"),
    "C2": Workload("C2", 300, 300, 90, 4.0, 4.0, 2.0, 0.05, 1000, 2,
                   0.30, 2, 16, 5, 40, "power", 6.0, 0.2),
    "C3": Workload("C3", 1024, 1024, 96, 4.0, 4.0, 2.0, 0.05, 200, 3,
                   0.35, 2, 16, 5, 60, "power", 6.0, 0.2),
}


def building_heights(nx: int, ny: int, nz: int, coverage: float,
                     foot_min: int, foot_max: int, h_min: int, h_max: int,
                     seed: int, margin_x: int = 8, margin_y: int = 4) -> np.ndarray:
    """Column heights h[j, i] (in cells, 0 = no building) of a random block city.

    Axis-aligned rectangles with footprint sides uniform in
    [foot_min, foot_max] are dropped until the covered fraction of ground
    columns reaches ``coverage``.  Blocks keep ``margin_x`` cells clear of
    the inflow and outflow planes and ``margin_y`` cells clear of the side
    walls; overlapping blocks keep the taller height.  Heights are uniform
    integers in [h_min, h_max], capped at nz - 4.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    h = np.zeros((ny, nx), dtype=np.int32)
    if coverage <= 0.0:
        return h
    i_lo, i_hi = margin_x, nx - margin_x          # usable [i_lo, i_hi)
    j_lo, j_hi = margin_y, ny - margin_y
    if i_hi - i_lo < foot_min or j_hi - j_lo < foot_min:
        return h
    cap = max(1, nz - 4)
    target = coverage * nx * ny
    for _ in range(1_000_000):
        if np.count_nonzero(h) >= target:
            break
        sx = int(rng.integers(foot_min, foot_max + 1))
        sy = int(rng.integers(foot_min, foot_max + 1))
        sx = min(sx, i_hi - i_lo)
        sy = min(sy, j_hi - j_lo)
        i0 = int(rng.integers(i_lo, i_hi - sx + 1))
        j0 = int(rng.integers(j_lo, j_hi - sy + 1))
        hh = min(int(rng.integers(h_min, h_max + 1)), cap)
        blk = h[j0:j0 + sy, i0:i0 + sx]
        np.maximum(blk, hh, out=blk)
    return h


def building_mask(heights: np.ndarray, nz: int) -> np.ndarray:
    """uint8 cell mask m[k, j, i] (C order, i fastest): 1 where k < h[j, i]."""
    ny, nx = heights.shape
    k = np.arange(nz, dtype=np.int32)[:, None, None]
    return (k < heights[None, :, :]).astype(np.uint8)


def stretched_widths(n: int, h0: float, ratio: float, n_uniform: int = 0) -> np.ndarray:
    """Cell widths of a geometrically stretched axis (float64): n_uniform
    cells of width h0, then every cell ``ratio`` times wider than the one
    before (ratio 1 gives a uniform axis)."""
    e = np.maximum(np.arange(n) - n_uniform + 1, 0)
    return h0 * np.power(float(ratio), e, dtype=np.float64)


def smooth_widths(n: int, length: float, a: float) -> np.ndarray:
    """Cell widths of a smoothly stretched axis of the given length: the
    faces sit at length * f(s_m), s_m = m / n, f(s) = s + a sin(2 pi s) / (2 pi)
    (|a| < 1 keeps f increasing).  Refining n keeps the same mapping, which
    is what a grid-convergence study needs."""
    s = np.arange(n + 1, dtype=np.float64) / n
    faces = length * (s + a * np.sin(2 * np.pi * s) / (2 * np.pi))
    return np.diff(faces)


def cell_centres(n: int, h) -> np.ndarray:
    """Centre coordinates of n cells of width h (a scalar or n widths),
    starting from 0 (float64)."""
    w = np.broadcast_to(np.asarray(h, dtype=np.float64), (n,))
    faces = np.concatenate(([0.0], np.cumsum(w)))
    return 0.5 * (faces[:-1] + faces[1:])


def log_law_profile(nz: int, dz, u_star_over_kappa: float = 0.3 / 0.4,
                    z0: float = 0.1) -> np.ndarray:
    """Log-law inflow speed at the cell-centre heights (dz a spacing or the
    nz cell heights of a stretched axis; uniform: z_k = (k + 1/2) dz).

    Evaluated in float64 and rounded once to float32, so every consumer
    sees the same bytes.
    """
    z = cell_centres(nz, dz)
    return (u_star_over_kappa * np.log(z / z0)).astype(np.float32)


def power_law_profile(nz: int, dz, u_top: float, alpha: float) -> np.ndarray:
    """Power-law inflow U_top (z/H)^alpha at cell centres, H the domain
    height (dz a spacing or the nz cell heights; float32)."""
    z = cell_centres(nz, dz)
    H = float(np.sum(np.broadcast_to(np.asarray(dz, dtype=np.float64), (nz,))))
    return (u_top * (z / H) ** alpha).astype(np.float32)


def make_workload_inputs(w: Workload):
    """(mask uint8 [nz,ny,nx], profile float32 [nz]) for a workload."""
    h = building_heights(w.nx, w.ny, w.nz, w.coverage, w.foot_min, w.foot_max,
                         w.h_min, w.h_max, w.seed)
    mask = building_mask(h, w.nz)
    if w.profile == "log":
        prof = log_law_profile(w.nz, w.dz)
    else:
        prof = power_law_profile(w.nz, w.dz, w.u_top, w.alpha)
    return mask, prof


def ensemble_members(n: int = 32, base_seed: int = 1000,
                     nxy_range=(96, 256), nz_range=(64, 90)) -> List[Workload]:
    """Uneven ensemble: member i uses seed base_seed + i for everything it draws."""
    out = []
    for i in range(n):
        rng = np.random.Generator(np.random.PCG64(base_seed + i))
        nx = int(rng.integers(nxy_range[0], nxy_range[1] + 1))
        ny = int(rng.integers(nxy_range[0], nxy_range[1] + 1))
        nz = int(rng.integers(nz_range[0], nz_range[1] + 1))
        alpha = float(rng.uniform(0.1, 0.35))
        u_top = float(rng.uniform(2.0, 12.0))
        cov = float(rng.uniform(0.15, 0.35))
        hmax = int(min(40, nz // 2))
        out.append(Workload(f"E{i}", nx, ny, nz, 4.0, 4.0, 2.0, 0.05, 100,
                            base_seed + i, cov, 2, 16, 4, hmax, "power",
                            u_top, alpha))
    return out


def random_fields(nx: int, ny: int, nz: int, seed: int, scale: float = 1.0):
    """Seeded random owned velocity/pressure arrays in the staggered layout.

    u: [nz, ny, nx+1], v: [nz, ny+1, nx], w: [nz+1, ny, nx], p: [nz, ny, nx],
    all float32, uniform in [-scale, scale].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(-scale, scale, (nz, ny, nx + 1)).astype(np.float32)
    v = rng.uniform(-scale, scale, (nz, ny + 1, nx)).astype(np.float32)
    w = rng.uniform(-scale, scale, (nz + 1, ny, nx)).astype(np.float32)
    p = rng.uniform(-scale, scale, (nz, ny, nx)).astype(np.float32)
    return u, v, w, p


def random_rhs(nx: int, ny: int, nz: int, seed: int, smooth: int = 0) -> np.ndarray:
    """Seeded float32 right-hand side [nz, ny, nx]; optionally box-smoothed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.standard_normal((nz, ny, nx))
    for _ in range(smooth):
        r = (r + np.roll(r, 1, 0) + np.roll(r, 1, 1) + np.roll(r, 1, 2)) / 4.0
    return r.astype(np.float32)
