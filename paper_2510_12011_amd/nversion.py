"""Activation times along the P1-P8 diagonal of the N-version cuboid.

The verification section of the paper compares activation times (the first
time V passes 0 mV) at points on the diagonal from the stimulated corner
P1 = (0, 0, 0) to the opposite vertex P8 = (20, 7, 3) mm.  The nodal field
is evaluated at those points with the P1 interpolant of the Kuhn-split grid
the run used: in a hex with local coordinates sorted as
u_a >= u_b >= u_c, the point lies in the tet (c, c + e_a, c + e_a + e_b,
c + 1) with barycentric weights (1 - u_a, u_a - u_b, u_b - u_c, u_c).
"""
from __future__ import annotations

import numpy as np

DIAGONAL = np.array([20.0, 7.0, 3.0])


def diagonal_points(n: int) -> np.ndarray:
    """n points from P1 to P8 inclusive, [n, 3] mm."""
    s = np.linspace(0.0, 1.0, n)
    return s[:, None] * DIAGONAL[None, :]


def kuhn_interpolate(field: np.ndarray, dims, lengths, points: np.ndarray) -> np.ndarray:
    """P1 interpolant of a nodal field on the Kuhn grid of `dims` = (nx, ny,
    nz) hexes over `lengths` (node (i, j, k) has id (i (ny+1) + j)(nz+1) + k)
    at `points` [m, 3] inside the box."""
    nx, ny, nz = dims
    h = np.asarray(lengths, np.float64) / np.asarray(dims, np.float64)
    q = np.asarray(points, np.float64) / h
    cell = np.clip(np.floor(q).astype(np.int64), 0, np.asarray(dims) - 1)
    loc = np.clip(q - cell, 0.0, 1.0)
    order = np.argsort(-loc, axis=1, kind="stable")      # axes by decreasing local coordinate
    u = np.take_along_axis(loc, order, axis=1)
    w = np.stack([1.0 - u[:, 0], u[:, 0] - u[:, 1], u[:, 1] - u[:, 2], u[:, 2]], axis=1)
    out = np.zeros(points.shape[0])
    corner = cell.copy()
    rows = np.arange(points.shape[0])
    for v in range(4):
        if v > 0:
            corner[rows, order[:, v - 1]] += 1
        ids = (corner[:, 0] * (ny + 1) + corner[:, 1]) * (nz + 1) + corner[:, 2]
        out += w[:, v] * field[ids]
    return out


def run_to_activation(sim, spec, n_points: int = 21, chunk: int = 2000,
                      max_steps: int | None = None):
    """Advance `sim` (built from `spec`, an inputs.nversion) until every node
    has activated or `max_steps`; returns (diagonal activation times [n_points]
    in ms, steps taken, nodal LAT)."""
    max_steps = spec.n_steps if max_steps is None else max_steps
    steps = 0
    lat = None
    while steps < max_steps:
        k = min(chunk, max_steps - steps)
        sim.run(k)
        steps += k
        lat, _ = sim.times()
        if np.isfinite(lat).all():
            break
    dims = tuple(int(round(L / h)) for L, h in zip(DIAGONAL, _spacing(spec)))
    return kuhn_interpolate(lat, dims, DIAGONAL, diagonal_points(n_points)), steps, lat


def _spacing(spec):
    g = spec.mesh.grid
    return tuple(float(np.unique(np.round(g[:, a], 9))[1]) for a in range(3))
