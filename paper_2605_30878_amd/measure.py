"""FP64 post-processing of colour fields: interface points, circle/sphere fits,
measured contact angles on curved and flat solids, apex height.

This is measurement (Section 3 measures theta_m and h_max from the phi = 1/2
contour), not part of the time step; it takes plain numpy arrays and is
applied identically to any solver's output.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence, Tuple

import numpy as np


def interface_points(phi: np.ndarray, shape, solid: Optional[np.ndarray] = None,
                     level: float = 0.5) -> np.ndarray:
    """Points where phi crosses ``level`` between axis neighbours (linear
    interpolation), skipping pairs that touch a solid node.  Periodic axes are
    not wrapped (a pair across the box edge is skipped)."""
    nx, ny, nz = shape
    f = phi.reshape(nz, ny, nx)
    s = None if solid is None else solid.reshape(nz, ny, nx).astype(bool)
    pts = []
    for axis in (2, 1, 0):
        if f.shape[axis] < 2:
            continue
        a = np.take(f, np.arange(f.shape[axis] - 1), axis=axis)
        b = np.take(f, np.arange(1, f.shape[axis]), axis=axis)
        m = (a - level) * (b - level) < 0
        if s is not None:
            sa = np.take(s, np.arange(f.shape[axis] - 1), axis=axis)
            sb = np.take(s, np.arange(1, f.shape[axis]), axis=axis)
            m &= ~(sa | sb)
        idx = np.argwhere(m)
        if idx.size == 0:
            continue
        fa = a[m]
        fb = b[m]
        t = (level - fa) / (fb - fa)
        p = idx.astype(np.float64)  # (z, y, x)
        p[:, axis] += t
        pts.append(p[:, ::-1])  # -> (x, y, z)
    if not pts:
        return np.zeros((0, 3))
    return np.concatenate(pts, axis=0)


def fit_circle(pts: np.ndarray, dim: int = 2) -> Tuple[np.ndarray, float]:
    """Algebraic least-squares circle (dim 2, uses x, y) or sphere fit."""
    P = pts[:, :dim]
    A = np.concatenate([2.0 * P, np.ones((P.shape[0], 1))], axis=1)
    b = (P * P).sum(axis=1)
    sol, *_ = np.linalg.lstsq(A, b, rcond=None)
    c = sol[:dim]
    r = math.sqrt(sol[dim] + float((c * c).sum()))
    return c, r


def curved_contact_angle(phi: np.ndarray, shape, solid: np.ndarray, centre: Sequence[float],
                         R: float, W: float, dim: int = 2, margin: float = 2.0) -> dict:
    """theta_m on a disk/ball of radius R at ``centre``: fit the phi = 1/2
    points farther than margin*W from the solid, then
    cos theta_m = (R^2 + Rc^2 - d^2) / (2 R Rc)."""
    pts = interface_points(phi, shape, solid)
    c0 = np.asarray(centre[:dim], dtype=np.float64)
    dist = np.sqrt(((pts[:, :dim] - c0) ** 2).sum(axis=1))
    pts = pts[dist > R + margin * W]
    c, Rc = fit_circle(pts, dim)
    d = float(np.sqrt(((c - c0) ** 2).sum()))
    cos_t = (R * R + Rc * Rc - d * d) / (2.0 * R * Rc)
    cos_t = min(1.0, max(-1.0, cos_t))
    return {"theta": math.degrees(math.acos(cos_t)), "Rc": Rc, "d": d, "centre": c,
            "npts": int(pts.shape[0])}


def apex_height(phi: np.ndarray, shape, x_line: Sequence[int], start: float, axis: int,
                level: float = 0.5) -> float:
    """Coordinate (along ``axis``) of the last phi = level crossing on the grid
    line through ``x_line`` (the other coordinates), searching upward from
    ``start``.  Used for h_max on the symmetry axis."""
    nx, ny, nz = shape
    f = phi.reshape(nz, ny, nx)
    idx = [int(x_line[2]) if nz > 1 else 0, int(x_line[1]), int(x_line[0])]
    ax = 2 - axis
    idx[ax] = slice(None)
    line = f[tuple(idx)]
    k0 = int(math.ceil(start))
    last = None
    for k in range(k0, line.shape[0] - 1):
        a, b = line[k], line[k + 1]
        if (a - level) * (b - level) < 0 or a == level:
            last = k + (level - a) / (b - a) if b != a else float(k)
    if last is None:
        raise ValueError("no crossing on the line")
    return float(last)


def flat_contact_angle(phi: np.ndarray, shape, solid: np.ndarray, wall_y: float, W: float,
                       margin: float = 2.0) -> dict:
    """theta_m for a 2D cap on the wall surface y = wall_y: circle fit to the
    phi = 1/2 points more than margin*W above the wall; cos theta = -h_c/Rc
    with h_c the fitted centre's height above the wall."""
    pts = interface_points(phi, shape, solid)
    pts = pts[pts[:, 1] > wall_y + margin * W]
    c, Rc = fit_circle(pts, 2)
    h = float(c[1] - wall_y)
    cos_t = min(1.0, max(-1.0, -h / Rc))
    return {"theta": math.degrees(math.acos(cos_t)), "Rc": Rc, "centre": c,
            "npts": int(pts.shape[0])}
