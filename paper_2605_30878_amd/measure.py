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

# ---------------------------------------------------------------- closed forms
# Drop on a cylinder / sphere: at the contact point the wetting condition of
# Eq. 7 (n_s . n_phi = -cos theta, n_s out of the solid, n_phi into the
# liquid) fixes the angle between the two circles, so the centre distance d
# obeys d^2 = R^2 + Rc^2 - 2 R Rc cos(theta).  The drop area (2D) or volume
# (3D) outside the solid then fixes Rc; the apex height above the solid
# centre is h_max = d + Rc (Section 3.2 measures h_max / R).
# Drop on a flat plate: a circular cap of area A and contact angle theta has
# Rc = sqrt(2A / (2 theta - sin 2 theta)) (Section 3.1), height
# H = Rc (1 - cos theta) and half-base a = Rc sin theta, for which Eq. 12
# returns theta when its spread S is read as the half-base.


def lens_area(r1: float, r2: float, d: float) -> float:
    """Area of the intersection of two disks of radii r1, r2 at distance d."""
    if d >= r1 + r2:
        return 0.0
    if d <= abs(r1 - r2):
        return math.pi * min(r1, r2) ** 2
    a1 = r1 * r1 * math.acos((d * d + r1 * r1 - r2 * r2) / (2 * d * r1))
    a2 = r2 * r2 * math.acos((d * d + r2 * r2 - r1 * r1) / (2 * d * r2))
    k = 0.5 * math.sqrt((-d + r1 + r2) * (d + r1 - r2) * (d - r1 + r2) * (d + r1 + r2))
    return a1 + a2 - k


def lens_volume(r1: float, r2: float, d: float) -> float:
    """Volume of the intersection of two balls of radii r1, r2 at distance d."""
    if d >= r1 + r2:
        return 0.0
    if d <= abs(r1 - r2):
        return 4.0 / 3.0 * math.pi * min(r1, r2) ** 3
    return (math.pi * (r1 + r2 - d) ** 2
            * (d * d + 2 * d * r2 - 3 * r2 * r2 + 2 * d * r1 + 6 * r1 * r2 - 3 * r1 * r1) / (12 * d))


def centre_distance(R: float, Rc: float, theta_deg: float) -> float:
    th = math.radians(theta_deg)
    return math.sqrt(max(R * R + Rc * Rc - 2 * R * Rc * math.cos(th), 0.0))


def drop_on_solid(R: float, amount: float, theta_deg: float, dim: int = 2):
    """Solve for (Rc, d, h_max) of a drop of area (dim 2) or volume (dim 3)
    ``amount`` outside a disk/ball of radius R at contact angle theta."""
    def outside(Rc):
        d = centre_distance(R, Rc, theta_deg)
        if dim == 2:
            return math.pi * Rc * Rc - lens_area(R, Rc, d)
        return 4.0 / 3.0 * math.pi * Rc ** 3 - lens_volume(R, Rc, d)

    lo, hi = 1e-6, 1.0
    while outside(hi) < amount:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if outside(mid) < amount:
            lo = mid
        else:
            hi = mid
    Rc = 0.5 * (lo + hi)
    d = centre_distance(R, Rc, theta_deg)
    return Rc, d, d + Rc


def plate_cap(area: float, theta_deg: float):
    """(Rc, H, half_base) of a 2D circular cap of the given area."""
    th = math.radians(theta_deg)
    Rc = math.sqrt(2.0 * area / (2.0 * th - math.sin(2.0 * th)))
    return Rc, Rc * (1.0 - math.cos(th)), Rc * math.sin(th)


def angle_from_apex(R: float, amount: float, h: float, dim: int = 2) -> float:
    """Contact angle (degrees) whose equilibrium drop of the given area (2D)
    or volume (3D) on a disk/ball of radius R has apex height h above the
    solid centre (h_max grows with theta at fixed amount); clamped to
    [0, 180]."""
    lo, hi = 1e-6, 180.0 - 1e-6
    if h <= drop_on_solid(R, amount, lo, dim)[2]:
        return 0.0
    if h >= drop_on_solid(R, amount, hi, dim)[2]:
        return 180.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if drop_on_solid(R, amount, mid, dim)[2] < h:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def plate_angle(half_base: float, H: float) -> float:
    """Eq. 12 with S read as the half-base; returns degrees."""
    return math.degrees(math.acos((half_base ** 2 - H ** 2) / (half_base ** 2 + H ** 2)))


# ---------------------------------------------------------------- measurements
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
    if pts.shape[0] < dim + 2:
        raise ValueError("too few interface points away from the solid for a fit")
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


def plate_angle_eq12(phi: np.ndarray, shape, wall: float = 0.5) -> dict:
    """Contact angle of a 2D drop on the wall surface y = wall (solid rows
    below it) by Eq. 12 (Sec. 3.1) with its spread S read as the half-base:
    S is half the distance between the phi = 1/2 crossings on the first fluid
    row, H the height of the last phi = 1/2 crossing above the wall on the
    column through the drop's middle."""
    nx, ny, _ = shape
    f = phi.reshape(ny, nx)
    row = f[1]
    inside = np.flatnonzero(row > 0.5)
    if inside.size == 0:
        raise ValueError("drop does not touch the wall")
    lo, hi = inside.min(), inside.max()
    # linear interpolation of the two crossings on the first fluid row
    xl = lo - (row[lo] - 0.5) / (row[lo] - row[lo - 1])
    xr = hi + (row[hi] - 0.5) / (row[hi] - row[hi + 1])
    S = 0.5 * (xr - xl)
    xc = int(round(0.5 * (xl + xr)))
    top = apex_height(phi, shape, (xc, 0, 0), 1.0, axis=1)
    H = top - wall
    return {"theta_eq12": plate_angle(S, H), "S": S, "H": H}


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
