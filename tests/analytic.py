"""Closed-form equilibrium shapes used as pins (FP64).

Drop on a cylinder / sphere: at the contact point the wetting condition of
Eq. 7 (n_s . n_phi = -cos theta, n_s out of the solid, n_phi into the liquid)
fixes the angle between the two circles, so the centre distance d obeys
d^2 = R^2 + Rc^2 - 2 R Rc cos(theta).  The drop area (2D) or volume (3D)
outside the solid then fixes Rc; the apex height above the solid centre is
h_max = d + Rc (Section 3.2 measures h_max/R).

Drop on a flat plate: a circular cap of area A and contact angle theta has
Rc = sqrt(2A / (2 theta - sin 2 theta)) (Section 3.1), height
H = Rc (1 - cos theta) and half-base a = Rc sin theta, for which Eq. 12
returns theta when its spread S is read as the half-base.
"""
from __future__ import annotations

import math


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


def plate_angle(half_base: float, H: float) -> float:
    """Eq. 12 with S read as the half-base; returns degrees."""
    return math.degrees(math.acos((half_base ** 2 - H ** 2) / (half_base ** 2 + H ** 2)))
