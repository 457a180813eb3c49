"""Synthetic workloads: geometry, physical parameters and the initial colour field.

This module is the only code shared by the GPU library's callers and the CPU
oracle's callers.  It holds no part of the method's arithmetic: it describes
problems (box, solids, drops, parameters) and draws the initial diffuse drop
shape, which is an input of the simulation, not a step of it.  All shapes are
deterministic; the porous packing is seeded.

Node (x, y, z) has integer coordinates and flat index x + nx*(y + ny*z);
arrays returned here are FP64 with that ordering.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

D2Q9 = 0
D3Q19 = 1

FP64 = 0
FP32 = 1
FP16_OFS = 2
BF16_OFS = 3

PRECISION_NAMES = {FP64: "f64", FP32: "f32", FP16_OFS: "f16ofs", BF16_OFS: "bf16ofs"}


@dataclasses.dataclass
class Solid:
    """kind 0: ball/disk |x - center| <= radius (closed).
    kind 1: half-space (x - center) . normal <= 0, normal points out of the solid."""

    kind: int
    center: Tuple[float, float, float]
    radius: float = 0.0
    normal: Tuple[float, float, float] = (0.0, 0.0, 0.0)


@dataclasses.dataclass
class LiquidRegion:
    """A liquid (phi = 1) region with a tanh edge of the given width.

    kind "ball": |x - center| < radius (periodic minimum image along the axes
    in `periodic`; plain distance along the others, e.g. across walls).
    kind "slab": lo <= x_axis < hi along `axis` (periodic distance).
    kind "below": x_axis < lo along `axis`.
    """

    kind: str
    center: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    radius: float = 0.0
    axis: int = 0
    lo: float = 0.0
    hi: float = 0.0
    width: float = 4.0
    periodic: Tuple[bool, bool, bool] = (True, True, True)


@dataclasses.dataclass
class Workload:
    name: str
    lattice: int
    shape: Tuple[int, int, int]  # (nx, ny, nz); nz = 1 for D2Q9
    rho_l: float = 1000.0
    rho_g: float = 1.0
    mu_l: float = 10.0
    mu_g: float = 0.1
    sigma: float = 1e-2
    W: float = 4.0
    mobility: float = 0.02
    g: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    theta: float = 90.0
    solids: List[Solid] = dataclasses.field(default_factory=list)
    liquid: List[LiquidRegion] = dataclasses.field(default_factory=list)
    precision: int = FP64
    steps: int = 1000
    ghost_rule: int = 0
    probe: int = 0   # 0: probe interpolation over all corners; 1: fluid corners only
    fill: int = 0    # 1: fluid nodes with at most one fluid lattice neighbour become solid (repeated)

    @property
    def nodes(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _coords(shape):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def _periodic_delta(a, c, n):
    d = a - c
    return d - n * np.round(d / n)


def initial_phi(wl: Workload) -> np.ndarray:
    """Initial colour field: 1/2 (1 + tanh(2 s / width)) with s the signed
    distance into the liquid region (the diffuse drop shape the workload
    prescribes), max over regions.  Solid nodes are left as computed; each
    solver overwrites them with its own initial solid value."""
    nx, ny, nz = wl.shape
    x, y, z = _coords(wl.shape)
    phi = np.zeros((nz, ny, nx), dtype=np.float64)
    pos = (x, y, z)
    for reg in wl.liquid:
        if reg.kind == "ball":
            px, py, pz = reg.periodic
            dx = _periodic_delta(x, reg.center[0], nx) if px else x - reg.center[0]
            dy = _periodic_delta(y, reg.center[1], ny) if py else y - reg.center[1]
            if wl.lattice == D3Q19:
                dz = _periodic_delta(z, reg.center[2], nz) if pz else z - reg.center[2]
            else:
                dz = 0.0 * z
            s = reg.radius - np.sqrt(dx * dx + dy * dy + dz * dz)
        elif reg.kind == "slab":
            n = wl.shape[reg.axis]
            t = pos[reg.axis]
            mid = 0.5 * (reg.lo + reg.hi)
            half = 0.5 * (reg.hi - reg.lo)
            s = half - np.abs(_periodic_delta(t, mid, n))
        elif reg.kind == "below":
            s = reg.lo - pos[reg.axis]
        else:
            raise ValueError(f"unknown liquid region {reg.kind!r}")
        phi = np.maximum(phi, 0.5 * (1.0 + np.tanh(2.0 * s / reg.width)))
    return phi.reshape(-1)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def cylinder_d2q9_128(theta: float = 90.0, precision: int = FP64) -> Workload:
    """D2Q9 drop on a cylinder: 128x128 periodic box, disk radius 24 at
    (64, 48), drop radius 20 centred on the disk top (64, 72) with tanh width
    5; density and viscosity ratio 1 (rho = 1, mu = 0.1), sigma = 0.01,
    2000 steps.  The interface width of the model is also 5."""
    return Workload(
        name="d2q9_cylinder_128", lattice=D2Q9, shape=(128, 128, 1),
        rho_l=1.0, rho_g=1.0, mu_l=0.1, mu_g=0.1, sigma=0.01, W=5.0, mobility=0.02,
        theta=theta,
        solids=[Solid(0, (64.0, 48.0, 0.0), 24.0)],
        liquid=[LiquidRegion("ball", (64.0, 72.0, 0.0), 20.0, width=5.0)],
        precision=precision, steps=2000)


def sphere_d3q19(n: int = 256, theta: float = 90.0, precision: int = FP32,
                 steps: int = 20000) -> Workload:
    """D3Q19 drop on a sphere in a periodic n^3 box (z up).  At n = 256:
    sphere radius 48 at the centre, drop radius 40 centred on the sphere top;
    smaller boxes scale every length by n/256 (n = 64: radii 12 and 10).
    rho_l/rho_g = 1000/1, mu_l/mu_g = 10/0.1, W = 4, sigma = 0.01."""
    s = n / 256.0
    c = n / 2.0
    R = 48.0 * s
    Rd = 40.0 * s
    return Workload(
        name=f"d3q19_sphere_{n}", lattice=D3Q19, shape=(n, n, n),
        rho_l=1000.0, rho_g=1.0, mu_l=10.0, mu_g=0.1, sigma=0.01, W=4.0, mobility=0.02,
        theta=theta,
        solids=[Solid(0, (c, c, c), R)],
        liquid=[LiquidRegion("ball", (c, c, c + R), Rd, width=4.0)],
        precision=precision, steps=steps)


def sphere_cap_d3q19(n: int = 256, theta: float = 90.0, precision: int = FP32, probe: int = 0,
                     volume: Optional[float] = None, steps: int = 20000) -> Workload:
    """The drop on a sphere of `sphere_d3q19`, started at its equilibrium cap
    for theta instead of the radius-40n/256 drop: a ball of radius R_c whose
    centre is d above the sphere centre, with d^2 = R^2 + R_c^2 - 2 R R_c cos
    theta (the drop meets the sphere at theta, Sec. 3.2) and R_c fixed by the
    liquid volume outside the sphere.  The default volume is that of the
    transient benchmark's drop outside the sphere.  The cap is geometry
    (lens volumes of two balls), not a step of the method."""
    from . import measure

    s = n / 256.0
    c = n / 2.0
    R = 48.0 * s
    if volume is None:
        Rd = 40.0 * s
        volume = 4.0 / 3.0 * math.pi * Rd ** 3 - measure.lens_volume(R, Rd, R)
    Rc, d, _ = measure.drop_on_solid(R, volume, theta, 3)
    return sphere_d3q19(n, theta=theta, precision=precision, steps=steps).with_(
        name=f"sphere{n}_eq_t{theta:g}", probe=probe,
        liquid=[LiquidRegion("ball", (c, c, c + d), Rc, width=4.0)])


def free_drop(lattice: int, n: int, radius: float, rho_ratio: float = 1.0,
              mu_ratio: float = 1.0, W: float = 4.0, sigma: float = 0.01,
              precision: int = FP64) -> Workload:
    """A drop in a periodic box with no solid (Laplace-law workload)."""
    nz = n if lattice == D3Q19 else 1
    c = n / 2.0
    return Workload(
        name=f"free_drop_{'d3q19' if lattice else 'd2q9'}_{n}", lattice=lattice,
        shape=(n, n, nz), rho_l=rho_ratio, rho_g=1.0, mu_l=0.1 * mu_ratio, mu_g=0.1,
        sigma=sigma, W=W, theta=90.0,
        liquid=[LiquidRegion("ball", (c, c, c if lattice == D3Q19 else 0.0), radius, width=W)],
        precision=precision, steps=1000)


def plate_d2q9(nx: int, ny: int, theta: float, drop_radius: float, W: float = 4.0,
               rho_ratio: float = 1.0, mu_ratio: float = 1.0,
               precision: int = FP64) -> Workload:
    """A drop on a flat wall: solid rows y = 0 and y = ny - 1 (half-spaces),
    periodic in x, drop centred on the lower wall surface at y = 0.5."""
    return Workload(
        name=f"plate_d2q9_{nx}x{ny}", lattice=D2Q9, shape=(nx, ny, 1),
        rho_l=rho_ratio, rho_g=1.0, mu_l=0.1 * mu_ratio, mu_g=0.1, sigma=0.01, W=W,
        theta=theta,
        solids=[Solid(1, (0.0, 0.5, 0.0), normal=(0.0, 1.0, 0.0)),
                Solid(1, (0.0, ny - 1.5, 0.0), normal=(0.0, -1.0, 0.0))],
        liquid=[LiquidRegion("ball", (nx / 2.0, 0.5, 0.0), drop_radius, width=W)],
        precision=precision, steps=1000)


def porous_d3q19(n: int = 384, sphere_radius: float = 12.0, porosity: float = 0.40,
                 seed: int = 0, precision: int = FP32, front: Optional[float] = None,
                 max_iter: int = 20000, probe: int = 1, fill: int = 1) -> Workload:
    """Dynamic contact line in a random packing of non-overlapping spheres.

    Sphere count is chosen so that the continuous solid fraction equals
    1 - porosity; centres start uniform (seeded) and are pushed apart under the
    periodic minimum image until no pair overlaps.  The wetting liquid
    (theta = 45 deg) fills x < front with tanh interfaces at x = front and
    x = 0; rho_l/rho_g = 10, mu_l/mu_g = 10, body acceleration (1e-6, 0, 0).
    The ghost-rule probe interpolates fluid corners only (probe = 1), and a
    ghost whose probe cell has no fluid corner takes its fluid lattice
    neighbours: with all corners, probes in the gaps between touching spheres
    read the far solid's (1 + cos theta)/2 and the run diverges within a few
    hundred steps (oracle and library alike).  Fluid nodes joined to the
    pore space by at most one lattice link (fill = 1; 0.03 % of the pore
    nodes at 384^3, in the contacts between spheres) are made solid: left
    fluid, such a node between the two spheres' ghost values is driven
    unstable below 90 degrees."""
    centres = sphere_packing(n, sphere_radius, 1.0 - porosity, seed, max_iter)
    solids = [Solid(0, tuple(float(v) for v in c), sphere_radius) for c in centres]
    front = n / 4.0 if front is None else front
    return Workload(
        name=f"d3q19_porous_{n}", lattice=D3Q19, shape=(n, n, n),
        rho_l=10.0, rho_g=1.0, mu_l=1.0, mu_g=0.1, sigma=0.01, W=4.0, mobility=0.02,
        g=(1e-6, 0.0, 0.0), theta=45.0, solids=solids,
        liquid=[LiquidRegion("slab", axis=0, lo=0.0, hi=front, width=4.0)],
        precision=precision, steps=50000, probe=probe, fill=fill)


def sphere_packing(n: int, radius: float, solid_fraction: float, seed: int,
                   max_iter: int = 20000, tol: float = 1e-6) -> np.ndarray:
    """Seeded non-overlapping sphere centres in a periodic n^3 box.

    The count gives the requested continuous solid fraction; centres start
    uniform (seeded), then every overlapping pair (periodic minimum image,
    found with a periodic k-d tree) is pushed apart along its centre line by
    half the overlap each, until the largest overlap is below `tol`."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    count = int(round(solid_fraction * n ** 3 / ((4.0 / 3.0) * math.pi * radius ** 3)))
    pos = rng.uniform(0.0, n, size=(count, 3))
    dmin = 2.0 * radius
    for _ in range(max_iter):
        pairs = cKDTree(pos, boxsize=n).query_pairs(dmin, output_type="ndarray")
        if len(pairs) == 0:
            break
        a, b = pairs[:, 0], pairs[:, 1]
        dv = pos[b] - pos[a]
        dv -= n * np.round(dv / n)
        dist = np.sqrt((dv * dv).sum(axis=1))
        ov = dmin - dist
        if ov.max() < tol:
            break
        push = 0.5 * (ov + 1e-7)[:, None] * dv / np.maximum(dist, 1e-12)[:, None]
        disp = np.zeros_like(pos)
        np.add.at(disp, b, push)
        np.add.at(disp, a, -push)
        pos = (pos + disp) % n
    return pos


def lattice_name(lattice: int) -> str:
    return "D3Q19" if lattice == D3Q19 else "D2Q9"


def n_directions(lattice: int) -> int:
    return 19 if lattice == D3Q19 else 9
