"""Host-side logic on the CPU: the packing generator, the initial colour
field, the served-mix request generator and its latency summary, and the
closed forms the contact-angle measurement inverts.  Each is checked
against what its definition fixes (non-overlap, the distributions' ranges,
lens geometry by Monte Carlo, round trips)."""
import math

import numpy as np
import pytest

from paper_2605_30878_amd import measure
from paper_2605_30878_amd import serve
from paper_2605_30878_amd import workloads as W


def _min_image_distances(pos, n):
    d = pos[:, None, :] - pos[None, :, :]
    d -= n * np.round(d / n)
    r = np.sqrt((d * d).sum(axis=-1))
    return r[np.triu_indices(len(pos), 1)]


def test_sphere_packing_is_seeded_and_non_overlapping():
    n, R, frac = 64, 6.0, 0.5
    a = W.sphere_packing(n, R, frac, seed=3)
    b = W.sphere_packing(n, R, frac, seed=3)
    c = W.sphere_packing(n, R, frac, seed=4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert len(a) == int(round(frac * n ** 3 / (4.0 / 3.0 * math.pi * R ** 3)))
    assert np.all((a >= 0) & (a < n))
    assert _min_image_distances(a, n).min() >= 2 * R - 1e-6


def test_porous_workload_geometry_options():
    wl = W.porous_d3q19(n=40, sphere_radius=5.0, porosity=0.40, seed=0, front=10.0)
    assert wl.probe == 1 and wl.fill == 1 and wl.theta == 45.0
    assert wl.rho_l / wl.rho_g == 10.0 and (wl.mu_l / wl.rho_l) == pytest.approx(wl.mu_g / wl.rho_g)
    phi = W.initial_phi(wl).reshape(40, 40, 40)
    # liquid slab x in [0, 10) with tanh edges at x = 0 and x = 10 (periodic)
    assert phi[:, :, 5].min() > 0.99 and phi[:, :, 25].max() < 0.01
    assert np.allclose(phi[:, :, 10], 0.5) and np.allclose(phi[:, :, 0], 0.5)


@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_initial_drop_profile(lattice):
    n, Rd, width = 48, 10.0, 4.0
    wl = W.free_drop(lattice, n, Rd, W=width)
    phi = W.initial_phi(wl)
    nz = n if lattice == W.D3Q19 else 1
    f = phi.reshape(nz, n, n)
    z0 = n // 2 if lattice == W.D3Q19 else 0
    row = f[z0, n // 2, :]
    x = np.arange(n) - n / 2.0
    want = 0.5 * (1.0 + np.tanh(2.0 * (Rd - np.abs(x)) / width))
    assert np.allclose(row, want, atol=1e-15)
    assert 0.0 <= phi.min() and phi.max() <= 1.0


def test_mixed_requests_follow_their_distributions():
    reqs = serve.mixed_requests(256, seed=0)
    assert [r.rid for r in reqs] == list(range(256))
    d3 = [r for r in reqs if r.workload.lattice == W.D3Q19]
    d2 = [r for r in reqs if r.workload.lattice == W.D2Q9]
    assert 0.30 < len(d3) / 256 < 0.50
    for r in reqs:
        wl = r.workload
        L = wl.shape[0]
        lo, hi = (48, 192) if wl.lattice == W.D3Q19 else (64, 512)
        assert lo - 1 <= L <= hi + 1
        assert wl.shape == ((L, L, L) if wl.lattice == W.D3Q19 else (L, L, 1))
        assert 20.0 <= wl.theta <= 160.0
        ratio = wl.rho_l / wl.rho_g
        assert 1.0 <= ratio <= 1000.0
        assert wl.mu_l / wl.mu_g == pytest.approx(max(1.0, ratio / 10.0))
        assert 2000 <= r.steps <= 20000 and r.steps == wl.steps
        R = wl.solids[0].radius
        assert 0.2 * L <= R <= 0.35 * L
    assert min(r.workload.shape[0] for r in d2) < 128 and max(r.workload.shape[0] for r in d2) > 256
    # scaled runs shrink steps and sides
    small = serve.mixed_requests(8, seed=0, step_scale=0.01, size_scale=0.3)
    assert all(r.steps <= 200 for r in small)
    # seeded: the same seed gives the same mix, another seed another one
    a, b, c = (serve.mixed_requests(16, seed=k) for k in (5, 5, 6))
    assert [(r.workload.shape, r.workload.theta, r.steps) for r in a] == \
        [(r.workload.shape, r.workload.theta, r.steps) for r in b]
    assert [r.workload.theta for r in a] != [r.workload.theta for r in c]


def test_poisson_arrivals_and_summary():
    reqs = serve.mixed_requests(4000, seed=1, step_scale=0.01, size_scale=0.1)
    arr = serve.poisson_arrivals(reqs, rate=50.0, seed=2)
    t = np.array([r.arrival for r in arr])
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() * 50.0 - 1.0) < 0.05          # mean gap 1/rate (4000 draws)
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.08    # exponential: std = mean
    assert all(r.arrival == 0.0 for r in serve.poisson_arrivals(reqs[:5], rate=0.0))
    res = [serve.Result(k, 0.0, 0.0, float(k + 1), 100, 10, {}) for k in range(100)]
    s = serve.summarize(res, wall=50.0)
    assert s["jobs"] == 100 and s["throughput_jobs_s"] == 2.0
    assert s["p50_latency_s"] == pytest.approx(50.5) and s["p99_latency_s"] == pytest.approx(99.01)
    assert s["aggregate_mlups"] == pytest.approx(100 * 100 * 10 / 50.0 / 1e6)
    # unstable runs (retired early) stay out of the latency and job counts;
    # the updates they made still count in the aggregate rate
    res[3].status = "unstable"
    res[7].status = "unstable"
    s = serve.summarize(res, wall=50.0)
    assert s["jobs"] == 98 and s["unstable_jobs"] == 2 and s["throughput_jobs_s"] == pytest.approx(98 / 50.0)
    assert s["aggregate_mlups"] == pytest.approx(100 * 100 * 10 / 50.0 / 1e6)
    lat = np.array([r.latency for r in res if r.status == "ok"])
    assert s["p99_latency_s"] == pytest.approx(float(np.percentile(lat, 99)))


def test_lens_geometry_by_monte_carlo():
    """Area / volume of the intersection of two circles / balls (used to
    place equilibrium drops) against a seeded Monte-Carlo estimate."""
    rng = np.random.default_rng(0)
    r1, r2, d = 5.0, 3.5, 6.0
    pts = rng.uniform(-6.0, 6.0, size=(400000, 3))
    in1 = (pts ** 2).sum(1) <= r1 ** 2
    in2 = ((pts - [d, 0, 0]) ** 2).sum(1) <= r2 ** 2
    # box x in [-6, 6]: the lens lies in x in [d - r2, r1] = [2.5, 5] and |y|, |z| < 3.5
    vol = (in1 & in2).mean() * 12.0 ** 3
    assert measure.lens_volume(r1, r2, d) == pytest.approx(vol, rel=0.02)
    p2 = pts[:, :2]
    in1 = (p2 ** 2).sum(1) <= r1 ** 2
    in2 = ((p2 - [d, 0]) ** 2).sum(1) <= r2 ** 2
    area = (in1 & in2).mean() * 12.0 ** 2
    assert measure.lens_area(r1, r2, d) == pytest.approx(area, rel=0.02)
    assert measure.lens_area(r1, r2, r1 + r2 + 1.0) == 0.0


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("theta", [30.0, 90.0, 150.0])
def test_drop_on_solid_round_trip(dim, theta):
    """The equilibrium drop of a given amount outside the solid: the cap
    meets the solid at angle theta (with theta through the liquid, the radii
    to the two centres enclose theta at the contact line: d = R + Rc at 180
    degrees, orthogonal circles at 90), holds the amount, and
    angle_from_apex inverts its apex height."""
    R = 12.0
    amount = 900.0 if dim == 2 else 8000.0
    Rc, d, h = measure.drop_on_solid(R, amount, theta, dim)
    assert d * d == pytest.approx(R * R + Rc * Rc - 2 * R * Rc * math.cos(math.radians(theta)), rel=1e-9)
    assert measure.centre_distance(R, 5.0, 180.0) == pytest.approx(R + 5.0)
    assert measure.centre_distance(R, 5.0, 90.0) == pytest.approx(math.hypot(R, 5.0))
    held = (math.pi * Rc * Rc - measure.lens_area(R, Rc, d) if dim == 2 else
            4.0 / 3.0 * math.pi * Rc ** 3 - measure.lens_volume(R, Rc, d))
    assert held == pytest.approx(amount, rel=1e-9)
    assert h == pytest.approx(d + Rc)
    assert measure.angle_from_apex(R, amount, h, dim) == pytest.approx(theta, abs=1e-6)
