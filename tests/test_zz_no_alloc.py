"""lbm_observe_static, the diagnostics call that allocates nothing (its
reduction scratch is a static device array of the library, shared by every
context on the device): the same diagnostics as lbm_observe, bit for bit,
on two calls in a row (a 64^3 box, then a smaller 24^3 box and a D2Q9 box,
each checked right after the other so that the second call meets the
first one's scratch contents), and a non-finite state is reported the same
way."""
import numpy as np
import pytest

from paper_2605_30878_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("step", "n_fluid", "n_solid", "n_ghost", "nonfinite", "mass_blue", "mass_red", "momentum", "max_speed",
        "kinetic_energy", "rc")


def _lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_30878_amd import lbm

    lbm.load_library()
    return lbm


def _same(a, b):
    """Equal field by field (non-finite values included: NaN equals NaN)."""
    for k in KEYS:
        x, y = np.asarray(a[k], dtype=np.float64), np.asarray(b[k], dtype=np.float64)
        assert np.array_equal(x, y, equal_nan=True), (k, a[k], b[k])


def test_observe_static_equals_observe_on_calls_in_a_row():
    lbm = _lbm()
    cases = [W.sphere_d3q19(64, theta=60.0, precision=W.FP32),          # larger first
             W.sphere_d3q19(24, theta=120.0, precision=W.FP16_OFS),     # then smaller
             W.cylinder_d2q9_128(theta=30.0)]
    sims = []
    for wl in cases:
        s = lbm.Simulation(wl, W.initial_phi(wl))
        s.step(30)
        sims.append(s)
    for s in sims:
        a = s.observe(static_scratch=True)
        b = s.observe()
        c = s.observe(static_scratch=True)
        print(f"[no-alloc] {s.wl.name}: mass {a['mass_blue']!r} max|u| {a['max_speed']:.3e}", flush=True)
        _same(a, b)
        _same(c, b)
        assert a["nonfinite"] == 0 and a["step"] == 30
    for s in sims:
        s.close()


def test_observe_static_reports_non_finite_state():
    lbm = _lbm()
    wl = W.sphere_d3q19(24, theta=60.0, precision=W.FP32)
    s = lbm.Simulation(wl, W.initial_phi(wl))
    N = s.read(lbm.FIELD_N)
    fluid = np.flatnonzero((s.read(lbm.FIELD_FLAGS).astype(np.int64) & lbm.FLAG_SOLID) == 0)
    N[5, fluid[len(fluid) // 3]] = np.inf
    s.set_field(lbm.FIELD_N, N)
    a = s.observe(allow_unstable=True, static_scratch=True)
    b = s.observe(allow_unstable=True)
    assert a["rc"] == lbm.EUNSTABLE and a["nonfinite"] >= 1
    _same(a, b)
    s.close()
