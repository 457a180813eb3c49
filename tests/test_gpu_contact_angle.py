"""Reduced-precision runs of the D3Q19 drop on a sphere (64^3, density ratio
1000, viscosity ratio 100) against the FP64 oracle after 20000 steps: the
contact angle (from the apex height and liquid volume, Section 3.2's
measure) within 0.5 degrees, the spurious-current maximum within 10 %, the
Laplace pressure jump within 2 % for FP32 and FP16-offset storage.

Two starts, two stored oracle references (tests/golden/, written by
tests/golden/make_sphere64.py from the oracle alone; the same FP64
measurement is applied to both sides):
  - the equilibrium cap of each angle (Sec. 3.2's start;
    sphere64_eq_oracle.json): the state at 20000 steps is the equilibrium
    drop, so this compares equilibrium angles;
  - a drop of radius 10 on the sphere top (sphere64_oracle.json), still
    relaxing at 20000 steps: this compares trajectories.
BF16 offsets (8 significant bits) meet the bar from the equilibrium start
up to 120 degrees (measured -0.04 / -0.07 / -0.38 degrees at 60 / 90 / 120,
spurious currents within 5 %) and miss it at 150 degrees (-1.81 degrees,
-27 % spurious current); in the transient they miss it too (-0.62 degrees
at 90 and -1.62 degrees at 150, +14 % and +17 % spurious currents).  Where
they miss, they are held to 2 degrees, 30 % and 2 % only as a regression
guard, not as a claim."""
import json
import os

import numpy as np
import pytest

from paper_2605_30878_amd import measure
from paper_2605_30878_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GOLDEN = {"transient": os.path.join(GOLDEN_DIR, "sphere64_oracle.json"),
          "equilibrium": os.path.join(GOLDEN_DIR, "sphere64_eq_oracle.json")}

# (angle, spurious current, Laplace jump) bars per storage and start
CLAIM, GUARD = (0.5, 0.10, 0.02), (2.0, 0.30, 0.02)


def bars(start: str, name: str, theta: float):
    if name != "bf16ofs":
        return CLAIM
    return CLAIM if start == "equilibrium" and theta <= 120.0 else GUARD


def _golden(start):
    if not os.path.exists(GOLDEN[start]):
        return {}
    with open(GOLDEN[start]) as f:
        return json.load(f)


def _measure(lbm, sim, wl):
    n = wl.shape[0]
    flags = sim.read(lbm.FIELD_FLAGS).astype(np.int64)
    solid = (flags & lbm.FLAG_SOLID) > 0
    phi = sim.read(lbm.FIELD_PHI)
    p = sim.read(lbm.FIELD_P)
    c = n / 2.0
    R = wl.solids[0].radius
    apex = measure.apex_height(phi, wl.shape, (n // 2, n // 2, 0), c + R, axis=2) - c
    rho = wl.rho_g + (wl.rho_l - wl.rho_g) * phi
    ph = rho * p
    fluid = ~solid
    o = sim.observe()
    return {"theta_apex": measure.angle_from_apex(R, o["mass_blue"], apex, dim=3), "apex": apex,
            "dp_h": float(ph[fluid & (phi > 0.999)].mean() - ph[fluid & (phi < 0.001)].mean()),
            "max_speed": o["max_speed"], "mass_blue": o["mass_blue"]}


def _workload(start, theta, prec, steps, probe):
    if start == "equilibrium":
        return W.sphere_cap_d3q19(64, theta=theta, precision=prec, probe=probe, steps=steps)
    return W.sphere_d3q19(64, theta=theta, precision=prec, steps=steps).with_(probe=probe)


@pytest.mark.parametrize("start", ["equilibrium", "transient"])
def test_reduced_precision_contact_angle_against_oracle(start):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gold = _golden(start)
    if not gold:
        pytest.skip("no oracle reference yet")
    from paper_2605_30878_amd import lbm

    keys = sorted(gold, key=lambda k: (gold[k].get("theta", float(k.split("/")[0])), k))
    precs = [W.FP32, W.FP16_OFS, W.BF16_OFS]
    cases = [(k, p) for k in keys for p in precs]
    steps = int(gold[keys[0]]["steps"])
    print(f"[angle] start={start} cases={cases} steps={steps}", flush=True)
    wls = [_workload(start, gold[k].get("theta", float(k.split("/")[0])), p, steps, int(gold[k].get("probe", 0)))
           for k, p in cases]
    sims = [lbm.Simulation(wl, W.initial_phi(wl)) for wl in wls]
    batch = lbm.Batch(max_jobs=len(sims))
    for _ in range(steps // 2000):
        batch.step(sims, [2000] * len(sims))
    batch.close()
    worst = {}
    for (t, p), wl, sim in zip(cases, wls, sims):
        g = gold[t]
        m = _measure(lbm, sim, wl)
        d_theta = m["theta_apex"] - g["theta_apex"]
        r_speed = m["max_speed"] / g["max_speed"] - 1.0
        r_dp = m["dp_h"] / g["dp_h"] - 1.0
        r_mass = m["mass_blue"] / g["mass_blue"] - 1.0
        name = W.PRECISION_NAMES[p]
        print(f"[angle] {start} theta={t} {name}: theta {m['theta_apex']:.3f} (oracle {g['theta_apex']:.3f}, "
              f"diff {d_theta:+.3f}); max|u| {m['max_speed']:.3e} ({r_speed:+.2%}); "
              f"dp_h {m['dp_h']:.4e} ({r_dp:+.2%}); mass {r_mass:+.2e}", flush=True)
        worst[(t, name)] = (d_theta, r_speed, r_dp)
        sim.close()
    for (t, name), (d_theta, r_speed, r_dp) in worst.items():
        b_theta, b_speed, b_dp = bars(start, name, gold[t].get("theta", float(t.split("/")[0])))
        assert abs(d_theta) <= b_theta, (t, name, d_theta)
        assert abs(r_speed) <= b_speed, (t, name, r_speed)
        if np.isfinite(gold[t]["dp_h"]):   # a thin cap (30 degrees) has no bulk liquid node to measure
            assert abs(r_dp) <= b_dp, (t, name, r_dp)
