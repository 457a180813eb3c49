"""Write the FP64 oracle's measurements of the D3Q19 drop on a sphere in a
64^3 box (sphere radius 12 at the centre, density ratio 1000, viscosity
ratio 100, W = 4, sigma = 0.01) after 20000 steps, for each contact angle
(at 30 degrees with the fluid-only probe interpolation: with all probe
corners that run diverges within 250 steps).

    tests/golden/sphere64_oracle.json     drop of radius 10 on the sphere
        top: the drops are still relaxing from that starting shape at 20000
        steps, so this is a trajectory;
    tests/golden/sphere64_eq_oracle.json  (--equilibrium) the drop started
        at its equilibrium cap for the angle with the same liquid volume
        outside the sphere (Sec. 3.2's start), so the state at 20000 steps is
        the equilibrium shape.

Only the oracle computes the fields; the FP64 numpy post-processing in
paper_2605_30878_amd/measure.py (the same fit the GPU test applies to the
library's output) turns them into angles and heights.  Run:
    OMP_NUM_THREADS=8 python tests/golden/make_sphere64.py [--equilibrium] [theta[p] ...]
(about 20 minutes per angle on 8 cores)."""
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2605_30878_amd import measure  # noqa: E402
from paper_2605_30878_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "sphere64_oracle.json")
OUT_EQ = os.path.join(HERE, "sphere64_eq_oracle.json")
STEPS = 20000


def measure_state(sim, wl):
    n = wl.shape[0]
    solid = sim.get(oracle.F_SOLID) > 0.5
    phi = sim.get(oracle.F_PHI)
    u = sim.get(oracle.F_U)
    p = sim.get(oracle.F_P)
    rho = sim.get(oracle.F_RHO)
    c = n / 2.0
    R = wl.solids[0].radius
    apex = measure.apex_height(phi, wl.shape, (n // 2, n // 2, 0), c + R, axis=2) - c
    ph = rho * p
    fluid = ~solid
    speed = np.sqrt((u * u).sum(axis=0))
    mass = float(phi[fluid].sum())
    rec = {"apex": apex, "theta_apex": measure.angle_from_apex(R, mass, apex, dim=3),
           "dp_h": float(ph[fluid & (phi > 0.999)].mean() - ph[fluid & (phi < 0.001)].mean()),
           "max_speed": float(speed[fluid].max()), "mass_blue": mass}
    try:
        fit = measure.curved_contact_angle(phi, wl.shape, solid, (c, c, c), R, wl.W, dim=3, margin=1.0)
        rec.update({"theta_fit": fit["theta"], "Rc": fit["Rc"], "d": fit["d"]})
    except ValueError:
        rec.update({"theta_fit": None, "Rc": None, "d": None})
    return rec


def workload(th: float, probe: int, equilibrium: bool) -> W.Workload:
    if equilibrium:
        return W.sphere_cap_d3q19(64, theta=th, precision=W.FP64, probe=probe, steps=STEPS)
    return W.sphere_d3q19(64, theta=th, precision=W.FP64, steps=STEPS).with_(probe=probe)


def main(cases, equilibrium=False):
    """cases: angles in degrees; an angle followed by "p" (e.g. "30p") runs
    with the fluid-only probe interpolation."""
    out = OUT_EQ if equilibrium else OUT
    for case in cases:
        probe = 1 if case.endswith("p") else 0
        th = float(case.rstrip("p"))
        wl = workload(th, probe, equilibrium)
        sim = oracle.OracleSim(wl, W.initial_phi(wl))
        t0 = time.time()
        rec = {"steps": STEPS, "theta": th, "probe": probe, "checkpoints": {},
               "start": "equilibrium cap" if equilibrium else "drop of radius 10 on the sphere top"}
        for k in range(1, 5):
            sim.step(STEPS // 4)
            rec["checkpoints"][str(k * STEPS // 4)] = measure_state(sim, wl)
            print(th, k * STEPS // 4, rec["checkpoints"][str(k * STEPS // 4)], f"{time.time() - t0:.0f}s",
                  flush=True)
        rec.update(rec["checkpoints"][str(STEPS)])
        data = json.load(open(out)) if os.path.exists(out) else {}   # merge with other writers
        data[str(float(th)) + ("/probe" if probe else "")] = rec
        with open(out, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    eq = "--equilibrium" in args
    args = [a for a in args if a != "--equilibrium"]
    main(args or ["30p", "60", "90", "120", "150"], equilibrium=eq)
