"""Timing of the paper's own benchmark boxes (D2Q9, Table 1 sizes) with this
library, for comparison with the MLUPS the paper reports for its JAX code
on an A100 (a different machine: context, not a target).

Drop on a plate (Section 3.1) at 500 x 300, 1000 x 600, 1500 x 900 (drop
area scaled with the box) and drop on a cylinder (Section 3.2) at 201^2,
401^2, 601^2 (R = L/5), both at density ratio 1000, viscosity ratio 100,
W = 4, theta = 60, equilibrium-shaped drops.  MLUPS = box nodes x steps /
(seconds x 1e6) over `steps` steps after 200 untimed ones.

    python -m paper_2605_30878_amd.context [--steps 5000]
"""
from __future__ import annotations

import argparse
import json
import time

from . import lbm
from . import sweeps
from . import workloads as W

PAPER_A100 = {  # Table 1: (FP32, FP64) MLUPS
    ("plate", 500): (759, 285), ("plate", 1000): (877, 257), ("plate", 1500): (768, 263),
    ("cylinder", 201): (374, 216), ("cylinder", 401): (740, 310), ("cylinder", 601): (844, 283),
}


def case(kind: str, size: int, precision: int) -> W.Workload:
    if kind == "plate":
        s = size / 500.0
        return sweeps.plate_case(60.0, 0, nx=size, ny=int(round(300 * s)), area=1e4 * s * s, precision=precision)
    R = size / 5.0
    return sweeps.cylinder_case(60.0, 0, R=R, area=3000.0 * (R / 40.0) ** 2, precision=precision).with_(
        shape=(size, size, 1))


def main():
    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=5000)
    args = ap.parse_args()
    lbm.load_library()
    rows = []
    for (kind, size), (p32, p64) in PAPER_A100.items():
        for prec, paper in ((W.FP32, p32), (W.FP64, p64)):
            wl = case(kind, size, prec)
            sim = lbm.Simulation(wl, W.initial_phi(wl))
            sim.step(200)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(args.steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            o = sim.observe()
            sim.close()
            mlups = wl.nodes * args.steps / dt / 1e6
            rows.append({"benchmark": kind, "grid": list(wl.shape[:2]), "precision": W.PRECISION_NAMES[prec],
                         "mlups": round(mlups, 1), "paper_a100_mlups": paper, "nonfinite": o["nonfinite"]})
            print(json.dumps(rows[-1]), flush=True)


if __name__ == "__main__":
    main()
