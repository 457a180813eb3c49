"""Continuous-batching server for many wetting simulations on one GPU.

Requests (a workload, a step count and an arrival time) are admitted while
a slot is free and their device footprint fits the HBM budget.  Every tick
advances all resident runs by up to `tick_steps` steps with one
`lbm_batch_step` call (shared launches for runs of the same lattice and
precision); runs that arrive during a tick join at the next one, runs that
finish leave and free their memory.  An admitted run is prepared (initial
field, geometry, device state on its own stream) by worker threads while the
resident batch computes, and joins the batch at the first tick after it is
ready.  Latency is completion time minus arrival time on the host's
monotonic clock.

A run that goes non-finite is retired on its own with status "unstable"
(checked when it finishes and every `check_ticks` ticks while it runs):
the other runs of the batch, each in its own device buffer, go on and
compute exactly what they compute alone.
"""
from __future__ import annotations

import dataclasses
import math
import sys
import time
from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor, wait
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import lbm
from . import workloads as W


@dataclasses.dataclass
class Request:
    rid: int
    workload: W.Workload
    steps: int
    arrival: float = 0.0          # seconds after the start of the run


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    nodes: int
    steps: int
    obs: Dict[str, object]
    state: Optional[Dict[str, np.ndarray]] = None
    status: str = "ok"            # "ok", or "unstable" (non-finite state; retired early)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def mixed_requests(count: int, seed: int = 0, step_scale: float = 1.0, size_scale: float = 1.0,
                   precision: int = W.FP32, d3q19_fraction: float = 0.4, probe: int = 0) -> List[Request]:
    """The served mix: 60 % D2Q9 boxes with side log-uniform in [64, 512] and
    40 % D3Q19 boxes with side log-uniform in [48, 192] (periodic), a disk or
    ball of radius U(0.2, 0.35) of the side at 0.35 of the box height, a drop
    of radius max(R/2, 10) on its top, contact angle U(20, 160) degrees,
    density ratio log-uniform in [1, 1000] (rho_g = 1), viscosity ratio
    max(1, ratio/10) (mu_g = 0.1), steps U(2000, 20000).  `step_scale` and
    `size_scale` shrink steps and sides for quick runs; `probe` = 1 sets the
    fluid-only probe interpolation of the ghost rule for every request."""
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(count):
        d3 = rng.uniform() < d3q19_fraction
        lo, hi = (48, 192) if d3 else (64, 512)
        L = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))) * size_scale))
        L = max(L, 24 if d3 else 32)
        R = rng.uniform(0.2, 0.35) * L
        theta = rng.uniform(20.0, 160.0)
        ratio = math.exp(rng.uniform(0.0, math.log(1000.0)))
        mu_ratio = max(1.0, ratio / 10.0)
        steps = max(1, int(round(rng.uniform(2000, 20000) * step_scale)))
        c = L / 2.0
        zc = 0.35 * L
        Rd = max(0.5 * R, min(10.0, 0.2 * L))
        if d3:
            solids = [W.Solid(0, (c, c, zc), R)]
            liquid = [W.LiquidRegion("ball", (c, c, zc + R), Rd, width=4.0)]
            shape = (L, L, L)
        else:
            solids = [W.Solid(0, (c, zc, 0.0), R)]
            liquid = [W.LiquidRegion("ball", (c, zc + R, 0.0), Rd, width=4.0)]
            shape = (L, L, 1)
        wl = W.Workload(name=f"req{k}", lattice=W.D3Q19 if d3 else W.D2Q9, shape=shape, rho_l=ratio, rho_g=1.0,
                        mu_l=0.1 * mu_ratio, mu_g=0.1, sigma=0.01, W=4.0, mobility=0.02, theta=theta,
                        solids=solids, liquid=liquid, precision=precision, steps=steps, probe=probe)
        reqs.append(Request(k, wl, steps))
    return reqs


def poisson_arrivals(reqs: Sequence[Request], rate: float, seed: int = 1) -> List[Request]:
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in reqs:
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        out.append(dataclasses.replace(r, arrival=t))
    return out


class Server:
    def __init__(self, hbm_budget: float = 64e9, max_slots: int = 256, tick_steps: int = 200,
                 device: str = "cuda:0", keep_state: bool = False, progress_s: float = 0.0,
                 prep_workers: int = 2, check_ticks: int = 10):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.budget = float(hbm_budget)
        self.max_slots = int(max_slots)
        self.tick = int(tick_steps)
        self.keep_state = keep_state
        self.progress_s = float(progress_s)   # > 0: a progress line on stderr this often
        self.prep_workers = max(1, int(prep_workers))
        self.check_ticks = int(check_ticks)   # > 0: look for non-finite runs this often (in ticks)
        self.stream = torch.cuda.current_stream(self.device)
        self.init_stream = torch.cuda.Stream(device=self.device)
        self.batch = lbm.Batch(max_jobs=max_slots, device=device, stream=self.stream)

    def _prepare(self, r: Request):
        # worker thread: host set-up and the run's initial state on the init stream
        torch = self.torch
        with torch.cuda.stream(self.init_stream):
            return lbm.Simulation(r.workload, W.initial_phi(r.workload), device=str(self.device),
                                  stream=self.init_stream)

    def run(self, requests: Sequence[Request]) -> List[Result]:
        torch = self.torch
        pending = sorted(requests, key=lambda r: r.arrival)
        waiting: List[Request] = []
        preparing = []  # [req, future, reserved bytes, admitted]
        resident = []   # [req, sim, remaining, admitted, bytes]
        used = 0.0
        results: List[Result] = []
        t0 = time.monotonic()
        i = 0
        busy = False
        ticks = 0
        last_report = 0.0
        pool = ThreadPoolExecutor(max_workers=self.prep_workers)
        try:
            while i < len(pending) or waiting or preparing or resident:
                now = time.monotonic() - t0
                if self.progress_s > 0 and now - last_report >= self.progress_s:
                    last_report = now
                    print(f"[serve] t={now:.0f}s done={len(results)} resident={len(resident)} "
                          f"preparing={len(preparing)} waiting={len(waiting)} pending={len(pending) - i}",
                          file=sys.stderr, flush=True)
                while i < len(pending) and pending[i].arrival <= now:
                    waiting.append(pending[i])
                    i += 1
                # admission by slot and HBM footprint; preparation overlaps the GPU
                while waiting and len(resident) + len(preparing) < self.max_slots:
                    r = waiting[0]
                    need = self._footprint(r.workload)
                    if used + need > self.budget and (resident or preparing):
                        break
                    waiting.pop(0)
                    used += need
                    preparing.append([r, pool.submit(self._prepare, r), need, now])
                # prepared runs join the batch
                still = []
                for rec in preparing:
                    r, fut, need, adm = rec
                    if fut.done():
                        sim = fut.result()
                        used += sim.device_bytes - need
                        resident.append([r, sim, r.steps, adm, sim.device_bytes])
                    else:
                        still.append(rec)
                preparing = still
                if busy:
                    self.stream.synchronize()
                    busy = False
                    ticks += 1
                    check = self.check_ticks > 0 and ticks % self.check_ticks == 0
                    still = []
                    for rec in resident:
                        r, sim, remaining, adm, nb = rec
                        obs = None
                        if remaining == 0 or check:
                            # a non-finite run is reported, not raised: it
                            # leaves alone and the batch goes on
                            obs = sim.observe(allow_unstable=True)
                        if remaining == 0 or (obs is not None and obs["nonfinite"] != 0):
                            status = "ok" if obs["nonfinite"] == 0 else "unstable"
                            state = None
                            if self.keep_state and status == "ok":
                                state = {"N": sim.read(lbm.FIELD_N_OFFSET), "B": sim.read(lbm.FIELD_B)}
                            results.append(Result(r.rid, r.arrival, adm, time.monotonic() - t0, r.workload.nodes,
                                                  int(obs["step"]), obs, state, status))
                            sim.close()
                            del sim
                            used -= nb
                        else:
                            still.append(rec)
                    resident = still
                    continue
                if not resident:
                    if preparing:
                        wait([rec[1] for rec in preparing], timeout=0.05, return_when=FIRST_COMPLETED)
                    elif i < len(pending):
                        time.sleep(max(0.0, min(0.05, pending[i].arrival - (time.monotonic() - t0))))
                    continue
                self.init_stream.synchronize()
                steps = [min(self.tick, rec[2]) for rec in resident]
                self.batch.step([rec[1] for rec in resident], steps)
                for rec, s in zip(resident, steps):
                    rec[2] -= s
                busy = True
        finally:
            pool.shutdown(wait=True)
        torch.cuda.synchronize(self.device)
        return sorted(results, key=lambda r: r.rid)

    def _footprint(self, wl: W.Workload) -> int:
        # device bytes of the run (populations dominate)
        Q = W.n_directions(wl.lattice)
        s = {W.FP64: 8, W.FP32: 4}.get(wl.precision, 2)
        t = 8 if wl.precision == W.FP64 else 4
        return wl.nodes * (2 * Q * s + Q * t + 2 * 4 * t + 2 * t + 1 + 32)

    def close(self):
        self.batch.close()


def summarize(results: Sequence[Result], wall: float) -> Dict[str, float]:
    """Latency percentiles and throughput over the runs that completed; the
    lattice updates of unstable runs (up to their retirement) count in the
    aggregate rate, the runs themselves are counted apart."""
    done = [r for r in results if r.status == "ok"]
    lat = np.array([r.latency for r in done]) if done else np.zeros(1)
    lups = sum(r.nodes * r.steps for r in results)
    return {"jobs": len(done), "unstable_jobs": len(results) - len(done),
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()), "throughput_jobs_s": len(done) / wall,
            "aggregate_mlups": lups / wall / 1e6, "wall_s": wall}


def serve_mix(count: int = 64, step_scale: float = 0.1, size_scale: float = 1.0, precision: int = W.FP32,
              load: float = 0.9, tick_steps: int = 200, seed: int = 0, hbm_budget: float = 64e9,
              probe: int = 0, progress_s: float = 0.0) -> Dict[str, object]:
    """Closed-loop capacity run (all requests at t = 0), then an open-loop run
    with Poisson arrivals at `load` x that capacity; returns both summaries."""
    reqs = mixed_requests(count, seed=seed, step_scale=step_scale, size_scale=size_scale, precision=precision,
                          probe=probe)
    srv = Server(hbm_budget=hbm_budget, tick_steps=tick_steps, progress_s=progress_s)
    t0 = time.monotonic()
    res = srv.run(reqs)
    closed = summarize(res, time.monotonic() - t0)
    rate = load * closed["throughput_jobs_s"]
    t0 = time.monotonic()
    res = srv.run(poisson_arrivals(reqs, rate, seed=seed + 1))
    opened = summarize(res, time.monotonic() - t0)
    srv.close()
    return {"closed_loop": closed, "open_loop": opened, "arrival_rate_jobs_s": rate, "requests": count,
            "step_scale": step_scale, "precision": W.PRECISION_NAMES[precision],
            "nonfinite_jobs": sum(1 for r in res if r.status != "ok")}


def main():
    import argparse
    import json

    ap = argparse.ArgumentParser(description="served mix: closed-loop capacity, then open-loop latency")
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--step-scale", type=float, default=1.0)
    ap.add_argument("--precision", choices=["f32", "f16ofs"], default="f32")
    ap.add_argument("--probe", type=int, default=0, help="1: fluid-only probe interpolation for every request")
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    prec = W.FP32 if args.precision == "f32" else W.FP16_OFS
    out = serve_mix(count=args.count, step_scale=args.step_scale, precision=prec, seed=args.seed, probe=args.probe,
                    progress_s=30.0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
