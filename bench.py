#!/usr/bin/env python3
"""Benchmark of the colour-gradient LBM update with curved-boundary wetting.

One "step" is one full lattice update of the D3Q19 drop-on-sphere box
(256^3, sphere radius 48 at the centre, drop radius 40 on its top, density
ratio 1000, viscosity ratio 100, FP32) with the state resident in HBM:
colour field, ghost-node update, fused collide-stream.  Prints one JSON line:
MLUPS (Eq. 14: box nodes x steps / (seconds x 1e6)), the roofline of the
dominant kernel (fused collide-stream) from HIP events on the library's
stream with its HBM traffic from the committed rocprofv3 counters, a short
served mix (p50 / p99 latency, FP32 and FP16 storage), and the FP64 CPU
oracle timed on the host on a few steps of the same box.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--size 256]
           [--precision f32|f64|f16ofs|bf16ofs] [--workload sphere|porous]
           [--layout box|sparse] [--no-serve] [--no-cpu-baseline]
       python bench.py --cpu-windows     (oracle timings only, no GPU)
       python bench.py --calibrate-copy  (plain 1 GiB copy, for counters)

--workload porous runs the 384^3 sphere packing (theta 45, density ratio
10, body force 1e-6) in the fluid-only storage layout by default.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2605_30878_amd", "csrc", "kernels.hip")


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary, or None when the kernel source changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    rec = t.get("kernels", {}).get(kernel, {}).get(workload)
    if not rec or rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(wl, steps: int):
    """The FP64 oracle, as it stands, on `steps` steps of the same box."""
    import numpy as np

    import oracle
    from paper_2605_30878_amd import workloads as W

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    wl64 = wl.with_(precision=W.FP64)
    phi0 = W.initial_phi(wl64)
    sim = oracle.OracleSim(wl64, phi0)
    sim.step(1)  # first touch of the arrays, not timed
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    del sim
    return {"value": wl.nodes * steps / (dt * 1e6), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{steps} steps of the full {wl.shape[0]}x{wl.shape[1]}x{wl.shape[2]} "
                      f"{W.lattice_name(wl.lattice)} box "
                      f"(FP64 oracle, OpenMP over nodes), after 1 untimed step"}


CPU_WINDOWS = {
    # name: (workload factory, steps); the oracle in FP64, as in cpu_baseline.
    # The 384^3 packing is left out: the oracle tests every node against
    # every one of its 4,694 spheres when it builds the geometry.
    "d2q9_cylinder_128": (lambda W: W.cylinder_d2q9_128(), 2000),
    "d3q19_sphere_64": (lambda W: W.sphere_d3q19(64, precision=W.FP64), 200),
    "d3q19_sphere_256": (lambda W: W.sphere_d3q19(256, precision=W.FP64), 3),
    "d3q19_sphere_256_1": (lambda W: W.sphere_d3q19(256, precision=W.FP64), 1),
}


def cpu_model() -> str:
    """The host CPU's model name (Linux), or the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def single_thread_window(name: str) -> dict:
    """One oracle window in a child process with one OpenMP thread."""
    import subprocess

    env = dict(os.environ, OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-window", name],
                         env=env, capture_output=True, text=True, check=True)
    return json.loads(res.stdout.strip().splitlines()[-1])


def cpu_window(name: str) -> dict:
    """One oracle timing window (this process's OpenMP threads)."""
    from paper_2605_30878_amd import workloads as W

    make, steps = CPU_WINDOWS[name]
    wl = make(W)
    r = cpu_baseline(wl, steps)
    r.update({"window": name, "steps": steps, "nodes": wl.nodes})
    return r


def cpu_windows(threads) -> list:
    """Every window at each thread count, each in a child process started
    with OMP_NUM_THREADS set (the OpenMP pool is sized at start-up).  No GPU
    is used."""
    import subprocess

    out = []
    for name in CPU_WINDOWS:
        if name.endswith("_1"):   # the single-thread sample of cpu_baseline
            continue
        for t in threads:
            env = dict(os.environ, OMP_NUM_THREADS=str(t))
            res = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-window", name],
                                 env=env, capture_output=True, text=True, check=True)
            rec = json.loads(res.stdout.strip().splitlines()[-1])
            print(f"[cpu] {rec}", file=sys.stderr, flush=True)
            out.append(rec)
    return out


def hbm_ceiling(gib: int = 4, repeats: int = 10) -> dict:
    """What plain streaming kernels reach on this device (lbm_hbm_probe over
    `gib` GiB): read-only, copy, and the colour kernel's pattern of 19 FP32
    plane reads and one plane write; GB/s of bytes moved, each the average
    launch after two untimed ones."""
    import torch

    from paper_2605_30878_amd import lbm

    nbytes = gib << 30
    src = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0")
    m = nbytes // 76                           # plane length of the 19-plane pattern
    out = {"bytes": nbytes}
    for name, kind, s, d, moved in (("read", lbm.PROBE_READ, src, dst, nbytes),
                                    ("copy", lbm.PROBE_COPY, src, dst, 2 * nbytes),
                                    ("planes19", lbm.PROBE_PLANES, src[: 19 * m], dst[:m], 80 * m)):
        lbm.hbm_probe(kind, s, d, 2)
        ms = lbm.hbm_probe(kind, s, d, repeats)
        out[name + "_gbs"] = round(moved / (ms * 1e-3) / 1e9, 1)
    del src, dst
    torch.cuda.empty_cache()
    return out


def inbox_values(shape, zc_blocks: int = 6144) -> int:
    """Values the collide-colour step writes to its inbox per launch: for
    each 64 x 8 x zc tile-chunk, the (node, direction) pairs whose source
    lies outside it, counted over the box geometry (solids included).  The
    chunk length follows the library's choice (about zc_blocks workgroups
    per launch, at least 4 planes)."""
    nx, ny, nz = shape
    KTX, KTY = 64, 8
    xt, yt = nx // KTX, ny // KTY
    zc = max(4, -(-(nz * xt * yt) // zc_blocks))
    zc = min(zc, nz)
    C = [(1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0), (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0), (0, 0, 1),
         (1, 0, 1), (0, 1, 1), (-1, 0, 1), (0, -1, 1), (0, 0, -1), (1, 0, -1), (0, 1, -1), (-1, 0, -1), (0, -1, -1)]
    total = 0
    for z0 in range(0, nz, zc):
        zl = min(zc, nz - z0)
        v = KTX * KTY * zl
        total += xt * yt * sum(v - (KTX - abs(a)) * (KTY - abs(b)) * max(zl - abs(c), 0) for a, b, c in C)
    return total


def hot_path(args, precision: str, form: str, layout: str) -> dict:
    """Time K steps of one configuration after W untimed ones; returns the
    JSON line of that run."""
    import torch

    from paper_2605_30878_amd import lbm
    from paper_2605_30878_amd import workloads as W

    prec = {"f32": W.FP32, "f64": W.FP64, "f16ofs": W.FP16_OFS, "bf16ofs": W.BF16_OFS}[precision]
    if args.workload == "porous":
        wl = W.porous_d3q19(n=384 if args.size == 256 else args.size, precision=prec)
    else:
        wl = W.sphere_d3q19(args.size, theta=args.theta, precision=prec)
    fused = form == "collide-colour" and layout == "box" and wl.shape[0] % 64 == 0 and wl.shape[1] % 8 == 0
    options = (lbm.OPT_FUSED if fused else 0) | (lbm.OPT_SPARSE if layout == "sparse" else 0)
    print(f"[bench] {wl.name} {precision} form={'collide-colour' if fused else 'two-pass'} layout={layout} "
          f"steps={args.steps} warmup={args.warmup}", file=sys.stderr, flush=True)
    sim = lbm.Simulation(wl, W.initial_phi(wl), device="cuda:0", options=options)
    obs0 = sim.observe()
    sim.step(args.warmup)
    torch.cuda.synchronize()

    # Timed region: exactly K steps; per-launch HIP events on the library's stream.
    t0 = time.perf_counter()
    ms = sim.step_profiled(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    obs1 = sim.observe()
    n_fluid = obs1["n_fluid"]
    s_n = {W.FP64: 8, W.FP32: 4}.get(prec, 2)   # bytes of one stored population
    s_t = 8 if prec == W.FP64 else 4            # bytes of phi, G, p
    Q, D = 19, 3
    mlups = wl.nodes * args.steps / (dt * 1e6)
    if fused:
        # collide-colour launch: N read and N* written (2 Q s_n), phi read
        # once and the next step's phi written (2 s_t) per fluid node, one
        # flag byte per box node, and the values handed across tile-chunk
        # faces written to the inbox
        inbox = inbox_values(wl.shape)
        alg_bytes = n_fluid * (2 * Q * s_n + 2 * s_t) + wl.nodes + inbox * s_t
        # + the fix-up: inbox read, and phi read and written at the nodes it touches
        impl_bytes = 2 * Q * s_n + 2 * s_t + (2 * inbox * s_t) / wl.nodes + 1
        kernel = "k_collide_colour"
    elif layout == "sparse":
        # the same per fluid node, with no flag bytes (the bounce-back links
        # come with the neighbour slots); the neighbour-slot table ((Q - 1) x
        # 4 bytes per fluid node, read by both launches) is layout overhead,
        # counted in impl_bytes only
        alg_bytes = n_fluid * (2 * Q * s_n + s_t + (D + 1) * s_t)
        impl_bytes = ((Q * s_n + 2 * s_t + (D + 1) * s_t) + (2 * Q * s_n + s_t + (D + 1) * s_t)
                      + 2 * (Q - 1) * 4)
        kernel = "k_collide_sparse"
    else:
        # collide-stream launch: N read and N* written (2 Q s_n), phi read
        # once, the record (G, p) written ((D + 1) s_t); one flag byte per node
        alg_bytes = n_fluid * (2 * Q * s_n + s_t + (D + 1) * s_t) + wl.nodes
        # colour launch (N, phi_prev, record in; phi out) + collide launch
        impl_bytes = (Q * s_n + 2 * s_t + (D + 1) * s_t) + (2 * Q * s_n + s_t + (D + 1) * s_t)
        kernel = "k_collide_stream"
    k_ms = ms["collide"] / args.steps
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    workload_key = f"d3q19_{args.workload}_{wl.shape[0]}_{precision}" + ("_sparse" if layout == "sparse" else "")
    traffic = measured_traffic(kernel, workload_key)
    # paper-state bytes per lattice update: N and B read once and written once
    step_bytes = 4 * Q * s_n
    result = {
        "metric": "D3Q19 two-phase MLUPS & % HBM roofline; p50/p99 job latency on served mix",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": precision,
        "data": ("synthetic (analytic sphere and tanh drop, deterministic)" if args.workload == "sphere" else
                 "synthetic (seeded random sphere packing, tanh liquid slab, deterministic)"),
        "config": ({"workload": f"D3Q19 drop on sphere {args.size}^3", "lattice": "D3Q19",
                    "box": [args.size] * 3, "sphere_radius": 48 * args.size / 256,
                    "drop_radius": 40 * args.size / 256, "rho_ratio": 1000, "mu_ratio": 100,
                    "theta_deg": args.theta, "W": 4.0, "sigma": 0.01, "storage": precision,
                    "n_fluid": n_fluid, "n_ghost": obs1["n_ghost"], "layout": layout,
                    "form": "collide-colour" if fused else "two-pass"} if args.workload == "sphere" else
                   {"workload": f"D3Q19 porous packing {wl.shape[0]}^3", "lattice": "D3Q19",
                    "box": list(wl.shape), "spheres": len(wl.solids), "sphere_radius": 12, "rho_ratio": 10,
                    "mu_ratio": 10, "theta_deg": 45, "body_accel": 1e-6, "storage": precision,
                    "n_fluid": n_fluid, "n_ghost": obs1["n_ghost"],
                    "porosity_nodes": round(n_fluid / wl.nodes, 4),
                    "ghost_probe": "fluid corners" if wl.probe else "all corners",
                    "dead_end_fill": bool(wl.fill), "layout": layout,
                    "mflups": round(n_fluid * args.steps / (dt * 1e6), 2)}),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": kernel, "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": round(k_ms, 5)} | ({"note": (
                         "the collide-colour kernel also forms the next colour field, so a step moves "
                         f"{impl_bytes:.0f} B per update against the two-pass form's "
                         f"{(Q * s_n + 2 * s_t + (D + 1) * s_t) + (2 * Q * s_n + s_t + (D + 1) * s_t)} B; its time is "
                         "set by instruction issue and a per-plane barrier at two workgroups per CU, not by HBM")}
                         if fused else {}),
        "step_roofline": {"bytes_per_update": step_bytes, "impl_bytes_per_update": round(impl_bytes, 2),
                          "roofline_mlups": round(HBM_PEAK_GBS * 1e9 / step_bytes / 1e6, 1),
                          "frac": round(mlups / (HBM_PEAK_GBS * 1e9 / step_bytes / 1e6), 4),
                          "target_frac": 0.70},
        "phase_ms_per_step": {k: round(v / args.steps, 5) for k, v in ms.items()},
        "mass_drift": abs(obs1["mass_blue"] / obs0["mass_blue"] - 1),
        "max_speed": obs1["max_speed"],
    }
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"line": result}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--workload", choices=["sphere", "porous"], default="sphere",
                    help="sphere: drop on a sphere (default); porous: 384^3 random sphere packing, "
                         "porosity 0.40, theta 45, body force 1e-6")
    ap.add_argument("--theta", type=float, default=90.0)
    ap.add_argument("--precision", choices=["f32", "f64", "f16ofs", "bf16ofs"], default="f32")
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", choices=["full", "reduced", "none"], default="full",
                    help="served mix: full = FP16 storage at the stated size (256 requests, full steps) plus a "
                         "reduced FP32 mix (64 requests, steps x 0.1); reduced = both reduced; none = skip")
    ap.add_argument("--no-serve", dest="serve", action="store_const", const="none",
                    help="same as --serve none")
    ap.add_argument("--form", choices=["collide-colour", "two-pass"], default=None,
                    help="step form: collide-colour (LBM_OPT_FUSED, default for the sphere box: the collide "
                         "kernel forms the next colour field) or two-pass (colour kernel + collide kernel)")
    ap.add_argument("--no-extra", action="store_true",
                    help="time only the requested configuration (no FP16 / two-pass lines, no HBM probe)")
    ap.add_argument("--layout", choices=["box", "sparse"], default=None,
                    help="device storage: box planes, or fluid-only slots with a neighbour table "
                         "(default: sparse for the porous packing, box otherwise)")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="only run the HBM reference kernels (read, copy, 19-plane pattern) over 4 GiB")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (for HBM counter calibration)")
    ap.add_argument("--cpu-windows", action="store_true",
                    help="only time the FP64 oracle on the host over fixed windows of several workloads, "
                         "with all cores and with one thread (no GPU use)")
    ap.add_argument("--cpu-window", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.cpu_window:
        print(json.dumps(cpu_window(args.cpu_window)), flush=True)
        return 0
    if args.cpu_windows:
        cores = os.cpu_count() or 1
        print(json.dumps({"cpu_windows": cpu_windows([int(os.environ.get("OMP_NUM_THREADS", "0")) or cores, 1])}),
              flush=True)
        return 0

    if args.gpus != 1:
        print(json.dumps({"error": "the library runs one lattice on one GPU; --gpus must be 1 (multi-GPU sharding is not built)",
                          "requested_gpus": args.gpus}), flush=True)
        return 2

    import torch

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": src.numel() * 4, "launches": 5}), flush=True)
        return 0

    if args.hbm_probe:
        print(json.dumps({"hbm_ceiling": hbm_ceiling()}), flush=True)
        return 0

    from paper_2605_30878_amd import lbm
    from paper_2605_30878_amd import workloads as W

    form = args.form or ("two-pass" if args.workload == "porous" else "collide-colour")
    layout = args.layout or ("sparse" if args.workload == "porous" else "box")
    main_run = hot_path(args, args.precision, form, layout)
    result = main_run.pop("line")
    if args.workload == "sphere" and args.precision == "f32" and not args.no_extra:
        # the same box in 16-bit offset storage, in both step forms (the
        # faster is reported: with half the population bytes the
        # collide-colour kernel's arithmetic outweighs the pass it saves),
        # and the two-pass form in FP32, each timed like the headline run
        forms16 = [form] + (["two-pass"] if form != "two-pass" else [])
        r16s = [hot_path(args, "f16ofs", f, layout)["line"] for f in forms16]
        r16 = min(r16s, key=lambda r: r["ms_per_step"])
        result["f16ofs"] = {"value": r16["value"], "unit": "MLUPS", "ms_per_step": r16["ms_per_step"],
                            "form": r16["config"]["form"],
                            "ms_per_step_by_form": {r["config"]["form"]: r["ms_per_step"] for r in r16s},
                            "speedup_over_f32": round(r16["value"] / result["value"], 3),
                            "roofline": r16["roofline"], "step_roofline": r16["step_roofline"],
                            "phase_ms_per_step": r16["phase_ms_per_step"], "mass_drift": r16["mass_drift"]}
        r2 = hot_path(args, "f32", "two-pass", layout)["line"]
        result["two_pass_f32"] = {"value": r2["value"], "ms_per_step": r2["ms_per_step"],
                                  "roofline": r2["roofline"], "phase_ms_per_step": r2["phase_ms_per_step"]}
    if not args.no_extra:
        ceil = hbm_ceiling()
        result["hbm_ceiling"] = ceil
        # the dominant kernel reads and writes the populations: a copy-like
        # pattern, so the copy kernel's rate is its attainable reference
        result["roofline"]["frac_of_copy_ceiling"] = round(result["roofline"]["achieved"] / ceil["copy_gbs"], 4)
    if args.serve != "none":
        from paper_2605_30878_amd import serve

        def mix_line(mix, count, scale):
            return {"requests": count, "steps": "U(2000, 20000)" + ("" if scale == 1.0 else " x %g" % scale),
                    "p50_s": round(mix["open_loop"]["p50_latency_s"], 4),
                    "p99_s": round(mix["open_loop"]["p99_latency_s"], 4),
                    "throughput_jobs_s": round(mix["open_loop"]["throughput_jobs_s"], 3),
                    "aggregate_mlups": round(mix["open_loop"]["aggregate_mlups"], 1),
                    "arrival_rate_jobs_s": round(mix["arrival_rate_jobs_s"], 3),
                    "closed_loop_jobs_s": round(mix["closed_loop"]["throughput_jobs_s"], 3),
                    "closed_loop_mlups": round(mix["closed_loop"]["aggregate_mlups"], 1),
                    "nonfinite_jobs": mix["nonfinite_jobs"]}

        full = args.serve == "full"
        # FP16 storage at the served mix's stated size (256 requests, full
        # step counts; Poisson arrivals at 0.9 x the closed-loop capacity);
        # FP32 as a reduced mix (64 requests, steps x 0.1) to bound the run
        count16, scale16 = (256, 1.0) if full else (64, 0.1)
        mix16 = serve.serve_mix(count=count16, step_scale=scale16, precision=W.FP16_OFS, progress_s=30.0)
        mix32 = serve.serve_mix(count=64, step_scale=0.1, precision=W.FP32, progress_s=30.0)
        result["served_mix"] = {"requests": count16, "steps": "U(2000, 20000)" + ("" if scale16 == 1.0 else
                                                                                  " x %g" % scale16),
                                "f16ofs": mix_line(mix16, count16, scale16),
                                "f32_reduced": mix_line(mix32, 64, 0.1)}
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        if args.workload == "porous":
            # the oracle tests every node against every sphere to build the
            # 384^3 packing; its bounded sample is a 96^3 packing of the same
            # spheres, porosity and physics
            sample = W.porous_d3q19(96, precision=W.FP64)
            cb = cpu_baseline(sample, args.cpu_steps)
            cb["sample"] = (f"{args.cpu_steps} steps of a 96^3 packing (radius-12 spheres, porosity 0.40, "
                            f"{len(sample.solids)} spheres; FP64 oracle, OpenMP over nodes), after 1 untimed step")
            result["cpu_baseline"] = cb
        else:
            cb = cpu_baseline(W.sphere_d3q19(args.size, theta=args.theta, precision=W.FP64), args.cpu_steps)
            cb["cpu_model"] = cpu_model()
            if args.size == 256:
                # the same box on one core: one step in a child process
                st = single_thread_window("d3q19_sphere_256_1")
                cb["single_thread"] = {"value": st["value"], "unit": "MLUPS", "cores": 1,
                                       "sample": "1 step of the same box (FP64 oracle, one OpenMP thread), "
                                                 "after 1 untimed step"}
            result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
