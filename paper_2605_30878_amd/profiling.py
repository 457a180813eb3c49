"""Summaries of rocprofv3 output for profiles/: per-kernel durations from a
--kernel-trace --stats run, and HBM bytes per dispatch from two --pmc runs
(FETCH_SIZE, WRITE_SIZE), each scaled by what the same counter reads for a
plain device copy of known size.

    python -m paper_2605_30878_amd.profiling stats <kernel_stats.csv> <out.md> "<command>"
    python -m paper_2605_30878_amd.profiling traffic <fetch.csv> <write.csv> <copy_fetch.csv> \
        <copy_write.csv> <copy_bytes> <workload_key> <out.md> "<commands>"
    python -m paper_2605_30878_amd.profiling counters <out.md> "<commands>" <pass.csv> [<pass.csv> ...]
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
KERNEL_SRC = os.path.join(HERE, "csrc", "kernels.hip")
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _itanium_short(base: str) -> str:
    """lbm::name<args> from an Itanium-mangled kernel name (the tracer leaves
    names with _Float16 / __bf16 arguments mangled): nested-name components,
    then lattice, float, double, _Float16, __bf16 and integer arguments."""
    i, comps = 3, []
    while i < len(base) and base[i].isdigit():
        j = i
        while base[j].isdigit():
            j += 1
        n = int(base[i:j])
        comps.append(base[j:j + n])
        i = j + n
    args = ""
    if i < len(base) and base[i] == "I":
        rest, k, toks = base[i + 1:], 0, []
        while k < len(rest) and rest[k] != "E":
            m = re.match(r"NS_(\d+)", rest[k:])
            if m:
                L = int(m.group(1))
                s = k + m.end()
                toks.append(rest[s:s + L])
                k = s + L + 1
            elif rest.startswith("DF16_", k):
                toks.append("_Float16")
                k += 5
            elif rest.startswith("DF16b", k):
                toks.append("__bf16")
                k += 5
            elif rest[k] in "fd":
                toks.append("float" if rest[k] == "f" else "double")
                k += 1
            elif rest.startswith("Lb1E", k) or rest.startswith("Lb0E", k):
                toks.append("true" if rest[k + 2] == "1" else "false")
                k += 4
            else:
                m = re.match(r"Li(\d+)E", rest[k:])
                if not m:
                    break
                toks.append(m.group(1))
                k += m.end()
        args = "<" + ", ".join(toks) + ">"
    return "::".join(comps) + args


def short_name(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    base = name.split("(")[0]
    if base.startswith("void "):
        base = base[5:]
    if base.startswith("_ZN"):
        return _itanium_short(base)
    return base


def stats_markdown(stats_csv: str, command: str) -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["| kernel | calls | average (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} % |")
    return "Command:\n\n```\n" + command + "\n```\n\n" + "\n".join(lines) + "\n"


def _counter_means(path: str):
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        acc[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes: float):
    """Per-kernel HBM bytes per dispatch, calibrated on the copy kernel
    (the dispatch with the largest counter value in the copy runs)."""
    cf = max(_counter_means(copy_fetch_csv).values())
    cw = max(_counter_means(copy_write_csv).values())
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    fetch = _counter_means(fetch_csv)
    write = _counter_means(write_csv)
    out = {}
    for k in fetch:
        fb = fetch[k] * 1024.0 * f_scale
        wb = write.get(k, 0.0) * 1024.0 * w_scale
        out[k] = {"fetch_bytes": fb, "write_bytes": wb, "hbm_bytes_per_launch": fb + wb}
    return out, f_scale, w_scale


COUNTER_KERNELS = ("k_colour_tile", "k_collide_stream", "k_collide_colour", "k_colour_fixup", "k_ghost")
PER_WAVE = ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR")
OF_WAVE_CYCLES = ("SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_SCA", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_ANY",
                  "SQ_WAIT_INST_ANY", "SQ_WAIT_ANY")


def counters_markdown(paths, command: str) -> str:
    """SQ / TA / TCC counters of the step kernels, averaged over dispatches
    (several single-pass runs of the same program): instructions per wave,
    activity and waits as a share of SQ_WAVE_CYCLES, and the raw means."""
    acc = defaultdict(lambda: defaultdict(list))
    for path in paths:
        for r in csv.DictReader(open(path)):
            name = short_name(r["Kernel_Name"])
            if any(k in name for k in COUNTER_KERNELS):
                acc[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = ["Commands:", "", "```", command, "```", "",
             "Instructions per wave; activity and waits as a share of SQ_WAVE_CYCLES "
             "(the sum over waves of their resident cycles).", ""]
    for name in sorted(acc):
        d = {c: sum(v) / len(v) for c, v in acc[name].items()}
        waves = d.get("SQ_WAVES", 0.0)
        lines.append(f"### `{name}`")
        lines.append("")
        lines.append("| counter | mean per dispatch | derived |")
        lines.append("|---|---|---|")
        for c in sorted(d):
            derived = ""
            if c in PER_WAVE and waves:
                derived = f"{d[c] / waves:.1f} per wave"
            elif c in OF_WAVE_CYCLES and d.get("SQ_WAVE_CYCLES"):
                derived = f"{100.0 * d[c] / d['SQ_WAVE_CYCLES']:.1f} % of wave-cycles"
            lines.append(f"| {c} | {d[c]:.4g} | {derived} |")
        lines.append("")
    return "\n".join(lines)


def main(argv):
    if argv[0] == "stats":
        md = stats_markdown(argv[1], argv[3])
        with open(argv[2], "w") as f:
            f.write(md)
        return 0
    if argv[0] == "traffic":
        fetch, write, cfetch, cwrite, cbytes, key, out_md, cmds = argv[1:9]
        per, fs, ws = traffic(fetch, write, cfetch, cwrite, float(cbytes))
        h = kernel_source_hash()
        data = {}
        if os.path.exists(TRAFFIC_JSON):
            data = json.load(open(TRAFFIC_JSON))
        data.setdefault("kernels", {})
        for k, v in per.items():
            name = k.split("<")[0].split("::")[-1]
            data["kernels"].setdefault(name, {})[key] = dict(v, kernel_source_hash=h)
        data["calibration"] = {"copy_bytes": float(cbytes), "fetch_scale": fs, "write_scale": ws}
        with open(TRAFFIC_JSON, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        lines = ["Commands:", "", "```", cmds, "```", "",
                 f"Calibration on a plain device copy of {float(cbytes) / 2**30:.0f} GiB: FETCH_SIZE x {fs:.4f}, "
                 f"WRITE_SIZE x {ws:.4f} (counters in KiB per dispatch).", "",
                 f"Kernel source hash: `{h}`", "",
                 "| kernel | fetch (MB) | write (MB) | HBM bytes per launch (MB) |", "|---|---|---|---|"]
        for k, v in sorted(per.items(), key=lambda kv: -kv[1]["hbm_bytes_per_launch"]):
            lines.append(f"| `{k}` | {v['fetch_bytes'] / 1e6:.1f} | {v['write_bytes'] / 1e6:.1f} | "
                         f"{v['hbm_bytes_per_launch'] / 1e6:.1f} |")
        with open(out_md, "w") as f:
            f.write("\n".join(lines) + "\n")
        return 0
    if argv[0] == "counters":
        md = counters_markdown(argv[3:], argv[2])
        with open(argv[1], "w") as f:
            f.write(md)
        return 0
    raise SystemExit(__doc__)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
