"""HBM traffic and kernel-time summaries of the N = 27 sweep, from rocprofv3 output.

Subcommands:

  run        the profiled workload: a plain device copy of a known size (the calibration
             kernel for the counters), then one fourth-order step of the N = 27 xyz chain
             on one complex128 vector with the library's default configuration.
             Used as  rocprofv3 --pmc FETCH_SIZE ... -- python3 -m paper_1305_0036_amd.profile_traffic run
             and again with WRITE_SIZE.
  traffic    reads the two counter CSVs, scales each sweep dispatch's FETCH_SIZE and
             WRITE_SIZE by what the same counter reads for the copy (bytes known), and
             writes a markdown summary with a JSON block that bench.py reads.
  stats      turns a rocprofv3 --kernel-trace --stats kernel_stats.csv into a short
             markdown table.
  counters   averages other rocprofv3 --pmc counters of the sweep dispatches by sweep kind
             (ping-pong sweeps: bit group, with or without a phase step; light-cone sweeps:
             each sweep of the step).
  run-dipolar   profiled workload: two fourth-order steps of the 5 x 6 dipolar lattice in
             complex64 at the library's default width (one warm-up, one traced).
  run-adjoint   profiled workload: the N = 20 gradient chain, a 40-step adjoint (warm-up),
             then the 300-step adjoint and a 300-step forward run.
  phase-split   from a kernel trace of run-dipolar: the traced step's sweeps with and
             without a phase step, their average durations and GB/s.

The summaries carry a hash of the kernel and planner sources; bench.py reports the
traffic only while the sources still hash the same.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = ["paper_1305_0036_amd/csrc/kernels.hip", "paper_1305_0036_amd/csrc/kernels.hpp",
           "paper_1305_0036_amd/csrc/tsspin.cpp", "paper_1305_0036_amd/csrc/plan.cpp",
           "paper_1305_0036_amd/csrc/plan.hpp"]
COPY_ELEMS = 1 << 27          # complex128 elements of the calibration copy (2 GiB each way)


def is_c128_sweep(name: str) -> bool:
    """A complex128 sweep dispatch: the light-cone kernel, the register-window kernels on
    doubles, or the half-LDS kernel (complex128 only) of the ping-pong sweeps on the top bit
    group."""
    return ("cone_c128_kernel" in name or "sweep_half_kernel" in name or
            (("sweep_reg_kernel" in name or "sweep_pipe_kernel" in name) and "double" in name))


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def cmd_run(args):
    sys.path.insert(0, ROOT)
    import torch

    from paper_1305_0036_amd import tsspin
    from paper_1305_0036_amd import workloads as W

    n = 27
    src = torch.ones(COPY_ELEMS, dtype=torch.complex128, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print("[profile] copy done", flush=True)
    del src, dst
    torch.cuda.empty_cache()
    w = W.xyz_chain(n=n, nsteps=1, state=False)
    g = torch.Generator(device="cpu").manual_seed(1)
    x = torch.polar(torch.full((1 << n,), 2.0 ** (-n / 2), dtype=torch.float64),
                    torch.rand(1 << n, dtype=torch.float64, generator=g) * 6.283).cuda()
    H = tsspin.Hamiltonian(n, w.bonds, w.fields)
    H.evolve(x, w.dt, 1, 4)
    torch.cuda.synchronize()
    cfg = H.kernel_config(tsspin.TS_C128, 4)
    print(f"[profile] step done {cfg}", flush=True)


def _dispatches(path):
    """Dispatch_Id -> (kernel name, counter value summed over the dimensions rocprofv3 lists)."""
    out = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            k = int(r["Dispatch_Id"])
            name, v = out.get(k, (r["Kernel_Name"], 0.0))
            out[k] = (name, v + float(r["Counter_Value"]))
    return out


def cmd_traffic(args):
    res = {}
    for counter, path in (("FETCH_SIZE", args.fetch), ("WRITE_SIZE", args.write)):
        d = _dispatches(path)
        copies = [v for name, v in d.values() if "copy" in name.lower() or "elementwise" in name.lower()]
        sweeps = [v for name, v in d.values() if is_c128_sweep(name)]
        if not copies or not sweeps:
            raise SystemExit(f"{path}: no copy or no complex128 sweep dispatch found")
        copy_kib = max(copies)          # the 2 GiB copy is the largest copy-like dispatch
        scale = (COPY_ELEMS * 16) / (copy_kib * 1024.0)
        res[counter] = dict(copy_kib=copy_kib, scale=scale, sweeps=len(sweeps),
                            sweep_kib_avg=sum(sweeps) / len(sweeps),
                            sweep_bytes_avg=scale * 1024.0 * sum(sweeps) / len(sweeps))
    alg = 2 * (1 << 27) * 16
    traffic = res["FETCH_SIZE"]["sweep_bytes_avg"] + res["WRITE_SIZE"]["sweep_bytes_avg"]
    summary = {"kernel": "complex128 sweep kernels (N=27, library defaults)",
               "source_hash": source_hash(), "traffic_bytes_per_launch": traffic,
               "algorithmic_bytes_per_launch": alg, "ratio": traffic / alg, "counters": res}
    lines = ["# HBM traffic of the complex128 sweep kernel, N = 27 xyz chain", "",
             "Commands (from the repository root, on the GPU; OUT is any output directory):", "",
             "```",
             "rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/pmc_fetch -o fetch -- "
             "python3 -m paper_1305_0036_amd.profile_traffic run",
             "rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/pmc_write -o write -- "
             "python3 -m paper_1305_0036_amd.profile_traffic run",
             "python3 -m paper_1305_0036_amd.profile_traffic traffic "
             "--fetch OUT/pmc_fetch/fetch_counter_collection.csv "
             f"--write OUT/pmc_write/write_counter_collection.csv --out {args.out}",
             "```", "",
             "Scaling: each counter is scaled by bytes / counter of a plain 2 GiB device copy "
             "(torch copy_ of 2^27 complex128 elements: 2 GiB read, 2 GiB written) measured in "
             "the same run.", "",
             "| counter | copy reads (KiB) | scale | sweep dispatches | sweep avg (KiB) | sweep avg scaled (GB) |",
             "|---|---|---|---|---|---|"]
    for c, r in res.items():
        lines.append(f"| {c} | {r['copy_kib']:.0f} | {r['scale']:.4f} | {r['sweeps']} | "
                     f"{r['sweep_kib_avg']:.0f} | {r['sweep_bytes_avg'] / 1e9:.3f} |")
    lines += ["", f"Traffic per launch: {traffic / 1e9:.3f} GB against {alg / 1e9:.3f} GB algorithmic "
              f"(one read and one write of the 2 GiB state): ratio {traffic / alg:.3f}.", "",
              "```json", json.dumps(summary, indent=1), "```", ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    print(json.dumps(summary))


def cmd_stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# {args.title}", "",
             "Commands (from the repository root, on the GPU; OUT is any output directory):", "",
             "```", args.command, "```", "",
             "| kernel | calls | total (ms) | average (us) | min (us) | max (us) | % |",
             "|---|---|---|---|---|---|---|"]
    for r in rows[: args.top]:
        name = r["Name"] if len(r["Name"]) < 90 else r["Name"][:87] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    sw = [r for r in rows if is_c128_sweep(r["Name"])]
    if sw:
        calls = sum(int(r["Calls"]) for r in sw)
        tot = sum(float(r["TotalDurationNs"]) for r in sw)
        lines += ["", f"complex128 sweep kernels together: {calls} calls, average "
                  f"{tot / calls / 1e3:.1f} us ({2 * (1 << 27) * 16 / (tot / calls) :.0f} GB/s at N = 27)."]
    lines += ["", f"Source hash of the kernels and planner: `{source_hash()}`.", ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))


def cmd_counters(args):
    """Average each counter over the complex128 sweep dispatches of one N = 27 step, grouped by
    the kind of sweep the plan says it is (bit group, with or without a phase step; each
    light-cone sweep on its own)."""
    sys.path.insert(0, ROOT)
    from paper_1305_0036_amd import tsspin
    from paper_1305_0036_amd import workloads as W

    w = W.xyz_chain(n=27, nsteps=1, state=False)
    H = tsspin.Hamiltonian(27, w.bonds, w.fields)
    nsw, cone = H.launches(tsspin.TS_C128, w.dt, 1, 4)
    if cone:
        labels = [f"light-cone sweep {i}" for i in range(nsw)]
    else:
        plan = H.plan(tsspin.TS_C128, w.dt, 1, 4)
        labels = [f"group {s['group']} {'phase' if s['axis'] >= 0 else 'layer'}" for s in plan]
    table = {}
    for path in args.csv:
        d = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if not is_c128_sweep(r["Kernel_Name"]):
                    continue
                k = int(r["Dispatch_Id"])
                d.setdefault(k, {})
                d[k][r["Counter_Name"]] = d[k].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        disp = [d[k] for k in sorted(d)]
        if len(disp) != len(labels):
            raise SystemExit(f"{path}: {len(disp)} sweep dispatches, plan has {len(labels)}")
        for lab, c in zip(labels, disp):
            for name, v in c.items():
                table.setdefault(lab, {}).setdefault(name, []).append(v)
    names = sorted({n for t in table.values() for n in t})
    lines = [f"# {args.title}", "",
             "Commands (from the repository root, on the GPU; OUT is any output directory):", "",
             "```", args.command, "```", "",
             "Average per dispatch, by sweep kind (" + ", ".join(
                 f"{lab}: {len(next(iter(t.values())))}" for lab, t in table.items()) + " dispatches).", "",
             "| counter | " + " | ".join(table) + " |", "|---|" + "---|" * len(table)]
    for n in names:
        lines.append(f"| {n} | " + " | ".join(
            f"{sum(t[n]) / len(t[n]):.4g}" if n in t else "" for t in table.values()) + " |")
    lines += ["", f"Source hash of the kernels and planner: `{source_hash()}`.", ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))


def cmd_run_dipolar(args):
    sys.path.insert(0, ROOT)
    import torch

    from paper_1305_0036_amd import tsspin
    from paper_1305_0036_amd import workloads as W

    w = W.dipolar_lattice(nsteps=1)
    H = tsspin.Hamiltonian(w.n, w.bonds, w.fields)
    x = torch.zeros(1 << w.n, dtype=torch.complex64, device="cuda")
    x[w.extra["init_index"]] = 1.0
    for _ in range(2):
        H.evolve(x, w.dt, 1, 4)
        torch.cuda.synchronize()
    plan = H.plan(tsspin.TS_C64, w.dt, 1, 4)
    print(json.dumps({"sweeps": len(plan), "phase": [int(0 <= p["axis"] < 3) for p in plan],
                      "group": [p["group"] for p in plan], "tile_bits": plan[0]["tile_bits"]}), flush=True)


def cmd_run_adjoint(args):
    sys.path.insert(0, ROOT)
    import time

    import torch

    from paper_1305_0036_amd import tsspin
    from paper_1305_0036_amd import workloads as W

    w = W.gradient_chain()
    H = tsspin.Hamiltonian(w.n, w.bonds, w.fields)
    x = torch.from_numpy(w.psi0).cuda()
    H.adjoint(x, w.dt, 40, 4, ("sz", 0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H.adjoint(x, w.dt, w.nsteps, 4, ("sz", 0))
    t1 = time.perf_counter()
    y = x.clone()
    H.evolve(y, w.dt, w.nsteps, 4)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"[profile] adjoint {1e3 * (t1 - t0):.1f} ms, forward {1e3 * (t2 - t1):.1f} ms", flush=True)


def cmd_phase_split(args):
    rows = sorted(csv.DictReader(open(args.csv)), key=lambda r: int(r["Start_Timestamp"]))
    sw = [r for r in rows if "sweep" in r["Kernel_Name"]]
    info = json.loads(open(args.plan).read().strip().splitlines()[-1])
    n = info["sweeps"]
    timed = sw[-n:]
    groups = {1: [], 0: []}
    for ph, r in zip(info["phase"], timed):
        groups[ph].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    moved = 2 * (1 << 30) * 8
    lines = [f"# {args.title}", "",
             "Commands (from the repository root, on the GPU; OUT is any output directory):", "",
             "```", args.command, "```", "",
             f"Kernel: `{timed[0]['Kernel_Name'][:100]}`, {n} sweeps in the traced step.", "",
             "| sweeps | count | average (us) | GB/s (16 GiB moved per sweep) |", "|---|---|---|---|"]
    for ph, label in ((1, "with a phase step"), (0, "layer only")):
        d = groups[ph]
        if d:
            avg = sum(d) / len(d)
            lines.append(f"| {label} | {len(d)} | {avg:.0f} | {moved / (avg * 1e-6) / 1e9:.0f} |")
    if "group" in info:
        lines += ["", "By bit group of the tile (group 0 holds the low index bits; the last, the top ones):",
                  "", "| group | phase step | count | average (us) | GB/s |", "|---|---|---|---|---|"]
        by = {}
        for g, ph, r in zip(info["group"], info["phase"], timed):
            by.setdefault((g, ph), []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        for (g, ph), d in sorted(by.items()):
            avg = sum(d) / len(d)
            lines.append(f"| {g} | {'yes' if ph else 'no'} | {len(d)} | {avg:.0f} | {moved / (avg * 1e-6) / 1e9:.0f} |")
    tot = sum(groups[0]) + sum(groups[1])
    lines += ["", f"Step: {tot / 1e3:.1f} ms of kernel time.", "",
              f"Source hash of the kernels and planner: `{source_hash()}`.", ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("run")
    sub.add_parser("run-dipolar")
    sub.add_parser("run-adjoint")
    ps = sub.add_parser("phase-split")
    ps.add_argument("--csv", required=True)
    ps.add_argument("--plan", required=True, help="the stdout of run-dipolar")
    ps.add_argument("--out", required=True)
    ps.add_argument("--title", required=True)
    ps.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--out", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--csv", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--top", type=int, default=8)
    c = sub.add_parser("counters")
    c.add_argument("--csv", required=True, nargs="+")
    c.add_argument("--out", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--command", required=True)
    args = ap.parse_args()
    {"run": cmd_run, "traffic": cmd_traffic, "stats": cmd_stats, "counters": cmd_counters,
     "run-dipolar": cmd_run_dipolar, "run-adjoint": cmd_run_adjoint,
     "phase-split": cmd_phase_split}[args.cmd](args)


if __name__ == "__main__":
    main()
