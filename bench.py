"""Benchmark: fourth-order Trotter-Suzuki evolution of the N = 27 open XYZ chain on one GPU.

Workload (seeded, synthetic): N = 27 open XYZ chain, J^a_i ~ U[0.5, 1.5] per bond,
h^z_i ~ U[-0.5, 0.5], random-phase state Phi, dt = 0.02, fourth-order fractal Suzuki.
One benchmark step is one Trotter step: U4(dt) applied to one 2^27-amplitude state
vector.  The workload is the infinite-temperature autocorrelation
C(t) = <a(t)|S^z_0|c(t)> with a(0) = Phi, c(0) = S^z_0 Phi: each time step advances both
vectors (two Trotter steps) and records C(t) (FP64), so K steps are K/2 time steps.  It
runs in complex128 and complex64; the complex64 C(t) is compared with the complex128 one
at every recorded time step.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]   (K, W even)

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(w, psi):
    """Time the FP64 oracle on a bounded sample of the same workload: one second-order block
    U2(a dt) of the full N = 27 state (z, y, x, x, y, z sub-steps).  A fourth-order Trotter
    step (the benchmark step: one vector) is five such blocks."""
    import numpy as np

    import oracle

    H = oracle.Hamiltonian(w.n, w.bonds, w.fields)
    x = np.array(psi, dtype=np.complex128)
    a = oracle.suzuki_a()
    t0 = time.perf_counter()
    oracle.evolve(H, x, a * w.dt, 1, 2)
    t_blk = time.perf_counter() - t0
    step = 5.0 * t_blk
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    return {"value": 1.0 / step, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "sample": f"one second-order block U2(a*dt) of the N=27 complex128 state "
                      f"({t_blk:.1f} s), scaled to the 5 blocks of one fourth-order step"}


def measured_traffic(kernel_hash):
    """HBM bytes per sweep launch from the committed counter summary, if it was taken on
    the current kernel sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", "sweep_traffic_c128_n27.md")
    try:
        text = open(path).read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("source_hash") != kernel_hash:
        return None
    return blob.get("traffic_bytes_per_launch")


def extra_workloads(torch, tsspin, W, log):
    """Secondary measurements of the other hot-path forms (not the headline number):
    the 512-chain disordered batch (complex64, one captured graph per segment), the N = 20
    adjoint gradient (complex128), and the N = 30 dipolar lattice (complex64, 8 GiB)."""
    import numpy as np

    out = {}
    ev = lambda: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

    # batched: 512 open XXZ chains, N ~ U{10..20}
    chains = W.disordered_xxz_batch()
    B = tsspin.Batch([(c.n, c.bonds, c.fields) for c in chains])
    packed = torch.from_numpy(np.concatenate([c.psi0 for c in chains])).to(torch.complex64).cuda()
    dt, kb = chains[0].dt, 40
    tuned_ms = B.autotune(tsspin.TS_C64, 4)   # tile width and register window for this batch
    B.evolve(packed, dt, 2, 4, record=[("sz", 0)], rec_every=1)
    torch.cuda.synchronize()
    e0, e1 = ev()
    e0.record()
    rec = B.evolve(packed, dt, kb, 4, record=[("sz", 0)], rec_every=1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    out["batch"] = {"workload": "disordered-xxz-batch: 512 open XXZ chains, N~U{10..20}, complex64, "
                                "order 4, dt=0.05, <S^z_0> recorded every step",
                    "chains": len(chains), "amplitudes": B.total, "steps": kb,
                    "chain_steps_per_s": round(len(chains) * kb / (ms / 1e3), 1),
                    "amplitude_steps_per_s": float(f"{B.total * kb / (ms / 1e3):.4g}"),
                    "ms_per_step": round(ms / kb, 4), "autotuned_ms_per_unrecorded_step": round(tuned_ms, 4),
                    "sz0_in_range": bool(np.abs(rec.cpu().numpy()).max() <= 0.5 + 1e-5)}
    log(f"batch: {out['batch']['chain_steps_per_s']} chain-steps/s")
    del packed, B
    torch.cuda.empty_cache()

    # adjoint: N = 20 chain, 300 steps, loss <S^z_0(T)>
    w = W.gradient_chain()
    H = tsspin.Hamiltonian(w.n, w.bonds, w.fields)
    x = torch.from_numpy(w.psi0).cuda()
    y = x.clone()
    H.evolve(y, w.dt, w.nsteps, 4)
    H.adjoint(x, w.dt, w.nsteps, 4, ("sz", 0))
    torch.cuda.synchronize()
    y = x.clone()
    e0, e1 = ev()
    e0.record()
    H.evolve(y, w.dt, w.nsteps, 4)
    e1.record()
    torch.cuda.synchronize()
    t_fwd = e0.elapsed_time(e1)
    t0 = time.perf_counter()
    H.adjoint(x, w.dt, w.nsteps, 4, ("sz", 0))
    t_adj = (time.perf_counter() - t0) * 1e3
    out["adjoint"] = {"workload": "gradient-chain: N=20 open XYZ chain, complex128, order 4, dt=0.02, "
                                  "300 steps, loss <S^z_0(T)>",
                      "parameters": 3 * len(w.bonds) + 3 * w.n, "forward_ms": round(t_fwd, 2),
                      "adjoint_ms": round(t_adj, 2), "adjoint_over_forward": round(t_adj / t_fwd, 2),
                      "central_fd_ms_77_params": round(2 * 77 * t_fwd, 1)}
    log(f"adjoint: {t_adj:.1f} ms (forward {t_fwd:.1f} ms)")
    del x, y, H

    # dipolar lattice: N = 30, 435 pairs, complex64 (8 GiB)
    w = W.dipolar_lattice(nsteps=3)
    H = tsspin.Hamiltonian(w.n, w.bonds, w.fields)
    x = torch.zeros(1 << w.n, dtype=torch.complex64, device="cuda")
    x[w.extra["init_index"]] = 1.0
    H.evolve(x, w.dt, 1, 4)
    torch.cuda.synchronize()
    e0, e1 = ev()
    e0.record()
    H.evolve(x, w.dt, w.nsteps, 4)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    nsw = H.launches(tsspin.TS_C64, w.dt, 1, 4)[0]
    gbs = 2 * (1 << w.n) * 8 * nsw * w.nsteps / (ms * 1e-3) / 1e9
    out["dipolar"] = {"workload": "dipolar-lattice: N=30 5x6 open lattice, 435 pairs, complex64, "
                                  "order 4, dt=0.01, Neel with site 0 flipped",
                      "steps_per_s": round(w.nsteps / (ms / 1e3), 3), "sweeps_per_step": nsw,
                      "sweep_GBps": round(gbs, 1), "sweep_frac": round(gbs / HBM_PEAK_GBS, 4)}
    log(f"dipolar: {out['dipolar']['steps_per_s']} steps/s, {gbs:.0f} GB/s")
    del x, H
    torch.cuda.empty_cache()

    # the ping-pong sweeps on the headline workload (HBM-bound form, one pass per layer part)
    w = W.xyz_chain(n=27, nsteps=4, state=False)
    for name, dt_t, code in (("c128", torch.complex128, tsspin.TS_C128), ("c64", torch.complex64, tsspin.TS_C64)):
        os.environ["TSSPIN_SWEEP_KERNEL"] = "half" if name == "c128" else "reg"
        try:
            H = tsspin.Hamiltonian(27, w.bonds, w.fields)
        finally:
            del os.environ["TSSPIN_SWEEP_KERNEL"]
        g = torch.Generator(device="cpu").manual_seed(3)
        x = torch.polar(torch.full((1 << 27,), 2.0 ** (-27 / 2), dtype=torch.float64),
                        torch.rand(1 << 27, dtype=torch.float64, generator=g) * 6.283).to(dt_t).cuda()
        H.evolve(x, w.dt, 1, 4)
        torch.cuda.synchronize()
        e0, e1 = ev()
        e0.record()
        H.evolve(x, w.dt, 4, 4)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 4
        nsw = len(H.plan(code, w.dt, 4, 4)) / 4
        gbs = 2 * (1 << 27) * (16 if name == "c128" else 8) * nsw / (ms * 1e-3) / 1e9
        out[f"pingpong_{name}"] = {"workload": "the headline xyz chain N=27, one vector, unrecorded",
                                   "steps_per_s": round(1e3 / ms, 3), "sweeps_per_step": nsw,
                                   "sweep_GBps": round(gbs, 1), "sweep_frac": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"ping-pong {name}: {1e3 / ms:.2f} steps/s, {gbs:.0f} GB/s per sweep")
        del x, H
        torch.cuda.empty_cache()
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--n", type=int, default=27)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--dtypes", default="c128,c64")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no "
              "sharded multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1305_0036_amd import tsspin
    from paper_1305_0036_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    n, K, Wm = args.n, args.steps, args.warmup
    if K < 2 or K % 2 or Wm % 2:
        print("--steps must be even and >= 2 and --warmup even: the C(t) workload advances "
              "its two vectors together (two Trotter steps per time step)", file=sys.stderr)
        sys.exit(2)
    kt, wt = K // 2, Wm // 2   # time steps of the pair
    log(f"generating workload n={n}")
    w = W.xyz_chain(n=n, nsteps=kt + wt, state=True)
    a0 = w.psi0
    c0 = W.sz_times(a0, n, 0)
    rec_spec = [("overlap_sz", 0, 0, 1)]
    dtypes = {"c128": torch.complex128, "c64": torch.complex64}
    results = {}
    for name in args.dtypes.split(","):
        dt_t = dtypes[name]
        code = tsspin.TS_C128 if name == "c128" else tsspin.TS_C64
        H = tsspin.Hamiltonian(n, w.bonds, w.fields)
        a = torch.from_numpy(a0).to(dt_t).cuda()
        c = torch.from_numpy(c0).to(dt_t).cuda()
        log(f"{name}: warmup {Wm}")
        rw = H.evolve([a, c], w.dt, wt, 4, record=rec_spec, rec_every=1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        rt = H.evolve([a, c], w.dt, kt, 4, record=rec_spec, rec_every=1)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        recs = np.concatenate([rw.cpu().numpy(), rt.cpu().numpy()[1:]], axis=0)
        # sweep-kernel duration: one vector, one step (the plan of the timed run's segments)
        # without recording, events around it
        ks = 1
        nsw, cone = H.launches(code, w.dt, ks, 4)
        H.evolve(a, w.dt, ks, 4)   # builds and uploads the ks-step plan outside the timed region
        torch.cuda.synchronize()
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record()
        H.evolve(a, w.dt, ks, 4)
        f1.record()
        torch.cuda.synchronize()
        sweep_ms = f0.elapsed_time(f1) / nsw
        nbytes = 2 * (1 << n) * (16 if name == "c128" else 8)
        cfg = H.kernel_config(code, 4)
        if cone:
            kname = f"cone_{name}_kernel<{cfg['tile_bits']}, 4> (light-cone sweeps)"
        else:
            v = 3 if (cfg["variant"] == 4 and name == "c128") else (0 if cfg["variant"] == 4 else cfg["variant"])
            kname = (f"{'sweep_pipe_kernel' if v == 2 else 'sweep_reg_kernel'}"
                     f"<{'double' if name == 'c128' else 'float'}, {cfg['tile_bits']}, {cfg['reg_bits']}>")
            if name == "c128" and v == 3 and cfg["tile_bits"] in (11, 12) and cfg["reg_bits"] == 4:
                kname += f" + sweep_half_kernel<{cfg['tile_bits']}, 4> (top bit group)"
        flops = None
        if cone:   # butterflies: 2 flops per amplitude and spin-layer; phase steps: one complex product
            sw1, _ = H.cone_plan(code, w.dt, 1, 4)
            sl = sum(bin(o["spins"]).count("1") for s in sw1 for o in s["ops"] if o["kind"] == "bfly")
            ph = sum(1 for s in sw1 for o in s["ops"] if o["kind"] == "phase")
            flops = (1 << n) * (2 * sl + 6 * ph) / len(sw1)
        results[name] = dict(ms=ms, steps_per_s=K / (ms / 1e3), C=recs, sweep_ms=sweep_ms,
                             sweep_bytes=nbytes, nsweeps=nsw, ks=ks, kernel=kname, cfg=cfg, cone=cone,
                             flops=flops, sweeps_per_vector_step=H.launches(code, w.dt, 1, 4)[0])
        log(f"{name}: {K} Trotter steps ({kt} time steps x 2 vectors) in {ms:.1f} ms -> "
            f"{K / (ms / 1e3):.2f} steps/s; "
            f"sweep {sweep_ms:.3f} ms = {nbytes / (sweep_ms * 1e-3) / 1e9:.0f} GB/s")
        del a, c, H
        torch.cuda.empty_cache()

    main_name = "c128" if "c128" in results else list(results)[0]
    r = results[main_name]
    achieved = r["sweep_bytes"] / (r["sweep_ms"] * 1e-3) / 1e9
    from paper_1305_0036_amd.profile_traffic import source_hash
    traffic = measured_traffic(source_hash()) if (main_name == "c128" and n == 27) else None
    out = {
        "metric": "Trotter steps/s at N=27 + % HBM peak; FP32 vs FP64 at <=1e-5 obs. error",
        "value": round(r["steps_per_s"], 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(r["ms"] / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_name,
        "data": "synthetic",
        "config": {
            "workload": "xyz-chain N=27 open, J~U[0.5,1.5], hz~U[-0.5,0.5], random-phase state, "
                        "dt=0.02, order 4; one step = U4(dt) on one 2^27 state vector; the C(t) "
                        "pair advances 2 vectors per time step and records C(t) every time step",
            "n_spins": n, "trotter_steps_per_time_step": 2, "time_steps": kt,
            "time_steps_per_s": round(r["steps_per_s"] / 2, 4), "order": 4, "dt": w.dt,
            "state_bytes": (1 << n) * (16 if main_name == "c128" else 8),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic / 1e9, 4),
            "traffic_unit": "GB per launch",
            "kernel": r["kernel"],
            "per_launch_bytes": r["sweep_bytes"],
            "launches_per_vector_step": r["sweeps_per_vector_step"],
            "avg_launch_ms": round(r["sweep_ms"], 4),
        },
    }
    if r["flops"]:
        # light-cone sweeps: arithmetic intensity below the ridge point (the roof is HBM),
        # but the kernel is limited by vector-instruction issue; its FP64 rate for reference
        out["roofline"]["flops_per_launch"] = round(r["flops"])
        out["roofline"]["achieved_tflops"] = round(r["flops"] / (r["sweep_ms"] * 1e-3) / 1e12, 2)
        out["roofline"]["fp64_peak_tflops"] = 78.6
    if "c64" in results and "c128" in results:
        c64 = results["c64"]
        dC = np.abs((results["c64"]["C"][:, 0] + 1j * results["c64"]["C"][:, 1])
                    - (results["c128"]["C"][:, 0] + 1j * results["c128"]["C"][:, 1]))
        a64 = c64["sweep_bytes"] / (c64["sweep_ms"] * 1e-3) / 1e9
        out["c64"] = {"value": round(c64["steps_per_s"], 4), "ms_per_step": round(c64["ms"] / K, 4),
                      "speedup_vs_c128": round(c64["steps_per_s"] / r["steps_per_s"], 3),
                      "max_abs_err_C_vs_c128": float(dC.max()),
                      "sweep_GBps": round(a64, 1), "sweep_frac": round(a64 / HBM_PEAK_GBS, 4)}
    if not args.no_extras and n == 27:
        out["other_forms"] = extra_workloads(torch, tsspin, W, log)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline(w, a0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
