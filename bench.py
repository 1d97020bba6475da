"""Benchmark: fourth-order Trotter-Suzuki evolution of the N = 27 open XYZ chain on one GPU.

Workload (seeded, synthetic): N = 27 open XYZ chain, J^a_i ~ U[0.5, 1.5] per bond,
h^z_i ~ U[-0.5, 0.5], random-phase state Phi, dt = 0.02, fourth-order fractal Suzuki.
One benchmark step is one Trotter step: U4(dt) applied to one 2^27-amplitude state
vector.  The workload is the infinite-temperature autocorrelation
C(t) = <a(t)|S^z_0|c(t)> with a(0) = Phi, c(0) = S^z_0 Phi: each time step advances both
vectors (two Trotter steps) and records C(t) (FP64).  K timed steps are K // 2 time steps
of the pair and, for odd K, one more Trotter step of a alone (unrecorded), so exactly K
Trotter steps are timed; the warm-up does the same with W steps on its own copies.  It runs
in complex128 and complex64; the complex64 C(t) is compared with the complex128 one at
every recorded time step.

Parity: the FP64 CPU oracle applies one second-order block U2(a dt) (a = 1/(4 - 4^(1/3)))
to the same N = 27 state; the GPU applies the same block (order 2, step a dt, one step) in
each dtype, and the relative L2 distance of the two states is reported.  The oracle run is
also the CPU baseline (all host cores; a one-thread sample at N = 24 beside it).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-extras]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# Rotation layers of one fourth-order step (five second-order blocks, four layers each after
# adjacent rotations are multiplied): the algorithmic floor moves the state in and out once
# per layer.
LAYERS_PER_STEP = 20
PARITY_TOL = {"c128": 1e-10, "c64": 1e-5}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="Trotter steps timed (>= 1)")
    ap.add_argument("--warmup", type=int, default=4, help="untimed Trotter steps first (>= 0)")
    ap.add_argument("--n", type=int, default=27)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle: no CPU baseline and no parity check")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--dtypes", default="c128,c64")
    args = ap.parse_args(argv)
    if args.steps < 1:
        ap.error("--steps must be >= 1")
    if args.warmup < 0:
        ap.error("--warmup must be >= 0")
    if args.gpus < 1:
        ap.error("--gpus must be >= 1")
    for d in args.dtypes.split(","):
        if d not in ("c128", "c64"):
            ap.error(f"unknown dtype {d!r} (c128, c64)")
    return args


def step_split(k: int):
    """(time steps of the C(t) pair, extra single-vector Trotter steps) for k Trotter steps:
    each time step advances both vectors once, an odd k adds one step of one vector."""
    return k // 2, k % 2


def algorithmic_bytes_per_step(n: int, esz: int) -> int:
    """Floor of the HBM bytes of one fourth-order step: one read and one write of the 2^n
    state per rotation layer."""
    return LAYERS_PER_STEP * 2 * (1 << n) * esz


def oracle_block(w, psi):
    """One second-order block U2(a dt) of the FP64 oracle on psi (all host cores): the
    parity reference and the CPU-baseline sample.  Returns (state, seconds)."""
    import oracle

    H = oracle.Hamiltonian(w.n, w.bonds, w.fields)
    a = oracle.suzuki_a()
    t0 = time.perf_counter()
    out = oracle.evolve(H, psi, a * w.dt, 1, 2)
    return out, time.perf_counter() - t0


_ONE_THREAD = r"""
import sys, time
sys.path.insert(0, sys.argv[1])
import oracle
from paper_1305_0036_amd import workloads as W
w = W.xyz_chain(n=int(sys.argv[2]), nsteps=1, state=True)
H = oracle.Hamiltonian(w.n, w.bonds, w.fields)
a = oracle.suzuki_a()
t0 = time.perf_counter()
oracle.evolve(H, w.psi0, a * w.dt, 1, 2)
print(time.perf_counter() - t0)
"""


def one_thread_sample(n_small: int):
    """Seconds of one U2(a dt) block of the oracle on one thread at n_small spins (same
    recipe), in a child process whose OpenMP runtime starts with one thread."""
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _ONE_THREAD, ROOT, str(n_small)], env=env,
                       capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-2000:])
    return float(r.stdout.strip().splitlines()[-1])


def cpu_baseline(n, t_block, t_one, n_small):
    """Oracle throughput in Trotter steps/s: a fourth-order step is five U2 blocks.  The
    one-thread sample at n_small spins is scaled to n by the state size and the number of
    single-spin passes (both grow with n)."""
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    out = {"value": float(f"{1.0 / (5.0 * t_block):.4g}"), "unit": "steps/s", "cores": cores,
           "kind": "oracle",
           "sample": f"one second-order block U2(a*dt) of the N={n} complex128 state on {cores} "
                     f"threads ({t_block:.1f} s), scaled to the 5 blocks of one fourth-order step"}
    if t_one is not None:
        scale = 2.0 ** (n - n_small) * n / n_small
        out["one_thread"] = {
            "value": float(f"{1.0 / (5.0 * t_one * scale):.4g}"), "unit": "steps/s", "cores": 1,
            "sample": f"one U2(a*dt) block of the N={n_small} chain of the same recipe on 1 thread "
                      f"({t_one:.2f} s), scaled by 2^{n - n_small}*{n}/{n_small} to N={n} and to "
                      f"5 blocks per step"}
    return out


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
    adjoint gradient (complex128), the N = 30 dipolar lattice (complex64, 8 GiB), the ping-
    pong sweeps of the headline chain, the Loschmidt echo (Sec. 4.2) and the order study."""
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
                    # the floor of every chain (20 layers, one read and one write each) over the
                    # recorded step time; chains of up to 14 spins stay in one workgroup's LDS
                    "algorithmic_GBps": round(sum(algorithmic_bytes_per_step(c.n, 8) for c in chains) * kb
                                              / (ms * 1e-3) / 1e9, 1),
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
    cfg = H.kernel_config(tsspin.TS_C64, 4)
    gbs = 2 * (1 << w.n) * 8 * nsw * w.nsteps / (ms * 1e-3) / 1e9
    alg = algorithmic_bytes_per_step(w.n, 8)
    out["dipolar"] = {"workload": "dipolar-lattice: N=30 5x6 open lattice, 435 pairs, complex64, "
                                  "order 4, dt=0.01, Neel with site 0 flipped",
                      "steps_per_s": round(w.nsteps / (ms / 1e3), 3), "sweeps_per_step": nsw,
                      "tile_bits": cfg["tile_bits"],
                      "frac": round(alg * w.nsteps / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "sweep_GBps": round(gbs, 1), "sweep_frac": round(gbs / HBM_PEAK_GBS, 4)}
    # the same steps with the phase read from the per-axis energy tables in HBM (variant 5)
    os.environ["TSSPIN_SWEEP_KERNEL"] = "etab"
    try:
        He = tsspin.Hamiltonian(w.n, w.bonds, w.fields)
    finally:
        del os.environ["TSSPIN_SWEEP_KERNEL"]
    x.zero_()
    x[w.extra["init_index"]] = 1.0
    He.evolve(x, w.dt, 1, 4)
    torch.cuda.synchronize()
    e0, e1 = ev()
    e0.record()
    He.evolve(x, w.dt, w.nsteps, 4)
    e1.record()
    torch.cuda.synchronize()
    ms_e = e0.elapsed_time(e1)
    out["dipolar"]["energy_table"] = {
        "config": {k: He.kernel_config(tsspin.TS_C64, 4)[k] for k in ("tile_bits", "reg_bits", "variant")},
        "steps_per_s": round(w.nsteps / (ms_e / 1e3), 3),
        "frac": round(alg * w.nsteps / (ms_e * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    He.close()
    del He
    torch.cuda.empty_cache()
    # the autotuner's choice for this system (one timed step per configuration)
    tuned = H.autotune(tsspin.TS_C64, 4, use_cache=False)
    x.zero_()
    x[w.extra["init_index"]] = 1.0
    H.evolve(x, w.dt, 1, 4)
    torch.cuda.synchronize()
    e0, e1 = ev()
    e0.record()
    H.evolve(x, w.dt, w.nsteps, 4)
    e1.record()
    torch.cuda.synchronize()
    ms_t = e0.elapsed_time(e1)
    out["dipolar"]["autotuned"] = {"config": {k: tuned[k] for k in ("tile_bits", "reg_bits", "variant")},
                                   "steps_per_s": round(w.nsteps / (ms_t / 1e3), 3),
                                   "frac": round(alg * w.nsteps / (ms_t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"dipolar: {out['dipolar']['steps_per_s']} steps/s, {gbs:.0f} GB/s per sweep; energy tables "
        f"{out['dipolar']['energy_table']['steps_per_s']} steps/s; autotuned "
        f"{out['dipolar']['autotuned']['steps_per_s']} steps/s {out['dipolar']['autotuned']['config']}")
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
    # the N = 12 Heisenberg chain: one workgroup holds the whole state for a recorded segment
    w = W.heisenberg_chain()
    H = tsspin.Hamiltonian(w.n, w.bonds, w.fields)
    x = torch.from_numpy(w.psi0).cuda()
    H.evolve(x, w.dt, 10, 4, record=[("sz", 0), ("norm",)], rec_every=1)
    x = torch.from_numpy(w.psi0).cuda()
    torch.cuda.synchronize()
    e0, e1 = ev()
    e0.record()
    rec = H.evolve(x, w.dt, w.nsteps, 4, record=[("sz", 0), ("norm",)], rec_every=1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    rc = rec.cpu().numpy()
    out["heisenberg_n12"] = {"workload": "heisenberg-chain: N=12 open chain, J=1, complex-Gaussian state, "
                                         "complex128, order 4, dt=0.05, 200 steps, <S^z_0> and norm every step",
                             "steps_per_s": round(w.nsteps / (ms / 1e3), 1), "ms_total": round(ms, 3),
                             "max_norm_dev": float(np.abs(rc[:, 1] - 1.0).max())}
    log(f"heisenberg n=12: {out['heisenberg_n12']['steps_per_s']} steps/s")
    del x, H
    out["echo"] = echo_study(torch, tsspin, W, log)
    out["order_study"] = order_study(torch, tsspin, W, log)
    return out


def echo_study(torch, tsspin, W, log, lengths=(100, 1000, 10000)):
    """The Loschmidt echo of Sec. 4.2 at N = 16: a periodic Heisenberg ring, and the ring
    plus double-quantum terms to the third neighbour, from |up>_0 (x) random phases;
    n order-4 steps with dt, then n with -dt; |1 - M_LE| with M_LE = |<psi_0|psi>|^2, in
    complex128 and complex64."""
    out = {"workload": "echo-ring: N=16 periodic Heisenberg ring (J=1), +/- S^xS^x - S^yS^y "
                       "(strength 1) to the 3rd neighbour, |up>_0 (x) random phases, dt=0.05, "
                       "order 4, n steps forward then n with -dt", "cases": []}
    for dq in (False, True):
        w = W.echo_ring(n=16, double_quantum=dq)
        H = tsspin.Hamiltonian(w.n, w.bonds, w.fields)
        for name, tdt in (("c128", torch.complex128), ("c64", torch.complex64)):
            x0 = torch.from_numpy(w.psi0).to(tdt).cuda()
            for n in lengths:
                x = x0.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                H.evolve(x, w.dt, n, 4)
                H.evolve(x, -w.dt, n, 4)
                ov = H.expect(x, [("overlap", x0)])[0]   # synchronises
                sec = time.perf_counter() - t0
                out["cases"].append({"double_quantum": dq, "dtype": name, "steps": n,
                                     "one_minus_M": float(f"{1.0 - abs(ov) ** 2:.6e}"),
                                     "ms_per_step": round(sec * 1e3 / (2 * n), 4)})
            del x0
        del H
    log("echo: " + ", ".join(f"{c['dtype']}{'+dq' if c['double_quantum'] else ''} n={c['steps']}: "
                             f"{c['one_minus_M']:.2e}" for c in out["cases"]))
    return out


def _dense_h(n, bonds, fields):
    """Dense H of Eq. 1 (bit j of the index = spin j, set = up) for the order study."""
    import numpy as np
    sx = np.array([[0, 1], [1, 0]], dtype=complex) / 2
    sy = np.array([[0, 1j], [-1j, 0]], dtype=complex) / 2   # basis (down, up)
    sz = np.diag([-0.5, 0.5]).astype(complex)

    def op(j, m):
        out = np.ones((1, 1), dtype=complex)
        for q in range(n - 1, -1, -1):
            out = np.kron(out, m if q == j else np.eye(2))
        return out
    S = [[op(j, m) for m in (sx, sy, sz)] for j in range(n)]
    H = np.zeros((1 << n, 1 << n), dtype=complex)
    for j in range(n):
        for a in range(3):
            if fields[j][a]:
                H += fields[j][a] * S[j][a]
    for (i, j, jx, jy, jz) in bonds:
        for a, c in enumerate((jx, jy, jz)):
            if c:
                H += c * S[i][a] @ S[j][a]
    return H


def order_study(torch, tsspin, W, log):
    """Accuracy against cost of the three orders (Sec. 2): the GPU's error against the exact
    propagator exp(-iHT) (dense, N = 10, T = 1) for three dt, beside the GPU time of one
    Trotter step of each order on the N = 27 benchmark chain."""
    import numpy as np
    import scipy.linalg as sla

    wq = W.xyz_chain(n=10, nsteps=1, state=True)
    Hd = _dense_h(wq.n, wq.bonds, wq.fields)
    exact = sla.expm(-1j * 1.0 * Hd) @ wq.psi0
    Hq = tsspin.Hamiltonian(wq.n, wq.bonds, wq.fields)
    w27 = W.xyz_chain(n=27, nsteps=1, state=False)
    H27 = tsspin.Hamiltonian(27, w27.bonds, w27.fields)
    x27 = torch.zeros(1 << 27, dtype=torch.complex128, device="cuda")
    x27[0] = 1.0
    rows = []
    for order in (1, 2, 4):
        H27.evolve(x27, w27.dt, 1, order)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        H27.evolve(x27, w27.dt, 4, order)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 4
        errs = []
        for dt in (0.1, 0.05, 0.025):
            x = torch.from_numpy(wq.psi0).cuda()
            Hq.evolve(x, dt, int(round(1.0 / dt)), order)
            errs.append(float(np.linalg.norm(x.cpu().numpy() - exact)))
        rows.append({"order": order, "errors_T1": {"0.1": errs[0], "0.05": errs[1], "0.025": errs[2]},
                     "error_ratio_per_halving": round(errs[1] / errs[2], 2),
                     "ms_per_step_n27_c128": round(ms, 3)})
    del x27, H27
    torch.cuda.empty_cache()
    log("order study: " + ", ".join(f"order {r['order']}: err(dt=0.05)={r['errors_T1']['0.05']:.2e}, "
                                    f"{r['ms_per_step_n27_c128']} ms/step" for r in rows))
    return {"workload": "xyz-chain recipe at N=10 (error vs dense exp(-iHT), T=1, complex128) and "
                        "N=27 (GPU ms per Trotter step, one vector, unrecorded)", "rows": rows}


def run_dtype(torch, tsspin, w, a0, c0, name, K, Wm, ref):
    """Warm-up, timed region and parity block of one dtype."""
    import numpy as np

    n = w.n
    dt_t = {"c128": torch.complex128, "c64": torch.complex64}[name]
    code = tsspin.TS_C128 if name == "c128" else tsspin.TS_C64
    esz = 16 if name == "c128" else 8
    rec_spec = [("overlap_sz", 0, 0, 1)]
    H = tsspin.Hamiltonian(n, w.bonds, w.fields)
    a = torch.from_numpy(a0).to(dt_t).cuda()
    c = torch.from_numpy(c0).to(dt_t).cuda()
    kt, kx = step_split(K)
    wt, wx = step_split(Wm)
    log(f"{name}: warmup {Wm} Trotter steps")
    if wt:
        wa, wc = a.clone(), c.clone()
        H.evolve([wa, wc], w.dt, wt, 4, record=rec_spec, rec_every=1)
        del wc
    if wx:
        wa = a.clone() if not wt else wa
        H.evolve(wa, w.dt, 1, 4)
    if Wm:
        del wa
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()   # the stream the library launches on
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    rt = H.evolve([a, c], w.dt, kt, 4, record=rec_spec, rec_every=1) if kt else None
    if kx:
        H.evolve(a, w.dt, 1, 4)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    recs = rt.cpu().numpy() if rt is not None else np.zeros((0, 2))
    # launches of the timed region: every Trotter step of one vector runs the one-step plan
    l1, cone = H.launches(code, w.dt, 1, 4)
    launches = K * l1
    # the same sweeps alone (one unrecorded step of one vector), for reference
    H.evolve(a, w.dt, 1, 4)
    torch.cuda.synchronize()
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record(stream)
    H.evolve(a, w.dt, 1, 4)
    f1.record(stream)
    torch.cuda.synchronize()
    kernel_only_ms = f0.elapsed_time(f1) / l1
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
    parity = None
    if ref is not None:
        x = torch.from_numpy(a0).to(dt_t).cuda()
        H.evolve(x, ref["a"] * w.dt, 1, 2)
        got = x.cpu().numpy().astype(np.complex128)
        parity = float(np.linalg.norm(got - ref["psi"]) / np.linalg.norm(ref["psi"]))
        del x, got
        log(f"{name}: parity vs oracle (one U2(a dt) block) rel L2 = {parity:.3e}")
    res = dict(ms=ms, steps_per_s=K / (ms / 1e3), C=recs, l1=l1, cone=cone, launches=launches,
               avg_launch_ms=ms / launches, kernel_only_ms=kernel_only_ms, esz=esz, kernel=kname,
               cfg=cfg, flops=flops, parity=parity)
    log(f"{name}: {K} Trotter steps ({kt} time steps x 2 vectors + {kx}) in {ms:.1f} ms -> "
        f"{res['steps_per_s']:.2f} steps/s; {l1} launches per step, {ms / launches:.3f} ms each")
    del a, c, H
    torch.cuda.empty_cache()
    return res


def roofline(r, n):
    """Roofline of the sweep kernel: algorithmic bytes per launch (the per-step floor over
    the launches of one step) over the average launch duration of the timed region."""
    alg_step = algorithmic_bytes_per_step(n, r["esz"])
    per_launch = alg_step / r["l1"]
    achieved = per_launch / (r["avg_launch_ms"] * 1e-3) / 1e9
    moved = 2 * (1 << n) * r["esz"]
    moved_gbs = moved / (r["avg_launch_ms"] * 1e-3) / 1e9
    return {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None,
        "kernel": r["kernel"],
        "algorithmic_bytes_per_step": alg_step,
        "launches_per_step": r["l1"],
        "algorithmic_bytes_per_launch": round(per_launch),
        "avg_launch_ms": round(r["avg_launch_ms"], 4),
        "avg_launch_ms_source": "HIP events around the timed region / its sweep launches "
                                "(the region's record reductions included)",
        "kernel_only_avg_launch_ms": round(r["kernel_only_ms"], 4),
        "moved_bytes_per_launch": moved,
        "moved_GBps": round(moved_gbs, 1),
        "moved_frac": round(moved_gbs / HBM_PEAK_GBS, 4),
    }


def main(argv=None):
    args = parse_args(argv)
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
    kt, kx = step_split(K)
    log(f"generating workload n={n}")
    w = W.xyz_chain(n=n, nsteps=kt + 1, state=True)
    a0 = w.psi0
    c0 = W.sz_times(a0, n, 0)
    ref = None
    t_block = t_one = None
    n_small = min(n, 24)
    if not args.no_cpu_baseline:
        import oracle
        log("oracle: one U2(a dt) block on the host cores (parity reference, CPU baseline)")
        psi_ref, t_block = oracle_block(w, a0)
        ref = {"psi": psi_ref, "a": oracle.suzuki_a()}
        log(f"oracle: {t_block:.1f} s; one-thread sample at n={n_small}")
        try:
            t_one = one_thread_sample(n_small)
        except (RuntimeError, subprocess.TimeoutExpired) as e:
            log(f"one-thread sample failed: {e}")
    results = {}
    for name in args.dtypes.split(","):
        results[name] = run_dtype(torch, tsspin, w, a0, c0, name, K, Wm, ref)

    main_name = "c128" if "c128" in results else list(results)[0]
    r = results[main_name]
    roof = roofline(r, n)
    from paper_1305_0036_amd.profile_traffic import source_hash
    traffic = measured_traffic(source_hash()) if (main_name == "c128" and n == 27) else None
    if traffic is not None:
        roof["traffic"] = round(traffic / 1e9, 4)
        roof["traffic_unit"] = "GB per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    if r["flops"]:
        # light-cone sweeps: arithmetic intensity below the FP64 ridge point (the roof is HBM)
        roof["flops_per_launch"] = round(r["flops"])
        roof["achieved_tflops"] = round(r["flops"] / (r["kernel_only_ms"] * 1e-3) / 1e12, 2)
        roof["fp64_peak_tflops"] = 78.6
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
            "workload": f"xyz-chain N={n} open, J~U[0.5,1.5], hz~U[-0.5,0.5], random-phase state, "
                        "dt=0.02, order 4; one step = U4(dt) on one 2^N state vector; the C(t) "
                        "pair advances 2 vectors per time step and records C(t) every time step",
            "n_spins": n, "time_steps": kt, "extra_single_vector_steps": kx,
            "time_steps_per_s": round((kt / (r["ms"] / 1e3)), 4), "order": 4, "dt": w.dt,
            "state_bytes": (1 << n) * r["esz"],
        },
        "roofline": roof,
    }
    if ref is not None:
        out["parity_rel_l2"] = {k: v["parity"] for k, v in results.items()}
        out["parity_rel_l2"]["tolerance"] = {k: PARITY_TOL[k] for k in results}
        out["parity_rel_l2"]["check"] = (f"one second-order block U2(a*dt) of the N={n} benchmark "
                                         "state: GPU (order 2, one step) vs the FP64 oracle")
        out["parity_rel_l2"]["pass"] = all(v["parity"] <= PARITY_TOL[k] for k, v in results.items())
    if "c64" in results and "c128" in results:
        c64 = results["c64"]
        C64, C128 = c64["C"], results["c128"]["C"]
        dC = np.abs((C64[:, 0] + 1j * C64[:, 1]) - (C128[:, 0] + 1j * C128[:, 1])) if len(C64) else np.zeros(1)
        r64 = roofline(c64, n)
        out["c64"] = {"value": round(c64["steps_per_s"], 4), "ms_per_step": round(c64["ms"] / K, 4),
                      "speedup_vs_c128": round(c64["steps_per_s"] / r["steps_per_s"], 3),
                      "max_abs_err_C_vs_c128": float(dC.max()), "kernel": c64["kernel"],
                      "frac": r64["frac"], "moved_frac": r64["moved_frac"],
                      "avg_launch_ms": r64["avg_launch_ms"], "launches_per_step": c64["l1"]}
    if not args.no_extras and n == 27:
        out["other_forms"] = extra_workloads(torch, tsspin, W, log)
    if t_block is not None:
        out["cpu_baseline"] = cpu_baseline(n, t_block, t_one, n_small)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
