"""GPU parity of libtsspin against the FP64 oracle (needs an MI355X).

Every case prints its name, size and seed before touching the GPU.  Tolerances:
complex128 states within 1e-10 relative L2 of the oracle; complex64 states within 1e-5
relative L2 (FP32 storage, FP64 phase arguments; about 6e-8 rounding per butterfly stage
and phase over a few hundred stages); observables as stated per test.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1305_0036_amd import workloads as W
from tests import dense_ref as D

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1305_0036_amd import tsspin
    return tsspin


def _say(*a):
    print("[case]", *a, flush=True)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _gpu(psi, dtype):
    return torch.from_numpy(np.ascontiguousarray(psi)).to(dtype).cuda()


C128, C64 = torch.complex128, torch.complex64
TOL = {C128: 1e-10, C64: 1e-5}


@pytest.mark.parametrize("dtype", [C128, C64])
@pytest.mark.parametrize("order", [1, 2, 4])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10, 12])
def test_resident_parity(n, order, dtype):
    ts = _dev()
    seed = 50 + 7 * n + order
    _say("resident", n, order, dtype, seed)
    rng = np.random.default_rng(seed)
    bonds, fields = D.random_xyz(rng, n, chain=n > 8)
    psi0 = D.random_state(rng, n)
    H = ts.Hamiltonian(n, bonds, fields)
    x = _gpu(psi0, dtype)
    H.evolve(x, 0.09, 5, order)
    torch.cuda.synchronize()
    ref = oracle.evolve(oracle.Hamiltonian(n, bonds, fields), psi0, 0.09, 5, order)
    assert _rel(x.cpu().numpy().astype(np.complex128), ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", [C128, C64])
@pytest.mark.parametrize("n,T", [(9, 8), (11, 8), (13, 8), (16, 8), (14, 10), (16, 11), (17, 12)])
def test_tiled_parity(n, T, dtype):
    ts = _dev()
    seed = 300 + n + 100 * T
    _say("tiled", n, T, dtype, seed)
    rng = np.random.default_rng(seed)
    bonds, fields = D.random_xyz(rng, n, chain=True)
    # a few long-range bonds so couplings cross the tile / outside boundary
    bonds += [(0, n - 1, 0.3, -0.2, 0.5), (2, n // 2 + 1, -0.4, 0.6, 0.1)]
    psi0 = D.random_state(rng, n)
    H = ts.Hamiltonian(n, bonds, fields)
    H.set_tile_bits(ts.TS_C128 if dtype == C128 else ts.TS_C64, T)
    x = _gpu(psi0, dtype)
    H.evolve(x, 0.07, 3, 4)
    torch.cuda.synchronize()
    ref = oracle.evolve(oracle.Hamiltonian(n, bonds, fields), psi0, 0.07, 3, 4)
    assert _rel(x.cpu().numpy().astype(np.complex128), ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", [C128, C64])
def test_observables_match_oracle(dtype):
    ts = _dev()
    n = 10
    _say("expect", n, dtype)
    rng = np.random.default_rng(77)
    bonds, fields = D.random_xyz(rng, n, chain=True)
    psi = D.random_state(rng, n)
    oth = D.random_state(rng, n)
    Ho = oracle.Hamiltonian(n, bonds, fields)
    H = ts.Hamiltonian(n, bonds, fields)
    x, y = _gpu(psi, dtype), _gpu(oth, dtype)
    obs = [("norm",), ("mz",), ("sz", 3), ("sx", 0), ("sx", 9), ("sy", 4), ("szsz", 1, 7),
           ("overlap_sz", 2, y)]
    got = H.expect(x, obs)
    ref = [oracle.expect(Ho, psi, "norm"), oracle.expect(Ho, psi, "mz"),
           oracle.expect(Ho, psi, "sz", 3), oracle.expect(Ho, psi, "sx", 0),
           oracle.expect(Ho, psi, "sx", 9), oracle.expect(Ho, psi, "sy", 4),
           oracle.expect(Ho, psi, "szsz", 1, 7), oracle.expect(Ho, psi, "overlap_sz", 2, other=oth)]
    tol = 1e-13 if dtype == C128 else 2e-6
    for g, r, o in zip(got, ref, obs):
        assert abs(g - r) < tol, (o[0], g, r)


def test_heisenberg_chain_record_vs_oracle():
    # N = 12 open Heisenberg chain, dt = 0.05, 200 steps, <S^z_0> and the norm every step
    ts = _dev()
    w = W.heisenberg_chain()
    _say("heisenberg-chain", w.n, w.nsteps)
    H = ts.Hamiltonian(w.n, w.bonds, w.fields)
    x = _gpu(w.psi0, C128)
    rec = H.evolve(x, w.dt, w.nsteps, w.order, record=[("sz", 0), ("norm",)], rec_every=1)
    rec = rec.cpu().numpy()
    Ho = oracle.Hamiltonian(w.n, w.bonds, w.fields)
    cur = w.psi0.copy()
    ref = [oracle.expect(Ho, cur, "sz", 0)]
    for _ in range(w.nsteps):
        cur = oracle.evolve(Ho, cur, w.dt, 1, w.order)
        ref.append(oracle.expect(Ho, cur, "sz", 0))
    assert np.abs(rec[:, 0] - np.array(ref)).max() < 1e-10
    assert np.abs(rec[:, 1] - 1.0).max() < 1e-12
    assert _rel(x.cpu().numpy(), cur) < 1e-10


@pytest.mark.parametrize("dtype", [C128, torch.complex64])
@pytest.mark.parametrize("n,nsteps,every,order", [(12, 40, 1, 4), (6, 25, 3, 2), (11, 9, 4, 1), (5, 4099, 1, 4)])
def test_resident_records_in_one_launch(monkeypatch, n, nsteps, every, order, dtype):
    """A single vector that fits one tile, recorded with real kinds only, runs every segment
    and record in one resident launch (4096 segments at most per launch: the last case takes
    two).  Against separate reductions after each segment (TSSPIN_NO_FUSE=1): the same
    operations, so the states agree bit for bit and the records to summation order."""
    ts = _dev()
    seed = 77 + n
    _say("resident records", n, nsteps, every, order, dtype, seed)
    rng = np.random.default_rng(seed)
    bonds, fields = D.random_xyz(rng, n, chain=True)
    psi0 = W.gaussian_state(rng, n)
    obs = [("sz", 0), ("norm",), ("sx", n - 1), ("sy", 1), ("szsz", 0, n - 1), ("mz",)]
    out = {}
    for nf in ("0", "1"):
        monkeypatch.setenv("TSSPIN_NO_FUSE", nf)
        H = ts.Hamiltonian(n, bonds, fields)
        x = _gpu(psi0, dtype)
        out[nf] = (H.evolve(x, 0.05, nsteps, order, record=obs, rec_every=every).cpu().numpy(), x.cpu())
    assert out["0"][0].shape == (nsteps // every + 1, len(obs))
    assert torch.equal(out["0"][1], out["1"][1])
    assert np.abs(out["0"][0] - out["1"][0]).max() < (1e-13 if dtype == C128 else 1e-6)


@pytest.mark.parametrize("dtype", [C128, torch.complex64])
@pytest.mark.parametrize("n,order", [(12, 4), (5, 2), (9, 1)])
def test_resident_precomputed_factors_bitwise(monkeypatch, n, order, dtype):
    """A state that fits one tile multiplies by phase factors formed once per plan (the
    plan's distinct phase steps applied to a tile of ones): the same amplitudes, bit for
    bit, as forming every phase in place (TSSPIN_RESIDENT_FACTORS=0), fields on every axis."""
    ts = _dev()
    seed = 310 + n
    _say("resident factors", n, order, dtype, seed)
    rng = np.random.default_rng(seed)
    bonds, fields = D.random_xyz(rng, n, chain=False)
    psi0 = W.gaussian_state(rng, n)
    out = {}
    for f in ("1", "0"):
        monkeypatch.setenv("TSSPIN_RESIDENT_FACTORS", f)
        H = ts.Hamiltonian(n, bonds, fields)
        x = _gpu(psi0, dtype)
        rec = H.evolve(x, 0.03, 7, order, record=[("sz", 0), ("norm",)], rec_every=2)
        out[f] = (x.cpu(), rec.cpu().numpy())
    assert torch.equal(out["1"][0], out["0"][0])
    assert np.array_equal(out["1"][1], out["0"][1])


def test_lockstep_vectors_and_overlap_record():
    # two vectors evolved together; <a|S^z_0|c> recorded every 2 steps (the C(t) pattern)
    ts = _dev()
    n = 11
    _say("pair", n)
    w = W.xyz_chain(n=n, nsteps=10)
    a0 = w.psi0
    c0 = W.sz_times(a0, n, 0)
    H = ts.Hamiltonian(n, w.bonds, w.fields)
    a, c = _gpu(a0, C128), _gpu(c0, C128)
    rec = H.evolve([a, c], w.dt, 10, 4, record=[("overlap_sz", 0, 0, 1), ("norm", 1)], rec_every=2)
    rec = rec.cpu().numpy()
    Ho = oracle.Hamiltonian(n, w.bonds, w.fields)
    ca, cc = a0.copy(), c0.copy()
    for r in range(6):
        ov = oracle.expect(Ho, cc, "overlap_sz", 0, other=ca)
        assert abs(complex(rec[r, 0], rec[r, 1]) - ov) < 1e-12
        assert abs(rec[r, 2] - oracle.expect(Ho, cc, "norm")) < 1e-12
        ca = oracle.evolve(Ho, ca, w.dt, 2, 4)
        cc = oracle.evolve(Ho, cc, w.dt, 2, 4)
    assert abs(rec[0, 0] - 0.25) < 1e-14   # C(0) = <Phi|S^z_0 S^z_0|Phi> = 1/4


# --------------------------------------------------------------- full size (N = 27)


def _blocks_of_xyz27():
    """Config-2 recipe at N = 27 with bonds (8,9) and (17,18) removed: three independent
    9-spin chains.  Returns the 27-spin bond list and the three block Hamiltonians."""
    w = W.xyz_chain(n=27, nsteps=1, state=False)
    bonds = [b for b in w.bonds if (b[0], b[1]) not in ((8, 9), (17, 18))]
    blocks = []
    for lo in (0, 9, 18):
        bb = [(i - lo, j - lo, jx, jy, jz) for (i, j, jx, jy, jz) in bonds if lo <= i < lo + 9]
        blocks.append(oracle.Hamiltonian(9, bb, w.fields[lo:lo + 9]))
    return w, bonds, blocks


@pytest.mark.parametrize("dtype", [C128, C64])
def test_full_size_factorized_evolution(dtype):
    # Exact property at any size: a Hamiltonian without bonds between blocks A, B, C and a
    # product state give psi(T) = psi_C(T) (x) psi_B(T) (x) psi_A(T), each block evolved by
    # the same Trotter product on its own.  Checked on all 2^27 amplitudes in the launch
    # configuration of the benchmark (13/14-bit tiles, three bit groups).
    ts = _dev()
    w, bonds, blocks = _blocks_of_xyz27()
    nsteps = 4
    _say("factorized-27", dtype, nsteps)
    rng = np.random.default_rng(2027)
    parts = [D.random_state(rng, 9) for _ in range(3)]
    evolved = [oracle.evolve(blocks[k], parts[k], w.dt, nsteps, 4) for k in range(3)]
    H = ts.Hamiltonian(27, bonds, w.fields)
    cd = torch.complex128
    x = torch.kron(torch.from_numpy(parts[2]).cuda(),
                   torch.kron(torch.from_numpy(parts[1]).cuda(), torch.from_numpy(parts[0]).cuda()))
    x = x.to(dtype).contiguous()
    H.evolve(x, w.dt, nsteps, 4)
    ref = torch.kron(torch.from_numpy(evolved[2]).cuda(),
                     torch.kron(torch.from_numpy(evolved[1]).cuda(), torch.from_numpy(evolved[0]).cuda()))
    err = torch.linalg.vector_norm(x.to(cd) - ref) / torch.linalg.vector_norm(ref)
    torch.cuda.synchronize()
    assert float(err) < TOL[dtype]


def test_full_size_echo_and_norm():
    # U4(-dt)^n U4(dt)^n = 1 (Sec. 4.2 echo with Sigma = 0): the full N = 27 workload
    ts = _dev()
    w = W.xyz_chain(n=27, nsteps=1, state=False)
    _say("echo-27")
    H = ts.Hamiltonian(27, w.bonds, w.fields)
    g = torch.Generator(device="cuda").manual_seed(27)
    phi = torch.rand(1 << 27, device="cuda", dtype=torch.float64, generator=g) * (2 * np.pi)
    x0 = torch.polar(torch.full_like(phi, 2.0 ** -13.5), phi)
    x = x0.clone()
    rec = H.evolve(x, w.dt, 6, 4, record=[("norm",)], rec_every=3)
    H.evolve(x, -w.dt, 6, 4)
    err = float(torch.linalg.vector_norm(x - x0))
    torch.cuda.synchronize()
    assert err < 1e-12
    assert np.abs(rec.cpu().numpy()[:, 0] - 1.0).max() < 1e-13


def test_full_size_pure_z_sampled_against_oracle_energies():
    # Single-part Hamiltonian (z couplings and fields of the N = 27 chain only): the
    # evolution is the exact phase exp(-i T D_z(b)) for any dt; 4096 sampled amplitudes
    # are compared one by one with the oracle's energy of that basis index.
    ts = _dev()
    w = W.xyz_chain(n=27, nsteps=1, state=False)
    bonds = [(i, j, 0.0, 0.0, jz) for (i, j, jx, jy, jz) in w.bonds]
    _say("pure-z-27")
    H = ts.Hamiltonian(27, bonds, w.fields)
    x = torch.full((1 << 27,), 2.0 ** -13.5, dtype=torch.complex128, device="cuda")
    steps = 7
    H.evolve(x, w.dt, steps, 4)
    rng = np.random.default_rng(9)
    idx = rng.integers(0, 1 << 27, size=4096, dtype=np.int64)
    got = x[torch.from_numpy(idx).cuda()].cpu().numpy()
    e = oracle.energies(oracle.Hamiltonian(27, bonds, w.fields), "z", idx.astype(np.uint64))
    ref = 2.0 ** -13.5 * np.exp(-1j * w.dt * steps * e)
    assert np.abs(got - ref).max() < 1e-12 * 2.0 ** -13.5 * 10


def test_autotune_writes_cache_and_tuned_run_matches_oracle(tmp_path, monkeypatch):
    ts = _dev()
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("TSSPIN_TUNE_CACHE", str(cache))
    n = 17
    _say("autotune", n)
    rng = np.random.default_rng(1717)
    bonds, fields = D.random_xyz(rng, n, chain=True)
    H = ts.Hamiltonian(n, bonds, fields)
    cfg = H.autotune(ts.TS_C128, 4, use_cache=False)
    assert 10 <= cfg["tile_bits"] <= 13 and cfg["ms_per_step"] > 0
    import json
    ent = json.loads(cache.read_text())["entries"]
    assert any(e["n"] == n and e["dtype"] == 0 and e["order"] == 4 for e in ent)
    # a new context picks the cached configuration on first use
    H2 = ts.Hamiltonian(n, bonds, fields)
    assert H2.kernel_config(ts.TS_C128, 4)["tile_bits"] == cfg["tile_bits"]
    psi0 = D.random_state(rng, n)
    x = _gpu(psi0, C128)
    H2.evolve(x, 0.07, 2, 4)
    ref = oracle.evolve(oracle.Hamiltonian(n, bonds, fields), psi0, 0.07, 2, 4)
    assert _rel(x.cpu().numpy(), ref) < 1e-10


@pytest.mark.parametrize("dtype", [C128, C64])
@pytest.mark.parametrize("variant,rb", [("reg", 4), ("reg", 3), ("pipe", 4), ("pipe", 3), ("lds", 4)])
def test_sweep_variants_match_oracle(monkeypatch, variant, rb, dtype):
    # 2^10 tiles of 2^10 amplitudes: the pipelined grid is smaller than the tile count, so
    # its workgroups walk several tiles each
    ts = _dev()
    n, T, seed = 20, 10, 4242
    _say("variant", variant, rb, n, T, dtype, seed)
    monkeypatch.setenv("TSSPIN_SWEEP_KERNEL", variant)
    monkeypatch.setenv("TSSPIN_REG_BITS", str(rb))
    rng = np.random.default_rng(seed)
    bonds, fields = D.random_xyz(rng, n, chain=True)
    bonds += [(1, n - 2, 0.25, -0.35, 0.45)]
    psi0 = D.random_state(rng, n)
    H = ts.Hamiltonian(n, bonds, fields)
    code = ts.TS_C128 if dtype == C128 else ts.TS_C64
    H.set_tile_bits(code, T)
    cfg = H.kernel_config(code, 4)
    assert cfg["variant"] == {"reg": 0, "lds": 1, "pipe": 2}[variant] and cfg["reg_bits"] == rb
    x = _gpu(psi0, dtype)
    H.evolve(x, 0.05, 2, 4)
    torch.cuda.synchronize()
    ref = oracle.evolve(oracle.Hamiltonian(n, bonds, fields), psi0, 0.05, 2, 4)
    assert _rel(x.cpu().numpy().astype(np.complex128), ref) < TOL[dtype]


@pytest.mark.parametrize("dtype,T,rb", [(C128, 10, 4), (C128, 12, 4), (C128, 12, 3), (C64, 12, 4),
                                         (C64, 13, 3)])
def test_pipelined_sweep_bitwise_equals_one_tile_per_workgroup(monkeypatch, dtype, T, rb):
    # same arithmetic in the same order: the two launch shapes must agree to the bit
    ts = _dev()
    n, seed = 24, 99
    _say("pipe-vs-reg", n, T, rb, dtype, seed)
    monkeypatch.setenv("TSSPIN_REG_BITS", str(rb))
    w = W.xyz_chain(n=n, nsteps=1, state=False)
    code = ts.TS_C128 if dtype == C128 else ts.TS_C64
    g = torch.Generator(device="cpu").manual_seed(seed)
    psi = torch.polar(torch.full((1 << n,), 2.0 ** (-n / 2), dtype=torch.float64),
                      torch.rand(1 << n, dtype=torch.float64, generator=g) * 6.283).to(dtype).cuda()
    out = {}
    for variant in ("reg", "pipe"):
        monkeypatch.setenv("TSSPIN_SWEEP_KERNEL", variant)
        H = ts.Hamiltonian(n, w.bonds, w.fields)
        H.set_tile_bits(code, T)
        assert H.kernel_config(code, 4)["variant"] == (2 if variant == "pipe" else 0)
        x = psi.clone()
        H.evolve(x, w.dt, 2, 4)
        torch.cuda.synchronize()
        out[variant] = x.cpu()
    assert torch.equal(out["reg"], out["pipe"])


@pytest.mark.parametrize("dtype", [C128, C64])
@pytest.mark.parametrize("T", [12, 8])
def test_dipolar_sublattice_against_oracle(dtype, T):
    # 3 x 4 sub-lattice of the dipolar workload: all 66 pairs coupled (J^z = 1/r^3,
    # J^x = J^y = -J^z/2), Neel with site 0 flipped; resident (T = 12) and tiled (T = 8)
    ts = _dev()
    w = W.dipolar_lattice(rows=3, cols=4, nsteps=40)
    _say("dipolar-sub", w.n, T, dtype)
    code = ts.TS_C128 if dtype == C128 else ts.TS_C64
    H = ts.Hamiltonian(w.n, w.bonds, w.fields)
    H.set_tile_bits(code, T)
    x = _gpu(w.psi0, dtype)
    rec = H.evolve(x, w.dt, w.nsteps, 4, record=[("sz", 0), ("sz", 5), ("norm",)], rec_every=10)
    torch.cuda.synchronize()
    Ho = oracle.Hamiltonian(w.n, w.bonds, w.fields)
    psi = w.psi0.copy()
    ref = [[oracle.expect(Ho, psi, "sz", 0), oracle.expect(Ho, psi, "sz", 5), 1.0]]
    for _ in range(w.nsteps // 10):
        psi = oracle.evolve(Ho, psi, w.dt, 10, 4)
        ref.append([oracle.expect(Ho, psi, "sz", 0), oracle.expect(Ho, psi, "sz", 5),
                    oracle.expect(Ho, psi, "norm")])
    got = rec.cpu().numpy()
    # complex64: 40 steps of FP32 storage and butterflies (about 800 rounded stages per
    # amplitude); the observable bound is the 1e-5 absolute target for complex64
    tol = 1e-11 if dtype == C128 else 1e-5
    assert np.abs(got - np.array(ref)).max() < tol
    assert _rel(x.cpu().numpy().astype(np.complex128), psi) < TOL[dtype]


def test_dipolar_full_lattice_complex64_against_complex128():
    # N = 30 (5 x 6, 435 pairs): complex64 state (8 GiB) against the complex128 run
    # (16 GiB) on the same GPU; phase arguments and sums are FP64 in both
    ts = _dev()
    w = W.dipolar_lattice(nsteps=4)
    _say("dipolar-full", w.n, w.nsteps)
    obs = [("sz", 0), ("sz", 1), ("sz", 29), ("szsz", 0, 1), ("norm",)]
    out = {}
    for dtype in (C128, C64):
        x = torch.zeros(1 << w.n, dtype=dtype, device="cuda")
        x[w.extra["init_index"]] = 1.0
        H = ts.Hamiltonian(w.n, w.bonds, w.fields)
        rec = H.evolve(x, w.dt, w.nsteps, 4, record=obs, rec_every=1)
        torch.cuda.synchronize()
        out[dtype] = rec.cpu().numpy()
        del x
        torch.cuda.empty_cache()
    # the initial record is exact: site 0 is the flipped site (down), the norm is 1
    assert out[C128][0, 0] == -0.5 and out[C128][0, 4] == 1.0
    assert np.abs(out[C64] - out[C128]).max() < 1e-5
    assert abs(out[C128][-1, 4] - 1.0) < 1e-12


@pytest.mark.parametrize("dtype", [C128, C64])
def test_long_run_over_several_plan_chunks(dtype):
    # 75 unrecorded steps run as 32 + 32 + 11 step plans; the records every 25 steps cut
    # the run differently (25-step segments): both must match the oracle
    ts = _dev()
    n, T, dt, ns = 14, 10, 0.03, 75
    _say("chunks", n, T, ns, dtype)
    rng = np.random.default_rng(75)
    bonds, fields = D.random_xyz(rng, n, chain=True)
    psi0 = D.random_state(rng, n)
    H = ts.Hamiltonian(n, bonds, fields)
    H.set_tile_bits(ts.TS_C128 if dtype == C128 else ts.TS_C64, T)
    x, y = _gpu(psi0, dtype), _gpu(psi0, dtype)
    H.evolve(x, dt, ns, 4)
    rec = H.evolve(y, dt, ns, 4, record=[("sz", 0)], rec_every=25)
    torch.cuda.synchronize()
    ref = oracle.evolve(oracle.Hamiltonian(n, bonds, fields), psi0, dt, ns, 4)
    assert _rel(x.cpu().numpy().astype(np.complex128), ref) < TOL[dtype]
    assert _rel(y.cpu().numpy().astype(np.complex128), ref) < TOL[dtype]
    assert abs(float(rec[-1, 0]) - oracle.expect(oracle.Hamiltonian(n, bonds, fields), ref, "sz", 0)) < 10 * TOL[dtype]


def test_full_size_one_magnon_against_exact_dynamics():
    # N = 27 XXZ chain with z fields from one up spin (site 13): the exact dynamics stays in
    # the 27-dimensional one-magnon sector, a tight-binding matrix whose exponential is
    # computed directly.  The GPU result differs by Trotter error only, and halving dt
    # must cut it by ~16 (fourth order); checked on all 27 sector amplitudes of the 2^27.
    import scipy.linalg as sla

    ts = _dev()
    n, J, delta, T, k0 = 27, 1.0, 0.8, 1.0, 13
    _say("one-magnon", n)
    rng = np.random.default_rng(2713)
    hz = rng.uniform(-0.5, 0.5, n)
    bonds = [(i, i + 1, J, J, delta) for i in range(n - 1)]
    fields = np.zeros((n, 3))
    fields[:, 2] = hz
    M = np.zeros((n, n))
    for k in range(n):
        e = sum(delta * (-0.25 if k in (i, i + 1) else 0.25) for i in range(n - 1))
        e += sum(0.5 * hz[q] if q == k else -0.5 * hz[q] for q in range(n))
        M[k, k] = e
    for i in range(n - 1):
        M[i, i + 1] = M[i + 1, i] = J / 2
    cT = sla.expm(-1j * T * M)[:, k0]
    H = ts.Hamiltonian(n, bonds, fields)
    idx = torch.tensor([1 << k for k in range(n)], device="cuda")
    errs, leak = [], []
    for ns in (20, 40):
        x = torch.zeros(1 << n, dtype=C128, device="cuda")
        x[1 << k0] = 1.0
        H.evolve(x, T / ns, ns, 4)
        got = x[idx].cpu().numpy()
        errs.append(np.abs(got - cT).max())
        leak.append(1.0 - float(np.sum(np.abs(got) ** 2)))
        del x
        torch.cuda.empty_cache()
    assert errs[0] < 1e-5 and 10 < errs[0] / errs[1] < 22, errs
    assert max(abs(v) for v in leak) < 1e-9, leak


def test_complex64_autocorrelation_over_1000_steps():
    # the C(t) pair of the xyz-chain workload (N = 24 here, same recipe), 1000 time steps:
    # complex64 storage against complex128, |Delta C(t)| <= 1e-5 at every recorded step
    ts = _dev()
    w = W.xyz_chain(n=24, nsteps=1000, state=True)
    _say("c64-long", w.n, w.nsteps)
    c0 = W.sz_times(w.psi0, w.n, 0)
    out = {}
    for dtype in (C128, C64):
        H = ts.Hamiltonian(w.n, w.bonds, w.fields)
        a, c = _gpu(w.psi0, dtype), _gpu(c0, dtype)
        rec = H.evolve([a, c], w.dt, w.nsteps, 4, record=[("overlap_sz", 0, 0, 1), ("norm",)],
                       rec_every=50)
        torch.cuda.synchronize()
        out[dtype] = rec.cpu().numpy()
        del a, c
    C = {d: out[d][:, 0] + 1j * out[d][:, 1] for d in out}
    assert abs(C[C128][0] - 0.25) < 1e-12
    _say("  max |C64 - C128|", float(np.abs(C[C64] - C[C128]).max()))
    assert np.abs(C[C64] - C[C128]).max() < 1e-5
    assert np.abs(out[C128][:, 2] - 1.0).max() < 1e-10


@pytest.mark.parametrize("T", [11, 12])
def test_half_lds_sweep_bitwise_equals_default(monkeypatch, T):
    # the complex128 variant that transposes real and imaginary parts through a buffer of
    # half the size runs the same arithmetic: results must agree to the bit, also for the
    # adjoint's paired ping-pong launches (the light-cone reverse pass, which would run
    # here otherwise, uses neither kernel and sums with atomic adds)
    ts = _dev()
    n, seed = 24, 2424
    _say("half-vs-reg", n, T, seed)
    monkeypatch.setenv("TSSPIN_ADJ_CONE", "0")
    w = W.xyz_chain(n=n, nsteps=1, state=False)
    g = torch.Generator(device="cpu").manual_seed(seed)
    psi = torch.polar(torch.full((1 << n,), 2.0 ** (-n / 2), dtype=torch.float64),
                      torch.rand(1 << n, dtype=torch.float64, generator=g) * 6.283).to(C128).cuda()
    out = {}
    for variant in ("reg", "half"):
        monkeypatch.setenv("TSSPIN_SWEEP_KERNEL", variant)
        H = ts.Hamiltonian(n, w.bonds, w.fields)
        H.set_tile_bits(ts.TS_C128, T)
        assert H.kernel_config(ts.TS_C128, 4)["variant"] == (3 if variant == "half" else 0)
        x = psi.clone()
        H.evolve(x, w.dt, 2, 4)
        torch.cuda.synchronize()
        grads = H.adjoint(psi, w.dt, 3, 4, ("sz", 0))
        out[variant] = (x.cpu(), grads)
    assert torch.equal(out["reg"][0], out["half"][0])
    assert out["reg"][1][0] == out["half"][1][0]
    assert np.array_equal(out["reg"][1][1], out["half"][1][1])
    assert np.array_equal(out["reg"][1][2], out["half"][1][2])


@pytest.mark.parametrize("axis", ["x", "y"])
def test_full_size_single_axis_eigenstate_phase(axis):
    # A Hamiltonian with only x (or only y) terms is evolved exactly by the Trotter product
    # for any dt, and a product of single-spin eigenstates of S^x (S^y) is one of its
    # eigenstates: psi(T) = exp(-i T E) psi(0) on all 2^27 amplitudes, with
    # E = sum_j h_j m_j + sum_bonds J m_i m_j and m_j = +-1/2 the chosen eigenvalues.
    # In the (down, up) order S^x = [[0,1],[1,0]]/2 and S^y = [[0,i],[-i,0]]/2: the +1/2
    # eigenvectors are (1, 1) and (1, -i), the -1/2 ones (1, -1) and (1, i), over sqrt 2.
    ts = _dev()
    n, T, ns = 27, 0.7, 13
    _say("single-axis", axis, n)
    rng = np.random.default_rng(27 + (axis == "y"))
    a = 0 if axis == "x" else 1
    J = rng.uniform(0.5, 1.5, n - 1)
    h = rng.uniform(-1.0, 1.0, n)
    bonds = [(i, i + 1, *(J[i] if k == a else 0.0 for k in range(3))) for i in range(n - 1)]
    bonds += [(0, n - 1, *(0.3 if k == a else 0.0 for k in range(3)))]
    fields = np.zeros((n, 3))
    fields[:, a] = h
    m = rng.choice([-0.5, 0.5], n)
    E = float(np.sum(h * m) + np.sum(J * m[:-1] * m[1:]) + 0.3 * m[0] * m[-1])
    # up-component factor of each spin: x: +-1 for m = +-1/2; y: -i for m = +1/2, +i for -1/2
    up = np.where(m > 0, 1.0, -1.0).astype(complex) if axis == "x" else np.where(m > 0, -1j, 1j)
    # psi0(b) = 2^(-n/2) prod over set bits j of up[j], built as an outer product on the GPU
    x = torch.ones(1, dtype=C128, device="cuda")
    for j in range(n):   # bit j = spin j; higher spins vary slower
        f = torch.tensor([1.0, up[j]], dtype=C128, device="cuda") / np.sqrt(2.0)
        x = torch.kron(f, x)
    psi0 = x.clone()
    H = ts.Hamiltonian(n, bonds, fields)
    H.evolve(x, T / ns, ns, 4)
    torch.cuda.synchronize()
    ratio = x * psi0.conj() * (2.0 ** n)     # |psi0(b)|^2 = 2^-n
    target = complex(np.exp(-1j * T * E))
    err = float((ratio - target).abs().max())
    assert err < 1e-11, err


@pytest.fixture(scope="module")
def xyz27_u2_block():
    """The benchmark's N = 27 xyz chain and random-phase state, and one second-order block
    U2(a dt) of it by the FP64 oracle (a = 1/(4 - 4^(1/3)), the first block of a
    fourth-order step)."""
    w = W.xyz_chain(n=27, nsteps=1, state=True)
    a = oracle.suzuki_a()
    ref = oracle.evolve(oracle.Hamiltonian(27, w.bonds, w.fields), w.psi0, a * w.dt, 1, 2)
    return w, a, ref


@pytest.mark.parametrize("dtype,mode", [(C128, 0), (C128, 2), (C64, -1)])
def test_full_size_benchmark_state_against_oracle(monkeypatch, xyz27_u2_block, dtype, mode):
    """The benchmarked Hamiltonian (all 26 bonds, every field) and state at N = 27: one U2(a dt)
    block on the GPU against the oracle on all 2^27 amplitudes, in the ping-pong (mode 0)
    and light-cone (mode 2) forms for complex128 and the default form for complex64."""
    ts = _dev()
    w, a, ref = xyz27_u2_block
    if mode >= 0:
        monkeypatch.setenv("TSSPIN_CONE", str(mode))
    _say("benchmark-state-27", dtype, "cone mode", mode)
    H = ts.Hamiltonian(27, w.bonds, w.fields)
    code = ts.TS_C128 if dtype == C128 else ts.TS_C64
    _, used = H.cone_plan(code, a * w.dt, 1, 2)
    if mode >= 0:
        assert used == (mode == 2)
    x = _gpu(w.psi0, dtype)
    H.evolve(x, a * w.dt, 1, 2)
    got = x.cpu().numpy().astype(np.complex128)
    del x
    err = _rel(got, ref)
    _say("  light-cone used:", used, "rel L2", err)
    assert err < TOL[dtype]


@pytest.mark.parametrize("n,T,dtype", [(17, 13, C128), (17, 13, C64), (18, 14, C64)])
def test_wide_tile_parity(n, T, dtype):
    """Tiles of 2^13 and 2^14 amplitudes (the widths chosen where they save a bit group)
    against the oracle, with bonds across the tile boundary."""
    ts = _dev()
    seed = 700 + n + 100 * T
    _say("wide-tile", n, T, dtype, seed)
    rng = np.random.default_rng(seed)
    bonds, fields = D.random_xyz(rng, n, chain=True)
    bonds += [(0, n - 1, 0.3, -0.2, 0.5), (3, n - 4, -0.4, 0.6, 0.1)]
    psi0 = D.random_state(rng, n)
    H = ts.Hamiltonian(n, bonds, fields)
    H.set_tile_bits(ts.TS_C128 if dtype == C128 else ts.TS_C64, T)
    x = _gpu(psi0, dtype)
    H.evolve(x, 0.07, 3, 4)
    torch.cuda.synchronize()
    ref = oracle.evolve(oracle.Hamiltonian(n, bonds, fields), psi0, 0.07, 3, 4)
    assert _rel(x.cpu().numpy().astype(np.complex128), ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", [C128, C64])
def test_dipolar_3x7_default_width_against_oracle(dtype):
    """3 x 7 dipolar lattice (all 210 pairs) at the library's default tile width for it
    (complex64: 2^13, where 2^12 would need one more bit group) against the oracle."""
    ts = _dev()
    w = W.dipolar_lattice(rows=3, cols=7, nsteps=2)
    _say("dipolar-3x7", dtype)
    code = ts.TS_C128 if dtype == C128 else ts.TS_C64
    H = ts.Hamiltonian(w.n, w.bonds, w.fields)
    assert H.kernel_config(code, 4)["tile_bits"] == (12 if dtype == C128 else 13)
    x = _gpu(w.psi0, dtype)
    rec = H.evolve(x, w.dt, w.nsteps, 4, record=[("sz", 0), ("energy",)], rec_every=2)
    torch.cuda.synchronize()
    Ho = oracle.Hamiltonian(w.n, w.bonds, w.fields)
    ref = oracle.evolve(Ho, w.psi0, w.dt, w.nsteps, 4)
    assert _rel(x.cpu().numpy().astype(np.complex128), ref) < TOL[dtype]
    got = rec.cpu().numpy()
    assert abs(got[-1, 0] - oracle.expect(Ho, ref, "sz", 0)) < (1e-12 if dtype == C128 else 2e-6)
    assert abs(got[-1, 1] - oracle.expect(Ho, ref, "energy")) < (1e-11 if dtype == C128 else 2e-5)


@pytest.mark.parametrize("dtype", [C128, C64])
@pytest.mark.parametrize("rb", [4, 3])
def test_energy_table_sweeps_match_oracle(monkeypatch, dtype, rb):
    """Phase steps from the per-axis energy tables in device memory (Sec. 3.1's precomputed
    phases, variant 5): a chain with fields on every axis plus two long bonds, tiles of 2^10
    (three bit groups at N = 20), against the oracle."""
    ts = _dev()
    n, T, seed = 20, 10, 5151
    _say("etab", n, T, rb, dtype, seed)
    monkeypatch.setenv("TSSPIN_SWEEP_KERNEL", "etab")
    monkeypatch.setenv("TSSPIN_REG_BITS", str(rb))
    rng = np.random.default_rng(seed)
    bonds, fields = D.random_xyz(rng, n, chain=True)
    bonds += [(1, n - 2, 0.25, -0.35, 0.45), (3, 11, -0.6, 0.3, 0.2)]
    psi0 = D.random_state(rng, n)
    H = ts.Hamiltonian(n, bonds, fields)
    code = ts.TS_C128 if dtype == C128 else ts.TS_C64
    H.set_tile_bits(code, T)
    cfg = H.kernel_config(code, 4)
    assert cfg["variant"] == 5 and cfg["reg_bits"] == rb
    x = _gpu(psi0, dtype)
    H.evolve(x, 0.05, 3, 4)
    torch.cuda.synchronize()
    ref = oracle.evolve(oracle.Hamiltonian(n, bonds, fields), psi0, 0.05, 3, 4)
    assert _rel(x.cpu().numpy().astype(np.complex128), ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", [C128, C64])
def test_energy_table_dipolar_sublattice_against_oracle(monkeypatch, dtype):
    """All 66 dipolar pairs of the 3 x 4 sub-lattice with the energies read from the tables,
    tiled at T = 8, 40 steps with <S^z> recorded, against the oracle (the same bounds as the
    factorised phase step)."""
    ts = _dev()
    monkeypatch.setenv("TSSPIN_SWEEP_KERNEL", "etab")
    w = W.dipolar_lattice(rows=3, cols=4, nsteps=40)
    _say("etab-dipolar-sub", w.n, dtype)
    code = ts.TS_C128 if dtype == C128 else ts.TS_C64
    H = ts.Hamiltonian(w.n, w.bonds, w.fields)
    H.set_tile_bits(code, 8)
    x = _gpu(w.psi0, dtype)
    rec = H.evolve(x, w.dt, w.nsteps, 4, record=[("sz", 0), ("sz", 5)], rec_every=10)
    torch.cuda.synchronize()
    Ho = oracle.Hamiltonian(w.n, w.bonds, w.fields)
    psi = w.psi0.copy()
    ref = [[oracle.expect(Ho, psi, "sz", 0), oracle.expect(Ho, psi, "sz", 5)]]
    for _ in range(w.nsteps // 10):
        psi = oracle.evolve(Ho, psi, w.dt, 10, 4)
        ref.append([oracle.expect(Ho, psi, "sz", 0), oracle.expect(Ho, psi, "sz", 5)])
    tol = 1e-11 if dtype == C128 else 1e-5
    assert np.abs(rec.cpu().numpy() - np.array(ref)).max() < tol
    assert _rel(x.cpu().numpy().astype(np.complex128), psi) < TOL[dtype]


def test_energy_table_matches_factorised_phase_at_n24(monkeypatch):
    """The two phase-step forms on the N = 24 xyz chain (complex128, two steps): the same
    product computed two ways (tables of factors against sin/cos of the stored energy)."""
    ts = _dev()
    n, seed = 24, 2424
    _say("etab-vs-tab", n, seed)
    w = W.xyz_chain(n=n, nsteps=1, state=False)
    g = torch.Generator(device="cpu").manual_seed(seed)
    psi = torch.polar(torch.full((1 << n,), 2.0 ** (-n / 2), dtype=torch.float64),
                      torch.rand(1 << n, dtype=torch.float64, generator=g) * 6.283).to(C128).cuda()
    out = {}
    for variant in ("reg", "etab"):
        monkeypatch.setenv("TSSPIN_SWEEP_KERNEL", variant)
        H = ts.Hamiltonian(n, w.bonds, w.fields)
        H.set_tile_bits(ts.TS_C128, 12)
        x = psi.clone()
        H.evolve(x, w.dt, 2, 4)
        torch.cuda.synchronize()
        out[variant] = x.cpu().numpy()
    assert _rel(out["etab"], out["reg"]) < 1e-12
