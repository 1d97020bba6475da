"""GPU parity of the light-cone sweeps (needs an MI355X).

The light-cone path is forced (TSSPIN_CONE=2) and compared with the FP64 oracle, with the
ping-pong sweeps of the same library (TSSPIN_CONE=0) and across storage precisions.  Every
case prints its name, size and seed before touching the GPU.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
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


def _ham(ts, monkeypatch, mode, n, bonds, fields):
    monkeypatch.setenv("TSSPIN_CONE", str(mode))
    return ts.Hamiltonian(n, bonds, fields)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("n,order,nsteps", [(13, 4, 2), (14, 2, 3), (16, 4, 2), (17, 1, 4), (20, 4, 1)])
def test_cone_parity_with_oracle(monkeypatch, n, order, nsteps, dtype):
    ts = _dev()
    seed = 900 + 10 * n + order
    _say("cone vs oracle", n, order, nsteps, dtype, seed)
    rng = np.random.default_rng(seed)
    bonds, fields = D.random_xyz(rng, n, chain=True)
    psi0 = D.random_state(rng, n)
    H = _ham(ts, monkeypatch, 2, n, bonds, fields)
    sweeps, used = H.cone_plan(ts.TS_C128, 0.07, nsteps, order)
    _say("  sweeps", len(sweeps), "light-cone path used:", used)
    assert used
    x = torch.from_numpy(psi0).to(dtype).cuda()
    H.evolve(x, 0.07, nsteps, order)
    torch.cuda.synchronize()
    ref = oracle.evolve(oracle.Hamiltonian(n, bonds, fields), psi0, 0.07, nsteps, order)
    err = _rel(x.cpu().numpy().astype(np.complex128), ref)
    _say("  rel L2", err)
    assert err < (1e-10 if dtype == torch.complex128 else 1e-5)


@pytest.mark.parametrize("n", [21, 24])
def test_cone_matches_ping_pong_with_records(monkeypatch, n):
    """Light-cone and ping-pong sweeps of the same library agree to rounding, including the
    observables recorded at every step (segments of one step, each back at the home layout)."""
    ts = _dev()
    seed = 40 + n
    _say("cone vs ping-pong", n, seed)
    rng = np.random.default_rng(seed)
    bonds = [(i, i + 1, *rng.uniform(0.5, 1.5, 3)) for i in range(n - 1)]
    fields = np.zeros((n, 3))
    fields[:, 2] = rng.uniform(-0.5, 0.5, n)
    g = torch.Generator().manual_seed(seed)
    psi = torch.polar(torch.full((1 << n,), 2.0 ** (-n / 2), dtype=torch.float64),
                      torch.rand(1 << n, dtype=torch.float64, generator=g) * 6.283).cuda()
    rec = [("sz", 0), ("szsz", 0, n - 1), ("sx", n // 2), ("norm",)]
    out = {}
    for mode in (0, 2):
        H = _ham(ts, monkeypatch, mode, n, bonds, fields)
        x = psi.clone()
        r = H.evolve(x, 0.02, 6, 4, record=rec)
        torch.cuda.synchronize()
        out[mode] = (x, r)
    d = float((out[0][0] - out[2][0]).abs().max())
    dr = float((out[0][1] - out[2][1]).abs().max())
    _say("  max |dpsi|", d, "max |drec|", dr)
    assert d < 1e-11 * float(out[0][0].abs().max()) and dr < 1e-12


def test_cone_complex64_close_to_complex128_at_n24(monkeypatch):
    ts = _dev()
    n, seed = 24, 77
    _say("cone c64 vs c128", n, seed)
    rng = np.random.default_rng(seed)
    bonds = [(i, i + 1, *rng.uniform(0.5, 1.5, 3)) for i in range(n - 1)]
    fields = np.zeros((n, 3))
    fields[:, 2] = rng.uniform(-0.5, 0.5, n)
    H = _ham(ts, monkeypatch, 2, n, bonds, fields)
    g = torch.Generator().manual_seed(seed)
    psi = torch.polar(torch.full((1 << n,), 2.0 ** (-n / 2), dtype=torch.float64),
                      torch.rand(1 << n, dtype=torch.float64, generator=g) * 6.283).cuda()
    a = psi.clone()
    b = psi.to(torch.complex64)
    ra = H.evolve(a, 0.02, 20, 4, record=[("sz", 0)])
    rb = H.evolve(b, 0.02, 20, 4, record=[("sz", 0)])
    torch.cuda.synchronize()
    err = float((ra - rb).abs().max())
    _say("  max |d<Sz0>|", err)
    assert err < 1e-5


@pytest.mark.parametrize("T,order,nsteps,every", [(11, 4, 5, 2), (12, 2, 40, 8), (12, 4, 70, 35)])
def test_cone_tile_widths_and_long_segments(monkeypatch, T, order, nsteps, every):
    """Tile width 11 and runs longer than one plan chunk (32 steps), with records every few
    steps: light-cone and ping-pong sweeps of the same library agree to rounding."""
    ts = _dev()
    n, seed = 18, 300 + T + nsteps
    _say("cone long", n, T, order, nsteps, every, seed)
    rng = np.random.default_rng(seed)
    bonds, fields = D.random_xyz(rng, n, chain=True)
    psi0 = D.random_state(rng, n)
    out = {}
    for mode in (0, 2):
        H = _ham(ts, monkeypatch, mode, n, bonds, fields)
        H.set_tile_bits(ts.TS_C128, T)
        x = torch.from_numpy(psi0).cuda()
        r = H.evolve(x, 0.03, nsteps, order, record=[("sz", 3), ("sx", 9), ("norm",)], rec_every=every)
        torch.cuda.synchronize()
        out[mode] = (x.cpu().numpy(), r.cpu().numpy())
    err = _rel(out[2][0], out[0][0])
    derr = float(np.abs(out[2][1] - out[0][1]).max())
    _say("  rel L2 cone vs ping-pong", err, "max |drec|", derr)
    assert err < 1e-11 and derr < 1e-12


@pytest.mark.parametrize("T", [11, 12])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_cone_all_to_all_with_oracle(monkeypatch, T, dtype):
    """All-to-all dipolar 2x7 lattice (N = 14, 91 pairs) in the light-cone form at tile
    widths 11 and 12, against the FP64 oracle."""
    ts = _dev()
    from paper_1305_0036_amd import workloads as W
    w = W.dipolar_lattice(2, 7, nsteps=2)
    _say("cone all-to-all vs oracle", w.n, T, dtype)
    H = _ham(ts, monkeypatch, 2, w.n, w.bonds, w.fields)
    code = ts.TS_C128 if dtype == torch.complex128 else ts.TS_C64
    H.set_tile_bits(code, T)
    sweeps, used = H.cone_plan(code, 0.05, 2, 4, tile_bits=T)
    _say("  sweeps", len(sweeps), "used", used)
    assert used
    rng = np.random.default_rng(77 + T)
    psi0 = D.random_state(rng, w.n)
    x = torch.from_numpy(psi0).to(dtype).cuda()
    H.evolve(x, 0.05, 2, 4)
    torch.cuda.synchronize()
    ref = oracle.evolve(oracle.Hamiltonian(w.n, w.bonds, w.fields), psi0, 0.05, 2, 4)
    err = _rel(x.cpu().numpy().astype(np.complex128), ref)
    _say("  rel L2", err)
    assert err < (1e-10 if dtype == torch.complex128 else 1e-5)


@pytest.mark.parametrize("case", ["dipolar-4x6", "hub-24"])
def test_cone_matches_ping_pong_beyond_chains(monkeypatch, case):
    """Non-chain Hamiltonians at N = 24 in complex128: the all-to-all dipolar 4x6 lattice
    (which the cost model sends to the light-cone form) and a chain with spin 0 coupled to
    every spin (phase steps reaching 12 outside spins, the kernel's row limit).  Light-cone
    and ping-pong sweeps of the same library agree to rounding."""
    ts = _dev()
    from paper_1305_0036_amd import workloads as W
    if case == "dipolar-4x6":
        w = W.dipolar_lattice(4, 6, nsteps=2)
        n, bonds, fields = w.n, w.bonds, w.fields
    else:
        n = 24
        rng = np.random.default_rng(31)
        pairs = sorted({(i, i + 1) for i in range(n - 1)} | {(0, j) for j in range(1, n)})
        bonds = [(i, j, *rng.uniform(0.5, 1.5, 3)) for i, j in pairs]
        fields = np.zeros((n, 3))
        fields[:, 2] = rng.uniform(-0.5, 0.5, n)
    _say("cone vs ping-pong", case, n)
    g = torch.Generator().manual_seed(5)
    psi = torch.polar(torch.full((1 << n,), 2.0 ** (-n / 2), dtype=torch.float64),
                      torch.rand(1 << n, dtype=torch.float64, generator=g) * 6.283).cuda()
    out = {}
    for mode in (0, 2):
        H = _ham(ts, monkeypatch, mode, n, bonds, fields)
        _, used = H.cone_plan(ts.TS_C128, 0.02, 2, 4)
        _say("  mode", mode, "light-cone used:", used)
        assert used == (mode == 2)
        x = psi.clone()
        H.evolve(x, 0.02, 2, 4)
        torch.cuda.synchronize()
        out[mode] = x
    err = float(torch.linalg.norm(out[2] - out[0]) / torch.linalg.norm(out[0]))
    _say("  rel L2", err)
    assert err < 1e-11


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_records_folded_into_the_last_sweep(monkeypatch, dtype):
    """Records of the light-cone form: norm, S^z, S^zS^z, M^z and the two overlaps (bra
    evolved before the ket) are accumulated by the last sweep of each vector's segment; S^x
    and the energy by a reduction after it.  Against separate reductions for everything
    (TSSPIN_NO_FUSE=1: the same states, so differences are summation order only) and against
    the oracle, for the C(t) pair of the benchmark's recipe at N = 20, three records of two
    steps each."""
    ts = _dev()
    from paper_1305_0036_amd import workloads as W
    n = 20
    w = W.xyz_chain(n=n, nsteps=6, state=True)
    _say("fused records", n, dtype)
    a0 = w.psi0
    c0 = W.sz_times(a0, n, 0)
    rec = [("overlap_sz", 0, 0, 1), ("norm", 1), ("sz", 3, 0), ("szsz", 2, 7, 1), ("mz", 0),
           ("overlap", 0, 1), ("sx", 4, 1), ("energy", 0)]
    out = {}
    for fuse in ("1", "0"):
        monkeypatch.setenv("TSSPIN_NO_FUSE", "0" if fuse == "1" else "1")
        H = _ham(ts, monkeypatch, 2, n, w.bonds, w.fields)
        a = torch.from_numpy(a0).to(dtype).cuda()
        c = torch.from_numpy(c0).to(dtype).cuda()
        out[fuse] = (H.evolve([a, c], w.dt, 6, 4, record=rec, rec_every=2).cpu().numpy(), a.cpu(), c.cpu())
    r1, r0 = out["1"][0], out["0"][0]
    assert torch.equal(out["1"][1], out["0"][1]) and torch.equal(out["1"][2], out["0"][2])
    tol = 1e-13 if dtype == torch.complex128 else 1e-6
    assert np.abs(r1 - r0).max() < tol
    # oracle: the same records from the oracle's states (complex128 only)
    if dtype == torch.complex128:
        Ho = oracle.Hamiltonian(n, w.bonds, w.fields)
        a, c = a0, c0
        for k in range(4):
            if k:
                a = oracle.evolve(Ho, a, w.dt, 2, 4)
                c = oracle.evolve(Ho, c, w.dt, 2, 4)
            ov = oracle.expect(Ho, c, "overlap_sz", 0, other=a)
            exp = [ov.real, ov.imag, oracle.expect(Ho, c, "norm"), oracle.expect(Ho, a, "sz", 3),
                   oracle.expect(Ho, c, "szsz", 2, 7), oracle.expect(Ho, a, "mz"),
                   np.vdot(a, c).real, np.vdot(a, c).imag, oracle.expect(Ho, c, "sx", 4),
                   oracle.expect(Ho, a, "energy")]
            assert np.abs(r1[k] - np.array(exp)).max() < 1e-11, k
