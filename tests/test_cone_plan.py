"""Light-cone plans of libtsspin, checked on the CPU (no GPU needed).

`ts_cone_describe` returns the light-cone form of a segment: sweeps over windows of spins,
each a list of butterflies on some spins and phase steps restricted to some terms, plus the
memory layout of every tile.  A test-only NumPy interpreter applies the operations in
order and the result is compared with the FP64 oracle; the bookkeeping is checked too:
every spin takes every layer once, every field / quarter-turn / bond term of every level
runs once, every tile holds the low memory bits, stores only permute a tile's own bits and
the layout ends where it started.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1305_0036_amd import tsspin
from tests import dense_ref as D
from tests.test_plan import _wht_bits


def _spins(mask, n):
    return [q for q in range(n) if (mask >> q) & 1]


def interpret_cone(sweeps, n, bonds, fields, psi, low_bits):
    """Apply a light-cone plan to psi (logical spin order); check its layout rules."""
    psi = np.array(psi, dtype=complex)
    idx = np.arange(1 << n, dtype=np.int64)
    bit = [((idx >> q) & 1) for q in range(n)]
    s = [b - 0.5 for b in bit]
    pos = list(range(n))
    layers = np.zeros(n, dtype=int)
    own_seen, bond_seen = set(), set()
    for sw in sweeps:
        tile = sw["tile"]
        mem = {p for _, p, _ in tile}
        assert {p for _, _, p in tile} == mem, "a store may only permute the tile's bits"
        assert set(range(low_bits)) <= mem, "every tile holds the low memory bits"
        assert all(pos[q] == p for q, p, _ in tile), "load layout"
        win = {q for q, _, _ in tile}
        assert sw["window"] == sum(1 << q for q in win)
        for op in sw["ops"]:
            if op["kind"] == "bfly":
                assert set(_spins(op["spins"], n)) <= win
                _wht_bits(psi, n, op["spins"])
                for q in _spins(op["spins"], n):
                    layers[q] += 1
                continue
            lv, ax, tau, c = op["level"], op["axis"], op["tau"], op["qturn"]
            ph = np.full(1 << n, 2.0 ** (-op["half_scale"] / 2) * np.exp(1j * np.pi * op["eighths"] / 4))
            for q in _spins(op["own"], n):
                assert q in win and layers[q] == lv
                assert (lv, q) not in own_seen
                own_seen.add((lv, q))
                ph = ph * (1j ** ((c * bit[q]) % 4))
                if ax < 3:
                    ph = ph * np.exp(-1j * tau * fields[q][ax] * s[q])
            for b in _spins(op["bonds"], len(bonds)):
                i, j = bonds[b][0], bonds[b][1]
                assert layers[i] == lv and layers[j] == lv and (i in win or j in win)
                assert (lv, b) not in bond_seen
                bond_seen.add((lv, b))
                if ax < 3:
                    ph = ph * np.exp(-1j * tau * bonds[b][2 + ax] * s[i] * s[j])
            psi *= ph
        for q, _, p in tile:
            pos[q] = p
    assert pos == list(range(n)), "the layout ends where it started"
    return psi, layers, own_seen, bond_seen


@pytest.mark.parametrize("order", [1, 2, 4])
@pytest.mark.parametrize("n,T,s,nsteps,adv", [(9, 6, 2, 2, 0), (10, 6, 2, 1, 0), (11, 7, 3, 3, 0),
                                              (12, 8, 4, 2, 0), (13, 8, 4, 1, 2), (14, 9, 4, 2, 0)])
def test_cone_plan_matches_oracle(order, n, T, s, nsteps, adv):
    rng = np.random.default_rng(7000 + 100 * n + 10 * T + order)
    bonds, fields = D.random_xyz(rng, n, chain=True)
    Hl = tsspin.Hamiltonian(n, bonds, fields)
    Ho = oracle.Hamiltonian(n, bonds, fields)
    psi = D.random_state(rng, n)
    dt = 0.09
    for dtype in (tsspin.TS_C128, tsspin.TS_C64):
        sweeps, _ = Hl.cone_plan(dtype, dt, nsteps, order, tile_bits=T, low_bits=s, max_adv=adv)
        pp = Hl.plan(dtype, dt, nsteps, order, tile_bits=T)
        got, layers, own, bnd = interpret_cone(sweeps, n, bonds, fields, psi, s)
        m = len({lv for lv, _ in own}) - 1   # levels 0..m
        assert (layers == m).all()
        assert len(own) == n * (m + 1) and len(bnd) == len(bonds) * (m + 1)
        ref = oracle.evolve(Ho, psi, dt, nsteps, order)
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12
        if adv:
            for sw in sweeps:
                per = {}
                for op in sw["ops"]:
                    if op["kind"] == "bfly":
                        for q in _spins(op["spins"], n):
                            per[q] = per.get(q, 0) + 1
                assert max(per.values(), default=0) <= adv
        if not adv:  # fewer passes over the state than the ping-pong plan
            assert len(sweeps) < len(pp)


def test_cone_plan_sizes_of_the_n27_chain():
    """The xyz chain at N = 27, T = 12: nine passes per fourth-order step (the ping-pong
    plan needs 41), every stage program within the kernel's limits."""
    rng = np.random.default_rng(5)
    bonds = [(i, i + 1, *rng.uniform(0.5, 1.5, 3)) for i in range(26)]
    fields = np.zeros((27, 3))
    fields[:, 2] = rng.uniform(-0.5, 0.5, 27)
    H = tsspin.Hamiltonian(27, bonds, fields)
    sweeps, _ = H.cone_plan(tsspin.TS_C128, 0.02, 1, 4)
    assert len(sweeps) == 9
    assert len(H.plan(tsspin.TS_C128, 0.02, 1, 4)) == 41
    for sw in sweeps:
        assert 0 < sw["stages"] <= 192 and 0 <= sw["transposes"] <= sw["stages"]
        assert sum(op["kind"] == "phase" for op in sw["ops"]) <= 32


def test_cone_plan_refused_for_a_small_register():
    H = tsspin.Hamiltonian(8, [(i, i + 1, 1.0, 1.0, 1.0) for i in range(7)], None)
    with pytest.raises(tsspin.TsError):
        H.cone_plan(tsspin.TS_C128, 0.05, 1, 4)   # 8 spins fit one tile of the default width


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("n,T", [(11, 8), (11, 9), (11, 10)])
def test_cone_plan_all_to_all_matches_oracle(order, n, T):
    """Every pair coupled (55 bonds at N = 11): the light-cone form of an all-to-all
    Hamiltonian, interpreted on the CPU, against the FP64 oracle."""
    rng = np.random.default_rng(8100 + 10 * n + T + order)
    bonds = [(i, j, *rng.uniform(-1.0, 1.0, 3)) for i in range(n) for j in range(i + 1, n)]
    fields = rng.uniform(-0.5, 0.5, (n, 3))
    Hl = tsspin.Hamiltonian(n, bonds, fields)
    psi = D.random_state(rng, n)
    sweeps, _ = Hl.cone_plan(tsspin.TS_C128, 0.05, 2, order, tile_bits=T, low_bits=4)
    got, layers, own, bnd = interpret_cone(sweeps, n, bonds, fields, psi, 4)
    m = len({lv for lv, _ in own}) - 1
    assert (layers == m).all() and len(bnd) == len(bonds) * (m + 1)
    ref = oracle.evolve(oracle.Hamiltonian(n, bonds, fields), psi, 0.05, 2, order)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12


def _outside_partners(sweep, bonds):
    """Largest number of distinct outside spins that one phase step's bonds reach."""
    win = {q for q, _, _ in sweep["tile"]}
    worst = 0
    for op in sweep["ops"]:
        if op["kind"] != "phase":
            continue
        ext = set()
        for b in _spins(op["bonds"], len(bonds)):
            i, j = bonds[b][0], bonds[b][1]
            ext |= {i, j} - win
        worst = max(worst, len(ext))
    return worst


def test_cone_refused_when_a_step_reaches_too_many_outside_spins():
    """A light-cone phase step selects its workgroup row by the bits of the outside spins its
    bonds reach; the kernel holds 12 such bits.  Plans that need more are never chosen (the
    ping-pong sweeps run instead), here for the all-to-all dipolar 5x5 lattice (N = 25)."""
    from paper_1305_0036_amd import workloads as W
    w = W.dipolar_lattice(5, 5, nsteps=1)
    H = tsspin.Hamiltonian(w.n, w.bonds, w.fields)
    for dtype in (tsspin.TS_C128, tsspin.TS_C64):
        _, used = H.cone_plan(dtype, w.dt, 1, 4)
        assert not used


@pytest.mark.parametrize("graph,n,refused", [("random", 22, False), ("hub", 24, False), ("hub", 26, True)])
def test_cone_row_limit_on_long_range_graphs(monkeypatch, graph, n, refused):
    """Chain plus long-range bonds (<= 63 bonds, so the plan lists them): random pairs, or
    spin 0 coupled to every spin.  Whenever the library would run the light-cone form, no
    phase step reaches more than 12 outside spins; the hub at N = 26 needs 14 and is refused,
    at N = 24 it needs exactly 12 and is kept."""
    monkeypatch.setenv("TSSPIN_CONE", "2")
    pairs = {(i, i + 1) for i in range(n - 1)}
    rng = np.random.default_rng(31)
    if graph == "random":
        while len(pairs) < 63:
            i, j = sorted(rng.choice(n, 2, replace=False))
            pairs.add((int(i), int(j)))
    else:
        pairs |= {(0, j) for j in range(1, n)}
    bonds = [(i, j, *rng.uniform(0.5, 1.5, 3)) for i, j in sorted(pairs)]
    H = tsspin.Hamiltonian(n, bonds, None)
    sweeps, used = H.cone_plan(tsspin.TS_C128, 0.02, 1, 4)
    worst = max(_outside_partners(sw, bonds) for sw in sweeps)
    assert worst <= 12 or not used
    assert used == (not refused)


@pytest.mark.parametrize("n,T,s,nsteps", [(11, 7, 3, 3), (12, 8, 4, 2)])
def test_light_cone_reverse_pass_gradient(n, T, s, nsteps):
    """The adjoint's light-cone reverse pass, run by the NumPy interpreter: psi(T) and
    lambda = S^z_0 psi(T) go through the light-cone plan of the inverse chain (for order 4
    the chain with -dt), and after every phase step each of its terms gains
    -2 tau / 2^e * sum_b f(b) Im(conj(lambda_b) psi_b), with e the butterflies' gain not yet
    paid back (spin-layers applied minus the steps' half_scale).  Against the oracle's
    forward-mode gradient; psi returns to psi0 and e to 0."""
    rng = np.random.default_rng(900 + n)
    bonds, fields = D.random_xyz(rng, n, chain=True)
    psi0 = D.random_state(rng, n)
    dt, order = 0.07, 4
    Ho = oracle.Hamiltonian(n, bonds, fields)
    Hl = tsspin.Hamiltonian(n, bonds, fields)
    psi = oracle.evolve(Ho, psi0, dt, nsteps, order)
    idx = np.arange(1 << n, dtype=np.int64)
    bit = [((idx >> q) & 1) for q in range(n)]
    sv = [b - 0.5 for b in bit]
    x = np.array(psi, dtype=complex)
    y = x * sv[0]
    sweeps, _ = Hl.cone_plan(tsspin.TS_C128, -dt, nsteps, order, tile_bits=T, low_bits=s)
    gb, gf = np.zeros((len(bonds), 3)), np.zeros((n, 3))
    e = 0
    for sw in sweeps:
        for op in sw["ops"]:
            if op["kind"] == "bfly":
                _wht_bits(x, n, op["spins"])
                _wht_bits(y, n, op["spins"])
                e += bin(op["spins"]).count("1")
                continue
            ax, tau, c = op["axis"], op["tau"], op["qturn"]
            ph = np.full(1 << n, 2.0 ** (-op["half_scale"] / 2) * np.exp(1j * np.pi * op["eighths"] / 4))
            for q in _spins(op["own"], n):
                ph = ph * (1j ** ((c * bit[q]) % 4))
                if ax < 3:
                    ph = ph * np.exp(-1j * tau * fields[q][ax] * sv[q])
            for b in _spins(op["bonds"], len(bonds)):
                i, j = bonds[b][0], bonds[b][1]
                if ax < 3:
                    ph = ph * np.exp(-1j * tau * bonds[b][2 + ax] * sv[i] * sv[j])
            x *= ph
            y *= ph
            e -= op["half_scale"]
            if ax < 3:
                w = (np.conj(y) * x).imag
                coef = -2.0 * tau / 2.0 ** e
                for q in _spins(op["own"], n):
                    gf[q, ax] += coef * np.sum(sv[q] * w)
                for b in _spins(op["bonds"], len(bonds)):
                    i, j = bonds[b][0], bonds[b][1]
                    gb[b, ax] += coef * np.sum(sv[i] * sv[j] * w)
    assert e == 0
    assert np.abs(x - psi0).max() < 1e-12
    _, gbo, gfo = oracle.grad_forward(Ho, psi0, dt, nsteps, order, "sz", 0, 0)
    scale = max(np.abs(gbo).max(), np.abs(gfo).max())
    assert np.abs(gb - gbo).max() < 1e-11 * scale and np.abs(gf - gfo).max() < 1e-11 * scale
