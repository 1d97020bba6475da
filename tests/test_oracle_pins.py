"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test fixes part of the oracle with a value or property that the paper or the
mathematics decides: the paper's worked examples (tests/golden), dense matrix
exponentials built a different way (tests/dense_ref.py), closed forms, invariants and
the order of accuracy of the Trotter products.
"""
from __future__ import annotations

import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from tests import dense_ref as D

GOLD = os.path.join(os.path.dirname(__file__), "golden")
EPS = np.finfo(float).eps


def _lines(name):
    with open(os.path.join(GOLD, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def _arrows_to_index(s: str) -> int:
    # leftmost character = highest spin; 'u' (up) is a set bit
    return sum(1 << k for k, ch in enumerate(reversed(s)) if ch == "u")


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def rotation_drift_bound(n, nsteps, order, slack=4.0):
    """Rounding bound on |1 - ||psi||| for the oracle.

    Every one-spin rotation multiplies by entries +-1/sqrt(2) rounded to double, so it
    scales the norm by 1 +- eps/2 at most; a step applies 2 rotations per spin in each
    x and y partial evolution (4, 4, 40 per spin for orders 1, 2, 4 -- counting both the
    V^dagger and the V sweep), plus O(eps) from each phase.
    """
    rot = {1: 4, 2: 8, 4: 40}[order] * n * nsteps
    ph = {1: 3, 2: 6, 4: 30}[order] * nsteps
    return slack * (rot * EPS / 2 + ph * EPS)


# ----------------------------------------------------------------- paper fixtures


def test_rotation_selfcheck():
    # The oracle's own V_a satisfy V^dagger S^a V = S^z and V^dagger V = 1.
    assert oracle.selfcheck() <= 1e-15


def test_pairing_example_spin2_of_4():
    # Sec. 3.2: rotating the second spin of four pairs n with n + 2^1.
    pairs = [(_arrows_to_index(a), _arrows_to_index(b)) for a, b in _lines("pairs_n4_spin2.txt")]
    assert len(pairs) == 8 == 2 ** (4 - 1)
    for lo, hi in pairs:
        assert hi == lo + 2
    # The oracle's one-spin pass on bit 1 with the swap matrix exchanges exactly those pairs.
    psi = np.arange(16, dtype=complex)
    out = oracle.apply_1spin(4, psi, 1, np.array([[0, 1], [1, 0]], dtype=complex))
    expect = psi.copy()
    for lo, hi in pairs:
        expect[lo], expect[hi] = psi[hi], psi[lo]
    assert np.array_equal(out, expect)


def test_fset_example_fixes_up_as_set_bit():
    # Sec. 3.3: F = {1,3} with spin 3 up and spin 1 down is {0100, 0110, 1100, 1110}.
    g = {ln[0]: ln[1:] for ln in _lines("fset_n4.txt")}
    states = [int(s, 2) for s in g["states"]]
    up = [int(s) - 1 for s in g["fixed_up"]]      # 0-based spin index = bit
    down = [int(s) - 1 for s in g["fixed_down"]]
    # z field of +1 on the fixed-up spin and -1 on the fixed-down spin: D_z = s_up - s_down
    fields = np.zeros((4, 3))
    fields[up[0], 2] = 1.0
    fields[down[0], 2] = -1.0
    H = oracle.Hamiltonian(4, [], fields)
    e = oracle.energies(H, "z", np.arange(16))
    # exactly the listed states have spin 3 up (+1/2) and spin 1 down (-1/2): energy 1
    assert sorted(np.nonzero(np.isclose(e, 1.0))[0].tolist()) == sorted(states)
    # and the set is closed under flipping the free spins
    for s in states:
        for f in g["free_spins"]:
            assert (s ^ (1 << (int(f) - 1))) in states


def test_paper_rotation_identities():
    # Sec. 2, Eq. Rotations and the two identities under it, in the textbook ordering.
    rows = {ln[0]: ln[1:] for ln in _lines("rotations.txt")}

    def mat(name):
        v = [complex(*map(float, t.split(","))) for t in rows[name]]
        return np.array(v).reshape(2, 2) / np.sqrt(2)

    Ry, Rx = mat("Ry_pi/2"), mat("Rx_-pi/2")
    SX = 0.5 * np.array([[0, 1], [1, 0]])
    SY = 0.5 * np.array([[0, -1j], [1j, 0]])
    SZ = 0.5 * np.diag([1, -1])
    assert np.abs(Ry.conj().T @ SX @ Ry - SZ).max() < 1e-15
    assert np.abs(Rx.conj().T @ SY @ Rx - SZ).max() < 1e-15


def test_zz_phase_pattern_and_sign_reading():
    # Sec. 2, Eq. ZZ-Phases prints exp(+itJ S^z S^z); the propagator is exp(-itH) (Sec. 2),
    # so the oracle's z partial evolution must be the complex conjugate of the printed one.
    pat = {ln[0]: float(ln[1]) for ln in _lines("zz_phases.txt")}
    J, tau = 0.83, 0.37
    H = oracle.Hamiltonian(2, [(0, 1, 0.0, 0.0, J)])
    idx = {"uu": 3, "ud": 2, "du": 1, "dd": 0}   # first letter = spin 2 (bit 1)
    psi = np.ones(4, dtype=complex)
    out = oracle.substep(H, psi, "z", tau)
    for k, c in pat.items():
        printed = np.exp(1j * tau * J * c)
        assert abs(out[idx[k]] - np.conj(printed)) < 4 * EPS


def test_suzuki_schedule_structure():
    # Sec. 2: U4 is five U2 factors, four at a*t and one at (1-4a)*t; every axis sums to dt.
    g = _lines("suzuki.txt")[0]
    assert int(g[2]) == 5 and int(g[4]) == 4 and int(g[6]) == 1
    a = oracle.suzuki_a()
    assert abs(4 * a + (1 - 4 * a) - 1) < 1e-15
    # 4^(1/3) is the real root of x^3 = 4
    assert abs((4 - 1 / a) ** 3 - 4) < 1e-13
    for order in (1, 2, 4):
        sch = oracle.step_schedule(order, 0.1)
        for ax in "xyz":
            assert abs(sum(t for a_, t in sch if a_ == ax) - 0.1) < 1e-15
    assert len(oracle.step_schedule(4, 0.1)) == 30


# -------------------------------------------------------- dense brute force (P1)


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_substeps_match_dense_expm(n):
    rng = np.random.default_rng(100 + n)
    bonds, fields = D.random_xyz(rng, n)
    H = oracle.Hamiltonian(n, bonds, fields)
    p = D.parts(n, bonds, fields)
    psi = D.random_state(rng, n)
    for ax in "xyz":
        tau = rng.uniform(-0.7, 0.7)
        ref = sla.expm(-1j * tau * p[ax]) @ psi
        assert _rel(oracle.substep(H, psi, ax, tau), ref) < 1e-13


@pytest.mark.parametrize("order", [1, 2, 4])
@pytest.mark.parametrize("n,chain", [(3, False), (4, True), (6, False)])
def test_evolution_matches_dense_trotter_product(order, n, chain):
    rng = np.random.default_rng(7 * n + order)
    bonds, fields = D.random_xyz(rng, n, chain=chain)
    H = oracle.Hamiltonian(n, bonds, fields)
    p = D.parts(n, bonds, fields)
    psi = D.random_state(rng, n)
    dt, ns = 0.13, 7
    ref = D.trotter(p, dt, ns, order) @ psi
    assert _rel(oracle.evolve(H, psi, dt, ns, order), ref) < 1e-12


def test_energies_match_dense_diagonal():
    rng = np.random.default_rng(5)
    n = 6
    bonds, fields = D.random_xyz(rng, n)
    H = oracle.Hamiltonian(n, bonds, fields)
    # energies of axis a are the z-diagonal of H_a with S^a replaced by S^z: rebuild each
    # axis as a pure-z dense Hamiltonian and read its diagonal
    for k, ax in enumerate("xyz"):
        b2 = [(i, j, 0.0, 0.0, (jx, jy, jz)[k]) for (i, j, jx, jy, jz) in bonds]
        f2 = np.zeros((n, 3))
        f2[:, 2] = fields[:, k]
        Hz = D.parts(n, b2, f2)["z"]
        assert np.allclose(oracle.energies(H, ax, np.arange(1 << n)), np.real(np.diag(Hz)),
                           atol=1e-14, rtol=0)


# --------------------------------------------------- order of accuracy (P2)


@pytest.mark.parametrize("order,lo,hi", [(1, 1.6, 2.4), (2, 3.3, 4.7), (4, 12.0, 20.0)])
def test_order_of_accuracy_against_exact_propagator(order, lo, hi):
    rng = np.random.default_rng(11)
    n = 6
    bonds, fields = D.random_xyz(rng, n)
    H = oracle.Hamiltonian(n, bonds, fields)
    psi = D.random_state(rng, n)
    T = 0.8
    exact = sla.expm(-1j * T * D.full_h(n, bonds, fields)) @ psi
    errs = []
    for ns in (8, 16, 32):
        errs.append(np.linalg.norm(oracle.evolve(H, psi, T / ns, ns, order) - exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert lo < r1 < hi and lo < r2 < hi, (errs, r1, r2)


# ------------------------------------------------ exact special cases (P3-P5)


def test_pure_z_part_is_exact_phase():
    rng = np.random.default_rng(3)
    n = 7
    bonds = [(i, j, 0.0, 0.0, rng.uniform(-1, 1)) for i in range(n) for j in range(i + 1, n)]
    fields = np.zeros((n, 3))
    fields[:, 2] = rng.uniform(-1, 1, n)
    H = oracle.Hamiltonian(n, bonds, fields)
    psi = D.random_state(rng, n)
    T, ns = 2.3, 17
    diag = np.real(np.diag(D.parts(n, bonds, fields)["z"]))
    ref = psi * np.exp(-1j * T * diag)
    # the x and y partial evolutions are the identity here, up to rotation rounding
    assert _rel(oracle.evolve(H, psi, T / ns, ns, 4), ref) < rotation_drift_bound(n, ns, 4)


@pytest.mark.parametrize("ax", ["x", "y"])
def test_single_axis_hamiltonian_is_exact(ax):
    rng = np.random.default_rng(4)
    n = 6
    k = "xyz".index(ax)
    bonds = []
    for i in range(n - 1):
        c = [0.0, 0.0, 0.0]
        c[k] = rng.uniform(0.5, 1.5)
        bonds.append((i, i + 1, *c))
    fields = np.zeros((n, 3))
    fields[:, k] = rng.uniform(-1, 1, n)
    H = oracle.Hamiltonian(n, bonds, fields)
    psi = D.random_state(rng, n)
    T, ns = 1.7, 9
    ref = sla.expm(-1j * T * D.full_h(n, bonds, fields)) @ psi
    for order in (1, 2, 4):
        assert _rel(oracle.evolve(H, psi, T / ns, ns, order), ref) < 1e-12


def test_larmor_precession_closed_form():
    # one spin, field along x, starting up: <S^z> = cos(hT)/2, <S^y> = -sin(hT)/2
    h = 1.3
    H = oracle.Hamiltonian(1, [], np.array([[h, 0.0, 0.0]]))
    psi = np.array([0, 1], dtype=complex)
    for T, ns in ((0.5, 5), (3.0, 40)):
        out = oracle.evolve(H, psi, T / ns, ns, 4)
        tol = rotation_drift_bound(1, ns, 4)
        assert abs(oracle.expect(H, out, "sz", 0) - 0.5 * np.cos(h * T)) < tol
        assert abs(oracle.expect(H, out, "sy", 0) + 0.5 * np.sin(h * T)) < tol
        assert abs(oracle.expect(H, out, "sx", 0)) < tol


def test_tilted_larmor_fourth_order():
    # field (hx, 0, hz): exact precession; the Trotter error falls 16x per halving of dt
    hx, hz = 0.9, 0.6
    H = oracle.Hamiltonian(1, [], np.array([[hx, 0.0, hz]]))
    psi = np.array([0, 1], dtype=complex)
    T = 2.0
    w = np.hypot(hx, hz)
    nx, nz = hx / w, hz / w
    # <S^z(t)> for precession about n of a spin starting along z: (nz^2 + nx^2 cos wt)/2
    ez = 0.5 * (nz ** 2 + nx ** 2 * np.cos(w * T))
    errs = [abs(oracle.expect(H, oracle.evolve(H, psi, T / ns, ns, 4), "sz", 0) - ez)
            for ns in (10, 20)]
    assert errs[0] < 1e-5 and 10 < errs[0] / errs[1] < 22


@pytest.mark.parametrize("init,sign", [(0b01, +1), (0b11, -1)])
def test_two_spin_flip_flop_closed_form(init, sign):
    # XX, YY and ZZ of a single bond commute, so the Trotter product is exact:
    # from |up,down>: <S^z_0> = cos((Jx+Jy)T/2)/2 ; from |up,up>: cos((Jx-Jy)T/2)/2
    jx, jy, jz = 0.7, 1.1, 0.4
    H = oracle.Hamiltonian(2, [(0, 1, jx, jy, jz)])
    psi = np.zeros(4, dtype=complex)
    psi[init] = 1
    T, ns = 4.0, 50
    out = oracle.evolve(H, psi, T / ns, ns, 4)
    ref = 0.5 * np.cos((jx + sign * jy) * T / 2)
    tol = rotation_drift_bound(2, ns, 4)
    assert abs(oracle.expect(H, out, "sz", 0) - ref) < tol


# ---------------------------------------------------- invariants (P6, P7, P12)


def test_norm_conservation_bound():
    rng = np.random.default_rng(8)
    n, ns = 8, 300
    bonds, fields = D.random_xyz(rng, n, chain=True)
    H = oracle.Hamiltonian(n, bonds, fields)
    psi = D.random_state(rng, n)
    out = oracle.evolve(H, psi, 0.05, ns, 4)
    assert abs(1 - np.linalg.norm(out)) < rotation_drift_bound(n, ns, 4)


def test_loschmidt_echo_returns_initial_state():
    # Sec. 4.2: the same partial evolutions with t -> -t undo the forward run
    rng = np.random.default_rng(9)
    n, ns = 8, 200
    bonds, fields = D.random_xyz(rng, n)
    H = oracle.Hamiltonian(n, bonds, fields)
    psi = D.random_state(rng, n)
    fwd = oracle.evolve(H, psi, 0.04, ns, 4)
    back = oracle.evolve(H, fwd, -0.04, ns, 4)
    tol = 2 * rotation_drift_bound(n, ns, 4)
    assert abs(1 - abs(np.vdot(psi, back)) ** 2) < 2 * tol
    assert np.linalg.norm(back - psi) < tol + 1e-13


def test_energy_bounded_fluctuation():
    rng = np.random.default_rng(10)
    n = 7
    bonds, fields = D.random_xyz(rng, n, chain=True)
    H = oracle.Hamiltonian(n, bonds, fields)
    psi = D.random_state(rng, n)
    e0 = oracle.expect(H, psi, "energy")
    es = []
    cur = psi
    for _ in range(20):
        cur = oracle.evolve(H, cur, 0.05, 10, 4)
        es.append(oracle.expect(H, cur, "energy"))
    dev = np.abs(np.array(es) - e0)
    assert dev.max() < 1e-5
    # no drift: the last values are not systematically further away than the first
    assert dev[-5:].mean() < 3 * dev[:5].mean() + 1e-9


# --------------------------------------------------------- observables vs dense


def test_observables_match_dense():
    rng = np.random.default_rng(12)
    n = 5
    bonds, fields = D.random_xyz(rng, n)
    H = oracle.Hamiltonian(n, bonds, fields)
    psi = D.random_state(rng, n)
    oth = D.random_state(rng, n)
    def ev(M):
        return np.vdot(psi, M @ psi)
    for i in range(n):
        for ax in "xyz":
            M = D.site_op(n, i, D.ONE_SPIN[ax])
            assert abs(oracle.expect(H, psi, "s" + ax, i) - ev(M).real) < 1e-14
        Mz = D.site_op(n, i, D.ONE_SPIN["z"])
        assert abs(oracle.expect(H, psi, "overlap_sz", i, other=oth) - np.vdot(oth, Mz @ psi)) < 1e-14
    i, j = 1, 3
    M = D.site_op(n, i, D.ONE_SPIN["z"]) @ D.site_op(n, j, D.ONE_SPIN["z"])
    assert abs(oracle.expect(H, psi, "szsz", i, j) - ev(M).real) < 1e-14
    Mz = sum(D.site_op(n, q, D.ONE_SPIN["z"]) for q in range(n))
    assert abs(oracle.expect(H, psi, "mz") - ev(Mz).real) < 1e-14
    assert abs(oracle.expect(H, psi, "energy") - ev(D.full_h(n, bonds, fields)).real) < 1e-13
    assert abs(oracle.expect(H, psi, "norm") - 1.0) < 1e-14


# ------------------------------------------------------- one-magnon sector (P8)


def test_one_magnon_sector_textbook():
    # XXZ chain with z fields from one up spin: the exact dynamics stays in the N-dim
    # one-magnon sector (a tight-binding matrix); the oracle differs by Trotter error only
    rng = np.random.default_rng(13)
    n, J, T = 9, 1.0, 1.0
    delta = 0.8
    hz = rng.uniform(-0.5, 0.5, n)
    bonds = [(i, i + 1, J, J, delta) for i in range(n - 1)]
    fields = np.zeros((n, 3))
    fields[:, 2] = hz
    # one-magnon basis |k> = spin k up, rest down; S^x S^x + S^y S^y hops with J/2
    M = np.zeros((n, n))
    for k in range(n):
        e = 0.0
        for i in range(n - 1):
            e += delta * (0.25 if (i != k and i + 1 != k) else -0.25)
        e += sum(0.5 * hz[q] if q == k else -0.5 * hz[q] for q in range(n))
        M[k, k] = e
    for i in range(n - 1):
        M[i, i + 1] = M[i + 1, i] = J / 2
    c0 = np.zeros(n, dtype=complex)
    c0[2] = 1
    cT = sla.expm(-1j * T * M) @ c0
    H = oracle.Hamiltonian(n, bonds, fields)
    psi = np.zeros(1 << n, dtype=complex)
    psi[1 << 2] = 1
    errs = []
    for ns in (20, 40):
        out = oracle.evolve(H, psi, T / ns, ns, 4)
        errs.append(np.abs(out[[1 << k for k in range(n)]] - cT).max())
    assert errs[0] < 1e-5 and 10 < errs[0] / errs[1] < 22


# ------------------------------------------------------------ gradients (P11)


def test_gradient_larmor_closed_form():
    h, T, ns = 0.9, 2.5, 25
    H = oracle.Hamiltonian(1, [], np.array([[h, 0.0, 0.0]]))
    psi = np.array([0, 1], dtype=complex)
    loss, gb, gf = oracle.grad_forward(H, psi, T / ns, ns, 4, "sz", 0)
    assert abs(loss - 0.5 * np.cos(h * T)) < rotation_drift_bound(1, ns, 4)
    assert abs(gf[0, 0] + 0.5 * T * np.sin(h * T)) < 1e-12
    assert abs(gf[0, 1]) < 1e-12 and abs(gf[0, 2]) < 1e-12


def test_gradient_flip_flop_closed_form():
    jx, jy, jz = 0.7, 1.1, 0.4
    T, ns = 3.0, 30
    H = oracle.Hamiltonian(2, [(0, 1, jx, jy, jz)])
    psi = np.zeros(4, dtype=complex)
    psi[0b01] = 1
    loss, gb, gf = oracle.grad_forward(H, psi, T / ns, ns, 4, "sz", 0)
    g = -(T / 4) * np.sin((jx + jy) * T / 2)
    assert abs(gb[0, 0] - g) < 1e-12 and abs(gb[0, 1] - g) < 1e-12
    assert abs(gb[0, 2]) < 1e-12


def test_gradient_matches_dense_finite_differences():
    rng = np.random.default_rng(14)
    n = 4
    bonds, fields = D.random_xyz(rng, n, chain=True)
    psi = D.random_state(rng, n)
    dt, ns, order = 0.1, 6, 4
    H = oracle.Hamiltonian(n, bonds, fields)
    loss, gb, gf = oracle.grad_forward(H, psi, dt, ns, order, "sx", 1)

    def L(bonds_, fields_):
        p = D.parts(n, bonds_, fields_)
        v = D.trotter(p, dt, ns, order) @ psi
        return np.vdot(v, D.site_op(n, 1, D.ONE_SPIN["x"]) @ v).real

    assert abs(loss - L(bonds, fields)) < 1e-13
    eps = 1e-5
    for k in range(len(bonds)):
        for a in range(3):
            bp = [list(b) for b in bonds]
            bm = [list(b) for b in bonds]
            bp[k][2 + a] += eps
            bm[k][2 + a] -= eps
            fd = (L(bp, fields) - L(bm, fields)) / (2 * eps)
            assert abs(gb[k, a] - fd) < 1e-8
    for q in range(n):
        for a in range(3):
            fp = fields.copy()
            fm = fields.copy()
            fp[q, a] += eps
            fm[q, a] -= eps
            fd = (L(bonds, fp) - L(bonds, fm)) / (2 * eps)
            assert abs(gf[q, a] - fd) < 1e-8


def test_energy_gradient_matches_dense_finite_differences():
    """Loss <psi(T)|H|psi(T)> with H of Eq. 1 itself: its derivative has the tangent term and
    the explicit <dH/dtheta>; central differences of the dense Trotter product and dense H,
    both rebuilt from the shifted parameters, pin the sum."""
    rng = np.random.default_rng(15)
    n = 4
    bonds, fields = D.random_xyz(rng, n, chain=False)
    psi = D.random_state(rng, n)
    dt, ns, order = 0.1, 5, 4
    H = oracle.Hamiltonian(n, bonds, fields)
    loss, gb, gf = oracle.grad_forward(H, psi, dt, ns, order, "energy")

    def L(bonds_, fields_):
        p = D.parts(n, bonds_, fields_)
        v = D.trotter(p, dt, ns, order) @ psi
        return np.vdot(v, D.full_h(n, bonds_, fields_) @ v).real

    assert abs(loss - L(bonds, fields)) < 1e-12
    eps = 1e-5
    worst = 0.0
    for k in range(len(bonds)):
        for a in range(3):
            bp = [list(b) for b in bonds]
            bm = [list(b) for b in bonds]
            bp[k][2 + a] += eps
            bm[k][2 + a] -= eps
            fd = (L(bp, fields) - L(bm, fields)) / (2 * eps)
            worst = max(worst, abs(gb[k, a] - fd))
    for q in range(n):
        for a in range(3):
            fp = fields.copy()
            fm = fields.copy()
            fp[q, a] += eps
            fm[q, a] -= eps
            fd = (L(bonds, fp) - L(bonds, fm)) / (2 * eps)
            worst = max(worst, abs(gf[q, a] - fd))
    assert worst < 1e-8
    # the explicit term is far above that bound, so dropping it fails the check
    v = D.trotter(D.parts(n, bonds, fields), dt, ns, order) @ psi
    explicit = [abs(np.vdot(v, D.site_op(n, q, D.ONE_SPIN[a]) @ v).real)
                for q in range(n) for a in "xyz"]
    assert max(explicit) > 1e-2


@pytest.mark.parametrize("axis", ["x", "y"])
def test_single_axis_product_eigenstate_closed_form(axis):
    # only x (or only y) terms: the axis parts commute, the Trotter product is exact, and a
    # product of S^x (S^y) eigenstates picks up exp(-i T E), E = sum h m + sum J m m.
    # (down, up) order: S^x eigenvectors (1, +-1)/sqrt2 for m = +-1/2; S^y: (1, -+i)/sqrt2
    n, T, ns = 7, 0.7, 5
    rng = np.random.default_rng(71 + (axis == "y"))
    a = 0 if axis == "x" else 1
    J = rng.uniform(0.5, 1.5, n - 1)
    h = rng.uniform(-1, 1, n)
    bonds = [(i, i + 1, *(J[i] if k == a else 0.0 for k in range(3))) for i in range(n - 1)]
    bonds += [(0, n - 1, *(0.3 if k == a else 0.0 for k in range(3)))]
    fields = np.zeros((n, 3))
    fields[:, a] = h
    m = rng.choice([-0.5, 0.5], n)
    E = float(np.sum(h * m) + np.sum(J * m[:-1] * m[1:]) + 0.3 * m[0] * m[-1])
    up = np.where(m > 0, 1.0, -1.0).astype(complex) if axis == "x" else np.where(m > 0, -1j, 1j)
    psi = np.ones(1, complex)
    for j in range(n):
        psi = np.kron(np.array([1, up[j]]) / np.sqrt(2), psi)
    out = oracle.evolve(oracle.Hamiltonian(n, bonds, fields), psi, T / ns, ns, 4)
    assert np.abs(out * psi.conj() * 2 ** n - np.exp(-1j * T * E)).max() < 1e-12
