"""Seeded synthetic inputs for the benchmark workloads and the tests.

Input construction only: Hamiltonian parameters (Sec. 2, Eq. 1) and initial states
(Sec. 2, Eq. 2; the random-phase states of Appendix A, Eq. entanglado).  Nothing here
evolves a state.  Both the oracle side and the GPU side of a test take their inputs from
these functions.

Random numbers come from NumPy's PCG64 (`default_rng(13050036 + k)` for workload k) in
FP64, drawn in the order: bonds in index order with (Jx, Jy, Jz) per bond, then fields,
then the initial state.  complex64 states are the FP64 arrays rounded.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED0 = 13050036


@dataclass
class Workload:
    name: str
    n: int
    bonds: list
    fields: np.ndarray
    dt: float
    nsteps: int
    order: int = 4
    psi0: np.ndarray | None = None          # complex128, or None when built lazily
    extra: dict = field(default_factory=dict)


def chain(n, couplings):
    """Open chain bonds (i, i+1) with couplings[i] = (Jx, Jy, Jz)."""
    return [(i, i + 1, *map(float, couplings[i])) for i in range(n - 1)]


def gaussian_state(rng, n):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def random_phase_state(rng, n):
    """|Phi> = 2^(-n/2) sum_b exp(i phi_b)|b>, phi_b ~ U[0, 2 pi)."""
    phi = rng.uniform(0.0, 2.0 * np.pi, size=1 << n)
    return np.exp(1j * phi) * (2.0 ** (-n / 2))


def polarized_random_phase_state(rng, n, up_spin=0):
    """|up>_{up_spin} (x) random phases on the other spins (Appendix A, Eq. entanglado)."""
    phi = rng.uniform(0.0, 2.0 * np.pi, size=1 << (n - 1))
    rest = np.exp(1j * phi) * (2.0 ** (-(n - 1) / 2))
    psi = np.zeros(1 << n, dtype=np.complex128)
    idx = np.arange(1 << (n - 1), dtype=np.int64)
    lo = idx & ((1 << up_spin) - 1)
    full = ((idx >> up_spin) << (up_spin + 1)) | (1 << up_spin) | lo
    psi[full] = rest
    return psi


def basis_state(n, b):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[b] = 1.0
    return psi


def neel_index(n):
    """Chain Neel state: spin i up iff i is even."""
    return sum(1 << i for i in range(0, n, 2))


def sz_times(psi, n, i):
    """S^z_i |psi>: amplitude b times +-1/2 (input of the autocorrelation C(t))."""
    b = np.arange(psi.size, dtype=np.int64)
    return psi * np.where((b >> i) & 1, 0.5, -0.5)


# ------------------------------------------------------------------------ workloads


def heisenberg_chain(n=12, nsteps=200):
    """N-spin open Heisenberg chain, J = 1, no fields, complex-Gaussian initial state."""
    rng = np.random.default_rng(SEED0 + 1)
    bonds = chain(n, [(1.0, 1.0, 1.0)] * (n - 1))
    psi = gaussian_state(rng, n)
    return Workload("heisenberg-chain", n, bonds, np.zeros((n, 3)), 0.05, nsteps, 4, psi,
                    dict(record=[("sz", 0), ("norm",)]))


def xyz_chain(n=27, nsteps=1000, state=True):
    """Open XYZ chain, J^a_i ~ U[0.5, 1.5] per bond, h^z_i ~ U[-0.5, 0.5], random-phase
    state; the autocorrelation C(t) = <a(t)|S^z_0|c(t)> with a(0) = Phi, c(0) = S^z_0 Phi."""
    rng = np.random.default_rng(SEED0 + 2)
    J = rng.uniform(0.5, 1.5, size=(n - 1, 3))
    hz = rng.uniform(-0.5, 0.5, size=n)
    fields = np.zeros((n, 3))
    fields[:, 2] = hz
    psi = random_phase_state(rng, n) if state else None
    return Workload("xyz-chain", n, chain(n, J), fields, 0.02, nsteps, 4, psi)


def dipolar_lattice(rows=5, cols=6, nsteps=500):
    """Open rows x cols lattice, all pairs J^z = 1/r^3, J^x = J^y = -J^z/2, Neel state with
    site 0 flipped; site i = cols*r + c, up iff r + c even."""
    n = rows * cols
    bonds = []
    for a in range(n):
        for b in range(a + 1, n):
            ra, ca = divmod(a, cols)
            rb, cb = divmod(b, cols)
            r = np.hypot(ra - rb, ca - cb)
            jz = 1.0 / r ** 3
            bonds.append((a, b, -jz / 2, -jz / 2, jz))
    up = sum(1 << i for i in range(n) if sum(divmod(i, cols)) % 2 == 0)
    up ^= 1  # flip site 0
    return Workload("dipolar-lattice", n, bonds, np.zeros((n, 3)), 0.01, nsteps, 4,
                    basis_state(n, up) if n <= 26 else None, dict(init_index=up))


def disordered_xxz_batch(n_chains=512, nmin=10, nmax=20, nsteps=400):
    """Independent open XXZ chains: N ~ U{nmin..nmax}, Jx = Jy = 1, Jz = Delta ~ U[0.5, 1.5],
    h^z ~ U[-W, W] with W = (2, 4, 8)[c mod 3]; |up>_0 (x) random phases."""
    rng = np.random.default_rng(SEED0 + 4)
    ns = rng.integers(nmin, nmax + 1, size=n_chains)
    chains = []
    for c in range(n_chains):
        n = int(ns[c])
        delta = rng.uniform(0.5, 1.5)
        W = (2.0, 4.0, 8.0)[c % 3]
        fields = np.zeros((n, 3))
        fields[:, 2] = rng.uniform(-W, W, size=n)
        chains.append(Workload(f"xxz-{c}", n, chain(n, [(1.0, 1.0, delta)] * (n - 1)), fields,
                               0.05, nsteps, 4, None, dict(W=W, seed_index=c)))
    # states are drawn after all Hamiltonians, chain by chain
    for w in chains:
        w.psi0 = polarized_random_phase_state(rng, w.n, 0)
    return chains


def gradient_chain(n=20, nsteps=300):
    """Open XYZ chain, 3(n-1) couplings ~ U[0.5, 1.5], h^x_i ~ U[-1, 1], Neel state;
    loss <S^z_0(T)>."""
    rng = np.random.default_rng(SEED0 + 5)
    J = rng.uniform(0.5, 1.5, size=(n - 1, 3))
    fields = np.zeros((n, 3))
    fields[:, 0] = rng.uniform(-1.0, 1.0, size=n)
    return Workload("gradient-chain", n, chain(n, J), fields, 0.02, nsteps, 4,
                    basis_state(n, neel_index(n)))


def echo_ring(n=16, double_quantum=False, nsteps=1000, dt=0.05):
    """The Loschmidt-echo workload of Sec. 4.2: a periodic ring of n spins with nearest-
    neighbour Heisenberg couplings J = 1, optionally plus the double-quantum terms
    S^x_j S^x_k - S^y_j S^y_k (coupling 1) between neighbours at distances 1, 2 and 3 around
    the ring (listed as separate bonds; coinciding bonds add up, as Eq. 1 sums them); the
    initial state is |up>_0 (x) random phases (Appendix A, Eq. entanglado).  The paper
    prints neither dt nor the double-quantum strength: dt = 0.05 and strength 1 are this
    workload's choices."""
    rng = np.random.default_rng(SEED0 + 6 + (1 if double_quantum else 0))
    bonds = [(i, (i + 1) % n, 1.0, 1.0, 1.0) for i in range(n)]
    if double_quantum:
        for d in (1, 2, 3):
            bonds += [(i, (i + d) % n, 1.0, -1.0, 0.0) for i in range(n)]
    name = "echo-ring-dq" if double_quantum else "echo-ring"
    return Workload(name, n, bonds, np.zeros((n, 3)), dt, nsteps, 4,
                    polarized_random_phase_state(rng, n, 0))
