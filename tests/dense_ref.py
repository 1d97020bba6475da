"""Dense-matrix construction of the model, used only to pin the oracle (N <= 10).

It is built a different way from the oracle: every spin operator is a Kronecker product
of the textbook spin-1/2 matrices, the partial evolutions are full matrix exponentials
(scipy.linalg.expm) of the dense axis parts, and the Trotter products are formed by
matrix multiplication straight from their definitions in Sec. 2 of the paper.
"""
from __future__ import annotations

from functools import reduce

import numpy as np
import scipy.linalg as sla

# Textbook spin-1/2 operators S = sigma/2 in the (up, down) ordering.
_SX_UD = 0.5 * np.array([[0, 1], [1, 0]], dtype=complex)
_SY_UD = 0.5 * np.array([[0, -1j], [1j, 0]], dtype=complex)
_SZ_UD = 0.5 * np.array([[1, 0], [0, -1]], dtype=complex)
# The state vector stores basis index 0 = down, 1 = up for every spin: reorder.
_SWAP = np.array([[0, 1], [1, 0]], dtype=complex)
ONE_SPIN = {a: _SWAP @ m @ _SWAP for a, m in (("x", _SX_UD), ("y", _SY_UD), ("z", _SZ_UD))}


def site_op(n: int, j: int, op: np.ndarray) -> np.ndarray:
    """op acting on spin j (bit j of the basis index) of an n-spin register."""
    # np.kron(A, B)[a*dimB + b] puts A on the more significant bits, so the factor list
    # runs from spin n-1 down to spin 0.
    mats = [np.eye(2, dtype=complex)] * n
    mats = list(mats)
    mats[n - 1 - j] = op
    return reduce(np.kron, mats)


def parts(n: int, bonds, fields) -> dict:
    """Dense H_x, H_y, H_z of Eq. 1 split by axis."""
    fields = np.zeros((n, 3)) if fields is None else np.asarray(fields, dtype=float)
    out = {}
    for k, a in enumerate("xyz"):
        H = np.zeros((1 << n, 1 << n), dtype=complex)
        for j in range(n):
            if fields[j, k] != 0.0:
                H += fields[j, k] * site_op(n, j, ONE_SPIN[a])
        for (i, j, jx, jy, jz) in bonds:
            c = (jx, jy, jz)[k]
            if c != 0.0:
                H += c * site_op(n, i, ONE_SPIN[a]) @ site_op(n, j, ONE_SPIN[a])
        out[a] = H
    return out


def full_h(n, bonds, fields):
    p = parts(n, bonds, fields)
    return p["x"] + p["y"] + p["z"]


def u1(p, t):
    """Eq. U1 with H_1, H_2, H_3 = H_x, H_y, H_z."""
    return sla.expm(-1j * t * p["x"]) @ sla.expm(-1j * t * p["y"]) @ sla.expm(-1j * t * p["z"])


def u2(p, t):
    return u1(p, -t / 2).conj().T @ u1(p, t / 2)


def u4(p, t):
    a = 1.0 / (4.0 - 4.0 ** (1.0 / 3.0))
    A = u2(p, a * t)
    B = u2(p, (1 - 4 * a) * t)
    return A @ A @ B @ A @ A


def trotter(p, dt, nsteps, order):
    U = {1: u1, 2: u2, 4: u4}[order](p, dt)
    return np.linalg.matrix_power(U, nsteps)


def random_xyz(rng, n, chain=False, with_fields=True):
    """Random couplings on all pairs (or a chain) and random fields on all axes."""
    pairs = [(i, i + 1) for i in range(n - 1)] if chain else \
        [(i, j) for i in range(n) for j in range(i + 1, n)]
    bonds = [(i, j, *rng.uniform(-1.5, 1.5, size=3)) for (i, j) in pairs]
    fields = rng.uniform(-1, 1, size=(n, 3)) if with_fields else None
    return bonds, fields


def random_state(rng, n):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)
