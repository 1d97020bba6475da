"""ctypes wrapper over ``oracle.c`` -- the plain FP64 CPU reference.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg use this module; the product path never does.

Every function takes the model of Sec. 2, Eq. 1 of the paper as a :class:`Hamiltonian`
(N spins, a bond list with (J^x, J^y, J^z) per bond, and fields h[N][3]) and works on the
2^N coefficient vector of Eq. 2 as a complex128 NumPy array.  Spin j is bit j of the basis
index and a set bit is spin up (Sec. 3.2 footnote, Sec. 3.3 F-set example).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OBS = {
    "norm": 0, "sx": 1, "sy": 2, "sz": 3, "szsz": 4, "mz": 5, "energy": 6, "overlap_sz": 7,
}
AXES = {"x": 0, "y": 1, "z": 2}


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, OpenMP, FP64, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        i32, i64, f64, u64 = C.c_int, C.c_int64, C.c_double, C.c_uint64
        lib.orc_selfcheck.restype = f64
        lib.orc_suzuki_a.restype = f64
        lib.orc_energy.restype = f64
        lib.orc_energy.argtypes = [i32, i32, P, P, P, P, i32, u64]
        lib.orc_energies.argtypes = [i32, i32, P, P, P, P, i32, P, i64, P]
        lib.orc_apply_1spin.argtypes = [i32, P, i32, P]
        lib.orc_substep.argtypes = [i32, i32, P, P, P, P, i32, f64, P]
        lib.orc_step_schedule.restype = i32
        lib.orc_step_schedule.argtypes = [i32, f64, P, P]
        lib.orc_evolve.restype = i32
        lib.orc_evolve.argtypes = [i32, i32, P, P, P, P, P, f64, i64, i32]
        lib.orc_apply_obs.restype = i32
        lib.orc_apply_obs.argtypes = [i32, i32, P, P, P, P, i32, i32, i32, P, P]
        lib.orc_expect.restype = i32
        lib.orc_expect.argtypes = [i32, i32, P, P, P, P, P, i32, i32, i32, P, P]
        lib.orc_grad_forward.restype = i32
        lib.orc_grad_forward.argtypes = [i32, i32, P, P, P, P, P, f64, i64, i32, i32, i32, i32,
                                         P, P, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


@dataclass
class Hamiltonian:
    """H of Eq. 1: ``bonds`` is a list of (i, j, Jx, Jy, Jz), ``fields`` is (n, 3)."""

    n: int
    bonds: list = field(default_factory=list)
    fields: np.ndarray | None = None

    def __post_init__(self):
        self.bi = np.ascontiguousarray([int(b[0]) for b in self.bonds], dtype=np.int32)
        self.bj = np.ascontiguousarray([int(b[1]) for b in self.bonds], dtype=np.int32)
        self.J = np.ascontiguousarray([[float(b[2]), float(b[3]), float(b[4])]
                                       for b in self.bonds], dtype=np.float64).reshape(-1, 3)
        if self.fields is None:
            self.h = np.zeros((self.n, 3), dtype=np.float64)
        else:
            self.h = np.ascontiguousarray(self.fields, dtype=np.float64).reshape(self.n, 3)

    def args(self):
        return (self.n, len(self.bonds), _ptr(self.bi), _ptr(self.bj), _ptr(self.J), _ptr(self.h))


def _state(psi) -> np.ndarray:
    a = np.ascontiguousarray(psi, dtype=np.complex128)
    return a


def selfcheck() -> float:
    return _load().orc_selfcheck()


def suzuki_a() -> float:
    return _load().orc_suzuki_a()


def step_schedule(order: int, dt: float):
    """[(axis, tau), ...] of one step, in the order the partial evolutions act."""
    axes = np.zeros(32, dtype=np.int32)
    taus = np.zeros(32, dtype=np.float64)
    k = _load().orc_step_schedule(order, dt, _ptr(axes), _ptr(taus))
    if k < 0:
        raise ValueError("order must be 1, 2 or 4")
    return [("xyz"[axes[i]], float(taus[i])) for i in range(k)]


def energies(H: Hamiltonian, axis: str, bs) -> np.ndarray:
    bs = np.ascontiguousarray(bs, dtype=np.uint64)
    out = np.empty(bs.shape, dtype=np.float64)
    _load().orc_energies(*H.args(), AXES[axis], _ptr(bs), bs.size, _ptr(out))
    return out


def apply_1spin(n: int, psi, q: int, U) -> np.ndarray:
    psi = _state(psi).copy()
    U = np.ascontiguousarray(U, dtype=np.complex128)
    _load().orc_apply_1spin(n, _ptr(psi), q, _ptr(U))
    return psi


def substep(H: Hamiltonian, psi, axis: str, tau: float) -> np.ndarray:
    psi = _state(psi).copy()
    _load().orc_substep(*H.args(), AXES[axis], tau, _ptr(psi))
    return psi


def evolve(H: Hamiltonian, psi, dt: float, nsteps: int, order: int = 4) -> np.ndarray:
    psi = _state(psi).copy()
    assert psi.size == 1 << H.n
    rc = _load().orc_evolve(*H.args(), _ptr(psi), dt, nsteps, order)
    if rc != 0:
        raise ValueError("order must be 1, 2 or 4")
    return psi


def apply_obs(H: Hamiltonian, psi, kind: str, i: int = 0, j: int = 0) -> np.ndarray:
    psi = _state(psi)
    out = np.empty_like(psi)
    rc = _load().orc_apply_obs(*H.args(), OBS[kind], i, j, _ptr(psi), _ptr(out))
    if rc != 0:
        raise ValueError(kind)
    return out


def expect(H: Hamiltonian, psi, kind: str, i: int = 0, j: int = 0, other=None):
    """<psi|O|psi> as a float, or the complex <other|S^z_i|psi> for 'overlap_sz'."""
    psi = _state(psi)
    out = np.zeros(2, dtype=np.float64)
    oth = _state(other) if other is not None else psi
    rc = _load().orc_expect(*H.args(), _ptr(psi), OBS[kind], i, j, _ptr(oth), _ptr(out))
    if rc != 0:
        raise ValueError(kind)
    if kind == "overlap_sz":
        return complex(out[0], out[1])
    return float(out[0])


def grad_forward(H: Hamiltonian, psi0, dt: float, nsteps: int, order: int, kind: str,
                 i: int = 0, j: int = 0):
    """(loss, grad_bonds[nb][3], grad_fields[n][3]) by forward-mode tangents."""
    psi0 = _state(psi0)
    nb = len(H.bonds)
    gb = np.zeros((nb, 3), dtype=np.float64)
    gf = np.zeros((H.n, 3), dtype=np.float64)
    loss = np.zeros(1, dtype=np.float64)
    rc = _load().orc_grad_forward(*H.args(), _ptr(psi0), dt, nsteps, order, OBS[kind], i, j,
                                  _ptr(loss), _ptr(gb), _ptr(gf))
    if rc != 0:
        raise ValueError("unsupported loss or order")
    return float(loss[0]), gb, gf
