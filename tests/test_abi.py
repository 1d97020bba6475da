"""C ABI of libtsspin on the CPU: the library loads, exports every symbol that
include/tsspin.h declares, and the host-only paths reject bad arguments."""
from __future__ import annotations

import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1305_0036_amd import tsspin

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "tsspin.h")).read()
    return sorted(set(re.findall(r"^(?:ts_status|const char \*)\s*(ts_\w+)\s*\(", text, re.M)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "ts_evolve" in names and "ts_create" in names
    out = subprocess.check_output(["nm", "-D", "--defined-only", tsspin.LIB_PATH], text=True)
    exported = set(re.findall(r" T (ts_\w+)", out))
    for n in names:
        assert n in exported, n
        assert hasattr(tsspin._lib, n)
    assert sorted(tsspin.EXPORTED) == names


def _create(n, bonds=(), fields=None):
    barr = (tsspin.ts_bond * max(1, len(bonds)))()
    for k, b in enumerate(bonds):
        barr[k].i, barr[k].j, barr[k].jx, barr[k].jy, barr[k].jz = b
    ctx = C.c_void_p()
    fp = None
    if fields is not None:
        f = np.ascontiguousarray(fields, dtype=np.float64)
        fp = f.ctypes.data_as(C.c_void_p)
    rc = tsspin._lib.ts_create(n, barr if bonds else None, len(bonds), fp, C.byref(ctx))
    return rc, ctx


@pytest.mark.parametrize("n,bonds,msg", [
    (0, (), "n_spins"),
    (36, (), "n_spins"),
    (4, ((0, 0, 1.0, 1.0, 1.0),), "i == j"),
    (4, ((0, 4, 1.0, 1.0, 1.0),), "out of range"),
    (4, ((-1, 2, 1.0, 1.0, 1.0),), "out of range"),
    (4, ((0, 1, math.nan, 1.0, 1.0),), "non-finite"),
    (4, ((0, 1, 1.0, math.inf, 1.0),), "non-finite"),
])
def test_create_rejects(n, bonds, msg):
    rc, ctx = _create(n, bonds)
    assert rc == tsspin.TS_EINVAL
    assert not ctx.value
    assert msg in tsspin.last_error()


def test_create_rejects_nan_field_and_null_out():
    f = np.zeros((3, 3))
    f[1, 2] = np.nan
    rc, _ = _create(3, (), f)
    assert rc == tsspin.TS_EINVAL and "field" in tsspin.last_error()
    assert tsspin._lib.ts_create(3, None, 0, None, None) == tsspin.TS_EINVAL


def test_destroy_null_and_balanced():
    assert tsspin._lib.ts_destroy(None) == tsspin.TS_OK
    for _ in range(50):
        rc, ctx = _create(5, ((0, 1, 1.0, 0.5, 0.2), (1, 0, 0.1, 0.1, 0.1)))
        assert rc == tsspin.TS_OK
        assert tsspin._lib.ts_destroy(ctx) == tsspin.TS_OK


def test_evolve_argument_checks_before_device():
    rc, ctx = _create(4, ((0, 1, 1.0, 1.0, 1.0),))
    assert rc == 0
    L = tsspin._lib
    dummy = (C.c_void_p * 1)(C.c_void_p(0x1000))
    # order, dt, n_psi, NULL, misalignment, dtype: rejected on the host
    assert L.ts_evolve(ctx, dummy, 1, 0, 0.1, 1, 3, None, 0, 1, None, None) == tsspin.TS_EINVAL
    assert "order" in tsspin.last_error()
    assert L.ts_evolve(ctx, dummy, 1, 0, math.nan, 1, 4, None, 0, 1, None, None) == tsspin.TS_EINVAL
    assert L.ts_evolve(ctx, dummy, 0, 0, 0.1, 1, 4, None, 0, 1, None, None) == tsspin.TS_EINVAL
    assert L.ts_evolve(ctx, None, 1, 0, 0.1, 1, 4, None, 0, 1, None, None) == tsspin.TS_EINVAL
    mis = (C.c_void_p * 1)(C.c_void_p(0x1008))
    assert L.ts_evolve(ctx, mis, 1, 0, 0.1, 1, 4, None, 0, 1, None, None) == tsspin.TS_EINVAL
    assert "misaligned" in tsspin.last_error()
    assert L.ts_evolve(ctx, dummy, 1, 7, 0.1, 1, 4, None, 0, 1, None, None) == tsspin.TS_EINVAL
    assert L.ts_evolve(ctx, dummy, 1, 0, 0.1, -1, 4, None, 0, 1, None, None) == tsspin.TS_EINVAL
    # observable checks
    ob = (tsspin.ts_observable * 1)()
    ob[0].kind, ob[0].i = tsspin.OBS["sz"], 9
    out = C.c_void_p(0x2000)
    assert L.ts_evolve(ctx, dummy, 1, 0, 0.1, 1, 4, ob, 1, 1, out, None) == tsspin.TS_EINVAL
    assert "spin index" in tsspin.last_error()
    ob[0].i, ob[0].ket = 0, 3
    assert L.ts_evolve(ctx, dummy, 1, 0, 0.1, 1, 4, ob, 1, 1, out, None) == tsspin.TS_EINVAL
    ob[0].ket = 0
    assert L.ts_evolve(ctx, dummy, 1, 0, 0.1, 1, 4, ob, 1, 0, out, None) == tsspin.TS_EINVAL
    assert L.ts_evolve(ctx, dummy, 1, 0, 0.1, 1, 4, ob, 1, 1, None, None) == tsspin.TS_EINVAL
    L.ts_destroy(ctx)


def test_c128_spin_limit():
    rc, ctx = _create(35)
    assert rc == 0
    dummy = (C.c_void_p * 1)(C.c_void_p(0x1000))
    assert tsspin._lib.ts_evolve(ctx, dummy, 1, tsspin.TS_C128, 0.1, 1, 4, None, 0, 1, None,
                                 None) == tsspin.TS_EINVAL
    assert "too many spins" in tsspin.last_error()
    tsspin._lib.ts_destroy(ctx)


def test_duplicate_bonds_are_summed_in_plan():
    # a bond listed twice must act like one bond with summed couplings
    a = tsspin.Hamiltonian(3, [(0, 1, 0.5, 0.0, 0.25), (1, 0, 0.5, 0.0, 0.25)])
    b = tsspin.Hamiltonian(3, [(0, 1, 1.0, 0.0, 0.5)])
    pa = a.plan(tsspin.TS_C128, 0.1, 2, 4)
    pb = b.plan(tsspin.TS_C128, 0.1, 2, 4)
    assert pa == pb


def test_one_hip_runtime_in_process():
    # the binding makes libtsspin bind to torch's HIP runtime (same soname); a second
    # runtime from /opt/rocm would see no device next to torch's
    assert len(tsspin._hip_runtimes()) <= 1
