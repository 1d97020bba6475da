"""ts_expect_noalloc (the allocation-free ts_expect, reductions in the library's fixed
scratch) called through the C ABI against ts_expect: the same values bit for bit, on two
calls in a row whose second has a smaller state (the scratch keeps the first call's
partials; the second must not read them)."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

from tests import dense_ref as D

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1305_0036_amd import tsspin
    return tsspin


def _noalloc(ts, H, x, observables):
    arr = (ts.ts_observable * len(observables))()
    slots = 0
    for k, ob in enumerate(observables):
        o = arr[k]
        o.kind = ts.OBS[ob[0]]
        if ob[0] == "szsz":
            o.i, o.j = ob[1], ob[2]
        elif ob[0] == "overlap_sz":
            o.i, o.other = ob[1], ob[2].data_ptr()
        elif ob[0] == "overlap":
            o.other = ob[1].data_ptr()
        elif ob[0] not in ("norm", "mz", "energy"):
            o.i = ob[1]
        slots += 2 if ob[0] in ("overlap_sz", "overlap") else 1
    out = torch.full((slots,), float("nan"), dtype=torch.float64, device=x.device)
    code = ts.TS_C128 if x.dtype == torch.complex128 else ts.TS_C64
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = ts._lib.ts_expect_noalloc(H._ctx, C.c_void_p(x.data_ptr()), code, arr, len(observables),
                                   C.c_void_p(out.data_ptr()), stream)
    return rc, out


@pytest.mark.parametrize("tdt", ["c128", "c64"])
def test_noalloc_expect_matches_expect(tdt):
    ts = _dev()
    dtype = torch.complex128 if tdt == "c128" else torch.complex64
    for n in (21, 12):   # the second call is smaller
        print(f"[case] noalloc n={n} {tdt}", flush=True)
        rng = np.random.default_rng(5000 + n)
        bonds, fields = D.random_xyz(rng, n, chain=True)
        H = ts.Hamiltonian(n, bonds, fields)
        x = torch.from_numpy(D.random_state(rng, n)).to(dtype).cuda()
        y = torch.from_numpy(D.random_state(rng, n)).to(dtype).cuda()
        obs = [("norm",), ("sz", 1), ("sx", 2), ("sy", n - 1), ("szsz", 0, n - 1), ("mz",),
               ("overlap_sz", 3, y), ("overlap", y)]
        ref = H.expect(x, obs)
        rc, out = _noalloc(ts, H, x, obs)
        assert rc == ts.TS_OK, ts.last_error()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        flat = []
        for v in ref:
            flat += [v.real, v.imag] if isinstance(v, complex) else [v]
        assert np.array_equal(got, np.array(flat)), (got, flat)
    # the energy needs the context's device copy of H: refused, nothing written
    rc, out = _noalloc(ts, H, x, [("energy",)])
    assert rc == ts.TS_EUNSUPPORTED and "energy" in ts.last_error()
    torch.cuda.synchronize()
    assert torch.isnan(out).all()
