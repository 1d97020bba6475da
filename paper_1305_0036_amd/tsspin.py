"""Thin ctypes binding of libtsspin (include/tsspin.h).

Argument marshalling only: every step of the evolution runs in the HIP kernels of the
library.  State vectors are torch tensors on the GPU (complex128 or complex64); torch
provides device memory and streams.  If the built library is missing this module raises
at import time; there is no other code path.
"""
from __future__ import annotations

import ctypes as C
import os
import struct

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsspin.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libtsspin.so not found at {LIB_PATH}; build it with "
        "`python -m paper_1305_0036_amd.build` (hipcc, gfx950)")

# torch first: its bundled HIP runtime has the same soname (libamdhip64.so.7) as the one
# libtsspin links, so the library then binds to torch's runtime instead of loading a second
# one from /opt/rocm.  Two HIP runtimes in one process do not share devices or streams.
import torch  # noqa: E402,F401


def _hip_runtimes():
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})
    except OSError:
        return []


_lib = C.CDLL(LIB_PATH)
if len(_hip_runtimes()) > 1:
    raise ImportError("two HIP runtimes are loaded in this process (%s); import torch before "
                      "anything that loads libamdhip64" % ", ".join(_hip_runtimes()))

TS_OK, TS_EINVAL, TS_ENOMEM, TS_EDEVICE, TS_EUNSUPPORTED, TS_ENUMERIC = 0, -1, -2, -3, -4, -5
TS_C128, TS_C64 = 0, 1
OBS = {"norm": 0, "sx": 1, "sy": 2, "sz": 3, "szsz": 4, "mz": 5, "energy": 6, "overlap_sz": 7,
       "overlap": 8}
_COMPLEX = ("overlap_sz", "overlap")


class ts_bond(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("jx", C.c_double), ("jy", C.c_double),
                ("jz", C.c_double)]


class ts_observable(C.Structure):
    _fields_ = [("kind", C.c_int32), ("i", C.c_int32), ("j", C.c_int32), ("ket", C.c_int32),
                ("bra", C.c_int32), ("other", C.c_void_p)]


_P = C.c_void_p
_I32, _I64, _F64, _INT = C.c_int32, C.c_int64, C.c_double, C.c_int
# every entry point of include/tsspin.h: name -> (restype, argtypes)
_SIGNATURES = {
    "ts_create": (_INT, [_I32, C.POINTER(ts_bond), _I32, _P, C.POINTER(_P)]),
    "ts_destroy": (_INT, [_P]),
    "ts_evolve": (_INT, [_P, C.POINTER(_P), _I32, _INT, _F64, _I64, _I32,
                         C.POINTER(ts_observable), _I32, _I32, _P, _P]),
    "ts_set_watchdog": (_INT, [_P, _F64]),
    "ts_expect": (_INT, [_P, _P, _INT, C.POINTER(ts_observable), _I32, _P, _P]),
    "ts_expect_noalloc": (_INT, [_P, _P, _INT, C.POINTER(ts_observable), _I32, _P, _P]),
    "ts_adjoint": (_INT, [_P, _P, _INT, _F64, _I64, _I32, C.POINTER(ts_observable), _P, _P, _P,
                          _P, _P]),
    "ts_create_batch": (_INT, [_I32, _P, _P, _P, _P, C.POINTER(_P)]),
    "ts_evolve_batch": (_INT, [_P, _P, _P, _INT, _F64, _I64, _I32, C.POINTER(ts_observable),
                               _I32, _I32, _P, _P]),
    "ts_set_tile_bits": (_INT, [_P, _INT, _I32]),
    "ts_batch_stats": (_INT, [_P, _P]),
    "ts_autotune": (_INT, [_P, _INT, _I32, _P, _I32, _P, _P]),
    "ts_get_kernel_config": (_INT, [_P, _INT, _I32, _P, _P, _P]),
    "ts_last_error": (C.c_char_p, []),
    "ts_plan_describe": (_INT, [_P, _INT, _F64, _I64, _I32, _I32, _P, _I64, C.POINTER(_I64)]),
    "ts_cone_describe": (_INT, [_P, _INT, _F64, _I64, _I32, _I32, _I32, _I32, _P, _I64,
                                C.POINTER(_I64), C.POINTER(_I32)]),
    "ts_dt_bound": (_INT, [_P, C.POINTER(_F64)]),
}
for _name, (_res, _args) in _SIGNATURES.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
EXPORTED = sorted(_SIGNATURES)


class TsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libtsspin error {code}: {msg}")
        self.code = code


def _check(rc: int):
    if rc != TS_OK:
        raise TsError(rc, _lib.ts_last_error().decode())


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.complex128:
        return TS_C128
    if t.dtype == torch.complex64:
        return TS_C64
    raise TypeError(f"state must be complex128 or complex64, got {t.dtype}")


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _obs_array(observables, n_psi):
    """('norm',), ('sz', i), ('szsz', i, j), ('sx', i), ('sy', i), ('mz',), ('energy',),
    ('overlap_sz', i, bra, ket), ('overlap', bra, ket) -- an optional trailing ket index
    selects the vector."""
    arr = (ts_observable * max(1, len(observables)))()
    slots = 0
    for k, ob in enumerate(observables):
        kind = ob[0]
        o = arr[k]
        o.kind = OBS[kind]
        o.ket = 0
        if kind in ("sx", "sy", "sz"):
            o.i = ob[1]
            o.ket = ob[2] if len(ob) > 2 else 0
        elif kind == "szsz":
            o.i, o.j = ob[1], ob[2]
            o.ket = ob[3] if len(ob) > 3 else 0
        elif kind in ("norm", "mz", "energy"):
            o.ket = ob[1] if len(ob) > 1 else 0
        elif kind == "overlap_sz":
            o.i, o.bra, o.ket = ob[1], ob[2], ob[3]
        elif kind == "overlap":
            o.bra, o.ket = ob[1], ob[2]
        slots += 2 if kind in _COMPLEX else 1
    return arr, slots


class Hamiltonian:
    """H of Eq. 1: bonds = [(i, j, Jx, Jy, Jz), ...], fields = (n, 3) or None."""

    def __init__(self, n: int, bonds=(), fields=None):
        self.n = int(n)
        self.bonds = list(bonds)
        nb = len(self.bonds)
        barr = (ts_bond * max(1, nb))()
        for k, b in enumerate(self.bonds):
            barr[k].i, barr[k].j = int(b[0]), int(b[1])
            barr[k].jx, barr[k].jy, barr[k].jz = float(b[2]), float(b[3]), float(b[4])
        self._fields = None
        fptr = None
        if fields is not None:
            self._fields = np.ascontiguousarray(fields, dtype=np.float64).reshape(self.n, 3)
            fptr = self._fields.ctypes.data_as(C.c_void_p)
        ctx = C.c_void_p()
        _check(_lib.ts_create(self.n, barr if nb else None, nb, fptr, C.byref(ctx)))
        self._ctx = ctx

    def close(self):
        if getattr(self, "_ctx", None):
            _lib.ts_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ evolution
    def evolve(self, psi, dt: float, nsteps: int, order: int = 4, record=(), rec_every: int = 1,
               rec_out=None, stream=None):
        """Evolve one tensor or a list of tensors in place.  Returns the record tensor
        (float64, [(nsteps // rec_every) + 1, slots], on the GPU) when `record` is given."""
        import torch
        vecs = list(psi) if isinstance(psi, (list, tuple)) else [psi]
        code = _dtype_code(vecs[0])
        for v in vecs:
            if not v.is_cuda or not v.is_contiguous() or v.numel() != (1 << self.n):
                raise ValueError("each state must be a contiguous CUDA tensor of 2^n amplitudes")
            if _dtype_code(v) != code:
                raise ValueError("all states must share one dtype")
        ptrs = (C.c_void_p * len(vecs))(*[v.data_ptr() for v in vecs])
        obs, slots = _obs_array(record, len(vecs))
        out = None
        out_ptr = None
        if record:
            nrec = nsteps // rec_every + 1
            out = rec_out if rec_out is not None else torch.empty(
                (nrec, slots), dtype=torch.float64, device=vecs[0].device)
            out_ptr = C.c_void_p(out.data_ptr())
        _check(_lib.ts_evolve(self._ctx, ptrs, len(vecs), code, float(dt), int(nsteps), int(order),
                              obs if record else None, len(record), int(rec_every), out_ptr,
                              _stream_ptr(stream)))
        return out

    def expect(self, psi, observables, stream=None):
        """Observables of one state: ('sz', i), ('szsz', i, j), ('norm',), ('mz',), ('energy',),
        ('sx', i), ('sy', i), ('overlap_sz', i, other_tensor), ('overlap', other_tensor)
        (<other|psi>).  Synchronises."""
        code = _dtype_code(psi)
        arr = (ts_observable * max(1, len(observables)))()
        slots = 0
        keep = []
        for k, ob in enumerate(observables):
            o = arr[k]
            o.kind = OBS[ob[0]]
            if ob[0] == "szsz":
                o.i, o.j = ob[1], ob[2]
            elif ob[0] == "overlap_sz":
                o.i = ob[1]
                o.other = ob[2].data_ptr()
                keep.append(ob[2])
            elif ob[0] == "overlap":
                o.other = ob[1].data_ptr()
                keep.append(ob[1])
            elif ob[0] not in ("norm", "mz", "energy"):
                o.i = ob[1]
            slots += 2 if ob[0] in _COMPLEX else 1
        out = np.zeros(max(1, slots), dtype=np.float64)
        _check(_lib.ts_expect(self._ctx, C.c_void_p(psi.data_ptr()), code, arr, len(observables),
                              out.ctypes.data_as(C.c_void_p), _stream_ptr(stream)))
        res, s = [], 0
        for ob in observables:
            if ob[0] in _COMPLEX:
                res.append(complex(out[s], out[s + 1]))
                s += 2
            else:
                res.append(float(out[s]))
                s += 1
        return res

    def adjoint(self, psi0, dt: float, nsteps: int, order: int, observable, workspace=None,
                stream=None):
        """(loss, grad_bonds[n_bonds][3], grad_fields[n][3]) of <psi(T)|O|psi(T)> by the
        adjoint pass of the library.  observable: ('sz', i), ('sx', i), ('sy', i),
        ('szsz', i, j), ('mz',) or ('energy',)."""
        import torch
        code = _dtype_code(psi0)
        if not psi0.is_cuda or not psi0.is_contiguous() or psi0.numel() != (1 << self.n):
            raise ValueError("psi0 must be a contiguous CUDA tensor of 2^n amplitudes")
        if workspace is None:
            workspace = torch.empty(2 << self.n, dtype=psi0.dtype, device=psi0.device)
        ob = ts_observable()
        ob.kind = OBS[observable[0]]
        if observable[0] == "szsz":
            ob.i, ob.j = observable[1], observable[2]
        elif observable[0] not in ("mz", "energy"):
            ob.i = observable[1]
        loss = np.zeros(1, dtype=np.float64)
        gb = np.zeros((max(1, len(self.bonds)), 3), dtype=np.float64)
        gf = np.zeros((self.n, 3), dtype=np.float64)
        _check(_lib.ts_adjoint(self._ctx, C.c_void_p(psi0.data_ptr()), code, float(dt), int(nsteps),
                               int(order), C.byref(ob), loss.ctypes.data_as(C.c_void_p),
                               gb.ctypes.data_as(C.c_void_p), gf.ctypes.data_as(C.c_void_p),
                               C.c_void_p(workspace.data_ptr()), _stream_ptr(stream)))
        return float(loss[0]), gb[: len(self.bonds)], gf

    def set_tile_bits(self, dtype: int, tile_bits: int):
        """Tile width used by evolve for dtype (0 = library default)."""
        _check(_lib.ts_set_tile_bits(self._ctx, dtype, tile_bits))

    def set_watchdog(self, max_drift: float):
        """Norm watchdog of evolve (see ts_set_watchdog): a relative drift bound, < 0 = off.
        A tripped watchdog raises TsError with code TS_ENUMERIC."""
        _check(_lib.ts_set_watchdog(self._ctx, float(max_drift)))

    def dt_bound(self) -> float:
        """Local time scale of the Hamiltonian (Sec. 2, Eq. SegundoMomento, see
        ts_dt_bound): the Trotter step dt must be much smaller than it."""
        out = C.c_double()
        _check(_lib.ts_dt_bound(self._ctx, C.byref(out)))
        return out.value

    def autotune(self, dtype: int, order: int = 4, use_cache: bool = True, stream=None):
        """Time the kernel configurations for this system (see ts_autotune); returns the
        chosen configuration and its time per step."""
        import torch
        tdt = torch.complex128 if dtype == TS_C128 else torch.complex64
        scratch = torch.zeros(1 << self.n, dtype=tdt, device="cuda")
        scratch[0] = 1.0
        ms = np.zeros(1, dtype=np.float64)
        _check(_lib.ts_autotune(self._ctx, dtype, order, C.c_void_p(scratch.data_ptr()),
                                int(use_cache), ms.ctypes.data_as(C.c_void_p), _stream_ptr(stream)))
        cfg = self.kernel_config(dtype, order)
        cfg["ms_per_step"] = float(ms[0])
        return cfg

    def kernel_config(self, dtype: int, order: int = 4):
        """Tile width, register window and kernel variant evolve uses (ts_get_kernel_config)."""
        t, r, v = C.c_int32(), C.c_int32(), C.c_int32()
        _check(_lib.ts_get_kernel_config(self._ctx, dtype, order, C.byref(t), C.byref(r),
                                         C.byref(v)))
        return {"tile_bits": t.value, "reg_bits": r.value, "variant": v.value}

    # --------------------------------------------------------------- introspection
    def plan(self, dtype: int, dt: float, nsteps: int, order: int = 4, tile_bits: int = 0):
        """Sweep plan as a list of dicts (host only, see ts_plan_describe)."""
        n = C.c_int64()
        _check(_lib.ts_plan_describe(self._ctx, dtype, dt, nsteps, order, tile_bits, None, 0,
                                     C.byref(n)))
        buf = np.zeros((max(1, n.value), 16), dtype=np.int64)
        _check(_lib.ts_plan_describe(self._ctx, dtype, dt, nsteps, order, tile_bits,
                                     buf.ctypes.data_as(C.c_void_p), n.value, C.byref(n)))
        out = []
        for r in buf[: n.value]:
            info = int(r[13])
            nst = (info >> 24) & 0xFF
            words = [int(r[14]) & ((1 << 64) - 1), int(r[15]) & ((1 << 64) - 1)]
            codes = [(words[k // 7] >> (9 * (k % 7))) & 0x1FF for k in range(nst)]
            out.append(dict(tile=int(r[0]) & ((1 << 64) - 1), pre=int(r[1]), post=int(r[2]),
                            axis=int(r[3]), qturn=int(r[4]), mag_exp=int(r[5]),
                            mag_sqrt=int(r[6]), eighths=int(r[7]), tile_bits=int(r[8]),
                            group=int(r[9]),
                            tau=struct.unpack("<d", struct.pack("<q", int(r[10])))[0],
                            reg_bits=int(r[12]), load_win=info & 0xFF,
                            store_win=(info >> 8) & 0xFF, phase_win=((info >> 16) & 0xFF) - 1,
                            transposes=(info >> 32) & 0xFF,
                            stages=[(c & 15, (c >> 4) & 1, c >> 5) for c in codes]))
        return out

    def cone_plan(self, dtype: int, dt: float, nsteps: int, order: int = 4, tile_bits: int = 0,
                  low_bits: int = 0, max_adv: int = 0):
        """Light-cone form of the segment (host only, see ts_cone_describe): a list of sweeps,
        each a dict with the window, the tile-bit layout and the operation list; plus whether
        ts_evolve would run it."""
        n = C.c_int64()
        used = C.c_int32()
        _check(_lib.ts_cone_describe(self._ctx, dtype, dt, nsteps, order, tile_bits, low_bits,
                                     max_adv, None, 0, C.byref(n), C.byref(used)))
        buf = np.zeros((max(1, n.value), 10), dtype=np.int64)
        _check(_lib.ts_cone_describe(self._ctx, dtype, dt, nsteps, order, tile_bits, low_bits,
                                     max_adv, buf.ctypes.data_as(C.c_void_p), n.value, C.byref(n),
                                     None))
        sweeps = []
        for r in buf[: n.value]:
            kind = int(r[0])
            if kind == 1:
                sweeps.append(dict(window=int(r[1]), low_load=int(r[2]), low_store=int(r[3]),
                                   remap=bool(r[4]), stages=int(r[6]), transposes=int(r[7]),
                                   tile=[], ops=[]))
            elif kind == 4:
                sweeps[-1]["tile"].append((int(r[2]), int(r[3]), int(r[4])))
            elif kind == 5:
                if int(r[1]) == -1:
                    sweeps[-1]["program"] = dict(load_win=int(r[5]), stages=[])
                elif int(r[1]) == -2:
                    sweeps[-1]["program"]["store_win"] = int(r[5])
                else:
                    sweeps[-1]["program"]["stages"].append(
                        dict(win=int(r[1]), phase=bool(r[2]), mask=int(r[3]), step=int(r[4])))
            elif kind == 2:
                sweeps[-1]["ops"].append(dict(kind="bfly", spins=int(r[1])))
            elif kind == 3:
                sweeps[-1]["ops"].append(dict(
                    kind="phase", level=int(r[1]), own=int(r[2]), bonds=int(r[3]),
                    half_scale=int(r[4]), eighths=int(r[5]), axis=int(r[6]), qturn=int(r[7]),
                    tau=struct.unpack("<d", struct.pack("<q", int(r[8])))[0], win=int(r[9])))
        return sweeps, bool(used.value)

    def launches(self, dtype: int, dt: float, nsteps: int, order: int = 4):
        """(sweep launches per vector for a segment of nsteps steps, light-cone form used)."""
        try:
            sw, used = self.cone_plan(dtype, dt, nsteps, order)
        except TsError:
            sw, used = [], False
        return (len(sw), True) if used else (len(self.plan(dtype, dt, nsteps, order)), False)


def last_error() -> str:
    return _lib.ts_last_error().decode()


_CTX_CACHE: "dict" = {}
_CTX_CACHE_MAX = 4


def _cached_hamiltonian(n, pairs, J, h):
    """The Hamiltonian object for these exact parameter values, reused across calls so that
    its plans and tables survive (a few most recent parameter sets are kept)."""
    Jn = np.ascontiguousarray(J.detach().cpu().numpy(), dtype=np.float64).reshape(len(pairs), 3)
    hn = np.ascontiguousarray(h.detach().cpu().numpy(), dtype=np.float64).reshape(n, 3)
    key = (int(n), tuple((int(i), int(j)) for i, j in pairs), Jn.tobytes(), hn.tobytes())
    H = _CTX_CACHE.pop(key, None)
    if H is None:
        bonds = [(int(i), int(j), *Jn[k]) for k, (i, j) in enumerate(pairs)]
        H = Hamiltonian(n, bonds, hn)
        while len(_CTX_CACHE) >= _CTX_CACHE_MAX:
            _CTX_CACHE.pop(next(iter(_CTX_CACHE))).close()
    _CTX_CACHE[key] = H
    return H


def _make_autograd():
    import torch

    class TSExpectation(torch.autograd.Function):
        """L = <psi(T)|O|psi(T)> as a differentiable function of the couplings J[n_bonds][3]
        and fields h[n][3] (float64 CPU tensors).  forward runs the evolution and backward
        returns the adjoint gradient computed by the library (ts_adjoint)."""

        @staticmethod
        def forward(ctx, J, h, n, pairs, psi0, dt, nsteps, order, observable):
            H = _cached_hamiltonian(n, pairs, J, h)
            loss, gb, gf = H.adjoint(psi0, dt, nsteps, order, observable)
            ctx.save_for_backward(torch.from_numpy(gb.copy()), torch.from_numpy(gf.copy()))
            return torch.tensor(loss, dtype=torch.float64)

        @staticmethod
        def backward(ctx, g):
            gb, gf = ctx.saved_tensors
            return g * gb, g * gf, None, None, None, None, None, None, None

    return TSExpectation


_AUTOGRAD = []


def expectation(J, h, n, pairs, psi0, dt, nsteps, order, observable):
    """Differentiable <psi(T)|O|psi(T)>: see TSExpectation."""
    if not _AUTOGRAD:
        _AUTOGRAD.append(_make_autograd())
    return _AUTOGRAD[0].apply(J, h, n, pairs, psi0, dt, nsteps, order, observable)


class Batch:
    """Independent systems evolved together: systems = [(n, bonds, fields), ...]."""

    def __init__(self, systems):
        self.ns = [int(s[0]) for s in systems]
        nb = [len(s[1]) for s in systems]
        off = np.zeros(len(systems) + 1, dtype=np.int32)
        off[1:] = np.cumsum(nb)
        barr = (ts_bond * max(1, int(off[-1])))()
        k = 0
        for s in systems:
            for b in s[1]:
                barr[k].i, barr[k].j = int(b[0]), int(b[1])
                barr[k].jx, barr[k].jy, barr[k].jz = float(b[2]), float(b[3]), float(b[4])
                k += 1
        fields = np.concatenate([np.zeros((s[0], 3)) if s[2] is None else
                                 np.asarray(s[2], dtype=np.float64).reshape(s[0], 3) for s in systems])
        self._fields = np.ascontiguousarray(fields)
        self._ns = np.ascontiguousarray(self.ns, dtype=np.int32)
        self._off = off
        ctx = C.c_void_p()
        _check(_lib.ts_create_batch(len(systems), self._ns.ctypes.data_as(C.c_void_p),
                                    barr, off.ctypes.data_as(C.c_void_p),
                                    self._fields.ctypes.data_as(C.c_void_p), C.byref(ctx)))
        self._ctx = ctx
        self.offsets = np.concatenate([[0], np.cumsum([1 << n for n in self.ns])[:-1]]).astype(np.int64)
        self.total = int(sum(1 << n for n in self.ns))

    def autotune(self, dtype: int, order: int = 4, stream=None):
        """Time one step of the whole batch for each tile width and register window (see
        ts_autotune) and keep the fastest on this batch; returns its time per step (ms)."""
        import torch
        tdt = torch.complex128 if dtype == TS_C128 else torch.complex64
        scratch = torch.zeros(self.total, dtype=tdt, device="cuda")
        ms = np.zeros(1, dtype=np.float64)
        _check(_lib.ts_autotune(self._ctx, dtype, order, C.c_void_p(scratch.data_ptr()), 0,
                                ms.ctypes.data_as(C.c_void_p), _stream_ptr(stream)))
        return float(ms[0])

    def close(self):
        if getattr(self, "_ctx", None):
            _lib.ts_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tile_bits(self, dtype: int, tile_bits: int):
        _check(_lib.ts_set_tile_bits(self._ctx, dtype, tile_bits))

    def stats(self):
        """Counters of evolve (see ts_batch_stats): graph replays, uncaptured runs, failed
        captures, captured programs kept."""
        out = np.zeros(4, dtype=np.int64)
        _check(_lib.ts_batch_stats(self._ctx, out.ctypes.data_as(C.c_void_p)))
        return dict(graph_replays=int(out[0]), eager_runs=int(out[1]), capture_failures=int(out[2]),
                    programs=int(out[3]))

    def evolve(self, packed, dt: float, nsteps: int, order: int = 4, record=(), rec_every: int = 1,
               rec_out=None, stream=None):
        """Evolve the packed states (system c at self.offsets[c]) in place.  Returns the
        records [n_systems, nsteps // rec_every + 1, len(record)] (float64, GPU) if asked."""
        import torch
        code = _dtype_code(packed)
        if not packed.is_cuda or not packed.is_contiguous() or packed.numel() != self.total:
            raise ValueError("packed must be a contiguous CUDA tensor of sum(2^n) amplitudes")
        obs, slots = _obs_array(record, 1)
        out, out_ptr = None, None
        if record:
            nrec = nsteps // rec_every + 1
            out = rec_out if rec_out is not None else torch.empty(
                (len(self.ns), nrec, slots), dtype=torch.float64, device=packed.device)
            out_ptr = C.c_void_p(out.data_ptr())
        off = np.ascontiguousarray(self.offsets)
        _check(_lib.ts_evolve_batch(self._ctx, C.c_void_p(packed.data_ptr()),
                                    off.ctypes.data_as(C.c_void_p), code, float(dt), int(nsteps),
                                    int(order), obs if record else None, len(record), int(rec_every),
                                    out_ptr, _stream_ptr(stream)))
        return out
