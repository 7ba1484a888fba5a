"""Python binding of the itse C ABI: argument marshalling only.

Every step of the method runs in the HIP library; torch provides device memory
(through the allocator callbacks of ``itse_create``) and the HIP stream.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _lib
from ._lib import check

_PREC = {"fp64": _lib.FP64, "fp32": _lib.FP32}
_CENTER = {"cell": _lib.CENTER_CELL, "origin": _lib.CENTER_ORIGIN}


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the itse HIP path needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


class _TorchAllocator:
    """Device memory for the library from torch's caching allocator."""

    def __init__(self):
        self.torch = _torch()
        self.live: Dict[int, object] = {}
        self._alloc = _lib.ALLOC_FN(self.alloc)
        self._free = _lib.FREE_FN(self.free)

    def alloc(self, nbytes, user):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device="cuda")
        except Exception:  # out of memory -> NULL, the library reports ITSE_ENOMEM
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def free(self, ptr, user):
        self.live.pop(ptr, None)


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream), stream


def _is_device_tensor(x):
    try:
        import torch
        return isinstance(x, torch.Tensor) and x.is_cuda
    except ImportError:
        return False


def _dtype_code(x):
    if _is_device_tensor(x):
        import torch
        if x.dtype == torch.float32:
            return _lib.DTYPE_F32
        if x.dtype == torch.float64:
            return _lib.DTYPE_F64
    else:
        if x.dtype == np.float32:
            return _lib.DTYPE_F32
        if x.dtype == np.float64:
            return _lib.DTYPE_F64
    raise TypeError(f"unsupported dtype {x.dtype}; use float32 or float64")


def make_opts(nstates: int, ortho_every: int = 1, moments: bool = False,
              parity: Optional[Sequence[int]] = None, axes: Optional[Sequence[int]] = None):
    o = _lib.StepOpts()
    o.ortho_every = int(ortho_every)
    o.moments = 1 if moments else 0
    for i in range(_lib.MAX_STATES):
        o.parity[i] = int(parity[i]) if parity is not None and i < len(parity) else 0
        o.axes[i] = int(axes[i]) if axes is not None and i < len(axes) else 7
    return o


class Lattice:
    """One N^3 lattice with `nstates` states evolved by the imaginary-time map.

    complex_psi=True: one complex state in a complex potential (set_potential takes
    a complex array; set_state(0, psi) / get_state(0) complex arrays; the library
    holds Re psi and Im psi as its states 0 and 1)."""

    def __init__(self, n: int, a: float, mass: float, dtau: float, kin: int = _lib.KIN_REL_LAT,
                 subtract_rest_mass: bool = True, precision: str = "fp64", center: str = "origin",
                 nstates: int = 1, stream=None, torch_memory: bool = True, complex_psi: bool = False):
        self._L = _lib.load()
        self.n, self.nstates = int(n), int(nstates)
        self.complex_psi = bool(complex_psi)
        self.precision = precision
        self.desc = _lib.Desc(int(n), float(a), float(mass), float(dtau), int(kin),
                              1 if subtract_rest_mass else 0, _PREC[precision], _CENTER[center],
                              int(nstates), 1 if complex_psi else 0)
        self._stream_ptr, self.stream = _stream_handle(stream)
        self._alloc = _TorchAllocator() if torch_memory else None
        handle = ctypes.c_void_p()
        af = self._alloc._alloc if self._alloc else _lib.ALLOC_FN(0)
        ff = self._alloc._free if self._alloc else _lib.FREE_FN(0)
        check(self._L.itse_create(ctypes.byref(self.desc), self._stream_ptr, af, ff, None,
                                  ctypes.byref(handle)))
        self.h = handle
        self._opts = make_opts(self.nstates)

    # -- lifetime -----------------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self._L.itse_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @staticmethod
    def footprint(n, nstates=1, precision="fp64", complex_psi=False, **kw) -> int:
        d = _lib.Desc(int(n), 1.0, 1.0, 1e-3, _lib.KIN_NR_CONT, 1, _PREC[precision], 0, int(nstates),
                      1 if complex_psi else 0)
        return int(_lib.load().itse_footprint_bytes(ctypes.byref(d)))

    # -- data -----------------------------------------------------------------------------
    def _in(self, arr):
        if _is_device_tensor(arr):
            t = arr.contiguous()
            assert t.numel() == self.n ** 3, "expected N^3 values"
            return ctypes.c_void_p(t.data_ptr()), _dtype_code(t), 1, t
        a = np.ascontiguousarray(arr)
        if a.dtype not in (np.float32, np.float64):
            a = a.astype(np.float64)
        assert a.size == self.n ** 3, "expected N^3 values"
        return a.ctypes.data_as(ctypes.c_void_p), _dtype_code(a), 0, a

    @staticmethod
    def _parts(x):
        """Real and imaginary parts of a complex array or tensor (contiguous copies)."""
        if _is_device_tensor(x):
            return x.real.contiguous(), x.imag.contiguous()
        x = np.asarray(x)
        return np.ascontiguousarray(x.real), np.ascontiguousarray(x.imag)

    def set_potential(self, v):
        if self.complex_psi:
            vr, vi = self._parts(v)
            p, dt, dev, keep = self._in(vr)
            check(self._L.itse_set_potential(self.h, p, dt, dev))
            self.set_potential_imag(vi)
            return
        p, dt, dev, keep = self._in(v)
        check(self._L.itse_set_potential(self.h, p, dt, dev))

    def set_potential_imag(self, vi):
        """Imaginary part of the potential (complex lattices only)."""
        p, dt, dev, keep = self._in(vi)
        check(self._L.itse_set_potential_imag(self.h, p, dt, dev))
        if dev:
            self.sync()

    def set_state(self, i: int, psi):
        if self.complex_psi and int(i) == 0:
            re, im = self._parts(psi)
            for part, arr in ((0, re), (1, im)):
                p, dt, dev, keep = self._in(arr)
                check(self._L.itse_set_state(self.h, part, p, dt, dev))
                if dev:
                    self.sync()
            return
        p, dt, dev, keep = self._in(psi)
        check(self._L.itse_set_state(self.h, int(i), p, dt, dev))
        if dev:
            self.sync()

    def get_state(self, i: int, dtype=np.float64, device: bool = False):
        if self.complex_psi and int(i) == 0:
            re = self._get_part(0, dtype, device)
            im = self._get_part(1, dtype, device)
            return re + 1j * im if not device else _torch().complex(re, im)
        return self._get_part(i, dtype, device)

    def _get_part(self, i: int, dtype=np.float64, device: bool = False):
        n = self.n
        if device:
            torch = _torch()
            tdt = torch.float32 if dtype in (np.float32, torch.float32) else torch.float64
            out = torch.empty((n, n, n), dtype=tdt, device="cuda")
            code = _lib.DTYPE_F32 if tdt == torch.float32 else _lib.DTYPE_F64
            check(self._L.itse_get_state(self.h, int(i), ctypes.c_void_p(out.data_ptr()), code, 1))
            return out
        out = np.empty((n, n, n), dtype=dtype)
        code = _lib.DTYPE_F32 if out.dtype == np.float32 else _lib.DTYPE_F64
        check(self._L.itse_get_state(self.h, int(i), out.ctypes.data_as(ctypes.c_void_p), code, 0))
        return out

    # -- stepping -------------------------------------------------------------------------
    def set_options(self, ortho_every: int = 1, moments: bool = False,
                    parity: Optional[Sequence[int]] = None, axes: Optional[Sequence[int]] = None):
        self._opts = make_opts(self.nstates, ortho_every, moments, parity, axes)
        check(self._L.itse_set_step_opts(self.h, ctypes.byref(self._opts)))

    def step(self, nsteps: int = 1):
        check(self._L.itse_step(self.h, int(nsteps), None))

    def evaluate(self, moments: bool = True):
        check(self._L.itse_evaluate(self.h, 1 if moments else 0))

    def observe(self, i: int) -> dict:
        o = _lib.Obs()
        check(self._L.itse_observe(self.h, int(i), ctypes.byref(o)))
        return o.as_dict()

    def observe_all(self) -> List[dict]:
        return [self.observe(i) for i in range(self.nstates)]

    def history(self, count: int) -> List[List[dict]]:
        buf = (_lib.Obs * (count * self.nstates))()
        check(self._L.itse_history(self.h, int(count), buf))
        k = self.nstates
        return [[buf[c * k + i].as_dict() for i in range(k)] for c in range(count)]

    @property
    def step_count(self) -> int:
        return int(self._L.itse_step_count(self.h))

    def orthogonalise(self, i: int):
        check(self._L.itse_orthogonalise(self.h, int(i)))

    def project_parity(self, i: int, sign: int, axes: int = 7) -> float:
        w = ctypes.c_double()
        check(self._L.itse_project_parity(self.h, int(i), int(sign), int(axes), ctypes.byref(w)))
        return w.value

    def apply_kinetic(self, i: int):
        torch = _torch()
        dt = torch.float32 if self.precision == "fp32" else torch.float64
        out = torch.empty((self.n,) * 3, dtype=dt, device="cuda")
        check(self._L.itse_apply_kinetic(self.h, int(i), ctypes.c_void_p(out.data_ptr())))
        self.sync()
        return out

    def spectrum(self, i: int):
        torch = _torch()
        dt = torch.float32 if self.precision == "fp32" else torch.float64
        n = self.n
        out = torch.empty((n, n, n // 2 + 1, 2), dtype=dt, device="cuda")
        check(self._L.itse_spectrum(self.h, int(i), ctypes.c_void_p(out.data_ptr())))
        self.sync()
        return out

    def polish(self, i: int) -> dict:
        o = _lib.Obs()
        check(self._L.itse_polish(self.h, int(i), ctypes.byref(o)))
        return o.as_dict()

    def sync(self):
        check(self._L.itse_sync(self.h))

    # -- analysis (itse_analyse, itse_momentum_radial) ---------------------------------
    def analyse(self, i: int, min_sep_edge: float = 0.3) -> dict:
        """Box normalisation, average radius (lattice units) and parity weights of
        state i in the effective volume of side (1 - min_sep_edge) A N."""
        out = _lib.Analysis()
        check(self._L.itse_analyse(self.h, int(i), float(min_sep_edge), ctypes.byref(out)))
        return out.as_dict()

    def analyse_noalloc(self, i: int, min_sep_edge: float = 0.3) -> dict:
        """analyse() through itse_analyse_noalloc: the same results with no device
        allocation (the library's fixed per-GPU workspace)."""
        out = _lib.Analysis()
        check(self._L.itse_analyse_noalloc(self.h, int(i), float(min_sep_edge), ctypes.byref(out)))
        return out.as_dict()

    def momentum_radial(self, i: int, nbins: int) -> dict:
        """Radial momentum-space wave-function of state i in bins of 2 pi / (N A):
        arrays count, p, psi (mean |Psi(p)|) and y = sqrt(4 pi) p psi."""
        arrs = {k: np.zeros(int(nbins)) for k in ("count", "p", "psi", "y")}
        ptr = {k: v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for k, v in arrs.items()}
        check(self._L.itse_momentum_radial(self.h, int(i), int(nbins), ptr["count"], ptr["p"], ptr["psi"],
                                           ptr["y"]))
        return arrs

    # -- snapshot-overlap extraction (itse_snapshot_*) ---------------------------------
    def snapshot(self):
        """Keep the current state 0 as the newest snapshot (the ring holds two)."""
        check(self._L.itse_snapshot_push(self.h))

    @property
    def snapshot_count(self) -> int:
        c = ctypes.c_int()
        check(self._L.itse_snapshot_count(self.h, ctypes.byref(c)))
        return c.value

    def clear_snapshots(self):
        check(self._L.itse_snapshot_clear(self.h))

    def extract(self, states: bool = False, dtype=np.float64):
        """Estimates from the current state 0 and the snapshots, newest first:
        list of observable dicts, and with states=True also the estimates as an
        array [1 + snapshot_count, N, N, N] of `dtype`."""
        outs = (_lib.Obs * 3)()
        n_out = ctypes.c_int()
        arr = None
        ptr = None
        code = _lib.DTYPE_F64
        if states:
            n = self.n
            arr = np.empty((1 + self.snapshot_count, n, n, n), dtype=dtype)
            code = _lib.DTYPE_F32 if arr.dtype == np.float32 else _lib.DTYPE_F64
            ptr = arr.ctypes.data_as(ctypes.c_void_p)
        check(self._L.itse_snapshot_extract(self.h, outs, ctypes.byref(n_out), ptr, code, 0))
        obs = [outs[k].as_dict() for k in range(n_out.value)]
        return (obs, arr) if states else obs

    def profile_step(self, nsteps: int = 5):
        """Mean duration (ms) of each pass of a step, measured with HIP events."""
        import json
        ms = (ctypes.c_double * 16)()
        npass = ctypes.c_int(16)
        names = ctypes.create_string_buffer(1024)
        check(self._L.itse_profile_step(self.h, int(nsteps), ms, ctypes.byref(npass), names, 1024))
        return dict(zip(json.loads(names.value.decode()), [ms[p] for p in range(npass.value)]))


class Batch:
    """Independent lattices stepped together (one graph launch per chunk of steps)."""

    def __init__(self, lattices: Sequence[Lattice], stream=None):
        self._L = _lib.load()
        self.lattices = list(lattices)
        self._stream_ptr, self.stream = _stream_handle(stream)
        arr = (ctypes.c_void_p * len(self.lattices))(*[l.h.value for l in self.lattices])
        handle = ctypes.c_void_p()
        check(self._L.itse_batch_create(len(self.lattices), arr, self._stream_ptr, ctypes.byref(handle)))
        self.h = handle

    def step(self, nsteps: int):
        check(self._L.itse_batch_step(self.h, int(nsteps)))

    def set_persistent(self, on: bool = True):
        """Step through the persistent kernel (one cooperative launch per call of
        step) instead of graph replay; raises ItseError (EINVAL) for batches it does
        not take."""
        check(self._L.itse_batch_set_persistent(self.h, 1 if on else 0))

    def close(self):
        if getattr(self, "h", None):
            self._L.itse_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(n: int, precision: str = "fp32", stream=None) -> str:
    L = _lib.load()
    sp, _ = _stream_handle(stream)
    buf = ctypes.create_string_buffer(4096)
    check(L.itse_autotune(int(n), _PREC[precision], sp, buf, 4096))
    return buf.value.decode()


def autotune_batch(n: int, precision: str = "fp32", count: int = 1, nstates: int = 2, stream=None) -> str:
    """Time every schedule of (n, precision) on a batch of `count` lattices with
    `nstates` states and keep the fastest for that kind of lattice; JSON report."""
    L = _lib.load()
    sp, _ = _stream_handle(stream)
    buf = ctypes.create_string_buffer(4096)
    check(L.itse_autotune_batch(int(n), _PREC[precision], int(count), int(nstates), sp, buf, 4096))
    return buf.value.decode()


def schedule(n: int, precision: str = "fp32") -> str:
    L = _lib.load()
    buf = ctypes.create_string_buffer(1024)
    check(L.itse_schedule_get(int(n), _PREC[precision], buf, 1024))
    return buf.value.decode()


def set_schedule(n: int, precision: str, variant: int, nstates: Optional[int] = None):
    """Select the transform schedule variant used by lattices created afterwards:
    for all of them, or (nstates given) only for one-state (nstates = 1) or
    multi-state lattices."""
    if nstates is None:
        check(_lib.load().itse_schedule_set(int(n), _PREC[precision], int(variant)))
    else:
        check(_lib.load().itse_schedule_set_states(int(n), _PREC[precision], int(nstates), int(variant)))


def schedule_variants(n: int, precision: str = "fp32") -> int:
    import json
    return int(json.loads(schedule(n, precision))["variants"])


class Server:
    """Eigensolve requests admitted by HBM footprint and stepped together
    (continuous batching).  Thin wrapper of the itse_server_* calls."""

    def __init__(self, hbm_budget: int, max_slots: int = 64, chunk: int = 100, stream=None):
        self._L = _lib.load()
        self._stream_ptr, self.stream = _stream_handle(stream)
        handle = ctypes.c_void_p()
        check(self._L.itse_server_create(int(hbm_budget), int(max_slots), int(chunk), self._stream_ptr,
                                         ctypes.byref(handle)))
        self.h = handle

    def submit(self, n, a, mass, dtau, potential, states, kin=_lib.KIN_REL_LAT, subtract_rest_mass=True,
               precision="fp32", center="origin", parity=None, axes=None, ortho_every=1, tol=1e-8,
               relative=True, keep_states=False, max_steps=100000) -> int:
        pot = np.ascontiguousarray(potential)
        sts = [np.ascontiguousarray(s) for s in states]
        desc = _lib.Desc(int(n), float(a), float(mass), float(dtau), int(kin), 1 if subtract_rest_mass else 0,
                         _PREC[precision], _CENTER[center], len(sts))
        ptrs = (ctypes.c_void_p * len(sts))(*[s.ctypes.data for s in sts])
        req = _lib.Request(desc, pot.ctypes.data, _dtype_code(pot), ptrs, _dtype_code(sts[0]),
                           make_opts(len(sts), ortho_every, False, parity, axes), float(tol),
                           1 if relative else 0, 1 if keep_states else 0, int(max_steps))
        rid = ctypes.c_uint64()
        check(self._L.itse_server_submit(self.h, ctypes.byref(req), ctypes.byref(rid)))
        return int(rid.value)

    def progress(self):
        live, queued = ctypes.c_int(), ctypes.c_int()
        check(self._L.itse_server_progress(self.h, ctypes.byref(live), ctypes.byref(queued)))
        return live.value, queued.value

    def poll(self, max_results: int = 256):
        buf = (_lib.Result * max_results)()
        n = ctypes.c_int()
        check(self._L.itse_server_poll(self.h, buf, int(max_results), ctypes.byref(n)))
        out = []
        for r in buf[: n.value]:
            out.append({"id": int(r.id), "status": int(r.status), "converged": bool(r.converged),
                        "steps": int(r.steps), "energy": list(r.energy), "t_submit": r.t_submit,
                        "t_admit": r.t_admit, "t_done": r.t_done})
        return out

    def state(self, rid: int, i: int, n: int, dtype=np.float64):
        out = np.empty((n, n, n), dtype=dtype)
        code = _lib.DTYPE_F32 if out.dtype == np.float32 else _lib.DTYPE_F64
        check(self._L.itse_server_state(self.h, ctypes.c_uint64(rid), int(i),
                                        out.ctypes.data_as(ctypes.c_void_p), code))
        return out

    def release(self, rid: int):
        check(self._L.itse_server_release(self.h, ctypes.c_uint64(rid)))

    @property
    def bytes_in_use(self) -> int:
        return int(self._L.itse_server_bytes_in_use(self.h))

    def close(self):
        if getattr(self, "h", None):
            self._L.itse_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
