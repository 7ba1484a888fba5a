"""ctypes declarations for libitse.so (the C ABI of include/itse.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libitse.so")

MAX_STATES = 8

ITSE_OK = 0
STATUS_NAMES = {0: "ITSE_OK", -1: "ITSE_EINVAL", -2: "ITSE_ENOMEM", -3: "ITSE_EUNSTABLE",
                -4: "ITSE_ENONFINITE", -5: "ITSE_EDEVICE", -6: "ITSE_ESTATE", -7: "ITSE_ENOTFOUND"}

KIN_FDTD, KIN_NR_CONT, KIN_NR_LAT, KIN_REL_LAT, KIN_REL_CONT = 0, 1, 2, 3, 4
FP64, FP32 = 0, 1
CENTER_CELL, CENTER_ORIGIN = 0, 1
DTYPE_F32, DTYPE_F64 = 1, 2


class ItseError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


class Desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("a", ctypes.c_double), ("mass", ctypes.c_double),
                ("dtau", ctypes.c_double), ("kin", ctypes.c_int),
                ("subtract_rest_mass", ctypes.c_int), ("precision", ctypes.c_int),
                ("center", ctypes.c_int), ("nstates", ctypes.c_int), ("complex_psi", ctypes.c_int)]


OBS_FIELDS = ("energy", "kinetic", "potential", "norm2", "x", "y", "z", "r2", "parity_even", "energy_imag")


class Analysis(ctypes.Structure):
    _fields_ = [("box_norm2", ctypes.c_double), ("rho_box", ctypes.c_double), ("w_plus", ctypes.c_double),
                ("w_minus", ctypes.c_double), ("w_minus_axis", ctypes.c_double * 3)]

    def as_dict(self):
        d = {f: getattr(self, f) for f in ("box_norm2", "rho_box", "w_plus", "w_minus")}
        for k in range(3):
            d[f"w_minus_e{k + 1}"] = self.w_minus_axis[k]
        return d


class Obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_longlong)] + [(f, ctypes.c_double) for f in OBS_FIELDS]

    def as_dict(self):
        d = {f: getattr(self, f) for f in OBS_FIELDS}
        d["step"] = self.step
        return d


class StepOpts(ctypes.Structure):
    _fields_ = [("ortho_every", ctypes.c_int), ("moments", ctypes.c_int),
                ("parity", ctypes.c_int * MAX_STATES), ("axes", ctypes.c_int * MAX_STATES)]


class Request(ctypes.Structure):
    _fields_ = [("desc", Desc), ("potential", ctypes.c_void_p), ("potential_dtype", ctypes.c_int),
                ("states", ctypes.POINTER(ctypes.c_void_p)), ("state_dtype", ctypes.c_int),
                ("opts", StepOpts), ("tol", ctypes.c_double), ("tol_relative", ctypes.c_int),
                ("keep_states", ctypes.c_int), ("max_steps", ctypes.c_longlong)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int), ("converged", ctypes.c_int),
                ("steps", ctypes.c_longlong), ("energy", ctypes.c_double * MAX_STATES),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def load():
    """Load the HIP library; raises if it has not been built (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch's HIP runtime must be the one the library binds to (same soname
    # libamdhip64.so.7): load torch first so the library does not pull in a
    # second HIP/HSA runtime from /opt/rocm.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -m paper_2006_16935_amd.build, or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER
    sigs = {
        "itse_last_error": ([], ctypes.c_char_p),
        "itse_version": ([], ctypes.c_char_p),
        "itse_footprint_bytes": ([P(Desc)], ctypes.c_size_t),
        "itse_create": ([P(Desc), vp, ALLOC_FN, FREE_FN, vp, P(vp)], ip),
        "itse_destroy": ([vp], ip),
        "itse_set_stream": ([vp, vp], ip),
        "itse_set_potential": ([vp, vp, ip, ip], ip),
        "itse_set_potential_imag": ([vp, vp, ip, ip], ip),
        "itse_set_state": ([vp, ip, vp, ip, ip], ip),
        "itse_get_state": ([vp, ip, vp, ip, ip], ip),
        "itse_set_step_opts": ([vp, P(StepOpts)], ip),
        "itse_step": ([vp, ip, P(StepOpts)], ip),
        "itse_evaluate": ([vp, ip], ip),
        "itse_observe": ([vp, ip, P(Obs)], ip),
        "itse_history": ([vp, ip, P(Obs)], ip),
        "itse_step_count": ([vp], ctypes.c_longlong),
        "itse_orthogonalise": ([vp, ip], ip),
        "itse_project_parity": ([vp, ip, ip, ip, P(dp)], ip),
        "itse_apply_kinetic": ([vp, ip, vp], ip),
        "itse_spectrum": ([vp, ip, vp], ip),
        "itse_polish": ([vp, ip, P(Obs)], ip),
        "itse_sync": ([vp], ip),
        "itse_analyse": ([vp, ip, ctypes.c_double, P(Analysis)], ip),
        "itse_analyse_noalloc": ([vp, ip, ctypes.c_double, P(Analysis)], ip),
        "itse_momentum_radial": ([vp, ip, ip, P(dp), P(dp), P(dp), P(dp)], ip),
        "itse_snapshot_push": ([vp], ip),
        "itse_snapshot_count": ([vp, P(ip)], ip),
        "itse_snapshot_clear": ([vp], ip),
        "itse_snapshot_extract": ([vp, P(Obs), P(ip), vp, ip, ip], ip),
        "itse_profile_step": ([vp, ip, P(dp), P(ip), ctypes.c_char_p, ctypes.c_size_t], ip),
        "itse_batch_create": ([ip, P(vp), vp, P(vp)], ip),
        "itse_batch_step": ([vp, ip], ip),
        "itse_batch_set_persistent": ([vp, ip], ip),
        "itse_batch_destroy": ([vp], ip),
        "itse_autotune": ([ip, ip, vp, ctypes.c_char_p, ctypes.c_size_t], ip),
        "itse_autotune_batch": ([ip, ip, ip, ip, vp, ctypes.c_char_p, ctypes.c_size_t], ip),
        "itse_schedule_get": ([ip, ip, ctypes.c_char_p, ctypes.c_size_t], ip),
        "itse_schedule_set": ([ip, ip, ip], ip),
        "itse_schedule_set_states": ([ip, ip, ip, ip], ip),
        "itse_server_create": ([ctypes.c_size_t, ip, ip, vp, P(vp)], ip),
        "itse_server_destroy": ([vp], ip),
        "itse_server_submit": ([vp, P(Request), P(ctypes.c_uint64)], ip),
        "itse_server_progress": ([vp, P(ip), P(ip)], ip),
        "itse_server_poll": ([vp, P(Result), ip, P(ip)], ip),
        "itse_server_state": ([vp, ctypes.c_uint64, ip, vp, ip], ip),
        "itse_server_release": ([vp, ctypes.c_uint64], ip),
        "itse_server_bytes_in_use": ([vp], ctypes.c_size_t),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def check(status: int):
    if status != ITSE_OK:
        msg = load().itse_last_error()
        raise ItseError(status, msg.decode() if msg else "")


def exported_symbols():
    """Names the library exports among those include/itse.h declares (for load checks)."""
    L = load()
    return [n for n in dir(L) if n.startswith("itse_")]
