"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/itse.h declares, and rejects bad arguments before
touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "itse.h")).read()
    return sorted(set(re.findall(r"\b(itse_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import paper_2006_16935_amd as pkg
    L = pkg.load()
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_footprint():
    import paper_2006_16935_amd as pkg
    from paper_2006_16935_amd import _lib
    L = pkg.load()
    assert b"gfx950" in L.itse_version()
    d = _lib.Desc(256, 0.025, 1.3, 0.00625, 3, 1, _lib.FP32, 1, 3)
    fp = L.itse_footprint_bytes(ctypes.byref(d))
    n3 = 256 ** 3
    # states + current states + spectra + potential at least
    assert fp > 3 * (2 * n3 * 4 + 256 * 256 * 129 * 8) + n3 * 4
    assert fp < 2 * 1024 ** 3
    # a complex state: Re and Im arrays, their spectra, Im V and K psi for both parts
    dc = _lib.Desc(256, 0.025, 1.3, 0.00625, 3, 1, _lib.FP32, 1, 1, 1)
    d2 = _lib.Desc(256, 0.025, 1.3, 0.00625, 3, 1, _lib.FP32, 1, 2)
    fc, f2 = L.itse_footprint_bytes(ctypes.byref(dc)), L.itse_footprint_bytes(ctypes.byref(d2))
    assert fc - f2 >= 3 * n3 * 4


def _create(**kw):
    from paper_2006_16935_amd import _lib
    L = _lib.load()
    base = dict(n=32, a=0.1, mass=1.0, dtau=0.00125, kin=1, subtract_rest_mass=1,
                precision=_lib.FP64, center=0, nstates=1, complex_psi=0)
    base.update(kw)
    d = _lib.Desc(*[base[k] for k, _ in _lib.Desc._fields_])
    h = ctypes.c_void_p()
    st = L.itse_create(ctypes.byref(d), None, _lib.ALLOC_FN(0), _lib.FREE_FN(0), None, ctypes.byref(h))
    return st, L.itse_last_error().decode()


@pytest.mark.parametrize("kw,status", [
    (dict(n=20), -1),            # factor 5
    (dict(n=4), -1),             # too small
    (dict(n=1024), -1),          # above the largest supported N (256)
    (dict(a=0.0), -1),
    (dict(mass=-1.0), -1),
    (dict(kin=7), -1),
    (dict(nstates=0), -1),
    (dict(nstates=9), -1),
    (dict(precision=5), -1),
    (dict(dtau=0.002), -3),      # dtau * max T = 2.96 for H_K^(1) at a = 0.1
    (dict(kin=3, dtau=0.06, a=0.05), -3),
    (dict(complex_psi=1, nstates=2), -1),   # a complex lattice holds one state
    (dict(complex_psi=2), -1),
])
def test_create_rejects_bad_descriptions(kw, status):
    st, msg = _create(**kw)
    assert st == status, msg
    assert msg


def test_stability_bound_matches_paper_map():
    """The first config's dtau = a^2/8 gives dtau max T = 1.8506 (< 1.95): accepted
    bound check happens before any device call, so only the rejection is testable here."""
    import math
    a = 0.1
    tmax = 3 * math.pi ** 2 / (2 * a * a)
    assert abs(a * a / 8 * tmax - 1.8506) < 1e-4
    st, msg = _create(dtau=1.95 / tmax * 1.001)
    assert st == -3
