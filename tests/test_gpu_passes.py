"""GPU parity of the three-pass step at the larger lattice sizes and for every
schedule variant (split factor of the y axis, workgroup shapes), through the C ABI,
against the FP64 oracle.

Tolerances: FP64 lattices 1e-12 (max-abs / max) for one transform or kinetic
application and 1e-10 relative for energies along trajectories.  FP32 lattices:
bounds at about four times the largest error measured on an MI355X (printed by
each run, see measure.py).
"""
import json

import numpy as np
import pytest

import synth
from measure import check, max_rel_energy

pytestmark = pytest.mark.gpu

CASES = [(32, "fp32", 1), (32, "fp32", 2), (48, "fp32", 1), (48, "fp32", 2),
         (64, "fp32", 1), (64, "fp32", 2), (96, "fp32", 1), (96, "fp32", 2), (96, "fp32", 3),
         (48, "fp64", 0), (96, "fp64", 0), (128, "fp32", 0), (128, "fp32", 1), (128, "fp64", 0),
         (192, "fp32", 0), (192, "fp64", 0), (256, "fp32", 0), (256, "fp32", 1), (256, "fp32", 2), (256, "fp32", 3),
         (256, "fp32", 4), (256, "fp32", 5),
         (256, "fp64", 0), (256, "fp64", 1)]


def _tol(prec):
    return 1e-12 if prec == "fp64" else 2e-6


def _rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def _lat(itse, n, prec, variant, kin=3, nstates=1, center="origin", a=None, mass=1.3):
    itse.set_schedule(n, prec, variant)
    a = 6.4 / n if a is None else a
    dtau = a * a * mass / 8 if kin in (1, 2) else a / 4
    return itse.Lattice(n, a, mass, dtau, kin=kin, subtract_rest_mass=True, precision=prec,
                        center=center, nstates=nstates)


@pytest.fixture(autouse=True)
def _reset_schedules(itse):
    yield
    for n, prec, _ in CASES:
        itse.set_schedule(n, prec, 0)


def _olat(orc, lat):
    d = lat.desc
    return orc.lattice(d.n, d.a, d.mass, d.dtau, d.kin, bool(d.subtract_rest_mass),
                       "cell" if d.center == 0 else "origin")


def test_schedule_per_kind(itse, orc):
    """One-state and multi-state lattices keep their own schedules; each runs with
    the one current at its creation."""
    itse.set_schedule(256, "fp32", 4, nstates=1)
    itse.set_schedule(256, "fp32", 3, nstates=3)
    js = json.loads(itse.schedule(256, "fp32"))
    assert js["variant"] == 3 and js["variant_one_state"] == 4
    lat = _lat(itse, 256, "fp32", 4, kin=3)      # created under variant 4 (both kinds)
    itse.set_schedule(256, "fp32", 0)
    psi = synth.random_state(256, 17, dtype=np.float32)
    lat.set_state(0, psi)
    got = lat.apply_kinetic(0).cpu().numpy().astype(np.float64)
    ref = orc.apply_kinetic(_olat(orc, lat), psi.astype(np.float64))
    check("passes.schedule_per_kind", _rel(got, ref), 2e-6)
    lat.close()


@pytest.mark.parametrize("n,prec,variant", CASES)
def test_spectrum_schedules(itse, orc, n, prec, variant):
    lat = _lat(itse, n, prec, variant)
    assert json.loads(itse.schedule(n, prec))["variant"] == variant
    dt = np.float32 if prec == "fp32" else np.float64
    psi = synth.random_state(n, 300 + n + variant, dtype=dt)
    lat.set_state(0, psi)
    spec = lat.spectrum(0).cpu().numpy().astype(np.float64)
    got = spec[..., 0] + 1j * spec[..., 1]
    ref = orc.fft3d(psi.astype(np.float64), -1)[:, :, : n // 2 + 1]
    if prec == "fp32":
        check(f"passes.spectrum[{n},{variant}]", _rel(got, ref), 7.5e-7)
    else:
        assert _rel(got, ref) < _tol(prec)
    lat.close()


@pytest.mark.parametrize("n,prec,variant", CASES)
@pytest.mark.parametrize("kin", [1, 3])
def test_kinetic_schedules(itse, orc, n, prec, variant, kin):
    lat = _lat(itse, n, prec, variant, kin=kin)
    dt = np.float32 if prec == "fp32" else np.float64
    psi = synth.random_state(n, 500 + n + kin, dtype=dt)
    lat.set_state(0, psi)
    got = lat.apply_kinetic(0).cpu().numpy().astype(np.float64)
    ref = orc.apply_kinetic(_olat(orc, lat), psi.astype(np.float64))
    if prec == "fp32":
        check(f"passes.kinetic[{n},{variant},{kin}]", _rel(got, ref), _tol(prec))
    else:
        assert _rel(got, ref) < _tol(prec)
    lat.close()


@pytest.mark.parametrize("n,prec,variant", [(96, "fp64", 0), (128, "fp64", 0), (128, "fp32", 1),
                                            (192, "fp32", 0), (256, "fp64", 0), (256, "fp64", 1),
                                            (48, "fp32", 2), (64, "fp32", 1), (96, "fp32", 2), (256, "fp32", 5),
                                            (32, "fp32", 2), (96, "fp32", 3)])
def test_multistate_steps_large(itse, orc, n, prec, variant):
    """Three states (even, odd, odd deflated against the odd one), Cornell potential,
    a few steps: every step's energies and the final states match the oracle."""
    steps = 4
    a = 6.4 / n
    lat = _lat(itse, n, prec, variant, kin=3, nstates=3, a=a)
    dt = np.float32 if prec == "fp32" else np.float64
    v = synth.potential_cornell(n, a, "origin", sigma=0.2, alpha=0.4, aniso=0.05).astype(dt)
    states = synth.random_states(n, 3, seed=40, dtype=dt)
    lat.set_potential(v)
    for i, s in enumerate(states):
        lat.set_state(i, s)
    lat.set_options(ortho_every=1, moments=True, parity=(1, -1, -1))
    lat.step(steps)
    hist = lat.history(steps)
    ostates, ohist = orc.step(_olat(orc, lat), [s.astype(np.float64) for s in states],
                              v.astype(np.float64), steps, parity=(1, -1, -1))
    e = max_rel_energy(hist, ohist, ("energy", "norm2", "x", "r2", "parity_even"), floor=1.0)
    st = max(_rel(lat.get_state(i), ostates[i]) for i in range(3))
    if prec == "fp64":
        assert e <= 1e-10 and st <= 1e-10, (e, st)
    else:
        check(f"passes.multistate_large[{n}].energies", e, 2.2e-7)
        check(f"passes.multistate_large[{n}].states", st, 1.7e-6)
    lat.close()


@pytest.mark.parametrize("n,prec,parity,axes,ortho", [
    (24, "fp64", (1, -1, -1), (4, 2, 7), 1),     # three different reflections: projected one by one
    (32, "fp64", (0, -1, 1), (7, 6, 6), 2),      # shared axes, Gram-Schmidt every other step
    (32, "fp32", (1, 0, -1), (1, 7, 1), 3),
    (24, "fp64", (-1, 1, 0), (7, 7, 7), 0),      # projections without Gram-Schmidt
])
def test_projection_modes(itse, orc, n, prec, parity, axes, ortho):
    """Reflection projections with shared or different axes, with and without
    Gram-Schmidt: energies and states follow the oracle."""
    steps = 12
    a = 0.2
    lat = _lat(itse, n, prec, 0, kin=2, nstates=3, center="cell", a=a, mass=1.1)
    dt = np.float32 if prec == "fp32" else np.float64
    v = synth.potential_harmonic(n, a, "cell", 0.5).astype(dt)
    states = synth.random_states(n, 3, seed=60, dtype=dt)
    lat.set_potential(v)
    for i, s in enumerate(states):
        lat.set_state(i, s)
    lat.set_options(ortho_every=ortho, moments=True, parity=parity, axes=axes)
    lat.step(steps)
    hist = lat.history(steps)
    ostates, ohist = orc.step(_olat(orc, lat), [s.astype(np.float64) for s in states],
                              v.astype(np.float64), steps, ortho_every=ortho, parity=parity, axes=axes)
    e = max_rel_energy(hist, ohist, ("energy", "norm2", "z", "parity_even"), floor=1.0)
    st = max(_rel(lat.get_state(i), ostates[i]) for i in range(3))
    if prec == "fp64":
        assert e <= 1e-10 and st <= 1e-10, (e, st)
    else:
        check(f"passes.projection_modes[{n},{parity},{axes}].energies", e, 2.7e-7)
        check(f"passes.projection_modes[{n},{parity},{axes}].states", st, 2.1e-6)
    lat.close()


@pytest.mark.parametrize("n,prec,parity,axes", [
    (12, "fp32", (1, -1, 0), (7, 7, 7)),      # three vectors per row
    (16, "fp64", (-1, 1, 1), (4, 4, 4)),      # z alone (element 0 pairs across lanes)
    (48, "fp32", (0, 1, -1), (5, 5, 5)),      # x and z
    (24, "fp64", (1, -1, -1), (3, 3, 3)),     # x and y, z kept
    (192, "fp64", (1, -1, 0), (7, 7, 7)),     # rows longer than one wave of vectors
])
def test_projection_origin_axes(itse, orc, n, prec, parity, axes):
    """Reflections about the origin (z -> -z mod N pairs element 0 of one vector with
    the neighbouring vector) on shared axes, with Gram-Schmidt every step: energies,
    parity weights and states follow the oracle."""
    steps = 6
    a = 0.25
    lat = _lat(itse, n, prec, 0, kin=2, nstates=3, center="origin", a=a, mass=1.1)
    dt = np.float32 if prec == "fp32" else np.float64
    v = synth.potential_harmonic(n, a, "origin", 0.5).astype(dt)
    states = synth.random_states(n, 3, seed=70 + n, dtype=dt)
    lat.set_potential(v)
    for i, s in enumerate(states):
        lat.set_state(i, s)
    lat.set_options(ortho_every=1, moments=True, parity=parity, axes=axes)
    lat.step(steps)
    hist = lat.history(steps)
    ostates, ohist = orc.step(_olat(orc, lat), [s.astype(np.float64) for s in states],
                              v.astype(np.float64), steps, ortho_every=1, parity=parity, axes=axes)
    e = max_rel_energy(hist, ohist, ("energy", "norm2", "parity_even"), floor=1.0)
    st = max(_rel(lat.get_state(i), ostates[i]) for i in range(3))
    if prec == "fp64":
        assert e <= 1e-10 and st <= 1e-10, (e, st)
    else:
        check(f"passes.projection_origin_axes[{n},{parity},{axes}].energies", e, 1.9e-7)
        check(f"passes.projection_origin_axes[{n},{parity},{axes}].states", st, 1.5e-6)
    lat.close()


@pytest.mark.parametrize("variant", [2, 4, 5])
def test_bare_one_state_steps(itse, orc, variant):
    """The bare one-state 256^3 FP32 step of the benchmark (no projection, no
    Gram-Schmidt): energies of the first steps and the state after them match the
    FP64 oracle on the same FP32 inputs."""
    p = synth.config_precision(256)
    v = p.potential_array(np.float64).astype(np.float32)
    psi = p.initial_states()[0].astype(np.float32)
    itse.set_schedule(256, "fp32", variant, nstates=1)
    lat = itse.Lattice(p.n, p.a, p.mass, p.dtau, kin=p.kin, subtract_rest_mass=True,
                       precision="fp32", center=p.center, nstates=1)
    itse.set_schedule(256, "fp32", 0)
    lat.set_potential(v)
    lat.set_state(0, psi)
    lat.set_options(ortho_every=0)
    steps = 3
    lat.step(steps)
    hist = lat.history(steps)
    ostates, ohist = orc.step(_olat(orc, lat), [psi.astype(np.float64)], v.astype(np.float64), steps)
    check(f"passes.bare_one_state[{variant}].energies", max_rel_energy(hist, ohist, ("energy", "norm2")), 4.8e-8)
    check(f"passes.bare_one_state[{variant}].state", _rel(lat.get_state(0), ostates[0]), 1.9e-6)
    lat.close()
