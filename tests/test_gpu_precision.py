"""Element-wise parity of the benchmarked steps, at the sizes the benchmark runs
them, and the FP64 re-evaluation (polish) of FP32 states.

The 256^3 three-state workload (Cornell + anisotropy stored in FP32, H_K^(3) - M,
parity +, -, -, Gram-Schmidt every step) is stepped through the C ABI with the
step options the benchmark uses (no position moments, which selects the update
pass instance the benchmark times) in every schedule, and each state is compared
with the FP64 oracle site by site on the same FP32-rounded inputs.

Tolerances.  FP64 lattices: 1e-10 relative (the target for FP64 wave-functions
and eigenvalues).  FP32 lattices: bounds set at about four times the largest
error measured on an MI355X for that quantity (max |got - ref| / max |ref| for
states and spectra, |got - ref| / |ref| for energies); the measured figures are
listed beside each bound.
"""
import numpy as np
import pytest

import synth
from measure import check

pytestmark = pytest.mark.gpu

STEPS = 2

# FP32 bounds, about 4x the largest error measured on an MI355X
FP32_STATE_BOUND = 2e-6      # states after the steps, max-abs / max (measured 4.9e-7)
FP32_ENERGY_BOUND = 4e-8     # step energies and norms, relative (measured 9.9e-9)
FP32_KIN_BOUND = 2.1e-6      # one kinetic application, max-abs / max (measured 5.3e-7)


def _olat(orc, p):
    return orc.lattice(p.n, p.a, p.mass, p.dtau, p.kin, p.subtract_rest_mass, p.center)


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _oracle_run(orc, n, steps):
    p = synth.config_precision(n)
    v32 = p.potential_array(np.float64).astype(np.float32)
    s32 = [s.astype(np.float32) for s in p.initial_states()]
    ost, oh = orc.step(_olat(orc, p), [s.astype(np.float64) for s in s32], v32.astype(np.float64), steps,
                       parity=list(p.parity))
    return p, v32, s32, ost, oh


@pytest.fixture(scope="module")
def work256(orc):
    return _oracle_run(orc, 256, STEPS)


@pytest.fixture(scope="module")
def work128(orc):
    return _oracle_run(orc, 128, STEPS)


def _gpu_run(itse, p, v, states, prec, variant, steps):
    itse.set_schedule(p.n, prec, variant)
    dt = np.float32 if prec == "fp32" else np.float64
    lat = itse.Lattice(p.n, p.a, p.mass, p.dtau, kin=p.kin, subtract_rest_mass=p.subtract_rest_mass,
                       precision=prec, center=p.center, nstates=p.nstates)
    itse.set_schedule(p.n, prec, 0)
    lat.set_potential(v.astype(dt))
    for i, s in enumerate(states):
        lat.set_state(i, s.astype(dt))
    lat.set_options(ortho_every=1, moments=False, parity=list(p.parity))
    lat.step(steps)
    hist = lat.history(steps)
    got = [lat.get_state(i) for i in range(p.nstates)]
    lat.close()
    return hist, got


def _errors(hist, got, oh, ost):
    e = max(abs(hist[s][i][f] - oh[s][i][f]) / abs(oh[s][i][f])
            for s in range(len(hist)) for i in range(len(got)) for f in ("energy", "norm2"))
    return e, [_rel(g, r) for g, r in zip(got, ost)]


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5])
def test_fp32_workload_states(itse, work256, variant):
    """The benchmarked 256^3 FP32 three-state step: energies and norms of every
    step, and all three states after the steps, site by site, in every schedule."""
    p, v32, s32, ost, oh = work256
    hist, got = _gpu_run(itse, p, v32, s32, "fp32", variant, STEPS)
    e, s = _errors(hist, got, oh, ost)
    check(f"precision.fp32_workload[{variant}].energies", e, FP32_ENERGY_BOUND)
    check(f"precision.fp32_workload[{variant}].states", max(s), FP32_STATE_BOUND)


@pytest.mark.parametrize("n,variant", [(128, 0), (256, 0), (256, 1)])
def test_fp64_workload_states(itse, work128, work256, n, variant):
    """The same three-state workload in FP64 without moments (the update pass with
    all loads issued up front, which FP64 lattices take from N = 128): energies,
    norms and states to 1e-10."""
    p, v32, s32, ost, oh = work128 if n == 128 else work256
    hist, got = _gpu_run(itse, p, v32, s32, "fp64", variant, STEPS)
    e, s = _errors(hist, got, oh, ost)
    print(f"[measured] fp64 {n}^3 workload schedule {variant}: energy/norm {e:.3e}, states "
          + ", ".join(f"{x:.3e}" for x in s), flush=True)
    assert e <= 1e-10
    assert max(s) <= 1e-10


KIN_FORMS = [(2, True), (4, True), (4, False), (3, False)]


@pytest.mark.parametrize("prec,variant", [("fp32", v) for v in range(6)] + [("fp64", 0), ("fp64", 1)])
@pytest.mark.parametrize("kin,sub", KIN_FORMS)
def test_kinetic_forms_256(itse, orc, prec, variant, kin, sub):
    """H_K^(2), the continuum-momentum relativistic form with and without the rest
    mass, and H_K^(3) with the rest mass, applied at 256^3 in every schedule (the
    multiply fused between the x transforms in registers)."""
    n, mass = 256, 1.3
    a = 6.4 / n
    dtau = a * a * mass / 8 if kin in (1, 2) else a / 4
    itse.set_schedule(n, prec, variant)
    lat = itse.Lattice(n, a, mass, dtau, kin=kin, subtract_rest_mass=sub, precision=prec, center="origin")
    itse.set_schedule(n, prec, 0)
    dt = np.float32 if prec == "fp32" else np.float64
    psi = synth.random_state(n, 700 + kin + 2 * sub, dtype=dt)
    lat.set_state(0, psi)
    got = lat.apply_kinetic(0).cpu().numpy().astype(np.float64)
    lat.close()
    ref = orc.apply_kinetic(orc.lattice(n, a, mass, dtau, kin, sub, "origin"), psi.astype(np.float64))
    err = _rel(got, ref)
    if prec == "fp64":
        assert err <= 1e-12, err
    else:
        check(f"precision.kinetic_forms[{kin},{int(sub)},{variant}]", err, FP32_KIN_BOUND)


def test_polish_equals_oracle_observe(itse, orc, work128):
    """itse_polish of FP32 states is the FP64 Rayleigh quotient of the same stored
    values: it equals the oracle's observe of the states read back and widened, to
    1e-12 (order of summation); the FP32-evaluated energy of the same states is
    printed beside it."""
    p, v32, s32, _, _ = work128
    lat = itse.Lattice(p.n, p.a, p.mass, p.dtau, kin=p.kin, subtract_rest_mass=p.subtract_rest_mass,
                       precision="fp32", center=p.center, nstates=p.nstates)
    lat.set_potential(v32)
    for i, s in enumerate(s32):
        lat.set_state(i, s)
    lat.set_options(ortho_every=1, parity=list(p.parity))
    lat.step(200)
    lat.evaluate(moments=False)
    e32 = [lat.observe(i)["energy"] for i in range(p.nstates)]
    pol = [lat.polish(i) for i in range(p.nstates)]
    ref = orc.observe(_olat(orc, p), [lat.get_state(i) for i in range(p.nstates)], v32.astype(np.float64))
    lat.close()
    for i in range(p.nstates):
        for f in ("energy", "kinetic", "potential"):
            assert abs(pol[i][f] - ref[i][f]) <= 1e-12 * abs(ref[i][f]), (i, f)
        print(f"[measured] 128^3 state {i} after 200 steps: FP32 energy - FP64 energy of the same state "
              f"{(e32[i] - ref[i]['energy']) / abs(ref[i]['energy']):.3e} relative", flush=True)


def test_polish_of_converged_fp32_solve(itse, orc):
    """A converged FP32 solve of the workload at 64^3 (60 000 steps, tau = 1500):
    the FP64 evaluation of each returned FP32 state (polish) is within 1e-8 relative
    of the eigenvalue of the same solve run in FP64 on the GPU, whose states the
    oracle certifies (residual of its step map) and whose energies the oracle
    recomputes.  The FP32-evaluated energies' errors are printed per eigenvalue."""
    p = synth.config_precision(64)
    v32 = p.potential_array(np.float64).astype(np.float32)
    s32 = [s.astype(np.float32) for s in p.initial_states()]
    steps = 60000
    res = {}
    for prec in ("fp32", "fp64"):
        dt = np.float32 if prec == "fp32" else np.float64
        lat = itse.Lattice(p.n, p.a, p.mass, p.dtau, kin=p.kin, subtract_rest_mass=p.subtract_rest_mass,
                           precision=prec, center=p.center, nstates=p.nstates)
        lat.set_potential(v32.astype(dt))
        for i, s in enumerate(s32):
            lat.set_state(i, s.astype(dt))
        lat.set_options(ortho_every=1, parity=list(p.parity))
        lat.step(steps)
        lat.evaluate(moments=False)
        res[prec] = {"E": [lat.observe(i)["energy"] for i in range(p.nstates)],
                     "polish": [lat.polish(i)["energy"] for i in range(p.nstates)],
                     "states": [lat.get_state(i) for i in range(p.nstates)]}
        lat.close()
    L = _olat(orc, p)
    cert = [orc.certify(L, st, v32.astype(np.float64)) for st in res["fp64"]["states"]]
    for i in range(p.nstates):
        ref = cert[i]["energy"]
        assert cert[i]["resid"] < 1e-9, (i, cert[i])
        assert abs(res["fp64"]["E"][i] - ref) <= 1e-10 * abs(ref), i
        err32 = abs(res["fp32"]["E"][i] - ref) / abs(ref)
        errp = abs(res["fp32"]["polish"][i] - ref) / abs(ref)
        print(f"[measured] 64^3 converged state {i}: E = {ref:.12f}, FP32 energy {err32:.3e}, "
              f"FP32 state polished {errp:.3e} relative, oracle residual {cert[i]['resid']:.2e}", flush=True)
        assert errp <= 1e-8, (i, errp)
