"""The GPU path against a value the paper prints: the relativistic harmonic
oscillator of its H_K^(3) section (kinetic term H_K^(3) with the rest mass
subtracted, V = r^2, M = 30 GeV, A = 0.006 fm), whose ground-state E0 - M the
paper compares with Li's analytic 0.38627 GeV at the 0.5 permille level
(fixture tests/golden/relativistic_oscillator.txt).

The solve runs the step map to convergence on the GPU in FP64.  The reported
energy is the Rayleigh quotient of H at the map's fixed point.  That fixed point
is an eigenvector of K + c V with c = 1 - O(dtau), so the quotient differs from
H's eigenvalue only at second order in dtau; it is also compared with the
oracle's eigenvalue of the same lattice operator (a Lanczos solve on the CPU)."""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "relativistic_oscillator.txt")


def _golden():
    vals = {}
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_relativistic_oscillator_ground_state(itse, orc):
    from scipy.sparse.linalg import LinearOperator, eigsh
    g = _golden()
    A = g["A_fm"] / g["hbar_c_GeV_fm"]
    M = g["M_GeV"]
    n = 96
    lat = itse.Lattice(n, A, M, A / 4, kin=itse.KIN_REL_LAT, subtract_rest_mass=True, precision="fp64",
                       center="cell")
    v = synth.potential_harmonic(n, A, "cell", coef=1.0)
    _, _, _, r = synth.radius_grid(n, A, "cell")
    w0 = np.sqrt(2.0 / M)
    guess = np.exp(-0.5 * M * w0 * r * r)
    lat.set_potential(v)
    lat.set_state(0, guess)
    lat.set_options(parity=(1,))
    res = itse.run_to_convergence(lat, tol=1e-12, relative=True, check_every=1000, max_steps=40000)
    assert res.converged
    e_gpu = res.energies[0]
    ref = g["E0_minus_M_analytic"]
    assert abs(e_gpu - ref) <= g["E0_relative_agreement"] * ref, (e_gpu, ref)
    # the oracle's lowest eigenvalue of the same lattice operator
    L = orc.lattice(n, A, M, kin=3, subtract_rest=True, center="cell")

    def mv(x):
        x = np.asarray(x).reshape(n, n, n)
        return (orc.apply_kinetic(L, x) + v * x).ravel()

    w, _ = eigsh(LinearOperator((n ** 3, n ** 3), matvec=mv, dtype=np.float64), k=1, which="SA", tol=1e-10,
                 v0=guess.ravel())
    print(f"\nE0 - M: GPU {e_gpu:.8f}, oracle eigenvalue {float(w[0]):.8f}, paper (analytic) {ref}", flush=True)
    assert abs(e_gpu - float(w[0])) <= 1e-6 * abs(float(w[0])), (e_gpu, float(w[0]))
    lat.close()
