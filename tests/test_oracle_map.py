"""Pins for the oracle's step map (paper, equation iter_proced with the A, B
factors of section "The iterative procedure"), its normalisation, Gram-Schmidt
deflation, reflection projections (section "Parity projection") and observables.

Independent references used here:

* constant potential: every plane wave is an exact eigenvector of the map with
  lambda(k) = (1 - dtau V0/2 - dtau T(k)) / (1 + dtau V0/2) (closed form);
* separable harmonic oscillator: the fixed point of the map is the ground state
  of K + sV with s = (1 + lambda)/2 (rearranging the update), which for
  V = sum_l v(x_l) reduces to dense 1D eigensolves (numpy ``eigh`` on a 1D
  kinetic matrix built from numpy's DFT for H_K^(1) or the 3-point stencil for
  H_K^(2)); the oracle's converged energies must equal the Rayleigh quotients of
  those fixed points (3D oscillator levels 3/2, 5/2, 7/2 up to the map's bias);
* projector identities P^2 = P, P+ + P- = 1, w+ + w- = 1; orthonormality after
  Gram-Schmidt; a one-site state for the position moments.
"""
import numpy as np
import pytest

import synth


def _k1d(n, a, m, kin):
    if kin == 1:
        F = np.fft.fft(np.eye(n), axis=0)
        idx = np.arange(n)
        mm = np.where(2 * idx <= n, idx, idx - n)
        k = 2 * np.pi * mm / n
        return np.fft.ifft(np.diag(k * k / (2 * a * a * m)) @ F, axis=0).real
    K = np.zeros((n, n))
    for i in range(n):
        K[i, i] = 2.0
        K[i, (i + 1) % n] -= 1.0
        K[i, (i - 1) % n] -= 1.0
    return K / (2 * a * a * m)


def _fixed_point(n, a, kin, dtau, quanta, center="cell"):
    """Rayleigh quotient of H = K + V at the map's fixed point for the separable
    oscillator V = r^2/2, for the product state with 1D quantum numbers `quanta`."""
    c = synth.axis_coords(n, a, center)
    v = 0.5 * c * c
    K = _k1d(n, a, 1.0, kin)
    s = 1.0
    for _ in range(300):
        e, U = np.linalg.eigh(K + s * np.diag(v))
        lam = 1.0 - dtau * sum(e[q] for q in quanta)
        s = 0.5 * (1.0 + lam)
    e, U = np.linalg.eigh(K + s * np.diag(v))
    return sum(U[:, q] @ K @ U[:, q] + U[:, q] @ (v * U[:, q]) for q in quanta), U


def test_constant_potential_closed_form(orc):
    n, a, m, dtau, v0 = 12, 0.2, 1.0, 0.004, 0.7
    for kin in (1, 2, 3):
        L = orc.lattice(n, a, m, dtau=dtau, kin=kin)
        T = orc.kinetic_symbol(L)
        v = np.full((n, n, n), v0)
        idx = np.indices((n, n, n))
        for mv in ((0, 0, 0), (1, 2, 0), (n // 2, 0, 5)):
            psi = np.cos(2 * np.pi * (mv[0] * idx[0] + mv[1] * idx[1] + mv[2] * idx[2]) / n)
            lam_exact = (1 - 0.5 * dtau * v0 - dtau * T[mv]) / (1 + 0.5 * dtau * v0)
            cert = orc.certify(L, psi, v)
            assert abs(cert["lambda"] - lam_exact) < 1e-14
            assert cert["resid"] < 1e-13
            out, _ = orc.step(L, [psi], v, 1, record=False)
            expect = np.sign(lam_exact) * psi / np.linalg.norm(psi)
            assert np.abs(out[0] - expect).max() < 1e-14


def test_plain_config_map_fixed_point(orc):
    """32^3, a = 0.1, H_K^(1), V = r^2/2 at the cell centre, dtau = a^2/8: the
    product of 1D ground states of K + sV (s = (1+lambda)/2, solved self-
    consistently with dense 1D eigensolves) is left invariant by the oracle's
    step, and its energy 1.08243497202... sits 7.1e-8 above the lattice-exact
    eigenvalue 1.0824349011 of K + V."""
    p = synth.config_plain_fp64()
    e_fp, U = _fixed_point(p.n, p.a, 1, p.dtau, (0, 0, 0))
    c = synth.axis_coords(p.n, p.a, "cell")
    e_exact = np.linalg.eigvalsh(_k1d(p.n, p.a, 1.0, 1) + np.diag(0.5 * c * c))[0] * 3
    assert abs(e_exact - 1.0824349011) < 1e-9
    assert abs(e_fp - 1.0824349720) < 1e-9
    u = U[:, 0]
    start = u[:, None, None] * u[None, :, None] * u[None, None, :]
    L = orc.lattice(p.n, p.a, p.mass, dtau=p.dtau, kin=p.kin, center="cell")
    v = p.potential_array()
    out, hist = orc.step(L, [start], v, 200)
    assert abs(hist[0][0]["energy"] - e_fp) < 1e-12
    assert abs(hist[-1][0]["energy"] - e_fp) < 1e-12
    assert np.abs(out[0] - start).max() < 1e-10
    assert orc.certify(L, start, v)["resid"] < 1e-12


@pytest.mark.slow
def test_oscillator_levels_three_halves_five_halves_seven_halves(orc):
    """H_K^(1), N = 32, a = 0.4 (the lattice oscillator is exact to 1e-13 here).
    State 0 even, state 1 odd, state 2 even and deflated against states 0, 1.

    States 0 and 1 are exact eigenvectors of the map, so their energies equal the
    separable fixed points to 1e-9.  State 2 is the fixed point of "map, then
    remove the (Euclidean) projection on state 0", which is not an eigenvector of
    the map; its bias, like the others, is second order in dtau, so the Richardson
    combination of runs at dtau = a^2/8 and a^2/16 must land on 3/2, 5/2, 7/2."""
    n, a = 32, 0.4
    v = synth.potential_harmonic(n, a, "cell", 0.5)
    runs = []
    for dtau, nsteps in ((a * a / 8, 700), (a * a / 16, 1000)):
        L = orc.lattice(n, a, 1.0, dtau=dtau, kin=1, center="cell")
        states = synth.random_states(n, 3, seed=0)
        out, hist = orc.step(L, states, v, nsteps, parity=(1, -1, 1))
        last = hist[-1]
        e0, _ = _fixed_point(n, a, 1, dtau, (0, 0, 0))
        e1, _ = _fixed_point(n, a, 1, dtau, (1, 0, 0))
        assert abs(last[0]["energy"] - e0) < 1e-9
        assert abs(last[1]["energy"] - e1) < 1e-9
        assert abs(last[0]["parity_even"] - 1) < 1e-12
        assert abs(last[1]["parity_even"]) < 1e-12
        assert abs(last[2]["parity_even"] - 1) < 1e-12
        g = np.einsum("iabc,jabc->ij", out, out)
        assert np.abs(g - np.eye(3)).max() < 1e-13
        runs.append([last[i]["energy"] for i in range(3)])
    for i, level in enumerate((1.5, 2.5, 3.5)):
        coarse, fine = runs[0][i], runs[1][i]
        assert 0 < fine - level < coarse - level < 1e-3
        assert abs((4 * fine - coarse) / 3 - level) < 2e-6


def test_hk2_oscillator_map_fixed_point(orc):
    """H_K^(2) at N = 32, a = 0.1: the fixed point built from the 3-point-stencil
    1D matrix (an operator independent of the oracle's FFT) is invariant under
    the oracle's step."""
    n, a = 32, 0.1
    dtau = a * a / 8
    e_fp, U = _fixed_point(n, a, 2, dtau, (0, 0, 0))
    u = U[:, 0]
    start = u[:, None, None] * u[None, :, None] * u[None, None, :]
    L = orc.lattice(n, a, 1.0, dtau=dtau, kin=2, center="cell")
    v = synth.potential_harmonic(n, a, "cell", 0.5)
    out, hist = orc.step(L, [start], v, 100)
    assert abs(hist[-1][0]["energy"] - e_fp) < 1e-12
    assert np.abs(out[0] - start).max() < 1e-10
    assert abs(e_fp - 1.0818558310) < 1e-6


@pytest.mark.parametrize("center", ["cell", "origin"])
@pytest.mark.parametrize("axes", [7, 4, 2, 1, 3])
def test_projection_identities(orc, center, axes):
    n = 10
    L = orc.lattice(n, 0.1, 1.0, center=center)
    psi = synth.random_state(n, 5)
    pp = orc.project(L, psi, +1, axes)
    pm = orc.project(L, psi, -1, axes)
    assert np.abs(pp + pm - psi).max() < 1e-15
    assert np.abs(orc.project(L, pp, +1, axes) - pp).max() < 1e-15
    assert np.abs(orc.project(L, pp, -1, axes)).max() < 1e-15
    assert abs(np.sum(pp * pm)) < 1e-12 * np.sum(psi * psi)


@pytest.mark.parametrize("center", ["cell", "origin"])
def test_parity_weight(orc, center):
    n = 12
    L = orc.lattice(n, 0.1, 1.0, dtau=1e-3, center=center)
    psi = synth.random_state(n, 9)
    v = np.zeros((n, n, n))
    pp = orc.project(L, psi, +1, 7)
    w = orc.observe(L, [psi, pp, psi - pp], v)
    assert abs(w[0]["parity_even"] - np.sum(pp * pp) / np.sum(psi * psi)) < 1e-13
    assert abs(w[1]["parity_even"] - 1.0) < 1e-13
    assert abs(w[2]["parity_even"]) < 1e-13


def test_orthonormalise(orc):
    n = 12
    states = synth.random_states(n, 4, seed=3)
    out = orc.orthonormalise(states)
    g = np.einsum("iabc,jabc->ij", out, out)
    assert np.abs(g - np.eye(4)).max() < 1e-14
    # spans are nested: state i lies in span(states 0..i)
    for i in range(4):
        A = np.stack([s.ravel() for s in states[: i + 1]], axis=1)
        coef, *_ = np.linalg.lstsq(A, out[i].ravel(), rcond=None)
        assert np.abs(A @ coef - out[i].ravel()).max() < 1e-12


@pytest.mark.parametrize("center", ["cell", "origin"])
def test_position_moments_one_site(orc, center):
    n, a = 8, 0.25
    L = orc.lattice(n, a, 1.0, dtau=1e-3, center=center)
    psi = np.zeros((n, n, n))
    site = (1, 6, 4)
    psi[site] = 2.0
    o = orc.observe(L, [psi], np.zeros_like(psi))[0]
    c = synth.axis_coords(n, a, center)
    assert abs(o["x"] - c[1]) < 1e-15 and abs(o["y"] - c[6]) < 1e-15 and abs(o["z"] - c[4]) < 1e-15
    assert abs(o["r2"] - (c[1] ** 2 + c[6] ** 2 + c[4] ** 2)) < 1e-14
    assert abs(o["norm2"] - 4.0) < 1e-15


def test_chunked_steps_equal_one_run(orc):
    """Stepping 7 then 5 steps (global step counter carried) equals 12 steps."""
    n = 12
    L = orc.lattice(n, 0.2, 1.0, dtau=0.004, kin=3, center="origin")
    v = synth.potential_cornell(n, 0.2, "origin")
    s0 = synth.random_states(n, 2, seed=1)
    full, _ = orc.step(L, s0, v, 12, ortho_every=3, record=False)
    a, _ = orc.step(L, s0, v, 7, ortho_every=3, record=False)
    b, _ = orc.step(L, a, v, 5, step0=7, ortho_every=3, record=False)
    assert np.array_equal(full, b)


def test_snapshot_extraction_plane_waves(orc):
    """Snapshot-overlap extraction (section "The iterative procedure") pinned by a
    closed form: with V = 0 the map multiplies each plane wave by
    lambda(k) = 1 - dtau T(k), so a mix of three orthonormal cosine waves stays a
    mix whose coefficients at step n are a_k lambda_k^n.  Gram-Schmidt of the
    coefficient vectors (latest, then earlier snapshots) gives the estimates and
    their energies sum_k q_k^2 T(k) exactly; the oracle, stepping the full
    lattice with its FFTs, must reproduce both."""
    n, a, m, dtau = 8, 0.5, 1.0, 0.03            # dtau max T = 1.78, inside the stable range
    L = orc.lattice(n, a, m, dtau, orc.KIN_NR_CONT, True, "cell")
    x = np.arange(n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    waves, T = [], []
    for mv in [(0, 0, 0), (1, 0, 0), (1, 1, 0)]:
        w = np.cos(2 * np.pi * (mv[0] * X + mv[1] * Y + mv[2] * Z) / n)
        waves.append(w / np.sqrt((w * w).sum()))
        k2 = sum((2 * np.pi * c / n) ** 2 for c in mv)
        T.append(k2 / (2 * a * a * m))
    T = np.array(T)
    coef0 = np.array([1.0, 0.8, 0.6])
    psi0 = sum(c * w for c, w in zip(coef0, waves))
    v = np.zeros((n, n, n))
    marks = [5, 20, 50]                    # snapshot steps, the last one is "current"
    snaps, state, done = [], psi0[None], 0
    for mk in marks:
        state, _ = orc.step(L, state, v, mk - done, step0=done, record=False)
        done = mk
        snaps.append(state[0].copy())
    est, obs = orc.snapshot_extract(L, snaps[-1], snaps[-2::-1], v)
    lam = 1.0 - dtau * T
    cols = [coef0 * lam ** mk for mk in marks[::-1]]     # latest first
    q = []
    for c in cols:
        c = c.copy()
        for b in q:
            c -= (b @ c) * b
        q.append(c / np.linalg.norm(c))
    for i in range(3):
        ref = sum(q[i][k] * waves[k] for k in range(3))
        assert np.abs(est[i] - ref).max() < 1e-12
        assert abs(obs[i]["energy"] - (q[i] ** 2) @ T) < 1e-12
    # the estimates approach the eigenstates in order of energy
    assert obs[0]["energy"] < obs[1]["energy"] < obs[2]["energy"]


def test_complex_map_reduces_to_real(orc):
    """Complex map with a real potential and a real state is the real map."""
    n, a = 12, 0.3
    L = orc.lattice(n, a, 1.2, dtau=a * a * 1.2 / 8, kin=2, center="cell")
    v = synth.potential_harmonic(n, a, "cell", 0.5)
    psi = synth.random_state(n, 3)
    out_c, rec_c = orc.step_complex(L, psi, v, 5)
    out_r, rec_r = orc.step(L, [psi], v, 5)
    assert np.abs(out_c.imag).max() == 0.0
    assert np.abs(out_c.real - out_r[0]).max() < 1e-14
    for s in range(5):
        assert abs(rec_c[s]["energy"] - rec_r[s][0]["energy"]) < 1e-13
        assert rec_c[s]["energy_imag"] == 0.0


def test_complex_constant_potential_closed_form(orc):
    """Closed form: with a constant complex V0 a plane wave is an eigenvector of the
    map with lambda = (1 - dtau V0/2 - dtau T(k)) / (1 + dtau V0/2); after n
    normalised steps the state is the start times (lambda/|lambda|)^n, and its
    energy is T(k) + V0."""
    n, a, m, dtau = 12, 0.25, 1.0, 0.01
    L = orc.lattice(n, a, m, dtau=dtau, kin=1, center="cell")
    v0 = 0.7 - 0.3j
    idx = np.indices((n, n, n))
    mv = (2, 1, 0)
    wave = np.cos(2 * np.pi * (mv[0] * idx[0] + mv[1] * idx[1] + mv[2] * idx[2]) / n)
    wave /= np.linalg.norm(wave)
    T = orc.kinetic_symbol(L)[mv]
    lam = (1 - 0.5 * dtau * v0 - dtau * T) / (1 + 0.5 * dtau * v0)
    out, rec = orc.step_complex(L, wave.astype(complex), np.full((n, n, n), v0), 7)
    assert np.abs(out - (lam / abs(lam)) ** 7 * wave).max() < 1e-13
    for r in rec:
        assert abs(r["energy"] - (T + v0.real)) < 1e-12 and abs(r["energy_imag"] - v0.imag) < 1e-12


def test_complex_map_global_phase(orc):
    """A real potential and a state e^{i theta} phi: the map is complex-linear with
    real A, B and H_K, so the result is e^{i theta} times the real map of phi, and
    every observable (moments and parity weight included) is that of phi."""
    n, a = 12, 0.3
    L = orc.lattice(n, a, 1.2, dtau=a * a * 1.2 / 8, kin=3, center="origin")
    v = synth.potential_harmonic(n, a, "origin", 0.5)
    phi = synth.random_state(n, 5)
    ph = np.exp(0.7j)
    out_c, rec_c = orc.step_complex(L, ph * phi, v, 4, parity=-1, axes=7, moments=True)
    out_r, rec_r = orc.step(L, [phi], v, 4, parity=[-1], axes=[7])
    assert np.abs(out_c - ph * out_r[0]).max() < 1e-14
    ob = orc.observe(L, [phi], v)[0]
    for k in ("x", "y", "z", "r2", "parity_even"):
        assert abs(rec_c[0][k] - ob[k]) < 1e-12, k
    for s in range(4):
        for k in ("energy", "kinetic", "potential"):
            assert abs(rec_c[s][k] - rec_r[s][0][k]) < 1e-12, (s, k)
        assert abs(rec_c[s]["energy_imag"]) < 1e-15
