"""Pins for the oracle's kinetic terms (paper, equations HK1, HK2, HK3 and the
eigenmode set of section "Kinetic terms").

Each form is checked against something other than its own symbol formula:

* H_K^(2) equals the periodic 7-point finite-difference Laplacian over 2 A^2 M
  (the paper gives the same momentum-space symbol for the FDTD term H_K^(0));
* H_K^(1) equals -nabla^2 / 2M on a smooth periodic function whose derivatives
  are known analytically (spectral accuracy);
* H_K^(3) squared equals (4/A^2 sin^2 symbol) + M^2, i.e. the lattice Laplacian
  stencil plus M^2, with and without the rest-mass subtraction;
* the relativistic analogue of H_K^(1) squared equals -nabla^2 + M^2 analytically;
* the paper's relativistic harmonic oscillator (V = r^2, M = 30 GeV, A = 0.006 fm)
  has E0 - M within the paper's stated 0.5 permille of Li's analytic 0.38627 GeV
  (golden fixture, Lanczos on the oracle's operator);
* plane waves, including the Nyquist mode, are eigenvectors (pins the momentum
  grid layout and the sign convention).
"""
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lap_stencil(psi, a):
    """Periodic 7-point stencil: (6 psi - sum of the six neighbours) / a^2."""
    out = 6.0 * psi
    for ax in range(3):
        out = out - np.roll(psi, 1, axis=ax) - np.roll(psi, -1, axis=ax)
    return out / (a * a)


def _smooth(n, a):
    """psi = f(x) g(y) h(z) with f = exp(c cos(theta x + phi)); returns psi and -nabla^2 psi."""
    L = n * a
    th = 2 * np.pi / L
    x = np.arange(n) * a
    parts = []
    for c, ph in ((1.0, 0.0), (0.8, 0.3), (0.6, 1.1)):
        f = np.exp(c * np.cos(th * x + ph))
        s = np.sin(th * x + ph)
        co = np.cos(th * x + ph)
        f2 = (c * c * th * th * s * s - c * th * th * co) * f
        parts.append((f, f2))
    (fx, fx2), (fy, fy2), (fz, fz2) = parts
    psi = fx[:, None, None] * fy[None, :, None] * fz[None, None, :]
    lap = (fx2[:, None, None] * fy[None, :, None] * fz[None, None, :]
           + fx[:, None, None] * fy2[None, :, None] * fz[None, None, :]
           + fx[:, None, None] * fy[None, :, None] * fz2[None, None, :])
    return psi, -lap


@pytest.mark.parametrize("n,a,m", [(12, 0.3, 1.0), (32, 0.1, 2.5), (48, 0.05, 0.7)])
def test_hk2_is_periodic_stencil(orc, n, a, m):
    psi = synth.random_state(n, 3)
    L = orc.lattice(n, a, m, kin=2)
    got = orc.apply_kinetic(L, psi)
    ref = _lap_stencil(psi, a) / (2 * m)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n,a,m", [(32, 0.2, 1.0), (48, 0.1, 3.0)])
def test_hk1_is_continuum_laplacian(orc, n, a, m):
    psi, mlap = _smooth(n, a)
    L = orc.lattice(n, a, m, kin=1)
    got = orc.apply_kinetic(L, psi)
    ref = mlap / (2 * m)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("sub", [False, True])
@pytest.mark.parametrize("n,a,m", [(16, 0.25, 1.3), (32, 0.05, 4.0)])
def test_hk3_squared_is_stencil_plus_mass(orc, n, a, m, sub):
    psi = synth.random_state(n, 11)
    L = orc.lattice(n, a, m, kin=3, subtract_rest=sub)

    def op(p):
        q = orc.apply_kinetic(L, p)
        return q + m * p if sub else q

    got = op(op(psi))
    ref = _lap_stencil(psi, a) + m * m * psi
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("sub", [False, True])
def test_relativistic_continuum_squared(orc, sub):
    n, a, m = 32, 0.2, 1.7
    psi, mlap = _smooth(n, a)
    L = orc.lattice(n, a, m, kin=4, subtract_rest=sub)

    def op(p):
        q = orc.apply_kinetic(L, p)
        return q + m * p if sub else q

    got = op(op(psi))
    ref = mlap + m * m * psi
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_rest_mass_subtraction_is_stable(orc):
    """sqrt(p^2+m^2)-m must keep full relative accuracy for p << m (lowest mode, heavy mass)."""
    n, a, m = 64, 0.4, 5.0
    L = orc.lattice(n, a, m, kin=3, subtract_rest=True)
    T = orc.kinetic_symbol(L)
    p2 = 4.0 * np.sin(np.pi / n) ** 2 / a ** 2          # lowest nonzero mode along one axis
    exact = p2 / (np.sqrt(p2 + m * m) + m)
    assert abs(T[1, 0, 0] - exact) <= 1e-15 * exact * 4
    # series check: p^2/(2m) - p^4/(8 m^3) + ...
    series = p2 / (2 * m) - p2 ** 2 / (8 * m ** 3) + p2 ** 3 / (16 * m ** 5)
    assert abs(T[1, 0, 0] - series) <= 1e-6 * exact


@pytest.mark.parametrize("kin,sub", [(1, True), (2, True), (3, True), (3, False), (4, True)])
def test_plane_waves_are_eigenvectors(orc, kin, sub):
    n, a, m = 16, 0.2, 1.3
    L = orc.lattice(n, a, m, kin=kin, subtract_rest=sub)
    idx = np.indices((n, n, n))
    for mv, ph in (((1, 0, 0), 0.2), ((n // 2, 3, n - 2), 0.0), ((5, n // 2, n // 2), 1.0)):
        psi = np.cos(2 * np.pi * (mv[0] * idx[0] + mv[1] * idx[1] + mv[2] * idx[2]) / n + ph)
        k = [2 * np.pi * (c if 2 * c <= n else c - n) / n for c in mv]
        s2 = sum(np.sin(kk / 2) ** 2 for kk in k)
        k2 = sum(kk * kk for kk in k)
        if kin == 1:
            t = k2 / (2 * a * a * m)
        elif kin == 2:
            t = 4 * s2 / (2 * a * a * m)
        else:
            p2 = 4 * s2 / a ** 2 if kin == 3 else k2 / a ** 2
            t = np.sqrt(p2 + m * m) - (m if sub else 0.0)
        got = orc.apply_kinetic(L, psi)
        assert np.abs(got - t * psi).max() <= 1e-12 * max(1.0, abs(t))


@pytest.mark.parametrize("kin,sub,expect", [(1, True, 0.0), (2, True, 0.0), (3, True, 0.0),
                                            (3, False, 1.3), (4, False, 1.3)])
def test_free_particle_constant_state(orc, kin, sub, expect):
    n = 12
    L = orc.lattice(n, 0.1, 1.3, dtau=1e-3, kin=kin, subtract_rest=sub)
    psi = np.full((n, n, n), 0.5)
    obs = orc.observe(L, [psi], np.zeros((n, n, n)))[0]
    assert abs(obs["energy"] - expect) < 1e-12
    cert = orc.certify(L, psi, np.zeros((n, n, n)))
    assert cert["resid"] < 1e-12


def _golden():
    vals = {}
    with open(os.path.join(GOLDEN, "relativistic_oscillator.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


@pytest.mark.slow
def test_relativistic_oscillator_worked_example(orc):
    """E0 - M of H_K^(3) + r^2 at M = 30 GeV, A = 0.006 fm agrees with Li's analytic
    value to the paper's 0.5 permille.  N = 96 keeps the box 5 widths wide."""
    from scipy.sparse.linalg import LinearOperator, eigsh
    g = _golden()
    A = g["A_fm"] / g["hbar_c_GeV_fm"]
    M = g["M_GeV"]
    n = 96
    L = orc.lattice(n, A, M, kin=3, subtract_rest=True, center="cell")
    v = synth.potential_harmonic(n, A, "cell", coef=1.0)
    _, _, _, r = synth.radius_grid(n, A, "cell")
    w0 = np.sqrt(2.0 / M)
    guess = np.exp(-0.5 * M * w0 * r * r).ravel()

    def mv(x):
        x = np.asarray(x).ravel()
        return orc.apply_kinetic(L, x.reshape(n, n, n)).ravel() + v.ravel() * x

    op = LinearOperator((n ** 3, n ** 3), matvec=mv, dtype=np.float64)
    w, _ = eigsh(op, k=1, which="SA", tol=1e-9, v0=guess)
    e0 = float(w[0])
    ref = g["E0_minus_M_analytic"]
    assert abs(e0 - ref) <= g["E0_relative_agreement"] * ref
    # the paper's own tau = 10 value lies above the converged lattice value
    assert e0 < g["E0_minus_M_numeric_tau10"]


@pytest.mark.slow
def test_relativistic_oscillator_radial_excitation(orc):
    """The first radially excited s state of the same problem agrees with Li's
    analytic E1 - M to the paper's sub-percent level.  The s states are isolated
    by restricting the operator to functions invariant under the cubic group
    (axis permutations and reflections about the cell centre), which H commutes
    with; the l = 2 levels have no invariant component, so the two lowest
    invariant levels are 1s and 2s.  The complement is shifted far above them."""
    import itertools
    from scipy.sparse.linalg import LinearOperator, eigsh
    g = _golden()
    A = g["A_fm"] / g["hbar_c_GeV_fm"]
    M = g["M_GeV"]
    n = 96
    L = orc.lattice(n, A, M, kin=3, subtract_rest=True, center="cell")
    v = synth.potential_harmonic(n, A, "cell", coef=1.0)
    _, _, _, r = synth.radius_grid(n, A, "cell")
    perms = list(itertools.permutations(range(3)))

    def invariant(x):
        e = x + x[::-1]
        e = e + e[:, ::-1]
        e = e + e[:, :, ::-1]
        return sum(np.transpose(e, q) for q in perms) / 48.0

    shift = 50.0  # GeV, far above both levels

    def mv(x):
        x = np.asarray(x).reshape(n, n, n)
        p = invariant(x)
        hp = orc.apply_kinetic(L, p) + v * p
        return (invariant(hp) + shift * (x - p)).ravel()

    w0 = np.sqrt(2.0 / M)
    gs = np.exp(-0.5 * M * w0 * r * r)
    guess = (gs + (M * w0 * r * r - 1.5) * gs).ravel()
    op = LinearOperator((n ** 3, n ** 3), matvec=mv, dtype=np.float64)
    w, _ = eigsh(op, k=2, which="SA", tol=1e-9, v0=guess)
    e0, e1 = sorted(float(x) for x in w)
    assert abs(e0 - g["E0_minus_M_analytic"]) <= g["E0_relative_agreement"] * g["E0_minus_M_analytic"]
    ref = g["E1_radial_minus_M_analytic"]
    assert abs(e1 - ref) <= 1e-2 * ref
    # the paper's tau = 10 value of this level (its second excited state) lies above
    assert e1 < g["E2_minus_M_numeric_tau10"]


# ---------------------------------------------------------------------------------
# H_K^(0) (paper, equation HK0): finite differences with Dirichlet boundaries, the
# wave-function vanishing outside the N^3 box.
# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("n,a,m", [(6, 0.3, 1.0), (12, 0.2, 2.0)])
def test_hk0_is_dirichlet_laplacian(orc, n, a, m):
    """Brute force: the dense Kronecker sum of 1D second-difference matrices with no
    wrap-around (Dirichlet walls), (2 delta_ij - delta_i,j+-1) / (2 M A^2) per axis,
    applied to a random state."""
    L = orc.lattice(n, a, m, kin=0)
    D = (2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)) / (2 * m * a * a)
    I = np.eye(n)
    H = np.kron(np.kron(D, I), I) + np.kron(np.kron(I, D), I) + np.kron(np.kron(I, I), D)
    psi = np.random.default_rng(n).standard_normal((n, n, n))
    ref = (H @ psi.reshape(-1)).reshape(n, n, n)
    assert np.abs(orc.apply_kinetic(L, psi) - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("modes", [(1, 1, 1), (2, 1, 3), (5, 4, 1)])
def test_hk0_sine_modes(orc, modes):
    """Closed form: products of sin(pi m (x + 1) / (N + 1)) vanish just outside the
    box and are eigenvectors with eigenvalue sum_l 4 sin^2(pi m_l / (2 (N + 1))) /
    (2 M A^2), the momentum-space form of the paper with k = pi m / (N + 1)."""
    n, a, m = 12, 0.25, 1.5
    L = orc.lattice(n, a, m, kin=0)
    x = np.arange(n)
    f = [np.sin(np.pi * q * (x + 1) / (n + 1)) for q in modes]
    psi = f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :]
    lam = sum(4 * np.sin(np.pi * q / (2 * (n + 1))) ** 2 for q in modes) / (2 * m * a * a)
    assert np.abs(orc.apply_kinetic(L, psi) - lam * psi).max() < 1e-13 * lam


def test_hk0_step_fixed_point(orc):
    """The step map with H_K^(0) keeps the product of 1D ground states of the
    Dirichlet K + sV (s = (1 + lambda)/2, from dense 1D eigensolves) invariant, as
    for the periodic kinds."""
    n, a, m, dtau = 16, 0.3, 1.0, 0.01
    L = orc.lattice(n, a, m, dtau=dtau, kin=0, center="cell")
    c = (np.arange(n) - 0.5 * (n - 1)) * a
    v1 = 0.5 * c * c
    D = (2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)) / (2 * m * a * a)
    s = 1.0
    for _ in range(200):
        e, U = np.linalg.eigh(D + s * np.diag(v1))
        lam = 1.0 - dtau * 3 * e[0]
        s = 0.5 * (1.0 + lam)
    e, U = np.linalg.eigh(D + s * np.diag(v1))
    u = U[:, 0]
    start = u[:, None, None] * u[None, :, None] * u[None, None, :]
    v = v1[:, None, None] + v1[None, :, None] + v1[None, None, :]
    out, hist = orc.step(L, [start], v, 50)
    e_fp = 3 * (u @ D @ u + u @ (v1 * u))
    assert abs(hist[0][0]["energy"] - e_fp) < 1e-12
    assert np.abs(out[0] - start).max() < 1e-10
