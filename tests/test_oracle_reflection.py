"""The oracle's reflections pinned by states whose parity is known by construction.

Section "Parity projection" defines P^(+-) psi = (psi(r) +- psi(-r))/2, with -r the
point reflection about the potential centre (equation parity); the INITSYMMETRY
options of section "Basic configuration" reflect a single axis.  The states here
are products f1(x1) f2(x2) f3(x3) of factors that are even or odd in the signed
coordinate about the centre, so their parity under any set of reflected axes is
the product of the factors' parities on those axes, fixed before the oracle sees
them.  The coordinates are computed in this file from the centring conventions:

  cell centring:   c = idx - (N - 1)/2         (the mirror of idx is N - 1 - idx)
  origin centring: c = idx or idx - N, |c| <= N/2 (minimum image; the mirror of idx
                   is -idx mod N, and the sites 0 and N/2 are their own mirrors)

For origin centring an odd factor must vanish at both self-mirror sites; sin(2 pi k
c / N) does, and c g(c) is set to zero at c = N/2.  A Gaussian about site 0 is even
under -idx mod N but not under N - 1 - idx, so a mirror that confused the two
centrings fails these tests.
"""
import numpy as np
import pytest

N = 12


def _coords(n, center):
    idx = np.arange(n, dtype=np.float64)
    if center == "cell":
        return idx - 0.5 * (n - 1)
    return np.where(2 * idx <= n, idx, idx - n)


def _factor(kind, n, center):
    """(values along one axis, parity under that axis' reflection)."""
    c = _coords(n, center)
    g = np.exp(-c * c / (2.0 * 2.2 ** 2))
    if kind == "gauss":
        return g, +1
    if kind == "cos":
        return np.cos(2.0 * np.pi * 2.0 * c / n) + 0.3, +1
    if kind == "sin":
        return np.sin(2.0 * np.pi * c / n) * (1.0 + 0.2 * c * c), -1
    if kind == "xg":
        f = c * g
        if center == "origin":
            f = np.where(2 * np.arange(n) == n, 0.0, f)   # self-mirror site N/2
        return f, -1
    raise ValueError(kind)


FACTORS = [("gauss", "gauss", "gauss"), ("xg", "gauss", "cos"), ("gauss", "sin", "gauss"),
           ("cos", "gauss", "xg"), ("xg", "sin", "gauss"), ("sin", "cos", "xg"),
           ("xg", "xg", "sin"), ("sin", "xg", "cos")]


def _state(kinds, center, n=N):
    (f1, p1), (f2, p2), (f3, p3) = (_factor(k, n, center) for k in kinds)
    psi = f1[:, None, None] * f2[None, :, None] * f3[None, None, :]
    return psi, (p1, p2, p3)


def _sign(par, axes):
    s = 1
    for bit in range(3):
        if axes & (1 << bit):
            s *= par[bit]
    return s


@pytest.mark.parametrize("center", ["cell", "origin"])
@pytest.mark.parametrize("axes", [7, 4, 2, 1, 3, 5, 6])
@pytest.mark.parametrize("kinds", FACTORS)
def test_projection_of_definite_states(orc, center, axes, kinds):
    """P with the state's own sign leaves it unchanged, the other sign annihilates it."""
    L = orc.lattice(N, 0.1, 1.0, center=center)
    psi, par = _state(kinds, center)
    s = _sign(par, axes)
    scale = np.abs(psi).max()
    keep = orc.project(L, psi, s, axes)
    kill = orc.project(L, psi, -s, axes)
    assert np.abs(keep - psi).max() <= 1e-15 * scale
    assert np.abs(kill).max() <= 1e-15 * scale


@pytest.mark.parametrize("center", ["cell", "origin"])
@pytest.mark.parametrize("kinds", FACTORS)
def test_parity_weight_of_definite_states(orc, center, kinds):
    """The even-parity weight (full inversion) of a definite state is exactly 1 or 0."""
    L = orc.lattice(N, 0.1, 1.0, dtau=1e-3, center=center)
    psi, par = _state(kinds, center)
    w = orc.observe(L, [psi], np.zeros_like(psi))[0]["parity_even"]
    expect = 1.0 if _sign(par, 7) > 0 else 0.0
    assert abs(w - expect) <= 1e-14


@pytest.mark.parametrize("center", ["cell", "origin"])
def test_parity_weight_of_a_mixture(orc, center):
    """a e + b o with e even and o odd under inversion: the even weight is
    a^2 |e|^2 / (a^2 |e|^2 + b^2 |o|^2) (the cross terms cancel by symmetry)."""
    L = orc.lattice(N, 0.1, 1.0, dtau=1e-3, center=center)
    e, pe = _state(("xg", "sin", "gauss"), center)
    o, po = _state(("xg", "gauss", "cos"), center)
    assert _sign(pe, 7) == 1 and _sign(po, 7) == -1
    a, b = 0.7, -1.3
    psi = a * e + b * o
    w = orc.observe(L, [psi], np.zeros_like(psi))[0]["parity_even"]
    ee, oo = a * a * np.sum(e * e), b * b * np.sum(o * o)
    assert abs(w - ee / (ee + oo)) <= 1e-13


@pytest.mark.parametrize("axes", [7, 4, 2])
def test_origin_states_are_not_cell_symmetric(orc, axes):
    """The origin-centred test states are not symmetric under the cell mirror
    N - 1 - idx: projecting them with the cell-centred oracle changes them, so the
    tests above separate the two centrings."""
    psi, par = _state(("gauss", "gauss", "gauss"), "origin")
    Lc = orc.lattice(N, 0.1, 1.0, center="cell")
    moved = orc.project(Lc, psi, _sign(par, axes), axes)
    assert np.abs(moved - psi).max() > 1e-3 * np.abs(psi).max()


@pytest.mark.parametrize("center", ["cell", "origin"])
@pytest.mark.parametrize("n", [9, 16])
def test_reflection_other_lengths(orc, center, n):
    """Odd N (origin centring: site 0 the only self-mirror) and N = 16."""
    L = orc.lattice(n, 0.1, 1.0, center=center)
    for kinds in FACTORS[:4]:
        psi, par = _state(kinds, center, n)
        for axes in (7, 4, 2):
            s = _sign(par, axes)
            scale = np.abs(psi).max()
            assert np.abs(orc.project(L, psi, s, axes) - psi).max() <= 1e-15 * scale
            assert np.abs(orc.project(L, psi, -s, axes)).max() <= 1e-15 * scale
