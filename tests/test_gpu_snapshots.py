"""GPU parity of the snapshot-overlap extraction of excited states (paper, section
"The iterative procedure") through the C ABI: state 0 evolves, snapshots are kept,
and the estimates (the latest wave-function, then each snapshot, newest first,
with its projections on the earlier estimates removed and normalised) and their
energies are compared with the oracle doing the same on the same inputs.

Tolerances: FP64 lattices 1e-10 relative on energies and 1e-9 max-abs on the
estimates (Gram-Schmidt of nearly parallel snapshots amplifies rounding by the
condition number of the snapshot set, about 1e2 here); FP32 lattices about four
times the largest error measured on an MI355X, for the ground-state energy and
for the excited estimates apart (FP32 rounding of the evolution, amplified the
same way), printed by each run (see measure.py)."""
import numpy as np
import pytest

import synth
from measure import check

pytestmark = pytest.mark.gpu


def _setup(itse, orc, n, prec, kin, center, pot, seed):
    a = 6.4 / n if kin in (3, 4) else 0.3
    mass = 1.3
    dtau = a / 4 if kin in (3, 4) else a * a * mass / 8
    lat = itse.Lattice(n, a, mass, dtau, kin=kin, subtract_rest_mass=True, precision=prec, center=center,
                       nstates=1)
    dt = np.float32 if prec == "fp32" else np.float64
    if pot == "cornell":
        v = synth.potential_cornell(n, a, center, sigma=0.2, alpha=0.4).astype(dt)
    else:
        v = synth.potential_harmonic(n, a, center, 0.5).astype(dt)
    psi = synth.random_state(n, seed, dtype=dt)
    lat.set_potential(v)
    lat.set_state(0, psi)
    lat.set_options(ortho_every=0)
    L = orc.lattice(n, a, mass, dtau, kin, True, center)
    return lat, L, v.astype(np.float64), psi.astype(np.float64)


@pytest.mark.parametrize("n,prec,kin,center,pot", [
    (32, "fp64", 3, "origin", "cornell"),
    (24, "fp64", 1, "cell", "harmonic"),
    (48, "fp32", 2, "cell", "harmonic"),
])
def test_snapshot_extraction_matches_oracle(itse, orc, n, prec, kin, center, pot):
    lat, L, v, psi = _setup(itse, orc, n, prec, kin, center, pot, seed=90 + n)
    marks = [30, 90, 160]
    state, done = psi[None], 0
    snaps = []
    for mk in marks:
        lat.step(mk - done)
        state, _ = orc.step(L, state, v, mk - done, step0=done, record=False)
        done = mk
        if mk != marks[-1]:
            lat.snapshot()
            snaps.append(state[0].copy())
    assert lat.snapshot_count == 2
    before = lat.get_state(0)
    obs, est = lat.extract(states=True)
    assert np.array_equal(before, lat.get_state(0))        # the lattice is not changed
    oest, oobs = orc.snapshot_extract(L, state[0], snaps[::-1], v)
    assert len(obs) == 3
    errs = [abs(obs[k]["energy"] - oobs[k]["energy"]) / max(1.0, abs(oobs[k]["energy"])) for k in range(3)]
    nerr = max(abs(obs[k]["norm2"] - 1.0) for k in range(3))
    # estimates are orthonormal
    gram = np.einsum("aijk,bijk->ab", est, est)
    gerr = np.abs(gram - np.eye(3)).max()
    if prec == "fp64":
        assert max(errs) <= 1e-10 and nerr < 1e-12 and gerr < 1e-12, (errs, nerr, gerr)
        for k in range(3):
            assert np.abs(est[k] - oest[k]).max() < 1e-9, k
    else:
        check(f"snapshots.extract[{n}].ground_energy", errs[0], 5.8e-7)
        check(f"snapshots.extract[{n}].excited_energies", max(errs[1:]), 2.9e-7)
        # measured 3.8e-9 with FMA contraction fixed by the source (8e-10 before)
        check(f"snapshots.extract[{n}].norms", nerr, 1.5e-8)
        # measured 3.8e-9 with FMA contraction fixed by the source (8e-10 before)
        check(f"snapshots.extract[{n}].gram", gerr, 1.5e-8)
    lat.close()


def test_snapshot_ring(itse, orc):
    """The ring keeps the two latest snapshots; with none, the only estimate is the
    normalised current state; clearing drops them."""
    lat, L, v, psi = _setup(itse, orc, 16, "fp64", 1, "cell", "harmonic", seed=5)
    obs = lat.extract()
    assert len(obs) == 1
    ref = orc.observe(L, [psi / np.sqrt((psi * psi).sum())], v)[0]
    assert abs(obs[0]["energy"] - ref["energy"]) < 1e-12 * abs(ref["energy"])
    state, done, kept = psi[None], 0, []
    for mk in (10, 20, 30, 40):
        lat.step(mk - done)
        state, _ = orc.step(L, state, v, mk - done, step0=done, record=False)
        done = mk
        lat.snapshot()
        kept.append(state[0].copy())
    assert lat.snapshot_count == 2
    lat.step(10)
    state, _ = orc.step(L, state, v, 10, step0=done, record=False)
    obs = lat.extract()
    _, oobs = orc.snapshot_extract(L, state[0], [kept[-1], kept[-2]], v)
    for k in range(3):
        assert abs(obs[k]["energy"] - oobs[k]["energy"]) <= 1e-10 * abs(oobs[k]["energy"])
    lat.clear_snapshots()
    assert lat.snapshot_count == 0
    assert len(lat.extract()) == 1
    lat.close()
