"""GPU tests of persistent batched stepping (itse_batch_set_persistent): one
cooperative launch runs every pass of every lattice of a batch for all the steps
of a call, the passes separated by grid-wide barriers.

Its tiles are those of the passes' own kernels under the same schedules, so each
lattice's states after the steps are compared bitwise with the same lattice
stepped alone; step energies of sampled lattices are compared with the FP64
oracle within about four times the largest FP32 error measured on an MI355X
(printed by each run, see measure.py)."""
import numpy as np
import pytest

import synth
from measure import check, max_rel_energy

pytestmark = pytest.mark.gpu

SIZES = (32, 48, 64, 96)


def _olat(orc, p):
    return orc.lattice(p.n, p.a, p.mass, p.dtau, p.kin, p.subtract_rest_mass, p.center)


def _make(itse, p, parity=None, precision="fp32"):
    dt = np.float32 if precision == "fp32" else np.float64
    lat = itse.Lattice(p.n, p.a, p.mass, p.dtau, kin=p.kin, subtract_rest_mass=p.subtract_rest_mass,
                       precision=precision, center=p.center, nstates=p.nstates)
    lat.set_potential(p.potential_array(np.float64).astype(dt))
    for i, s in enumerate(p.initial_states()):
        lat.set_state(i, s.astype(dt))
    lat.set_options(ortho_every=1, parity=parity)
    return lat


def _pairs(itse, probs, variant, parities=None):
    """Lattices of `probs` created under schedule `variant` (1 or 2; 1 for N = 32,
    whose schedule 2 has plane workgroups of two waves, which the persistent kernel
    does not take), twice: one set to step alone, one for the batch."""
    for n in SIZES:
        itse.set_schedule(n, "fp32", 1 if n == 32 else variant)
    try:
        par = parities or [None] * len(probs)
        alone = [_make(itse, p, q) for p, q in zip(probs, par)]
        batched = [_make(itse, p, q) for p, q in zip(probs, par)]
    finally:
        for n in SIZES:
            itse.set_schedule(n, "fp32", 0)
    return alone, batched


def _assert_bitwise(probs, alone, batched):
    for j, (p, la, lb) in enumerate(zip(probs, alone, batched)):
        for i in range(p.nstates):
            assert np.array_equal(la.get_state(i, np.float32), lb.get_state(i, np.float32)), (j, p.n, i)
        assert la.step_count == lb.step_count
        ha, hb = la.history(4), lb.history(4)
        assert ha == hb, j


@pytest.mark.parametrize("variant", [1, 2])
def test_persistent_batch_matches_alone_and_oracle(itse, orc, variant):
    """The batched-form mix (N in {32, 48, 64, 96}, one and two states, Gram-Schmidt
    every step), persistent: every lattice's states and step records equal the
    same lattice stepped alone bitwise; sampled energies follow the oracle."""
    probs = synth.batch_problems(count=10, seed=11, nstates=2)
    probs += synth.batch_problems(count=4, seed=12, nstates=1)
    alone, batched = _pairs(itse, probs, variant)
    steps = 13
    for lat in alone:
        lat.step(steps)
    batch = itse.Batch(batched)
    batch.set_persistent(True)
    batch.step(steps)
    _assert_bitwise(probs, alone, batched)
    for j in (0, 5, 11):
        p = probs[j]
        v = p.potential_array(np.float64).astype(np.float32).astype(np.float64)
        states = [s.astype(np.float32).astype(np.float64) for s in p.initial_states()]
        _, oh = orc.step(_olat(orc, p), states, v, steps)
        check(f"persistent.schedule{variant}_energies[{j}]", max_rel_energy(batched[j].history(steps), oh), 2.5e-7)
    batch.close()
    for lat in alone + batched:
        lat.close()


def test_persistent_projection_and_chunks(itse):
    """Parity projection along one set of axes (the projection/Gram pass on every
    step), steps split over several calls, and a switch back to graph replay and to
    persistent again: bitwise equal to stepping alone."""
    probs = synth.batch_problems(count=6, seed=21, nstates=2)
    parities = [[1, -1], [-1, 1], [1, 1], [0, -1], [1, -1], [-1, -1]]
    alone, batched = _pairs(itse, probs, 1, parities)
    for lat in alone:
        lat.step(17)
    batch = itse.Batch(batched)
    batch.set_persistent(True)
    batch.step(5)
    batch.step(1)
    batch.set_persistent(False)
    batch.step(4)
    batch.set_persistent(True)
    batch.step(7)
    _assert_bitwise(probs, alone, batched)
    batch.close()
    for lat in alone + batched:
        lat.close()


def test_persistent_falls_back_for_moments(itse):
    """Steps that form position moments take the graph path (the persistent kernel
    has the update instance without them): results still equal stepping alone."""
    probs = synth.batch_problems(count=4, seed=31, nstates=2)
    alone, batched = _pairs(itse, probs, 1)
    for lat in alone + batched:
        lat.set_options(ortho_every=1, moments=True)
    for lat in alone:
        lat.step(6)
    batch = itse.Batch(batched)
    batch.set_persistent(True)
    batch.step(6)
    _assert_bitwise(probs, alone, batched)
    for la, lb in zip(alone, batched):
        assert la.observe(0)["r2"] == lb.observe(0)["r2"]
    batch.close()
    for lat in alone + batched:
        lat.close()


def test_persistent_rejects_other_batches(itse):
    """FP64 lattices, more than two states, sizes without tiles and schedule 0 are
    refused with EINVAL; the batch keeps stepping through graphs."""
    p = synth.batch_problems(count=1, seed=41, nstates=2)[0]
    cases = []
    cases.append(_make(itse, p, precision="fp64"))
    cases.append(_make(itse, synth.batch_problems(count=1, seed=42, nstates=3)[0]))
    cases.append(_make(itse, p))  # schedule 0
    big = synth.batch_problems(count=1, seed=43, sizes=(128,), nstates=2)[0]
    itse.set_schedule(128, "fp32", 1)
    try:
        cases.append(_make(itse, big))
    finally:
        itse.set_schedule(128, "fp32", 0)
    for lat in cases:
        b = itse.Batch([lat])
        with pytest.raises(itse.ItseError, match="EINVAL"):
            b.set_persistent(True)
        b.step(2)
        assert lat.step_count == 2
        b.close()
        lat.close()


def test_options_changed_during_persistent_steps(itse):
    """Options that change the step's passes while the batch steps persistently
    (here Gram-Schmidt switched on) also reach the graph path afterwards: graphs
    captured before the change are not replayed.  Bitwise equal to stepping alone
    with the same sequence of options."""
    probs = synth.batch_problems(count=5, seed=51, nstates=2)
    alone, batched = _pairs(itse, probs, 1)
    for lat in alone + batched:
        lat.set_options(ortho_every=0)
    batch = itse.Batch(batched)
    for lat in alone:
        lat.step(3)
    batch.step(3)                      # graphs captured without the Gram pass
    for lat in alone + batched:
        lat.set_options(ortho_every=1)
    batch.set_persistent(True)
    for lat in alone:
        lat.step(4)
    batch.step(4)                      # persistent, with the Gram pass
    batch.set_persistent(False)
    for lat in alone:
        lat.step(5)
    batch.step(5)                      # graph path again: must include the Gram pass
    _assert_bitwise(probs, alone, batched)
    batch.close()
    for lat in alone + batched:
        lat.close()
