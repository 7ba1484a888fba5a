"""GPU tests of the batched form (many lattices of uneven size in one graph launch
per chunk of steps) and of the serving loop (admission by HBM footprint,
continuous batching), through the C ABI, against the FP64 oracle.

Tolerances: FP32 lattices, step energies against the oracle on the same FP32
inputs within about four times the largest error measured on an MI355X (printed
by each run, see measure.py); batched against alone: bitwise.  Converged eigenpairs are
certified by the oracle's residual of the step map."""
import numpy as np
import pytest

import synth
from measure import check, max_rel_energy

pytestmark = pytest.mark.gpu


def _olat(orc, p):
    return orc.lattice(p.n, p.a, p.mass, p.dtau, p.kin, p.subtract_rest_mass, p.center)


def _make(itse, p, precision="fp32"):
    dt = np.float32 if precision == "fp32" else np.float64
    lat = itse.Lattice(p.n, p.a, p.mass, p.dtau, kin=p.kin, subtract_rest_mass=p.subtract_rest_mass,
                       precision=precision, center=p.center, nstates=p.nstates)
    lat.set_potential(p.potential_array(np.float64).astype(dt))
    for i, s in enumerate(p.initial_states()):
        lat.set_state(i, s.astype(dt))
    lat.set_options(ortho_every=1, parity=list(p.parity) if p.parity else None)
    return lat


def test_batched_mix_matches_oracle_and_alone(itse, orc):
    """Twelve solves from the batched-form recipe (N in {32, 48, 64, 96}, masses,
    Cornell couplings and kinetic terms drawn as the recipe says, two states each):
    the batched trajectory equals each lattice stepped alone bitwise, and its
    energies follow the oracle."""
    probs = synth.batch_problems(count=12, seed=3, nstates=2)
    assert len({p.n for p in probs}) >= 3
    steps = 24
    alone = [_make(itse, p) for p in probs]
    for lat in alone:
        lat.step(steps)
    mixed = [_make(itse, p) for p in probs]
    batch = itse.Batch(mixed)
    batch.step(steps)
    for p, la, lb in zip(probs, alone, mixed):
        ha, hb = la.history(steps), lb.history(steps)
        for s in range(steps):
            for i in range(p.nstates):
                assert ha[s][i]["energy"] == hb[s][i]["energy"]
        for i in range(p.nstates):
            assert np.array_equal(la.get_state(i, np.float32), lb.get_state(i, np.float32))
    for j in (0, 5, 11):
        p = probs[j]
        v = p.potential_array(np.float64).astype(np.float32).astype(np.float64)
        states = [s.astype(np.float32).astype(np.float64) for s in p.initial_states()]
        _, oh = orc.step(_olat(orc, p), states, v, steps)
        hb = mixed[j].history(steps)
        check(f"batch.mix_energies[{j}]", max_rel_energy(hb, oh), 2.5e-7)
    batch.close()
    for lat in alone + mixed:
        lat.close()


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_batched_mix_under_other_schedules(itse, orc, variant):
    """The batched-form mix under the other schedules of the batch sizes (column
    workgroups of four waves; the y axis split in two where the size has it; plane
    workgroups of two or three waves, each owning whole update rounds): the batch
    equals each lattice stepped alone bitwise, and the energies follow the
    oracle."""
    probs = synth.batch_problems(count=8, seed=5, nstates=2)
    for n in (32, 48, 64, 96):
        itse.set_schedule(n, "fp32", min(variant, itse.schedule_variants(n, "fp32") - 1))
    try:
        steps = 12
        alone = [_make(itse, p) for p in probs]
        mixed = [_make(itse, p) for p in probs]
    finally:
        for n in (32, 48, 64, 96):
            itse.set_schedule(n, "fp32", 0)
    for lat in alone:
        lat.step(steps)
    batch = itse.Batch(mixed)
    batch.step(steps)
    for p, la, lb in zip(probs, alone, mixed):
        for i in range(p.nstates):
            assert np.array_equal(la.get_state(i, np.float32), lb.get_state(i, np.float32))
    for j in (0, 3, 7):
        p = probs[j]
        v = p.potential_array(np.float64).astype(np.float32).astype(np.float64)
        states = [s.astype(np.float32).astype(np.float64) for s in p.initial_states()]
        _, oh = orc.step(_olat(orc, p), states, v, steps)
        check(f"batch.schedule{variant}_energies[{j}]", max_rel_energy(mixed[j].history(steps), oh), 2.5e-7)
    batch.close()
    for lat in alone + mixed:
        lat.close()


def _request(itse, server, p, tol=1e-7, keep=False, precision="fp32", max_steps=20000):
    dt = np.float32 if precision == "fp32" else np.float64
    return server.submit(p.n, p.a, p.mass, p.dtau, p.potential_array(np.float64).astype(dt),
                         [s.astype(dt) for s in p.initial_states()], kin=p.kin,
                         subtract_rest_mass=p.subtract_rest_mass, precision=precision, center=p.center,
                         ortho_every=1, tol=tol, relative=True, keep_states=keep, max_steps=max_steps)


def _drain(server, limit=100000):
    results = {}
    for _ in range(limit):
        live, queued = server.progress()
        for r in server.poll():
            results[r["id"]] = r
        if live == 0 and queued == 0:
            break
    return results


def test_server_result_same_alone_and_in_mix(itse):
    """A request solved alone and the same request admitted later into a mix of
    other requests of several sizes give bitwise the same energies and step count."""
    probs = synth.batch_problems(count=6, seed=11, sizes=(32, 48, 64), nstates=2)
    target = probs[0]
    alone = itse.Server(hbm_budget=8 << 30, max_slots=8, chunk=50)
    rid = _request(itse, alone, target)
    ra = _drain(alone)[rid]
    alone.close()
    assert ra["status"] == 0 and ra["converged"]
    mix = itse.Server(hbm_budget=8 << 30, max_slots=3, chunk=50)
    ids = [_request(itse, mix, p) for p in probs[1:3]]
    mix.progress()                           # the first two start before the target arrives
    ids.append(_request(itse, mix, target))
    ids += [_request(itse, mix, p) for p in probs[3:]]
    res = _drain(mix)
    mix.close()
    assert set(ids) <= set(res)
    rm = res[ids[2]]
    assert rm["status"] == 0 and rm["converged"]
    assert rm["steps"] == ra["steps"]
    assert rm["energy"][:2] == ra["energy"][:2]
    for i in ids:
        assert res[i]["status"] == 0


def test_server_admission_by_footprint(itse):
    """With a budget that holds two 64^3 requests, at most two are live at once,
    the rest wait in arrival order, and all device memory is returned."""
    probs = synth.batch_problems(count=5, seed=5, sizes=(64,), nstates=2)
    fp = itse.Lattice.footprint(64, 2, "fp32")
    server = itse.Server(hbm_budget=2 * fp + fp // 2, max_slots=16, chunk=40)
    ids = [_request(itse, server, p, tol=1e-6) for p in probs]
    peak = 0
    results = {}
    for _ in range(100000):
        live, queued = server.progress()
        peak = max(peak, live)
        assert server.bytes_in_use <= 2 * fp + fp // 2
        for r in server.poll():
            results[r["id"]] = r
        if live == 0 and queued == 0:
            break
    assert peak == 2
    assert server.bytes_in_use == 0
    assert sorted(results) == sorted(ids)
    # admitted in arrival order
    admits = [results[i]["t_admit"] for i in ids]
    assert admits == sorted(admits)
    with pytest.raises(itse.ItseError) as e:
        _request(itse, itse.Server(hbm_budget=fp // 2, max_slots=1, chunk=10), probs[0])
    assert e.value.status == -2
    server.close()


def test_server_converged_eigenpair_certified(itse, orc):
    """An FP64 request run to 1e-10 relative: the oracle certifies the returned
    ground state as a fixed point of the step map (small residual), with the
    same energy."""
    p = synth.Problem(n=32, a=0.2, mass=1.3, kin=3, dtau=0.05, center="origin", nstates=1,
                      potential="cornell", pot_args={"sigma": 0.2, "alpha": 0.4}, seed=7)
    server = itse.Server(hbm_budget=1 << 30, max_slots=2, chunk=100)
    rid = _request(itse, server, p, tol=1e-10, keep=True, precision="fp64", max_steps=40000)
    r = _drain(server)[rid]
    assert r["status"] == 0 and r["converged"]
    psi = server.state(rid, 0, p.n)
    server.release(rid)
    server.close()
    cert = orc.certify(_olat(orc, p), psi, p.potential_array(np.float64))
    assert abs(cert["energy"] - r["energy"][0]) <= 1e-10 * abs(r["energy"][0])
    assert cert["resid"] < 1e-5


def test_autotuners_report_and_set_schedules(itse):
    """itse_autotune times every schedule of a size on a three-state and a one-state
    step and keeps the fastest of each; itse_autotune_batch times a batch of the
    given count and state number and keeps the fastest for that kind of lattice.
    Bad counts and state numbers are refused."""
    import json
    n = 48
    nv = itse.schedule_variants(n, "fp32")
    try:
        single = json.loads(itse.autotune(n, "fp32"))
        assert len(single["times_ms"]) == nv and len(single["times_ms_one_state"]) == nv
        assert all(t > 0 for t in single["times_ms"] + single["times_ms_one_state"])
        assert single["times_ms"][single["best"]] == min(single["times_ms"])
        cur = json.loads(itse.schedule(n, "fp32"))
        assert cur["variant"] == single["best"] and cur["variant_one_state"] == single["best_one_state"]
        batch = json.loads(itse.autotune_batch(n, "fp32", 6, 2))
        assert batch["count"] == 6 and batch["nstates"] == 2 and len(batch["times_ms"]) == nv
        assert batch["times_ms"][batch["best"]] == min(batch["times_ms"])
        assert json.loads(itse.schedule(n, "fp32"))["variant"] == batch["best"]
        with pytest.raises(itse.ItseError, match="EINVAL"):
            itse.autotune_batch(n, "fp32", 0, 2)
        with pytest.raises(itse.ItseError, match="EINVAL"):
            itse.autotune_batch(n, "fp32", 2, 0)
    finally:
        itse.set_schedule(n, "fp32", 0)
