"""Benchmark of the imaginary-time step on one MI355X.

Workload (default): the precision-form solve at 256^3 - three states (parity
even, odd, odd deflated against the odd one), FP32 wave-functions and transforms
with FP64 norms/energies/Gram sums, relativistic lattice kinetic term
sqrt(p^2+m^2)-m with m = 1.3, a = 0.025, dtau = a/4, Cornell potential
-0.4/r + 0.2 r + 0.05 (x^2-y^2)/r (r >= a/2) stored as FP32, origin centring.

A step = one application of the whole hot path to every state: transforms,
kinetic multiply, update, parity projections, Gram-Schmidt, normalisation and
energies.  value = site-steps/s counting each state's N^3 sites per step.

Prints ONE JSON line (rank 0).  Extra keys: per-pass times and bytes, the same
workload in FP64, the bare one-state step, the batched form (64 lattices), the
serving form (Poisson arrivals: p50/p90/p99 latency and site-steps/s), the H_K^(0)
and complex forms, and the CPU oracle baseline on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def pass_bytes(n: int, w: int, nstates: int, parity, ortho: bool, axes=None):
    """Algorithmic bytes of each kernel of one step (all states): what each kernel
    must read and write once.  States are kept as psi_i = sum_(j<=i) c_ji u_j, so
    the two plane passes read i+1 arrays for state i when Gram-Schmidt is on.  When
    all projected states reflect the same axes, the projection shares one pass with
    the Gram sums (k_project_gram); otherwise k_project projects each state alone."""
    sites = n ** 3
    s = 2.0 * w * (n // 2 + 1) / n        # half-spectrum bytes per lattice site
    k = nstates
    reads = sum((i + 1) if ortho else 1 for i in range(k))
    proj = [i for i in range(k) if parity and parity[i]]
    ax = [(axes[i] if axes else 7) for i in proj]
    uniform = len(set(ax)) <= 1
    gram_pass = (ortho and k > 1) or bool(proj)
    return {
        "k_plane_fwd": sites * (reads * w + k * s),
        "k_columns": sites * k * 2 * s,
        "k_plane_inv": sites * (k * s + reads * w + k * w + k * w),
        "k_project": 0.0 if uniform else sites * 2 * w * len(proj),
        "k_project_gram": sites * (k * w + (len(proj) * w if uniform else 0)) if gram_pass else 0.0,
        "k_finalize": 0.0,
    }


def model_step_bytes(n: int, w: int, nstates: int, lazy: bool) -> float:
    """Bytes of one step of all states in the three-pass model: per state and site
    8 w (1 + 1/N) (P1 reads psi and writes the half spectrum, P2 reads and writes
    it, P3 reads it, psi and V and writes psi'; the half spectrum holds
    2 w (1/2 + 1/N) bytes per site), plus 2 w i for state i when the states are
    lazy combinations of the raw arrays (P1 and P3 read i more arrays).  A separate
    projection or Gram pass, and the finalisation, are not in the model: they are
    reported as overhead time."""
    per_state = 8.0 * w * (1.0 + 1.0 / n)
    extra = sum(2.0 * w * i for i in range(nstates)) if lazy else 0.0
    return float(n) ** 3 * (nstates * per_state + extra)


OVERHEAD_PASSES = ("k_project", "k_project_gram", "k_finalize")


def measured_traffic(kernel: str, variant: int):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, scaled by a plain
    copy) from the committed counter summary of the 256^3 FP32 three-state step, if
    it holds a record for this schedule variant taken from the current kernel
    sources."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        lines = open(os.path.join(root, "profiles", "step_256_fp32_k3.md")).read().splitlines()
    except OSError:
        return None
    rec = None
    for ln in lines:
        if ln.startswith("traffic-json: "):
            rec = json.loads(ln[len("traffic-json: "):])
    per_variant = (rec or {}).get("bytes")
    got = per_variant.get(str(variant), {}).get(kernel) if isinstance(per_variant, dict) else None
    if got is None:
        return None
    h = hashlib.sha256()
    for name in ("itse_pass.h", "itse_fft.h", "itse_launch.h", "itse_internal.h"):
        with open(os.path.join(root, "paper_2006_16935_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return got if h.hexdigest() == rec["sources_sha256"] else None


def build_workload(n: int, fp32: bool):
    import synth
    p = synth.config_precision(n)
    dt = np.float32 if fp32 else np.float64
    v = p.potential_array(np.float64).astype(np.float32).astype(dt)  # FP32-stored potential
    states = [s.astype(dt) for s in p.initial_states()]
    return p, v, states


def make_lattice(itse, p, v, states, fp32: bool):
    lat = itse.Lattice(p.n, p.a, p.mass, p.dtau, kin=p.kin, subtract_rest_mass=p.subtract_rest_mass,
                       precision="fp32" if fp32 else "fp64", center=p.center, nstates=p.nstates)
    lat.set_potential(v)
    for i, s in enumerate(states):
        lat.set_state(i, s)
    lat.set_options(ortho_every=p.ortho_every, moments=False, parity=list(p.parity))
    return lat


def make_fdtd_lattice(itse, p, v, states, nstates=None):
    """The workload with H_K^(0) (finite differences, Dirichlet walls) and the
    dtau = a^2 M / 8 its stability bound allows; nstates=1 gives the bare step."""
    import dataclasses
    pf = dataclasses.replace(p, kin=0, dtau=p.a * p.a * p.mass / 8)
    if nstates == 1:
        pf = dataclasses.replace(pf, nstates=1, parity=(0,))
        states = states[:1]
    return make_lattice(itse, pf, v, states, fp32=True)


def make_complex_lattice(itse, p, v, states):
    """One complex state at the workload's size: Re V the workload's potential,
    Im V = 0.5 r^2 (the paper's complex-oscillator shape), psi = states[0] + i
    states[1], parity of state 0."""
    import synth
    lat = itse.Lattice(p.n, p.a, p.mass, p.dtau, kin=p.kin, subtract_rest_mass=p.subtract_rest_mass,
                       precision="fp32", center=p.center, complex_psi=True)
    vi = synth.potential_harmonic_complex(p.n, p.a, p.center, 0.5, 1.0).imag.astype(np.float32)
    lat.set_potential(v.astype(np.float32) + 1j * vi)
    lat.set_state(0, states[0] + 1j * states[1])
    lat.set_options(moments=False, parity=(p.parity[0],))
    return lat


def timed_steps(torch, lat, steps: int, warmup: int):
    lat.step(warmup)
    lat.sync()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    stream = lat.stream
    start.record(stream)
    lat.step(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    lat.sync()
    return start.elapsed_time(stop) / 1000.0


def cpu_baseline(p, v, states, target_s: float = 14.0, max_steps: int = 50):
    """The FP64 oracle on the same 256^3 workload: one untimed step of all states,
    then as many steps as fill about target_s seconds (at most max_steps), timed."""
    import oracle
    L = oracle.lattice(p.n, p.a, p.mass, p.dtau, p.kin, p.subtract_rest_mass, p.center)
    st = [s.astype(np.float64) for s in states]
    v64 = v.astype(np.float64)
    t0 = time.perf_counter()
    oracle.step(L, st, v64, 1, parity=list(p.parity), record=False)
    steps = max(1, min(max_steps, int(round(target_s / (time.perf_counter() - t0)))))
    t0 = time.perf_counter()
    oracle.step(L, st, v64, steps, parity=list(p.parity), record=False)
    dt = time.perf_counter() - t0
    sites = p.n ** 3 * p.nstates
    return {"value": sites * steps / dt, "unit": "site-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} steps of all {p.nstates} states of the {p.n}^3 workload in FP64 "
                      f"({dt:.1f} s, after one untimed step)"}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_scaling():
    """The FP64 oracle at the smaller configuration sizes, on one thread and on all
    threads: the plain 32^3 oscillator (one state, 20 steps) and the 128^3
    relativistic Cornell solve (three states with Gram-Schmidt, 1 step); the 256^3
    figure is the cpu_baseline (all threads only: one thread would take minutes)."""
    import oracle
    import synth
    out = {"cpu_model": _cpu_model(), "nproc": os.cpu_count(), "runs": []}
    all_threads = oracle.num_threads()
    cases = [(synth.config_plain_fp64(), 20), (synth.config_relativistic_fp64(128), 1)]
    for prob, steps in cases:
        L = oracle.lattice(prob.n, prob.a, prob.mass, prob.dtau, prob.kin, prob.subtract_rest_mass, prob.center)
        v = prob.potential_array(np.float64)
        st = [s.astype(np.float64) for s in prob.initial_states()]
        for threads in (1, all_threads):
            oracle.set_num_threads(threads)
            t0 = time.perf_counter()
            oracle.step(L, st, v, steps, parity=list(prob.parity) if prob.parity else None,
                        ortho_every=prob.ortho_every, record=False)
            dt = time.perf_counter() - t0
            out["runs"].append({"n": prob.n, "states": prob.nstates, "steps": steps, "threads": threads,
                                "site_steps_per_s": prob.n ** 3 * prob.nstates * steps / dt})
    oracle.set_num_threads(all_threads)
    return out


def batch_leg(torch, itse, steps: int, warmup: int, count: int = 64):
    """The batched form: `count` independent solves (N in {32, 48, 64, 96}, masses,
    Cornell couplings and kinetic terms drawn by synth.batch_problems), two states
    each, FP32 with FP64 sums, stepped together; aggregate site-steps/s."""
    import synth
    probs = synth.batch_problems(count=count, seed=0, nstates=2)
    # schedules per size picked by the library's autotuner before the lattices are
    # created (a lattice takes the schedule current at its creation): each size timed
    # as a batch of as many lattices as the mix holds of it
    sizes = {}
    for p in probs:
        sizes[p.n] = sizes.get(p.n, 0) + 1
    tuned = {n: json.loads(itse.autotune_batch(n, "fp32", c, 2)) for n, c in sorted(sizes.items())}
    lats = []
    for p in probs:
        lat = itse.Lattice(p.n, p.a, p.mass, p.dtau, kin=p.kin, subtract_rest_mass=p.subtract_rest_mass,
                           precision="fp32", center=p.center, nstates=p.nstates)
        lat.set_potential(p.potential_array(np.float64).astype(np.float32))
        for i, st in enumerate(p.initial_states(np.float32)):
            lat.set_state(i, st)
        lat.set_options(ortho_every=1)
        lats.append(lat)
    b = itse.Batch(lats)
    b.step(warmup)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(b.stream)
    b.step(steps)
    stop.record(b.stream)
    torch.cuda.synchronize()
    secs = start.elapsed_time(stop) / 1000.0
    for lat in lats:
        lat.sync()
    sites = sum(p.n ** 3 * p.nstates for p in probs)
    b.close()
    for lat in lats:
        lat.close()
    # the three-pass model's bytes of every lattice's step (Gram-Schmidt every step,
    # so the states are lazy combinations) against 8 TB/s
    model_bytes = sum(model_step_bytes(p.n, 4, p.nstates, True) for p in probs)
    return {"site_steps_per_s": sites * steps / secs, "ms_per_step": secs * 1000.0 / steps,
            "lattices": count, "sizes": sizes, "steps": steps, "site_steps_per_step": sites,
            "step_bytes": model_bytes, "step_hbm_frac": model_bytes / (secs / steps) / 1e9 / HBM_PEAK_GBS,
            "schedules": {n: t["best"] for n, t in tuned.items()}}


def serving_run(torch, itse, count: int, qps: float, budget: int, seed: int = 1, burst: bool = False):
    """The serving form: `count` requests arriving as a Poisson stream at `qps`
    (synth.serving_requests: N in {64, 128, 192, 256}, two states, relative tolerance
    1e-8; burst: all arrive at time 0, for the saturated capacity), admitted by
    footprint against `budget` bytes; latency = arrival to result.  The requests'
    input arrays are generated before the clock starts."""
    import time as _time
    import synth
    reqs = synth.serving_requests(count, qps, seed=seed)
    if burst:
        reqs = [(0.0, p) for _, p in reqs]
    inputs = [(t, p, p.potential_array(np.float64).astype(np.float32), p.initial_states(np.float32))
              for t, p in reqs]
    server = itse.Server(hbm_budget=budget, max_slots=64, chunk=100)
    t0 = _time.perf_counter()
    nxt = 0
    arrival, done, ids = {}, {}, {}
    site_steps = 0
    while len(done) < count:
        now = _time.perf_counter() - t0
        while nxt < count and inputs[nxt][0] <= now:
            t_arr, p, v, st = inputs[nxt]
            rid = server.submit(p.n, p.a, p.mass, p.dtau, v, st, kin=p.kin,
                                subtract_rest_mass=p.subtract_rest_mass, precision="fp32", center=p.center,
                                ortho_every=1, tol=p.tol, relative=True, max_steps=60000)
            arrival[rid] = t_arr
            ids[rid] = p
            nxt += 1
        live, queued = server.progress()
        for r in server.poll():
            done[r["id"]] = (_time.perf_counter() - t0, r)
            site_steps += ids[r["id"]].n ** 3 * ids[r["id"]].nstates * r["steps"]
            print(f"serving: {len(done)}/{count} done at {done[r['id']][0]:.1f} s, live {live}, queued {queued}",
                  file=sys.stderr, flush=True)
        if live == 0 and queued == 0 and nxt < count:
            _time.sleep(max(0.0, inputs[nxt][0] - (_time.perf_counter() - t0)))
    wall = _time.perf_counter() - t0
    server.close()
    lat = np.array([done[i][0] - arrival[i] for i in done])
    conv = sum(1 for i in done if done[i][1]["converged"])
    return {"requests": count, "qps": None if burst else qps, "burst": burst, "budget_bytes": budget,
            "p50_latency_s": float(np.percentile(lat, 50)), "p90_latency_s": float(np.percentile(lat, 90)),
            # linear interpolation between order statistics; with fewer than 100 requests it
            # falls between the largest two
            "p99_latency_s": float(np.percentile(lat, 99)), "max_latency_s": float(lat.max()),
            "mean_latency_s": float(lat.mean()), "site_steps_per_s": site_steps / wall, "wall_s": wall,
            "completions_per_s": count / wall, "converged": conv,
            "steps_mean": float(np.mean([done[i][1]["steps"] for i in done]))}


def _solve(itse, p, v, states, precision, tol, relative, max_steps, parity):
    """Run one solve to |dE| <= tol per 100 steps; returns (energies, steps, seconds, lattice)."""
    from paper_2006_16935_amd.solver import run_to_convergence
    lat = itse.Lattice(p.n, p.a, p.mass, p.dtau, kin=p.kin, subtract_rest_mass=p.subtract_rest_mass,
                       precision=precision, center=p.center, nstates=len(states))
    lat.set_potential(v)
    for i, st in enumerate(states):
        lat.set_state(i, st)
    lat.set_options(ortho_every=1, parity=list(parity) if parity else None)
    res = run_to_convergence(lat, tol, relative=relative, check_every=100, max_steps=max_steps)
    return res, lat


def _fixed_solve(itse, p, v, states, precision, steps, parity, chunk=5000):
    """Run exactly `steps` steps (progress on stderr every `chunk`); returns a result
    with the energies, the energy change over the last chunk per state, and the
    lattice."""
    import types
    lat = itse.Lattice(p.n, p.a, p.mass, p.dtau, kin=p.kin, subtract_rest_mass=p.subtract_rest_mass,
                       precision=precision, center=p.center, nstates=len(states))
    lat.set_potential(v)
    for i, st in enumerate(states):
        lat.set_state(i, st)
    lat.set_options(ortho_every=1, parity=list(parity) if parity else None)
    t0 = time.perf_counter()
    prev = None
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        lat.step(k)
        done += k
        cur = [o["energy"] for o in lat.observe_all()]
        if done < steps:
            prev = cur
        print(f"study {precision}: {done}/{steps} steps, E = {cur}", file=sys.stderr, flush=True)
    res = types.SimpleNamespace(energies=cur, steps=done, converged=True, wall_s=time.perf_counter() - t0,
                                last_change=[abs(a - b) for a, b in zip(cur, prev)] if prev else None)
    return res, lat


def study(torch, itse, which: str, max_steps: int, fixed_steps: int = 0):
    """Converged eigenpairs against the oracle.

    precision: the 256^3 precision-form solve (3 states, parity +,-,-) in FP32 (with
    FP64 sums) and in FP64 on the GPU, from the same FP32-rounded inputs; the oracle
    certifies each GPU state (residual of its step map) and evaluates its energy in
    FP64; errors are reported per eigenvalue for the FP32 energies, the FP64
    re-evaluation of the FP32 states (polish) and the FP64 energies.
    relativistic: the 128^3 FP64 relativistic Cornell solve with three states to
    |dE| < 1e-10 (the first excited level is a degenerate triplet of the cubic
    lattice, so E1 = E2); the oracle certifies the states."""
    import oracle
    import synth
    out = {"study": which}
    if which == "precision":
        p = synth.config_precision(256)
        v32 = p.potential_array(np.float64).astype(np.float32)
        s32 = [s.astype(np.float32) for s in p.initial_states()]
        if fixed_steps:
            r32, lat32 = _fixed_solve(itse, p, v32, s32, "fp32", fixed_steps, p.parity)
        else:
            r32, lat32 = _solve(itse, p, v32, s32, "fp32", p.tol, True, max_steps, p.parity)
        polish = [lat32.polish(i)["energy"] for i in range(p.nstates)]
        st32 = [lat32.get_state(i) for i in range(p.nstates)]
        lat32.close()
        s64 = [s.astype(np.float64) for s in s32]
        if fixed_steps:
            r64, lat64 = _fixed_solve(itse, p, v32.astype(np.float64), s64, "fp64", fixed_steps, p.parity)
        else:
            r64, lat64 = _solve(itse, p, v32.astype(np.float64), s64, "fp64", 1e-11, True, max_steps, p.parity)
        st64 = [lat64.get_state(i) for i in range(p.nstates)]
        lat64.close()
        L = oracle.lattice(p.n, p.a, p.mass, p.dtau, p.kin, p.subtract_rest_mass, p.center)
        c64 = [oracle.certify(L, st, v32.astype(np.float64)) for st in st64]
        c32 = [oracle.certify(L, st, v32.astype(np.float64)) for st in st32]
        ref = [c["energy"] for c in c64]
        out.update({
            "n": 256, "steps_fp32": r32.steps, "converged_fp32": r32.converged, "seconds_fp32": r32.wall_s,
            "steps_fp64": r64.steps, "converged_fp64": r64.converged, "seconds_fp64": r64.wall_s,
            "E_fp32": r32.energies, "E_polish": polish, "E_fp64": r64.energies, "E_oracle": ref,
            "resid_fp64_states": [c["resid"] for c in c64], "resid_fp32_states": [c["resid"] for c in c32],
            "E_oracle_of_fp32_states": [c["energy"] for c in c32],
            "relerr_fp32": [abs(a - b) / abs(b) for a, b in zip(r32.energies, ref)],
            "relerr_polish": [abs(a - b) / abs(b) for a, b in zip(polish, ref)],
            "relerr_fp64": [abs(a - b) / abs(b) for a, b in zip(r64.energies, ref)],
        })
        if fixed_steps:
            out["fixed_steps"] = fixed_steps
            out["last_chunk_change_fp32"] = r32.last_change
            out["last_chunk_change_fp64"] = r64.last_change
    else:
        p = synth.config_relativistic_fp64(128)
        v = p.potential_array(np.float64)
        r, lat = _solve(itse, p, v, p.initial_states(), "fp64", 1e-10, False, max_steps, None)
        st = [lat.get_state(i) for i in range(p.nstates)]
        lat.evaluate(moments=True)
        par = [lat.observe(i)["parity_even"] for i in range(p.nstates)]
        lat.close()
        L = oracle.lattice(p.n, p.a, p.mass, p.dtau, p.kin, p.subtract_rest_mass, p.center)
        cert = [oracle.certify(L, s_, v) for s_ in st]
        out.update({"n": 128, "steps": r.steps, "converged": r.converged, "seconds": r.wall_s,
                    "site_steps_per_s": p.n ** 3 * p.nstates * r.steps / r.wall_s,
                    "E": r.energies, "E_oracle": [c["energy"] for c in cert],
                    "resid": [c["resid"] for c in cert], "parity_even_weight": par,
                    "E1_minus_E2": r.energies[1] - r.energies[2]})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--schedule", type=int, default=-1,
                    help="schedule variant for the 256^3 FP32 lattice (default: autotune)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-lattice batched leg")
    ap.add_argument("--study", choices=["precision", "relativistic"], default=None,
                    help="only run a converged-solve study against the oracle and print its JSON line")
    ap.add_argument("--max-steps", type=int, default=60000)
    ap.add_argument("--fixed-steps", type=int, default=0,
                    help="with --study precision: run exactly this many steps in each precision "
                         "instead of stopping on |dE|")
    ap.add_argument("--serving", action="store_true",
                    help="only run the serving form (Poisson arrivals) and print its JSON line")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--qps", type=float, default=0.5)
    ap.add_argument("--burst", action="store_true",
                    help="with --serving: every request arrives at time 0 (the saturated capacity)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg of the default run")
    ap.add_argument("--serving-requests", type=int, default=40)
    ap.add_argument("--serving-qps", type=float, default=0.5)
    ap.add_argument("--budget-gb", type=float, default=288.0)
    ap.add_argument("--kernels-only", action="store_true",
                    help="only step the 256^3 FP32 workload a few times and profile its passes (for rocprofv3)")
    ap.add_argument("--form", choices=["precision", "fdtd", "complex", "batch", "fp64"], default="precision",
                    help="with --kernels-only: the workload (precision), its H_K^(0) form, one complex state, "
                         "the 64-lattice batch, or the workload in FP64 (schedule default 1)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 256 MiB five times (scale for HBM counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": x.numel() * 4, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the step runs on one GPU (each lattice lives whole on one GPU; "
                                   "no sharding across GPUs is implemented): --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_2006_16935_amd as itse

    torch.cuda.set_device(0)
    if args.study:
        print(json.dumps(study(torch, itse, args.study, args.max_steps, args.fixed_steps)), flush=True)
        return
    if args.serving:
        res = serving_run(torch, itse, args.requests, args.qps, int(args.budget_gb * (1 << 30)), burst=args.burst)
        print(json.dumps({"metric": "p50/p99 solve latency, serving form", **res}), flush=True)
        return
    n = args.n
    if args.kernels_only:
        # the timed workload's passes alone, for profilers: a few graph steps, then
        # eager launches of each pass (schedule from --schedule, default 2)
        itse.set_schedule(n, "fp32", args.schedule if args.schedule >= 0 else 2)
        if args.form == "batch":
            print(json.dumps({"batch64": batch_leg(torch, itse, 10, 2)}), flush=True)
            return
        if args.form == "fp64":
            itse.set_schedule(n, "fp64", args.schedule if args.schedule >= 0 else 1)
            p, v64, st64 = build_workload(n, fp32=False)
            lat = make_lattice(itse, p, v64, st64, fp32=False)
            lat.step(2)
            prof = lat.profile_step(args.profile_steps)
            lat.close()
            print(json.dumps({"passes_ms": prof}), flush=True)
            return
        p, v32, st32 = build_workload(n, fp32=True)
        if args.form == "fdtd":
            lat = make_fdtd_lattice(itse, p, v32, st32)
        elif args.form == "complex":
            lat = make_complex_lattice(itse, p, v32, st32)
        else:
            lat = make_lattice(itse, p, v32, st32, fp32=True)
        lat.step(2)
        prof = lat.profile_step(args.profile_steps)
        lat.close()
        print(json.dumps({"passes_ms": prof}), flush=True)
        return
    # schedule per (n, precision) picked by the library's autotuner (timed outside the
    # measured region; results are deterministic for a given schedule)
    if args.schedule >= 0:
        itse.set_schedule(n, "fp32", args.schedule)
        tune32 = None
    else:
        tune32 = json.loads(itse.autotune(n, "fp32"))
    tune64 = None if args.no_fp64 else json.loads(itse.autotune(n, "fp64"))
    p, v32, st32 = build_workload(n, fp32=True)
    lat = make_lattice(itse, p, v32, st32, fp32=True)
    secs = timed_steps(torch, lat, args.steps, args.warmup)
    sites = n ** 3 * p.nstates
    value = sites * args.steps / secs
    ms_per_step = secs * 1000.0 / args.steps

    # per-pass durations (HIP events between eager launches on the lattice stream)
    prof = lat.profile_step(args.profile_steps)
    pb = pass_bytes(n, 4, p.nstates, p.parity, p.ortho_every == 1)
    dom = max(prof, key=lambda k: prof[k])
    dom_ms = prof[dom]
    achieved = pb[dom] / (dom_ms * 1e-3) / 1e9
    step_bytes = model_step_bytes(n, 4, p.nstates, p.ortho_every == 1)
    e_fp32 = [lat.observe(i)["energy"] for i in range(p.nstates)]
    lat.close()

    extra = {}
    # the same lattice with one state and no projection or Gram-Schmidt: the bare
    # three-pass step (32 + 32/N bytes per site in FP32)
    import dataclasses
    p1 = dataclasses.replace(p, nstates=1, parity=(0,))
    lat1 = make_lattice(itse, p1, v32, st32[:1], fp32=True)
    steps1 = max(20, args.steps // 2)
    secs1 = timed_steps(torch, lat1, steps1, args.warmup)
    prof1 = lat1.profile_step(args.profile_steps)
    pb1 = pass_bytes(n, 4, 1, None, False)
    extra["k1_site_steps_per_s"] = n ** 3 * steps1 / secs1
    extra["k1_ms_per_step"] = secs1 * 1000.0 / steps1
    extra["k1_hbm_frac"] = model_step_bytes(n, 4, 1, False) / (secs1 / steps1) / 1e9 / HBM_PEAK_GBS
    extra["k1_passes_ms"] = prof1
    # snapshot-overlap extraction on the one-state lattice: keeping a snapshot,
    # and forming the three estimates with their energies (second call timed; the
    # first one creates the analysis lattice)
    lat1.snapshot()
    lat1.step(16)
    lat1.snapshot()
    lat1.step(16)
    lat1.extract()
    lat1.sync()
    t0 = time.perf_counter()
    for _ in range(10):
        lat1.snapshot()
    lat1.sync()
    push_ms = (time.perf_counter() - t0) * 100.0
    lat1.step(16)
    lat1.snapshot()
    lat1.step(16)
    lat1.sync()
    t0 = time.perf_counter()
    snap_obs = lat1.extract()
    extract_ms = (time.perf_counter() - t0) * 1000.0
    extra["snapshot_overlap"] = {"push_ms": push_ms, "extract_ms": extract_ms,
                                 "estimates": len(snap_obs)}
    # analysis of the state: box observables and parity weights, radial momentum space
    lat1.analyse(0, 0.3)
    t0 = time.perf_counter()
    ana = lat1.analyse(0, 0.3)
    analyse_ms = (time.perf_counter() - t0) * 1000.0
    lat1.momentum_radial(0, 128)
    t0 = time.perf_counter()
    lat1.momentum_radial(0, 128)
    momentum_ms = (time.perf_counter() - t0) * 1000.0
    extra["analysis"] = {"analyse_ms": analyse_ms, "momentum_radial_ms": momentum_ms,
                         "rho_box": ana["rho_box"], "w_plus": ana["w_plus"]}
    lat1.close()
    if not args.no_fp64:
        p64, v64, st64 = build_workload(n, fp32=False)
        lat64 = make_lattice(itse, p64, v64, st64, fp32=False)
        steps64 = max(10, args.steps // 4)
        secs64 = timed_steps(torch, lat64, steps64, max(2, args.warmup // 2))
        extra["fp64_site_steps_per_s"] = sites * steps64 / secs64
        extra["fp64_ms_per_step"] = secs64 * 1000.0 / steps64
        pb64 = model_step_bytes(n, 8, p.nstates, p.ortho_every == 1)
        extra["fp64_step_hbm_frac"] = pb64 / secs64 * steps64 / 1e9 / HBM_PEAK_GBS
        extra["fp64_step_hbm_frac_compulsory"] = 24.0 * sites * steps64 / secs64 / 1e9 / HBM_PEAK_GBS
        lat64.close()

    # H_K^(0) (finite differences, Dirichlet walls): the same three-state workload
    # with one fused stencil pass per state instead of the transforms, and the bare
    # one-state step (12 bytes per site in FP32: psi, V, psi')
    latf = make_fdtd_lattice(itse, p, v32, st32)
    secsf = timed_steps(torch, latf, args.steps, args.warmup)
    proff = latf.profile_step(args.profile_steps)
    latf.close()
    latf1 = make_fdtd_lattice(itse, p, v32, st32, nstates=1)
    secsf1 = timed_steps(torch, latf1, args.steps, args.warmup)
    proff1 = latf1.profile_step(args.profile_steps)
    latf1.close()
    fd_bytes = float(n ** 3) * 4 * sum(i + 1 + 2 for i in range(p.nstates))
    extra["fdtd"] = {
        "site_steps_per_s": sites * args.steps / secsf,
        "ms_per_step": secsf * 1000.0 / args.steps,
        "passes_ms": proff,
        "k_fdtd_gbs": fd_bytes / (proff["k_fdtd"] * 1e-3) / 1e9,
        "k_fdtd_frac": fd_bytes / (proff["k_fdtd"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "k1_site_steps_per_s": n ** 3 * args.steps / secsf1,
        "k1_ms_per_step": secsf1 * 1000.0 / args.steps,
        "k1_passes_ms": proff1,
        "k1_hbm_frac": 12.0 * n ** 3 / (secsf1 / args.steps) / 1e9 / HBM_PEAK_GBS,
    }

    # one complex state in a complex potential (Re V the workload's potential, Im V
    # = 0.5 r^2, the paper's complex-oscillator shape): both parts forward, the real
    # part's inverse pass writing K Re psi, then the imaginary part's inverse pass
    # applying the complex update to both parts.  The two inverse passes move 48
    # bytes per site in FP32: spectra 8, Re psi twice 8, Im psi 4, Re V twice 8,
    # Im V 4, K Re psi written and read 8, both new parts 8
    latc = make_complex_lattice(itse, p, v32, st32)
    secsc = timed_steps(torch, latc, args.steps, args.warmup)
    profc = latc.profile_step(args.profile_steps)
    latc.close()
    inv_bytes = (48.0 + 16.0 / n) * n ** 3
    extra["complex"] = {
        "site_steps_per_s": n ** 3 * args.steps / secsc,
        "ms_per_step": secsc * 1000.0 / args.steps,
        "passes_ms": profc,
        "inverse_passes_gbs": inv_bytes / (profc["k_plane_inv"] * 1e-3) / 1e9,
        "inverse_passes_frac": inv_bytes / (profc["k_plane_inv"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
    }

    out = {
        "metric": "site-steps/s at 256^3 (FP32 steps with FP64 reductions)",
        "value": value,
        "unit": "site-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"precision form: {n}^3, 3 states (parity +,-,- with Gram-Schmidt), "
                               f"FP32 states/FFT, FP64 reductions, sqrt(p^2+m^2)-m, Cornell+aniso FP32 V",
                   "n": n, "nstates": p.nstates, "site_steps_per_step": sites,
                   "schedule": json.loads(itse.schedule(n, "fp32")), "autotune_fp32": tune32,
                   "autotune_fp64": tune64},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom, json.loads(itse.schedule(n, "fp32"))["variant"]),
                     "kernel": dom,
                     "kernel_ms": dom_ms, "kernel_bytes": pb[dom]},
        "passes_ms": prof,
        "passes_bytes": pb,
        # the whole step against the three-pass byte model (per state 32 + 32/N bytes
        # per site in FP32, plus 8 i for state i kept as a lazy combination); passes
        # the model does not count are overhead time
        "step_bytes": step_bytes,
        "step_hbm_frac": step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "step_overhead_ms": {k: prof[k] for k in OVERHEAD_PASSES if k in prof},
        # against the compulsory floor of 12 bytes per site and state (psi in, V in,
        # psi' out), which the transforms cannot reach when a plane does not fit on chip
        "step_hbm_frac_compulsory": 12.0 * value / 1e9 / HBM_PEAK_GBS,
        "energies_fp32": e_fp32,
    }
    if not args.no_batch:
        extra["batch64"] = batch_leg(torch, itse, max(20, args.steps // 2), 5)
    if not args.no_serving:
        # the serving form at a fixed arrival rate, bounded to about a minute and a half
        extra["serving"] = serving_run(torch, itse, args.serving_requests, args.serving_qps, 288 << 30)
    out.update(extra)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, v32.astype(np.float64), [s.astype(np.float64) for s in st32])
        out["oracle_scaling"] = oracle_scaling()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
