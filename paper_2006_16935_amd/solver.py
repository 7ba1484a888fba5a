"""Convergence driver: step in chunks, read the energies, stop on |dE| <= tol.

The paper checks E_b(i) - E_b(i-1) < TOLERANCE every SNAPUPDATE steps (section
"Basic configuration"); the signed difference is immediately below any positive
tolerance while E decreases, so the absolute change is used here.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional, Sequence

from .lattice import Lattice


@dataclasses.dataclass
class SolveResult:
    energies: List[float]
    steps: int
    converged: bool
    trace: List[List[float]]          # energies per state at each check
    wall_s: float


def converged(prev: Sequence[float], cur: Sequence[float], tol: float, relative: bool) -> bool:
    for a, b in zip(prev, cur):
        scale = abs(b) if relative else 1.0
        if abs(b - a) > tol * scale:
            return False
    return True


def run_to_convergence(lat: Lattice, tol: float, relative: bool = False, check_every: int = 100,
                       max_steps: int = 200000) -> SolveResult:
    t0 = time.perf_counter()
    prev = None
    trace = []
    taken = 0
    ok = False
    while taken < max_steps:
        lat.step(check_every)
        taken += check_every
        # complex lattices: the complex energy (its change in modulus)
        cur = [complex(o["energy"], o["energy_imag"]) if lat.complex_psi else o["energy"]
               for o in lat.observe_all()]
        trace.append(cur)
        if prev is not None and converged(prev, cur, tol, relative):
            ok = True
            break
        prev = cur
    return SolveResult(energies=trace[-1] if trace else [], steps=taken, converged=ok, trace=trace,
                       wall_s=time.perf_counter() - t0)


@dataclasses.dataclass
class SnapshotResult:
    energies: List[float]             # ground state, then the excited-state estimates
    steps: int
    converged: bool
    trace: List[List[float]]          # estimate energies at each snapshot
    observables: List[dict]
    wall_s: float


def run_snapshot_overlap(lat: Lattice, snap_every: int, tol: float, relative: bool = False,
                         max_steps: int = 200000) -> SnapshotResult:
    """The paper's single-state run with snapshot-overlap extraction (section "The
    iterative procedure"; flag SNAPUPDATE of section "Basic configuration"): state 0
    evolves, a snapshot is kept every `snap_every` steps, and the run stops when the
    ground-state energy moved by at most `tol` since the previous snapshot.  The
    estimates come from the latest wave-function and the two latest snapshots."""
    t0 = time.perf_counter()
    lat.clear_snapshots()
    trace, prev, taken, ok = [], None, 0, False
    obs: List[dict] = []
    while taken < max_steps:
        lat.step(snap_every)
        taken += snap_every
        obs = lat.extract()
        cur = obs[0]["energy"]
        trace.append([o["energy"] for o in obs])
        lat.snapshot()
        if prev is not None and abs(cur - prev) <= tol * (abs(cur) if relative else 1.0):
            ok = True
            break
        prev = cur
    return SnapshotResult(energies=trace[-1] if trace else [], steps=taken, converged=ok, trace=trace,
                          observables=obs, wall_s=time.perf_counter() - t0)


def solve(n, a, mass, dtau, kin, potential, states, precision="fp64", center="origin",
          subtract_rest_mass=True, parity: Optional[Sequence[int]] = None, ortho_every: int = 1,
          tol: float = 1e-10, relative: bool = False, check_every: int = 100,
          max_steps: int = 200000, stream=None) -> SolveResult:
    lat = Lattice(n, a, mass, dtau, kin=kin, subtract_rest_mass=subtract_rest_mass,
                  precision=precision, center=center, nstates=len(states), stream=stream)
    try:
        lat.set_potential(potential)
        for i, s in enumerate(states):
            lat.set_state(i, s)
        lat.set_options(ortho_every=ortho_every, parity=parity)
        return run_to_convergence(lat, tol, relative, check_every, max_steps)
    finally:
        lat.close()
