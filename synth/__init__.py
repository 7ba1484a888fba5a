"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the eigensolver itself: it only draws random
initial wave-functions, evaluates potential formulas on lattice coordinates and
describes the benchmark workloads.  Both the FP64 oracle (``oracle/``) and the
HIP path receive the arrays produced here through their own entry points.

Conventions (paper, section "Overview and structure of the paper" and the
hard-coded potential list):

* the lattice is N^3, index order ``[x1][x2][x3]`` (C order, x3 fastest);
* ``center="cell"`` puts the potential centre at the off-grid point
  ``((N-1)/2, (N-1)/2, (N-1)/2)`` (0-based; the paper's 1-based
  ``N_H = (N+1)/2``); ``center="origin"`` puts it at site 0 with minimum-image
  distances (the paper's "add 100 to the potential code" option).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

CELL = "cell"
ORIGIN = "origin"

# Kinetic-term identifiers shared by name with both implementations.
KIN_NR_CONT = 1   # H_K^(1)
KIN_NR_LAT = 2    # H_K^(2)
KIN_REL_LAT = 3   # H_K^(3)
KIN_REL_CONT = 4  # relativistic analogue of H_K^(1)


def random_state(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """i.i.d. uniform[-1, 1] wave-function drawn from PCG64 ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(n, n, n)).astype(dtype, copy=False)


def random_states(n: int, k: int, seed: int = 0, dtype=np.float64) -> List[np.ndarray]:
    """State i is drawn from ``default_rng(seed + i)``."""
    return [random_state(n, seed + i, dtype) for i in range(k)]


def axis_coords(n: int, a: float, center: str) -> np.ndarray:
    """Signed physical coordinate of each index along one axis."""
    idx = np.arange(n, dtype=np.float64)
    if center == CELL:
        return (idx - (n - 1) / 2.0) * a
    if center == ORIGIN:
        return np.where(2 * idx <= n, idx, idx - n) * a
    raise ValueError(f"unknown centring {center!r}")


def radius_grid(n: int, a: float, center: str):
    c = axis_coords(n, a, center)
    x = c[:, None, None]
    y = c[None, :, None]
    z = c[None, None, :]
    r = np.sqrt(x * x + y * y + z * z)
    return x, y, z, r


def potential_harmonic(n: int, a: float, center: str = CELL, coef: float = 0.5) -> np.ndarray:
    """V = coef * r^2 (coef = 1/2 is the standard oscillator with m = omega = 1;
    coef = 1 is the oscillator without the 1/2 used for the relativistic example)."""
    _, _, _, r = radius_grid(n, a, center)
    return coef * r * r


def potential_harmonic_complex(n: int, a: float, center: str = CELL, coef: float = 0.5,
                               imag: float = 1.0) -> np.ndarray:
    """V = coef * (1 + i imag) r^2: with imag = 1 the paper's complex 3d harmonic
    oscillator shape (hard-coded potential 5) with a positive real part."""
    _, _, _, r = radius_grid(n, a, center)
    return coef * (1.0 + 1j * imag) * r * r


def random_state_complex(n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Real part from ``default_rng(seed)``, imaginary part from ``default_rng(seed + 1)``."""
    return (random_state(n, seed) + 1j * random_state(n, seed + 1)).astype(dtype, copy=False)


def potential_cornell(n: int, a: float, center: str = ORIGIN, sigma: float = 0.2,
                      alpha: float = 0.4, reg: Optional[float] = None,
                      aniso: float = 0.0) -> np.ndarray:
    """V = -alpha / r_eff + sigma * r_eff + aniso * (x^2 - y^2) / r_eff,
    with r_eff = max(r, reg) and reg = a/2 unless given."""
    x, y, _, r = radius_grid(n, a, center)
    reg = a / 2.0 if reg is None else reg
    r_eff = np.maximum(r, reg)
    v = -alpha / r_eff + sigma * r_eff
    if aniso != 0.0:
        v = v + aniso * (x * x - y * y) / r_eff
    return v


def potential_coulomb_clamped(n: int, a: float, center: str = CELL) -> np.ndarray:
    """The paper's hard-coded radial Coulomb potential: -1/(A rho) for rho > 1,
    -1/A for rho <= 1 (rho in lattice units)."""
    _, _, _, r = radius_grid(n, a, center)
    rho = r / a
    return np.where(rho > 1.0, -1.0 / (a * np.maximum(rho, 1.0)), -1.0 / a)


# --------------------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    """One eigensolve: lattice, kinetic term, potential recipe, step size, states."""
    n: int
    a: float
    mass: float
    kin: int
    dtau: float
    center: str
    nstates: int
    potential: str                 # "harmonic", "cornell", "cornell_aniso", "zero"
    pot_args: dict = dataclasses.field(default_factory=dict)
    subtract_rest_mass: bool = True
    seed: int = 0
    fp32: bool = False
    parity: Sequence[int] = ()     # per-state reflection sign (0 = none)
    ortho_every: int = 1
    tol: float = 1e-10
    tol_relative: bool = False
    check_every: int = 100

    def potential_array(self, dtype=np.float64) -> np.ndarray:
        if self.potential == "harmonic":
            v = potential_harmonic(self.n, self.a, self.center, **self.pot_args)
        elif self.potential == "cornell":
            v = potential_cornell(self.n, self.a, self.center, **self.pot_args)
        elif self.potential == "cornell_aniso":
            args = dict(self.pot_args)
            args.setdefault("aniso", 0.05)
            v = potential_cornell(self.n, self.a, self.center, **args)
        elif self.potential == "zero":
            v = np.zeros((self.n,) * 3)
        else:
            raise ValueError(self.potential)
        return v.astype(dtype)

    def initial_states(self, dtype=np.float64) -> List[np.ndarray]:
        return random_states(self.n, self.nstates, self.seed, dtype)

    def sites(self) -> int:
        return self.n ** 3


def config_plain_fp64() -> Problem:
    """32^3, a = 0.1, H_K^(1) with m = 1, V = r^2/2 at the cell centre,
    dtau = a^2/8, one state from seed 0, 2000 steps."""
    a = 0.1
    return Problem(n=32, a=a, mass=1.0, kin=KIN_NR_CONT, dtau=a * a / 8.0, center=CELL,
                   nstates=1, potential="harmonic", pot_args={"coef": 0.5}, seed=0)


def config_relativistic_fp64(n: int = 128) -> Problem:
    """128^3, a = 0.05, sqrt(p^2+m^2)-m with m = 1.3, Cornell -0.4/r + 0.2 r with
    r_eff = max(r, a/2) at the origin, dtau = a/4, ground + two excited states."""
    a = 0.05
    return Problem(n=n, a=a, mass=1.3, kin=KIN_REL_LAT, dtau=a / 4.0, center=ORIGIN,
                   nstates=3, potential="cornell",
                   pot_args={"sigma": 0.2, "alpha": 0.4}, seed=0, tol=1e-10)


def config_precision(n: int = 256) -> Problem:
    """256^3 FP32 steps with FP64 reductions; Cornell + 0.05 (x^2-y^2)/r stored as FP32;
    box 6.4 (a = 0.025); state 0 even, states 1 and 2 odd (2 deflated against 1)."""
    a = 6.4 / n
    return Problem(n=n, a=a, mass=1.3, kin=KIN_REL_LAT, dtau=a / 4.0, center=ORIGIN,
                   nstates=3, potential="cornell_aniso",
                   pot_args={"sigma": 0.2, "alpha": 0.4, "aniso": 0.05},
                   seed=0, fp32=True, parity=(1, -1, -1), tol=1e-8, tol_relative=True)


def batch_problems(count: int = 64, seed: int = 0, sizes=(32, 48, 64, 96),
                   nstates: int = 2) -> List[Problem]:
    """Independent solves with N ~ U{sizes}, m ~ U[1,5], sigma ~ U[0.1,0.3],
    alpha ~ U[0.2,0.5], kinetic term 50/50 relativistic / non-relativistic
    (the non-relativistic half alternates H_K^(1) / H_K^(2)); a = 0.1, origin centring."""
    rng = np.random.default_rng(seed)
    out = []
    nr_toggle = 0
    for j in range(count):
        n = int(rng.choice(sizes))
        m = float(rng.uniform(1.0, 5.0))
        sigma = float(rng.uniform(0.1, 0.3))
        alpha = float(rng.uniform(0.2, 0.5))
        rel = bool(rng.uniform() < 0.5)
        a = 0.1
        if rel:
            kin, dtau = KIN_REL_LAT, a / 4.0
        else:
            kin = KIN_NR_CONT if nr_toggle % 2 == 0 else KIN_NR_LAT
            nr_toggle += 1
            dtau = a * a * m / 8.0
        out.append(Problem(n=n, a=a, mass=m, kin=kin, dtau=dtau, center=ORIGIN,
                           nstates=nstates, potential="cornell",
                           pot_args={"sigma": sigma, "alpha": alpha},
                           seed=1000 + 10 * j, fp32=True, tol=1e-8, tol_relative=True))
    return out


def serving_requests(count: int, qps: float, seed: int = 1,
                     sizes=(64, 128, 192, 256), nstates: int = 2):
    """Poisson arrival stream: returns a list of (arrival_time_s, Problem)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for j in range(count):
        t += float(rng.exponential(1.0 / qps))
        n = int(rng.choice(sizes))
        m = float(rng.uniform(1.0, 5.0))
        sigma = float(rng.uniform(0.1, 0.3))
        alpha = float(rng.uniform(0.2, 0.5))
        rel = bool(rng.uniform() < 0.5)
        a = 0.1
        if rel:
            kin, dtau = KIN_REL_LAT, a / 4.0
        else:
            kin = KIN_NR_CONT if j % 2 == 0 else KIN_NR_LAT
            dtau = a * a * m / 8.0
        reqs.append((t, Problem(n=n, a=a, mass=m, kin=kin, dtau=dtau, center=ORIGIN,
                                nstates=nstates, potential="cornell",
                                pot_args={"sigma": sigma, "alpha": alpha},
                                seed=5000 + 10 * j, fp32=True, tol=1e-8,
                                tol_relative=True)))
    return reqs


__all__ = [name for name in dir() if not name.startswith("_")]
