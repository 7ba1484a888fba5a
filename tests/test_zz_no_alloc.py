"""itse_analyse_noalloc against itse_analyse through the C ABI: the same analysis
(box normalisation, average radius, parity weights) with no device allocation.

Two calls in a row, the second on a smaller lattice, each compared with the
allocating entry point on the same state: both run the same kernels with the same
fixed-order sums, so the results must be identical.  The torch allocator the
lattices draw from must see no allocation during the no-allocation calls."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _lattice(itse, n, prec, center, seed):
    a = 6.4 / n
    lat = itse.Lattice(n, a, 1.3, a / 4, kin=3, precision=prec, center=center, nstates=2)
    dt = np.float32 if prec == "fp32" else np.float64
    x = synth.axis_coords(n, a, center)
    g = np.exp(-(x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2) / 1.5)
    lat.set_state(0, synth.random_state(n, seed, dtype=dt))
    lat.set_state(1, (g * (0.7 + 0.5 * x[None, None, :] + 0.2 * x[:, None, None])).astype(dt))
    return lat


@pytest.mark.parametrize("order", [((128, "fp64", "origin"), (48, "fp32", "cell")),
                                   ((256, "fp32", "origin"), (32, "fp64", "origin"))])
def test_noalloc_analysis_equals_allocating_entry_point(itse, order):
    for call, (n, prec, center) in enumerate(order):
        lat = _lattice(itse, n, prec, center, seed=40 + call)
        for i, m in ((0, 0.3), (1, 0.0), (1, 0.45)):
            live = len(lat._alloc.live)
            got = lat.analyse_noalloc(i, m)
            assert len(lat._alloc.live) == live, "the no-allocation call allocated"
            ref = lat.analyse(i, m)
            for k, r in ref.items():
                assert got[k] == r, (n, prec, i, m, k, got[k], r)
        lat.close()


def test_noalloc_analysis_errors(itse):
    lat = _lattice(itse, 16, "fp64", "cell", seed=1)
    for bad in (-0.1, 1.0):
        with pytest.raises(itse.ItseError, match="EINVAL"):
            lat.analyse_noalloc(0, bad)
    with pytest.raises(itse.ItseError, match="EINVAL"):
        lat.analyse_noalloc(2, 0.3)
    lat.close()
    c = itse.Lattice(16, 0.25, 1.2, 0.05, kin=3, precision="fp32", complex_psi=True)
    with pytest.raises(itse.ItseError, match="ESTATE"):
        c.analyse_noalloc(0, 0.3)
    c.close()
