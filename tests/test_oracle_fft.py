"""Pins for the oracle's transform (paper, section "Kinetic terms": unnormalised
FFT with exp(-i k.x) and IFFT with exp(+i k.x)).

The oracle's 1D transform uses the DFT definition for lengths <= 16 and a
recursive radix-2/3 Cooley-Tukey split above.  Both are checked against numpy's
FFT (an independent library routine), against closed forms (delta <-> constant,
a single plane wave), round trip and Parseval.  A dropped twiddle, a wrong sign
or a transposed axis fails the numpy comparison at every size listed.
"""
import numpy as np
import pytest

NAIVE_LENGTHS = [1, 2, 3, 4, 6, 8, 9, 12, 16]
SPLIT_LENGTHS = [18, 24, 27, 32, 36, 48, 64, 96, 128, 192, 256]


def _rand_c(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("n", NAIVE_LENGTHS + SPLIT_LENGTHS)
def test_lines_match_numpy(orc, n):
    x = _rand_c((5, n), n)
    y = orc.fft_lines(x, -1)
    ref = np.fft.fft(x, axis=-1)
    assert np.abs(y - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    yi = orc.fft_lines(x, +1)
    refi = np.fft.ifft(x, axis=-1) * n
    assert np.abs(yi - refi).max() <= 1e-13 * max(1.0, np.abs(refi).max())


@pytest.mark.parametrize("n", [2, 6, 12, 16, 18, 24, 32, 48])
def test_3d_matches_numpy(orc, n):
    x = _rand_c((n, n, n), 100 + n)
    y = orc.fft3d(x, -1)
    ref = np.fft.fftn(x)
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    # axis order: transform of data varying along one axis only
    z = np.zeros((n, n, n), complex)
    z[:, 0, 0] = np.arange(n) + 1.0
    assert np.allclose(orc.fft3d(z, -1), np.fft.fftn(z), atol=1e-12 * n * n)


@pytest.mark.parametrize("n", [8, 12, 32, 48])
def test_closed_forms(orc, n):
    d = np.zeros((n, n, n), complex)
    d[0, 0, 0] = 1.0
    assert np.abs(orc.fft3d(d, -1) - 1.0).max() < 1e-14
    c = np.ones((n, n, n), complex)
    f = orc.fft3d(c, -1)
    expect = np.zeros_like(f)
    expect[0, 0, 0] = n ** 3
    assert np.abs(f - expect).max() < 1e-9
    # single plane wave exp(+2 pi i m.x / N) lands on bin m with weight N^3
    m = (1, n // 2, n - 3)
    idx = np.indices((n, n, n))
    pw = np.exp(2j * np.pi * (m[0] * idx[0] + m[1] * idx[1] + m[2] * idx[2]) / n)
    f = orc.fft3d(pw, -1)
    expect = np.zeros_like(f)
    expect[m] = n ** 3
    assert np.abs(f - expect).max() < 1e-9 * n ** 3


@pytest.mark.parametrize("n", [6, 16, 24, 64])
def test_roundtrip_and_parseval(orc, n):
    x = _rand_c((n, n, n), 7 * n)
    f = orc.fft3d(x, -1)
    back = orc.fft3d(f, +1) / n ** 3
    assert np.abs(back - x).max() < 1e-14 * max(1, np.log2(n)) * 10
    lhs = np.sum(np.abs(x) ** 2)
    rhs = np.sum(np.abs(f) ** 2) / n ** 3
    assert abs(lhs - rhs) <= 1e-13 * lhs
