"""Pins for the oracle's own FFT: brute-force DFT on tiny grids (the definition of
the discrete Fourier coefficients, Sec. 3.1), round trip, Parseval, and numpy.fft
as an independent library routine at larger sizes."""
import itertools

import numpy as np
import pytest

import oracle


def brute_dft(x, sign):
    """Direct sum over all index tuples; forward carries 1/N^d."""
    shape = x.shape
    out = np.zeros_like(x, dtype=np.complex128)
    Ntot = np.prod(shape)
    for k in itertools.product(*[range(n) for n in shape]):
        acc = 0.0
        for j in itertools.product(*[range(n) for n in shape]):
            ph = sum(jj * kk / n for jj, kk, n in zip(j, k, shape))
            acc += x[j] * np.exp(sign * 2j * np.pi * ph)
        out[k] = acc / Ntot if sign < 0 else acc
    return out


@pytest.mark.parametrize("shape", [(2,), (3,), (4,), (6,), (8,), (12,), (16,), (24,), (5,), (7,)])
def test_fft_1d_matches_brute_force(shape):
    # The oracle's transforms are 2D/3D; a 1D line is a 2D grid with one row.
    rng = np.random.default_rng(11)
    x = rng.standard_normal((1,) + shape) + 1j * rng.standard_normal((1,) + shape)
    for sign in (-1, +1):
        np.testing.assert_allclose(oracle.fft(x, sign), brute_dft(x, sign), rtol=0, atol=1e-14 * max(1, shape[0]))


@pytest.mark.parametrize("shape", [(4, 6), (6, 4), (8, 12), (3, 2, 4), (4, 4, 6)])
def test_fft_nd_matches_brute_force(shape):
    rng = np.random.default_rng(12)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    for sign in (-1, +1):
        np.testing.assert_allclose(oracle.fft(x, sign), brute_dft(x, sign), rtol=0, atol=2e-14 * np.prod(shape))


@pytest.mark.parametrize("shape", [(64, 64), (48, 96), (192, 192), (384, 128), (16, 32, 24)])
def test_fft_matches_numpy_and_round_trip(shape):
    rng = np.random.default_rng(13)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    X = oracle.fft(x, -1)
    ref = np.fft.fftn(x) / x.size
    assert np.abs(X - ref).max() <= 1e-15 * np.abs(ref).max() * 50
    # Parseval: sum |x|^2 = N^d sum |X|^2
    assert abs(np.sum(np.abs(x) ** 2) - x.size * np.sum(np.abs(X) ** 2)) <= 1e-12 * np.sum(np.abs(x) ** 2)
    back = oracle.fft(X, +1)
    assert np.abs(back - x).max() <= 1e-13
