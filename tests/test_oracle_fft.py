"""Pins of the oracle FFT: brute-force DFT, numpy.fft, Parseval, round trip."""
import cmath
import os

import numpy as np
import pytest

from oracle import fft as F


def brute_dft2(x, sign=-1):
    """Nested-loop 2D DFT straight from the definition."""
    n0, n1 = x.shape
    out = np.zeros((n0, n1), dtype=complex)
    for k0 in range(n0):
        for k1 in range(n1):
            acc = 0j
            for j0 in range(n0):
                for j1 in range(n1):
                    acc += x[j0, j1] * cmath.exp(sign * 2j * cmath.pi * (k0 * j0 / n0 + k1 * j1 / n1))
            out[k0, k1] = acc
    return out


@pytest.mark.parametrize("shape", [(8, 8), (6, 6), (12, 12), (8, 12)])
def test_fft2_matches_brute_force(shape):
    rng = np.random.default_rng(1)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = brute_dft2(x)
    assert np.abs(F.fft2(x) - ref).max() <= 1e-13 * np.abs(ref).max()
    refi = brute_dft2(x, +1) / x.size
    assert np.abs(F.ifft2(x) - refi).max() <= 1e-13 * np.abs(refi).max()


@pytest.mark.parametrize("n", [16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 1024])
def test_fft_matches_numpy(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    ref = np.fft.fft(x)
    assert np.abs(F.fft(x) - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.abs(F.ifft(x) - np.fft.ifft(x)).max() <= 1e-13 * np.abs(np.fft.ifft(x)).max()


def test_fft2_numpy_and_parseval():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 64, 64))
    G = F.fft2(x)
    assert np.abs(G - np.fft.fft2(x)).max() <= 1e-12 * np.abs(G).max()
    # Parseval: sum |G|^2 = N^2 sum |g|^2
    assert abs(np.sum(np.abs(G) ** 2) - x[0].size * np.sum(x ** 2)) <= 1e-12 * np.sum(np.abs(G) ** 2)
    assert np.abs(F.ifft2(G) - x).max() <= 1e-13


def test_3d_and_shifts():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((16, 16, 16)) + 1j * rng.standard_normal((16, 16, 16))
    assert np.abs(F.fftn3(x) - np.fft.fftn(x)).max() <= 1e-12 * np.abs(np.fft.fftn(x)).max()
    assert np.abs(F.ifftn3(x) - np.fft.ifftn(x)).max() <= 1e-13
    assert np.array_equal(F.shift_to_native(x, (0, 1, 2)), np.fft.ifftshift(x))
    assert np.array_equal(F.shift_to_centred(x, (0, 1, 2)), np.fft.fftshift(x))
