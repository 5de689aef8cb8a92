"""Plain FP64 discrete Fourier transforms for the oracle.

Forward transform X[k] = sum_x x[x] exp(-2 pi i k x / n), unnormalised;
the inverse uses exp(+2 pi i k x / n) and divides by n.  (The paper writes
its transform with exp(+i q.r), Eq. 1; intensities do not depend on the
sign, and the oracle uses one sign consistently for 2D and 3D.)

Method: a direct O(n^2) DFT for lengths up to 32 (any length, so the factor
3 of n = 3*2^k is handled there), and radix-2 decimation-in-time combine
steps above that.  No blocking or reordering beyond that textbook scheme.
"""
from __future__ import annotations

import numpy as np

_DIRECT_MAX = 32


def dft_direct(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Direct DFT along the last axis: X[k] = sum_j x[j] exp(sign*2*pi*i*j*k/n)."""
    n = x.shape[-1]
    j = np.arange(n)
    ang = (sign * 2.0 * np.pi / n) * ((j[:, None] * j[None, :]) % n)
    w = np.cos(ang) + 1j * np.sin(ang)          # w[j, k]
    return np.asarray(x, dtype=np.complex128) @ w


def _split(n: int):
    """n = n0 * 2^s with n0 <= 32 (n0 may contain the factor 3)."""
    s = 0
    while n > _DIRECT_MAX and n % 2 == 0:
        n //= 2
        s += 1
    if n > _DIRECT_MAX:
        raise ValueError("length must be (<=32) * 2^s")
    return n, s


def fft1(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Unnormalised DFT along the last axis with exponent sign `sign`."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    n0, s = _split(n)
    if s == 0:
        return dft_direct(x, sign)
    p = 1 << s
    lead = x.shape[:-1]
    # column r of the (n0, p) view is the subsequence x[r::p]
    sub = x.reshape(lead + (n0, p))
    # direct DFT of every subsequence along the n0 axis
    X = np.moveaxis(dft_direct(np.moveaxis(sub, -2, -1), sign), -1, -2)   # (.., n0, p)
    while X.shape[-1] > 1:
        half = X.shape[-1] // 2
        L = X.shape[-2]
        even = X[..., :half]                      # subsequence r::2*half ...
        odd = X[..., half:]                       # ... and r+half::2*half
        k = np.arange(L)
        f = np.exp(sign * 1j * np.pi * k / L)[:, None]   # exp(sign*2*pi*i*k/(2L))
        X = np.concatenate([even + f * odd, even - f * odd], axis=-2)
    return X[..., 0]


def fft(x, axis=-1):
    return np.moveaxis(fft1(np.moveaxis(np.asarray(x), axis, -1), -1), -1, axis)


def ifft(x, axis=-1):
    x = np.asarray(x)
    n = x.shape[axis]
    return np.moveaxis(fft1(np.moveaxis(x, axis, -1), +1), -1, axis) / n


def fft2(x):
    return fft(fft(x, -1), -2)


def ifft2(x):
    return ifft(ifft(x, -1), -2)


def ifftn3(x):
    return ifft(ifft(ifft(x, -1), -2), -3)


def fftn3(x):
    return fft(fft(fft(x, -1), -2), -3)


def shift_to_native(a, axes):
    """Move the origin from index N/2 (centred arrays) to index 0."""
    return np.roll(a, [-(a.shape[ax] // 2) for ax in axes], axis=axes)


def shift_to_centred(a, axes):
    """Move the origin from index 0 to index N/2."""
    return np.roll(a, [a.shape[ax] // 2 for ax in axes], axis=axes)
