"""Pins of the oracle's input preparation and random initial objects (step A's random guess, the
problem statement's I = |E|^2), checked with numpy's FFT as an independent library.

* amplitudes(): A = sqrt(I) moved from the centred layout (zero frequency at index N/2) to native
  order (zero frequency at index 0); I < 0 marks an unmeasured pixel and becomes -1.
* initial_object(): the random start of angle n is Re F2^-1(A e^{i phi}) with unmeasured
  amplitudes taken as 0.  The real part of an inverse transform has, as its own transform, the
  Hermitian part of what was inverted, so in native order
      F2(native(x))[q] = (a(q) e^{i phi(q)} + a(-q) e^{-i phi(-q)}) / 2,   a = max(A, 0).
  A mix-up of centred and native order, a missing zero for unmeasured pixels, a forward/inverse
  swap or a dropped 1/2 each break that identity on an input with A(q) != A(-q).
"""
import numpy as np
import pytest

from oracle import cpra as C
from oracle.rng import initial_phases


def _asymmetric_intensity(N, rng, holes=True):
    """Centred, non-centrosymmetric intensity with a one-sided block of unmeasured pixels."""
    I = rng.uniform(0.5, 4.0, size=(N, N)) ** 2
    if holes:
        I[N // 2 + 2:N // 2 + 5, N // 2 - 6:N // 2 - 3] = -1.0      # its mirror block stays measured
    return I


def test_amplitudes_layout_and_unmeasured():
    rng = np.random.default_rng(10)
    N = 16
    I = _asymmetric_intensity(N, rng)
    A = C.amplitudes(I)
    # centred index (N/2 + w, N/2 + u) holds frequency (w, u); native index (w mod N, u mod N)
    for w, u in [(0, 0), (1, 0), (0, 3), (-2, 5), (-8, -8), (7, -1)]:
        v = I[N // 2 + w, N // 2 + u]
        want = -1.0 if v < 0 else np.sqrt(v)
        assert A[w % N, u % N] == want
    assert np.count_nonzero(A < 0) == 9 and np.all(A[A >= 0] > 0)
    with pytest.raises(ValueError):
        C.amplitudes(np.where(I > 3, np.nan, I))


@pytest.mark.parametrize("N,n,seed", [(16, 0, 3), (24, 5, 77), (64, 2, 1002)])
def test_initial_object_spectrum_is_hermitian_part(N, n, seed):
    rng = np.random.default_rng(N + n)
    I = _asymmetric_intensity(N, rng)
    A = C.amplitudes(I)
    x = C.initial_object(A, seed, n)
    assert x.dtype == np.float64 and x.shape == (N, N)
    a = np.where(A >= 0, A, 0.0)
    phi = initial_phases(seed, n, N)
    E = a * np.exp(1j * phi)
    neg = (-np.arange(N)) % N
    E_minus = E[np.ix_(neg, neg)]                       # E(-q) in native order
    want = 0.5 * (E + np.conj(E_minus))
    got = np.fft.fft2(np.fft.ifftshift(x))              # native-order object -> spectrum
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    # the input really exercises the pairing: A(q) != A(-q) somewhere, and a pair with exactly one
    # unmeasured member
    A_minus = A[np.ix_(neg, neg)]
    assert np.count_nonzero(A != A_minus) > N * N // 2
    assert np.count_nonzero((A < 0) != (A_minus < 0)) > 0


def test_initial_object_depends_on_angle_and_seed_only_through_phases():
    N = 16
    A = C.amplitudes(_asymmetric_intensity(N, np.random.default_rng(0)))
    x1 = C.initial_object(A, 5, 1)
    assert np.array_equal(C.initial_object(A, 5, 1), x1)
    assert not np.allclose(C.initial_object(A, 5, 2), x1)
    assert not np.allclose(C.initial_object(A, 6, 1), x1)
    # doubling the amplitudes doubles the object exactly (power of two)
    assert np.array_equal(C.initial_object(np.where(A >= 0, 2 * A, -1.0), 5, 1), 2 * x1)
