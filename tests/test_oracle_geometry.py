"""Pins of the oracle's geometry: Fourier slice theorem, seam mirror, slice cells."""
import numpy as np
import pytest

from oracle import cpra as C
from oracle import fft as F
from oracle import geometry as G
from oracle import stepd as D


def _object(N=16, seed=0):
    rng = np.random.default_rng(seed)
    O = np.zeros((N, N, N))
    O[3:13, 4:12, 2:14] = rng.uniform(0, 1, size=(10, 8, 12))
    return O


@pytest.mark.parametrize("q", [0, 1, 2, 3])
def test_fourier_slice_theorem_right_angles(q):
    """F2 of the projection equals the central slice of the 3D transform (Eq. 2-3)."""
    N = 16
    O = _object(N)
    theta = q * np.pi / 2
    po = G.project_right_angle(O, q)
    E2 = F.shift_to_centred(C.forward(po), (0, 1))                 # centred [w][u]
    E3 = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(O)))         # centred [kz][ky][kx]
    kx, ky = D.slice_cells(N, [theta])
    sl = E3[:, ky[0], kx[0]]                                       # [kz][u]
    assert np.abs(E2 - sl).max() <= 1e-12 * np.abs(E3).max()


def test_seam_mirror_is_projection_at_theta_plus_pi():
    O = _object(16, 1)
    for q in (0, 1):
        assert np.array_equal(C.mirror_t(G.project_right_angle(O, q)), G.project_right_angle(O, q + 2))


def test_coupling_seam_against_direct_projections():
    """Np=2 at 0 and 90 deg: the wrapped neighbours are the POs at -90 and 180 deg."""
    O = _object(16, 2)
    po = np.stack([G.project_right_angle(O, 0), G.project_right_angle(O, 1)])
    alpha = (0.1, 0.6, 0.3)          # asymmetric: catches swapped sides
    out = C.couple(po, np.ones(2, bool), alpha, C.WRAP_MIRROR)
    exp0 = alpha[0] * G.project_right_angle(O, 3) + alpha[1] * po[0] + alpha[2] * po[1]
    exp1 = alpha[0] * po[0] + alpha[1] * po[1] + alpha[2] * G.project_right_angle(O, 2)
    assert np.abs(out[0] - exp0).max() <= 1e-12
    assert np.abs(out[1] - exp1).max() <= 1e-12


def test_plain_wrap_preserves_sum_and_single_angle_identity():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((7, 8, 8))
    out = C.couple(X, np.ones(7, bool), (0.2, 0.6, 0.2), C.WRAP_PLAIN)
    assert np.abs(out.sum(0) - X.sum(0)).max() <= 1e-12
    one = C.couple(X[:1], np.ones(1, bool), (0.3, 0.4, 0.3), C.WRAP_PLAIN)
    assert np.abs(one - X[:1]).max() <= 1e-15


def test_coupling_partial_set_renormalises():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((5, 4, 4))
    present = np.array([1, 1, 0, 1, 1], bool)
    out = C.couple(X, present, (0.2, 0.6, 0.2), C.WRAP_PLAIN)
    # angle 1: right neighbour 2 absent -> weights (0.2, 0.6)/0.8
    assert np.abs(out[1] - (0.25 * X[0] + 0.75 * X[1])).max() <= 1e-15
    assert np.array_equal(out[2], X[2])


def test_slice_cells_closed_forms():
    N = 16
    kx, ky = D.slice_cells(N, [0.0, np.pi / 2])
    u = np.arange(N) - N // 2
    assert np.array_equal(kx[0], np.full(N, N // 2))
    assert np.array_equal(ky[0], (u + N // 2) % N)
    assert np.array_equal(kx[1], (-u + N // 2) % N)
    assert np.array_equal(ky[1], np.full(N, N // 2))


def test_k_tap_coupling_reduces_and_closed_forms():
    """2K+1 taps: the 3-tap case equals Eq. 4's three-tap form; a one-hot tap is a ring shift
    (mirrored where it wraps); the plain-wrap ring sum is preserved; absent neighbours renormalise."""
    from oracle import cpra as C
    rng = np.random.default_rng(7)
    Np, N = 7, 8
    X = rng.standard_normal((Np, N, N))
    allp = np.ones(Np, bool)
    for wrap in (C.WRAP_MIRROR, C.WRAP_PLAIN):
        assert np.allclose(C.couple_taps(X, allp, (0.1, 0.6, 0.3), wrap), C.couple(X, allp, (0.1, 0.6, 0.3), wrap),
                           atol=1e-15)
    # one-hot alpha_{+2}: O_n = X_{n+2}, mirrored for n = Np-2, Np-1 (the wrap)
    taps = (0, 0, 1e-300, 0, 1.0)
    Y = C.couple_taps(X, allp, taps, C.WRAP_MIRROR)
    for n in range(Np):
        want = X[(n + 2) % Np] if n + 2 < Np else C.mirror_t(X[(n + 2) % Np])
        assert np.allclose(Y[n], want, atol=1e-12)
    # plain wrap: every column of the circulant sums to 1, so the ring sum is kept
    taps5 = (0.05, 0.15, 0.5, 0.2, 0.1)
    Z = C.couple_taps(X, allp, taps5, C.WRAP_PLAIN)
    assert np.allclose(Z.sum(0), X.sum(0), atol=1e-12)
    # absent neighbour n+1 of n = 2: its weight drops, the rest rescale
    pres = allp.copy()
    pres[3] = False
    W = C.couple_taps(X, pres, taps5, C.WRAP_PLAIN)
    s = 0.05 + 0.15 + 0.5 + 0.1
    assert np.allclose(W[2], (0.05 * X[0] + 0.15 * X[1] + 0.5 * X[2] + 0.1 * X[4]) / s, atol=1e-13)
    assert np.array_equal(W[3], X[3])
