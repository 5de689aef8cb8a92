"""Pins of the oracle's step D (Fourier-slice insertion + 3D inverse FFT)."""
import numpy as np

from oracle import geometry as G
from oracle import stepd as D


def test_two_exact_slices_against_numpy_masked_inverse():
    N = 16
    rng = np.random.default_rng(0)
    O = np.zeros((N, N, N))
    O[4:12, 5:11, 3:13] = rng.uniform(0, 1, size=(8, 6, 10))
    po = np.stack([G.project_right_angle(O, 0), G.project_right_angle(O, 1)])
    vol = D.assemble_volume(po, [0.0, np.pi / 2])
    E3 = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(O)))
    mask = np.zeros((N, N), bool)
    mask[:, N // 2] = True          # kx = 0 plane (theta = 0)
    mask[N // 2, :] = True          # ky = 0 plane (theta = 90 deg)
    ref = np.real(np.fft.fftshift(np.fft.ifftn(np.fft.ifftshift(E3 * mask[None]))))
    assert np.abs(vol - ref).max() <= 1e-12 * np.abs(ref).max()


def test_single_slice_is_a_back_projection_smear():
    N = 16
    rng = np.random.default_rng(1)
    po = rng.uniform(size=(1, N, N))
    vol = D.assemble_volume(po, [0.0])
    # only the kx = 0 plane is filled: the volume is PO[z][y]/N along every x
    assert np.abs(vol - po[0][:, :, None] / N).max() <= 1e-13


def test_volume_at_matches_literal_volume():
    """The sampled-voxel evaluation agrees with the full N^3 form at every voxel asked for."""
    N = 16
    rng = np.random.default_rng(2)
    po = rng.uniform(size=(5, N, N))
    theta = np.pi * np.arange(5) / 5
    vol = D.assemble_volume(po, theta)
    pts = np.stack([rng.integers(0, N, 3) for _ in range(12)] + [np.array([N // 2] * 3)])
    got = D.volume_at(po, theta, pts)
    ref = vol[pts[:, 0], pts[:, 1], pts[:, 2]]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(vol).max()
