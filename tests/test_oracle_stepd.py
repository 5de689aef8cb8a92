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
