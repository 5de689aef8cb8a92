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


def test_bilinear_weights_partition_unity_and_centroid():
    """Each sample's four weights sum to 1 and their weighted cell position is the sample's
    real position (bilinear interpolation reproduces linear functions)."""
    import math
    N, Np = 32, 7
    theta = np.pi * np.arange(Np) / Np
    iy, ix, w = D.bilinear_cells(N, theta)
    assert np.all(w >= 0) and np.allclose(w.sum(-1), 1.0, atol=1e-14)
    for n in range(Np):
        for iu in range(N):
            u = iu - N // 2
            x, y = -(u * math.sin(theta[n])), u * math.cos(theta[n])
            # unwrap the centred indices next to the sample before averaging
            cx = (ix[n, iu] - N // 2 - math.floor(x) + N // 2) % N - N // 2 + math.floor(x)
            cy = (iy[n, iu] - N // 2 - math.floor(y) + N // 2) % N - N // 2 + math.floor(y)
            assert abs(np.dot(w[n, iu], cx) - x) < 1e-12 and abs(np.dot(w[n, iu], cy) - y) < 1e-12


def test_bilinear_equals_nearest_on_axis_angles_and_averages_constants():
    """At theta = 0 every sample sits on a cell (weights 0/1), so bilinear insertion equals the
    nearest-voxel one; a constant spectrum inserts as that constant on every touched cell."""
    rng = np.random.default_rng(3)
    N = 16
    E = rng.standard_normal((1, N, N)) + 1j * rng.standard_normal((1, N, N))
    th = np.array([0.0])
    assert np.allclose(D.insert_slices(E, th, "bilinear"), D.insert_slices(E, th, "nearest"), atol=1e-15)
    th = np.pi * np.arange(5) / 5
    ones = np.ones((5, N, N), complex)
    g = D.insert_slices(ones, th, "bilinear")
    iy, ix, w = D.bilinear_cells(N, th)
    touched = np.zeros((N, N), bool)
    touched[iy[w > 0], ix[w > 0]] = True
    assert np.allclose(g[:, touched], 1.0, atol=1e-12) and np.all(g[:, ~touched] == 0)


def test_bilinear_volume_at_matches_literal_grid():
    rng = np.random.default_rng(4)
    N, Np = 16, 5
    obj = rng.standard_normal((Np, N, N))
    th = np.pi * np.arange(Np) / Np
    vol = D.assemble_volume(obj, th, "bilinear")
    pts = rng.integers(0, N, size=(20, 3))
    got = D.volume_at(obj, th, pts, "bilinear")
    assert np.allclose(got, vol[pts[:, 0], pts[:, 1], pts[:, 2]], atol=1e-12 * np.abs(vol).max())
