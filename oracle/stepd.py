"""FP64 oracle of step D: Fourier-slice insertion and one 3D inverse FFT.

TEST INFRASTRUCTURE ONLY (see cpra.py).

Step D of the paper interpolates the retrieved 2D spectra E_n into a 3D
spectrum E(q) and transforms back.  Reading taken here: E_n = F2 of the
final estimate O'_n; nearest-voxel insertion along the Fourier slice of
angle n, averaged over all (n, u) that land on a voxel, empty voxels zero;
the volume is the real part of the 3D inverse transform, centred.  No 3D
iterations follow (those are a later refinement).

Slice geometry (Fourier slice theorem, Eq. 2-3, rotation about z):
centred frequency (w, u) of angle n sits at
    k_x = -u sin(theta_n),  k_y = u cos(theta_n),  k_z = w,
rounded to the nearest voxel with floor(x + 0.5) in FP64 and wrapped mod N.
This is the literal N^3 form: it builds the whole 3D grid and calls the
oracle's own 3D inverse FFT.
"""
from __future__ import annotations

import math

import numpy as np

from . import fft as F


def slice_cells(N: int, theta) -> tuple[np.ndarray, np.ndarray]:
    """(kx_index, ky_index), each (Np, N) int64: centred voxel indices of frequency u of angle n."""
    Np = len(theta)
    kx = np.zeros((Np, N), dtype=np.int64)
    ky = np.zeros((Np, N), dtype=np.int64)
    for n in range(Np):
        s = math.sin(float(theta[n]))
        c = math.cos(float(theta[n]))
        for iu in range(N):
            u = float(iu - N // 2)
            x = -(u * s)
            y = u * c
            kx[n, iu] = (math.floor(x + 0.5) + N // 2) % N
            ky[n, iu] = (math.floor(y + 0.5) + N // 2) % N
    return kx, ky


def insert_slices(E_centred: np.ndarray, theta) -> np.ndarray:
    """Average the centred 2D spectra E_n[w][u] into a centred 3D grid [kz][ky][kx]."""
    Np, N, _ = E_centred.shape
    kx, ky = slice_cells(N, theta)
    grid = np.zeros((N, N, N), dtype=np.complex128)
    cnt = np.zeros((N, N), dtype=np.int64)
    for n in range(Np):
        for iu in range(N):
            grid[:, ky[n, iu], kx[n, iu]] += E_centred[n, :, iu]
            cnt[ky[n, iu], kx[n, iu]] += 1
    return grid / np.maximum(cnt, 1)[None, :, :]


def assemble_volume(objects_centred: np.ndarray, theta) -> np.ndarray:
    """Volume [z][y][x] (centred, float64) from the final POs of all angles."""
    E = F.shift_to_centred(F.fft2(F.shift_to_native(objects_centred, (-2, -1))), (-2, -1))
    grid = insert_slices(E, theta)
    vol = F.ifftn3(F.shift_to_native(grid, (-3, -2, -1)))
    return np.real(F.shift_to_centred(vol, (-3, -2, -1)))


def volume_at(objects_centred: np.ndarray, theta, points) -> np.ndarray:
    """The step-D volume at selected voxels only, straight from its definition.

    points: (M, 3) centred indices (z, y, x).  Builds the same averaged
    insertion as `insert_slices`, but only on occupied (ky, kx) cells, and sums
    the 3D inverse DFT directly over those cells for each requested voxel, so
    it stays cheap at N = 512 and 1024 where the N^3 grid is not.
    """
    Np, N, _ = objects_centred.shape
    E = F.shift_to_centred(F.fft2(F.shift_to_native(objects_centred, (-2, -1))), (-2, -1))   # [n][w][u]
    kx, ky = slice_cells(N, theta)
    cell = ky * N + kx                                     # (Np, N) cell id of (n, u)
    ids, inv = np.unique(cell.ravel(), return_inverse=True)
    acc = np.zeros((N, ids.size), dtype=np.complex128)     # [kz][cell]
    cnt = np.bincount(inv, minlength=ids.size).astype(np.float64)
    flat = E.transpose(1, 0, 2).reshape(N, -1)             # [kz][(n, u)]
    for w in range(N):
        acc[w] = np.bincount(inv, weights=flat[w].real, minlength=ids.size) + \
            1j * np.bincount(inv, weights=flat[w].imag, minlength=ids.size)
    acc /= cnt[None, :]
    kyc = ids // N - N // 2                                # centred frequencies of the cells
    kxc = ids % N - N // 2
    kz = np.arange(N) - N // 2
    out = np.zeros(len(points))
    for i, (z, y, x) in enumerate(points):
        zc, yc, xc = z - N // 2, y - N // 2, x - N // 2
        hz = np.exp(2j * np.pi * kz * zc / N) @ acc        # sum over kz for every cell
        out[i] = np.real(np.sum(hz * np.exp(2j * np.pi * (kyc * yc + kxc * xc) / N))) / N ** 3
    return out
