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
