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


def bilinear_cells(N: int, theta):
    """Bilinear insertion (the alternative reading of "interpolate"): sample (n, u) at the real
    position (x, y) = (-u sin t, u cos t) spreads over the four cells around it with weights
    (1-fy)(1-fx), (1-fy)fx, fy(1-fx), fy fx, fx = x - floor(x), fy = y - floor(y).
    Returns (ky_index, kx_index, weight), each (Np, N, 4), centred indices."""
    Np = len(theta)
    iy = np.zeros((Np, N, 4), dtype=np.int64)
    ix = np.zeros((Np, N, 4), dtype=np.int64)
    w = np.zeros((Np, N, 4))
    for n in range(Np):
        s = math.sin(float(theta[n]))
        c = math.cos(float(theta[n]))
        for iu in range(N):
            u = float(iu - N // 2)
            x = -(u * s)
            y = u * c
            x0, y0 = math.floor(x), math.floor(y)
            fx, fy = x - x0, y - y0
            corners = ((y0, x0, (1.0 - fy) * (1.0 - fx)), (y0, x0 + 1, (1.0 - fy) * fx),
                       (y0 + 1, x0, fy * (1.0 - fx)), (y0 + 1, x0 + 1, fy * fx))
            for k, (cy, cx, wk) in enumerate(corners):
                iy[n, iu, k] = (cy + N // 2) % N
                ix[n, iu, k] = (cx + N // 2) % N
                w[n, iu, k] = wk
    return iy, ix, w


def insert_slices(E_centred: np.ndarray, theta, interp: str = "nearest") -> np.ndarray:
    """Average the centred 2D spectra E_n[w][u] into a centred 3D grid [kz][ky][kx]: nearest voxel
    with a plain average per voxel, or bilinear with the weighted average sum(w E) / sum(w)."""
    Np, N, _ = E_centred.shape
    grid = np.zeros((N, N, N), dtype=np.complex128)
    if interp == "nearest":
        kx, ky = slice_cells(N, theta)
        cnt = np.zeros((N, N), dtype=np.int64)
        for n in range(Np):
            for iu in range(N):
                grid[:, ky[n, iu], kx[n, iu]] += E_centred[n, :, iu]
                cnt[ky[n, iu], kx[n, iu]] += 1
        return grid / np.maximum(cnt, 1)[None, :, :]
    if interp != "bilinear":
        raise ValueError("interp must be 'nearest' or 'bilinear'")
    iy, ix, w = bilinear_cells(N, theta)
    wsum = np.zeros((N, N))
    for n in range(Np):
        for iu in range(N):
            for k in range(4):
                grid[:, iy[n, iu, k], ix[n, iu, k]] += w[n, iu, k] * E_centred[n, :, iu]
                wsum[iy[n, iu, k], ix[n, iu, k]] += w[n, iu, k]
    return grid / np.where(wsum > 0, wsum, 1.0)[None, :, :]


def assemble_volume(objects_centred: np.ndarray, theta, interp: str = "nearest") -> np.ndarray:
    """Volume [z][y][x] (centred, float64) from the final POs of all angles."""
    E = F.shift_to_centred(F.fft2(F.shift_to_native(objects_centred, (-2, -1))), (-2, -1))
    grid = insert_slices(E, theta, interp)
    vol = F.ifftn3(F.shift_to_native(grid, (-3, -2, -1)))
    return np.real(F.shift_to_centred(vol, (-3, -2, -1)))


def volume_at(objects_centred: np.ndarray, theta, points, interp: str = "nearest") -> np.ndarray:
    """The step-D volume at selected voxels only, straight from its definition.

    points: (M, 3) centred indices (z, y, x).  Builds the same averaged
    insertion as `insert_slices`, but only on occupied (ky, kx) cells, and sums
    the 3D inverse DFT directly over those cells for each requested voxel, so
    it stays cheap at N = 512 and 1024 where the N^3 grid is not.
    """
    Np, N, _ = objects_centred.shape
    E = F.shift_to_centred(F.fft2(F.shift_to_native(objects_centred, (-2, -1))), (-2, -1))   # [n][w][u]
    flat = E.transpose(1, 0, 2).reshape(N, -1)             # [kz][(n, u)]
    if interp == "nearest":
        kx, ky = slice_cells(N, theta)
        cell = (ky * N + kx).ravel()                       # cell id of (n, u)
        wt = np.ones(cell.size)
        src = np.arange(cell.size)
    else:
        iy, ix, w4 = bilinear_cells(N, theta)
        cell = (iy * N + ix).reshape(-1)                   # (n, u, corner)
        wt = w4.reshape(-1)
        src = np.repeat(np.arange(Np * N), 4)
    ids, inv = np.unique(cell, return_inverse=True)
    acc = np.zeros((N, ids.size), dtype=np.complex128)     # [kz][cell]
    cnt = np.bincount(inv, weights=wt, minlength=ids.size)
    for w in range(N):
        acc[w] = np.bincount(inv, weights=wt * flat[w, src].real, minlength=ids.size) + \
            1j * np.bincount(inv, weights=wt * flat[w, src].imag, minlength=ids.size)
    acc /= np.where(cnt > 0, cnt, 1.0)[None, :]
    kyc = ids // N - N // 2                                # centred frequencies of the cells
    kxc = ids % N - N // 2
    kz = np.arange(N) - N // 2
    out = np.zeros(len(points))
    for i, (z, y, x) in enumerate(points):
        zc, yc, xc = z - N // 2, y - N // 2, x - N // 2
        hz = np.exp(2j * np.pi * kz * zc / N) @ acc        # sum over kz for every cell
        out[i] = np.real(np.sum(hz * np.exp(2j * np.pi * (kyc * yc + kxc * xc) / N))) / N ** 3
    return out
