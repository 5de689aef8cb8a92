"""FP64 oracle of the 3D refinement that follows step D.

TEST INFRASTRUCTURE ONLY (see cpra.py).

After the retrieved 2D spectra are inserted into the 3D grid (stepd.py), the paper refines the
volume with a few tens of 3D iterations in the manner of conventional 3D CXDI, but with the
inserted spectrum (phases included) as the Fourier constraint and a 3D support built from the 2D
supports.  Readings taken here:

* Fourier constraint: the Hermitian part of the inserted spectrum, E_h(k) = (E(k) + conj E(-k))/2,
  is imposed on every (k_y, k_x) cell that received a slice sample, and on its mirror cell, for
  all k_z (the insertion fills whole k_z lines); all other cells are free.  The volume is real, so
  its spectrum is Hermitian; the inserted one is not quite (the frequency -N/2 has no +N/2
  partner, and rounding ties break the symmetry of the cell map), and the step-D volume, the real
  part of its inverse transform, has exactly E_h there.
* Real-space constraint: the 3D support is the intersection over the angles of the
  back-projected 2D supports: voxel (z, y, x) (centred) belongs to it when, for every angle n,
  the projected coordinate t = floor(y cos t_n - x sin t_n + 1/2) (FP64) lies in the 2D support
  of angle n at row z (outside the N-pixel range counts as outside); positivity as in 2D.
* Iteration: error reduction, V <- P_S(Re F3^-1(P_F(F3 V))).  Every `shrink_every` iterations the
  support is replaced by the 3D shrinkwrap of V (separable periodic Gaussian k(dz) k(dy) k(dx)
  of cpra.gaussian_window, kept where the blur is >= threshold * its maximum).
The volume is centred [z][y][x]; transforms use the oracle's own FFT.
"""
from __future__ import annotations

import math

import numpy as np

from . import cpra as C
from . import fft as F
from . import stepd as D


def measured_grid(objects_centred: np.ndarray, theta, interp: str = "nearest"):
    """(Hermitian part of the inserted spectrum, centred [kz][ky][kx]; the sampled (ky, kx) cells
    and their mirrors) of the final POs."""
    E = F.shift_to_centred(F.fft2(F.shift_to_native(objects_centred, (-2, -1))), (-2, -1))
    Np, N, _ = E.shape
    E3 = D.insert_slices(E, theta, interp)
    sampled = np.zeros((N, N), bool)
    if interp == "nearest":
        kx, ky = D.slice_cells(N, theta)
        sampled[ky, kx] = True
    else:
        iy, ix, w = D.bilinear_cells(N, theta)
        sampled[iy[w > 0], ix[w > 0]] = True
    # Hermitian part and the mirrored cells (centred index i <-> (N - i) mod N)
    m = (N - np.arange(N)) % N
    E3h = 0.5 * (E3 + np.conj(E3[m][:, m][:, :, m]))
    sampled_h = sampled | sampled[m][:, m]
    return E3h, sampled_h


def support3d(S2: np.ndarray, theta) -> np.ndarray:
    """Intersection of the back-projected 2D supports (Np, N, N) [n][z][t] -> (N, N, N) [z][y][x]."""
    Np, N, _ = S2.shape
    r = np.arange(N, dtype=np.float64) - N // 2
    yc, xc = r[:, None], r[None, :]
    S3 = np.ones((N, N, N), bool)
    for n in range(Np):
        s, c = math.sin(float(theta[n])), math.cos(float(theta[n]))
        t = np.floor(((yc * c) - (xc * s)) + 0.5).astype(np.int64) + N // 2      # (y, x)
        inside = (t >= 0) & (t < N)
        tt = np.clip(t, 0, N - 1)
        S3 &= inside[None, :, :] & S2[n][:, tt]                                    # [z][y][x]
    return S3


def shrinkwrap3d(V: np.ndarray, sigma: float, threshold: float) -> np.ndarray:
    k = C.gaussian_window(sigma)
    W = (len(k) - 1) // 2
    b = V.astype(np.float64)
    for ax in range(3):
        acc = np.zeros_like(b)
        for d in range(-W, W + 1):
            acc += k[d + W] * np.roll(b, d, axis=ax)
        b = acc
    return b >= threshold * b.max()


def refine(V0, E3, sampled, S3, n_iter, positivity=True, shrink_every=0, sigma=1.0, threshold=0.1):
    """n_iter error-reduction iterations from V0 (centred); returns (V, final support)."""
    V = np.asarray(V0, dtype=np.float64).copy()
    Ef = F.shift_to_native(E3, (-3, -2, -1))
    mask = F.shift_to_native(sampled, (-2, -1))[None, :, :]
    S = S3.copy()
    for it in range(1, n_iter + 1):
        G = F.fftn3(F.shift_to_native(V, (-3, -2, -1)))
        G = np.where(mask, Ef, G)
        V = np.real(F.shift_to_centred(F.ifftn3(G), (-3, -2, -1)))
        keep = S & (V >= 0) if positivity else S
        V = np.where(keep, V, 0.0)
        if shrink_every and it % shrink_every == 0:
            S = shrinkwrap3d(V, sigma, threshold)
    return V, S
