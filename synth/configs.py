"""Seeded scans for the workloads the build is measured on.

Every scan is produced from seeds only: object seed = 1000*config + scan,
noise seed = object seed + 1, initial-phase seed = object seed + 2.
Intensities are I = |F2(PO)|^2 of the exact projections, centred (zero
frequency at index N/2), stored float32; supports are uint8 [z][t], centred.

Workload recipes (they stand in for the paper's layered-oxide particle and
bacterial cell, whose data are not public):
  1  N=64,  Np=16 : 5 random ellipsoids in a ball of radius 24, noise-free,
                    support = disc of radius 24.
  2  N=256, Np=180: convex polyhedron with voids and 5% texture, Poisson
                    noise at 1e6 photons peak, support = 1.2x dilated hull.
  4  N=512, Np=360: cell-like ellipsoidal shell with granules, noise-free,
                    support = projection of the 1.2x dilated outer ellipsoid.
Angles are evenly spaced over 180 degrees about z: theta_n = pi*n/Np.
"""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import objects as obj

DEFAULTS = {1: (64, 16), 2: (256, 180), 4: (512, 360)}


def angles(Np: int) -> np.ndarray:
    return np.pi * np.arange(Np, dtype=np.float64) / Np


def build_object(config: int, scan: int, N: int):
    rng = np.random.default_rng(1000 * config + scan)
    if config == 1:
        k = N / 64.0
        return obj.make_ellipsoids(rng, 5, centre_radius=20.0 * k, semi=(3.0 * k, 10.0 * k),
                                   support_radius=24.0 * k)
    if config == 2:
        return obj.make_polyhedron(rng, N)
    if config == 4:
        return obj.make_cell(rng, N)
    raise ValueError(f"unknown config {config}")


def _support(config, o, N, theta):
    if config == 1:
        c = np.arange(N) - N / 2
        zz, tt = np.meshgrid(c, c, indexing="ij")
        return zz * zz + tt * tt <= (24.0 * N / 64.0) ** 2
    return o.support(N, theta)


def _one_angle(args):
    config, scan, N, theta = args
    o = build_object(config, scan, N)
    po = o.project(N, theta)
    sup = _support(config, o, N, theta)
    spec = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(po)))
    return po, sup, (spec.real ** 2 + spec.imag ** 2)


def make_scan(config: int, scan: int = 0, N: int | None = None, Np: int | None = None,
              angle_subset=None, workers: int | None = None, keep_po: bool = False,
              peak: float | None = None):
    """Return a dict with I (Np,N,N) float32, support (Np,N,N) uint8, theta (Np,) float64.

    `angle_subset` restricts generation to the listed angle indices of the
    full Np-angle scan (the intensities are identical to those of the full
    scan at those indices).
    """
    dN, dNp = DEFAULTS.get(config, (None, None))
    N = N or dN
    Np = Np or dNp
    th = angles(Np)
    idx = np.arange(Np) if angle_subset is None else np.asarray(angle_subset)
    jobs = [(config, scan, N, float(th[i])) for i in idx]
    if workers is None:
        workers = min(len(jobs), max(1, min(16, (os.cpu_count() or 1))))
    if workers > 1 and len(jobs) > 4 and N >= 128:
        with ProcessPoolExecutor(workers) as ex:
            res = list(ex.map(_one_angle, jobs, chunksize=max(1, len(jobs) // (4 * workers))))
    else:
        res = [_one_angle(j) for j in jobs]
    po = np.stack([r[0] for r in res])
    sup = np.stack([r[1] for r in res]).astype(np.uint8)
    inten = np.stack([r[2] for r in res])
    if peak is None and config == 2:
        peak = 1e6
    if peak is not None:
        rng = np.random.default_rng(1000 * config + scan + 1)
        scale = peak / inten.reshape(len(idx), -1).max(axis=1)
        inten = rng.poisson(inten * scale[:, None, None]).astype(np.float64)
    out = {
        "I": inten.astype(np.float32),
        "support": sup,
        "theta": th[idx].copy(),
        "N": N,
        "Np": len(idx),
        "phase_seed": 1000 * config + scan + 2,
    }
    if keep_po:
        out["po"] = po
    return out
