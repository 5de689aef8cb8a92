"""Exact voxel projections at right angles (oracle pins for the Fourier slice theorem).

TEST INFRASTRUCTURE ONLY (see cpra.py).

For a voxel object O[z][y][x] (centred, coordinate = index - N/2) the PO at
angle theta sums along d = (cos t, sin t, 0) and is indexed by the
transverse coordinate along e_t = (-sin t, cos t, 0).  At multiples of 90
degrees the rays run along grid lines, so the projection is an exact sum:
  0   deg: d = +x, e_t = +y  -> PO[z][t] = sum_x O[z][t][x]
  90  deg: d = +y, e_t = -x  -> PO[z][t] = sum_y O[z][y][-t]
  180 deg: d = -x, e_t = -y  -> PO[z][t] = sum_x O[z][-t][x]
  270 deg: d = -y, e_t = +x  -> PO[z][t] = sum_y O[z][y][t]
(-t means index (N - t) mod N.)
"""
from __future__ import annotations

import numpy as np


def project_right_angle(O: np.ndarray, quarter_turns: int) -> np.ndarray:
    N = O.shape[-1]
    neg = (N - np.arange(N)) % N
    q = quarter_turns % 4
    if q == 0:
        return O.sum(axis=2)
    if q == 1:
        return O.sum(axis=1)[:, neg]
    if q == 2:
        return O.sum(axis=2)[:, neg]
    return O.sum(axis=1)
