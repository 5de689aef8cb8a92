"""Seeded non-centrosymmetric inputs for the GPU parity tests (no test functions here).

Poisson noise breaks I(q) = I(-q) pixel by pixel, and a beamstop that is not
symmetric about the origin leaves pairs (q, -q) with exactly one measured
member.  Both exercise the Hermitian-pair form of the modulus projection: the
pair packing of the amplitudes, the packed DC/Nyquist column and the
one-sided unmeasured rule.  Holds none of the method's arithmetic.
"""
from __future__ import annotations

import numpy as np

from synth import make_scan


def one_sided_beamstop(I):
    """Mark off-centre blocks of every map unmeasured (I = -1) whose point mirrors stay measured.

    Centred index c = N/2 is frequency 0.  Blocks: an interior block in the upper-left quadrant,
    rows of the zero-frequency column (u = 0) with w > 0 only, and rows of the Nyquist column
    (u = -N/2, centred index 0) with w > 0 only.  The Nyquist column is its own mirror in u, so
    its unmeasured rows w pair with measured rows -w."""
    I = np.array(I, dtype=np.float32, copy=True)
    N = I.shape[-1]
    c = N // 2
    b = max(2, N // 32)
    I[:, c - 3 * b:c - 2 * b, c - 5 * b:c - 3 * b] = -1.0      # w < 0, u < 0 block
    I[:, c + 2:c + 2 + b, c] = -1.0                            # u = 0, w in [2, 2 + b)
    I[:, c + 1:c + 1 + b, 0] = -1.0                            # u = -N/2, w in [1, 1 + b)
    return I


def asymmetry_counts(I):
    """(pixels whose amplitude differs from their point mirror's, pairs with exactly one measured
    member, the same two counts restricted to the u = 0 and u = -N/2 columns)."""
    I = np.asarray(I, dtype=np.float64)
    N = I.shape[-1]
    c = N // 2
    idx = (2 * c - np.arange(N)) % N                 # centred index of -q
    M = I[..., idx, :][..., :, idx]
    meas, mmeas = I >= 0, M >= 0
    diff = meas & mmeas & (I != M)
    one = meas ^ mmeas
    cols = [c, 0]
    return (int(diff.sum()), int(one.sum()), int(diff[..., cols].sum()), int(one[..., cols].sum()))


def noisy_scan(config, N=None, Np=None, peak=1e6, beamstop=False, **kw):
    scan = make_scan(config, N=N, Np=Np, peak=peak, **kw)
    if beamstop:
        scan = dict(scan, I=one_sided_beamstop(scan["I"]))
    return scan
