"""How far two correct implementations of HIO can drift apart on the 64^3 / 16-angle scan.

HIO's update off the object constraint, g - beta g', is an expansive feedback step, and which
pixels fall on the constraint (support and g' >= 0) is a sign decision.  A perturbation of the
random start at the level of FP64 rounding therefore grows geometrically until the sign
decisions differ, after which the two runs follow different trajectories.  This is a property of
the algorithm, measured here on the oracle against itself, and it is why a GPU run in FP32 (or in
FP64 with another summation order) is compared with the oracle step by step, from the oracle's own
state, and whole HIO runs only over the first few tens of iterations.
"""
import numpy as np

from oracle import cpra as C


def _run(scan, perturb, checkpoints):
    o = C.Oracle(scan["N"], scan["Np"], theta=scan["theta"], seed=scan["phase_seed"])
    o.submit(0, scan["I"], scan["support"])
    if perturb:
        rng = np.random.default_rng(123)
        rms = np.sqrt(np.mean(o.g ** 2))
        o.g = o.g + perturb * rms * rng.standard_normal(o.g.shape)
    out, k = {}, 0
    for c in checkpoints:
        o.iterate(c - k, C.HIO, 0.9)
        k = c
        out[c] = o.g.copy()
    return out


def test_hio_amplifies_a_rounding_level_perturbation(scan_c1):
    checks = [10, 30, 50, 100, 200]
    a = _run(scan_c1, 0.0, checks)
    b = _run(scan_c1, 1e-15, checks)
    rel = {c: float(np.linalg.norm(a[c] - b[c]) / np.linalg.norm(a[c])) for c in checks}
    print("relative L2 between the runs:", {c: f"{v:.1e}" for c, v in rel.items()})
    # early on the runs agree far beyond FP32 rounding ...
    assert rel[10] <= 1e-10
    assert rel[30] <= 1e-8
    # ... and by the end of the 200-iteration schedule they are different reconstructions
    assert rel[200] >= 1e-3
    assert rel[200] >= 1e5 * rel[30]
