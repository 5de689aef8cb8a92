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


def _run_er(scan, perturb, seed, n_iter=20):
    o = C.Oracle(scan["N"], scan["Np"], theta=scan["theta"], seed=scan["phase_seed"])
    o.submit(0, scan["I"], scan["support"])
    if perturb:
        rng = np.random.default_rng(seed)
        o.g = o.g * (1.0 + perturb * rng.standard_normal(o.g.shape))
    o.iterate(n_iter, C.ER, 0.0)
    return o.g


def test_er_amplifies_a_single_fp32_rounding(scan_c1):
    """ER (with positivity) over 20 iterations and two couplings: one relative perturbation of the
    random start at FP32 rounding level (6e-8, once, pixel by pixel) moves the result by about
    1e-5 over the whole scan and up to about 1e-4 on single angles, because pixels whose g' sits
    near 0 take the other side of the positivity decision.  An FP32 run rounds at every step, so
    the whole-run FP32 ER comparison with the oracle needs a tolerance of a few 1e-4."""
    a = _run_er(scan_c1, 0.0, 0)
    whole, worst = [], []
    for seed in (1, 2, 3):
        b = _run_er(scan_c1, 6e-8, seed)
        whole.append(float(np.linalg.norm(b - a) / np.linalg.norm(a)))
        worst.append(max(float(np.linalg.norm(b[n] - a[n]) / np.linalg.norm(a[n])) for n in range(a.shape[0])))
    print("whole-scan", [f"{v:.1e}" for v in whole], "worst angle", [f"{v:.1e}" for v in worst])
    assert max(whole) >= 1e-5 and max(worst) >= 5e-5
    assert max(whole) <= 1e-4
