"""GPU parity on non-centrosymmetric data (needs an MI355X).

Noise-free intensities satisfy I(q) = I(-q) exactly, so they never exercise the Hermitian-pair form
of the modulus projection with two different amplitudes.  These tests use inputs where that
symmetry is broken, as in measured data (Eq. 1 gives I = |E|^2; the paper's measured-cell
reconstruction has photon noise and a beamstop):

* Poisson noise (the 256^3 polyhedron scan, 180 angles, 1e6 photons at the peak), so that A(q) and
  A(-q) differ pixel by pixel, also on the packed DC/Nyquist column;
* a beamstop that is not point-symmetric, so that pairs (q, -q) have exactly one measured member,
  on interior pixels and on the u = 0 and u = -N/2 columns.

Every test first asserts that its input has such pixels.  Tolerances are those of the other
parity tests: one iteration 1e-5 (FP32) / 1e-12 (FP64), whole ER runs 1e-4 (FP32); every bound is
on the whole-scan relative L2, with every single angle within twice the bound.
"""
from types import SimpleNamespace

import numpy as np
import pytest

from gpu_util import banner, last_step_parity, rel_l2, require_gpu, run_gpu, run_oracle, scan_rel
from noisy_inputs import asymmetry_counts, noisy_scan

pytestmark = pytest.mark.gpu

F32, F64 = 0, 1
HIO, ER = 0, 1
ALPHA = (0.2, 0.6, 0.2)


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _state_step_check(torch, plan, scan, X, sample, algo, beta, *, boundary, estimate, tol):
    """One GPU iteration from the plan's current state X (all angles, as read back), checked on the
    sampled angles against one oracle iteration from the same state: Eq. 4 over X at a boundary,
    then the 2D iteration.  Also checks E_F of that iteration."""
    from oracle import cpra as C
    Np = scan["Np"]
    if boundary:
        g_prev_all = C.couple(X, np.ones(Np, bool), ALPHA, C.WRAP_MIRROR)
    else:
        g_prev_all = X
    err = plan.iterate(1, algo, beta, errors=True)
    torch.cuda.synchronize()
    got = plan.objects().cpu().numpy()
    A = {n: C.amplitudes(scan["I"][n]) for n in sample}
    S = {n: scan["support"][n] != 0 for n in sample}
    orc = SimpleNamespace(g_prev={n: g_prev_all[n] for n in sample}, A=A, S=S, positivity=True)
    rel, namb, valid, flips = last_step_parity(got, orc, algo=algo, beta=beta, estimate=estimate, amb=1e-5,
                                               angles=sample)
    print(f"  step: rel {rel:.2e}, ambiguous pixels {namb}, sign-ambiguous frequencies {flips}")
    assert valid and namb <= len(sample) * scan["N"] ** 2 * 1e-4
    assert rel <= tol
    for n in sample:
        ref = C.fourier_error(C.forward(orc.g_prev[n]), A[n])
        assert abs(err[0, n] - ref) <= tol * ref, (n, err[0, n], ref)
    return got


def test_polyhedron_poisson_trajectory(torch):
    """The 256^3 polyhedron scan with Poisson noise (N = 256, 180 angles), FP32: initial objects and
    the first coupled iteration against the oracle's own start; then one GPU iteration from the
    GPU's own state at k = 9 (episode estimate), 10 (boundary), 100 (boundary), 499 (estimate)
    of HIO and at 500 (boundary) of ER, each against one oracle iteration from that state."""
    import paper_2402_05283_amd as cp
    from oracle import cpra as C
    banner("noisy polyhedron: generating N=256 Np=180, Poisson 1e6")
    scan = noisy_scan(2)
    N, Np, seed = scan["N"], scan["Np"], scan["phase_seed"]
    assert (N, Np) == (256, 180)
    diff, one, diff_cols, _ = asymmetry_counts(scan["I"])
    print(f"pixels with I(q) != I(-q): {diff} (u = 0 and -N/2 columns: {diff_cols})")
    assert diff > 0.05 * scan["I"].size and diff_cols > 0

    sample = (0, 1, 2, 57, 89, 90, 133, 177, 178, 179)        # both sides of the seam, and inside
    need = sorted({(n + d) % Np for n in sample for d in (-1, 0, 1)})
    banner("noisy polyhedron: initial objects")
    plan = cp.Plan(N, Np, theta=scan["theta"], alpha=ALPHA, n_ei=10, seed=seed)
    plan.submit(0, torch.from_numpy(scan["I"]).cuda(), torch.from_numpy(scan["support"]).cuda())
    torch.cuda.synchronize()
    w0 = plan.objects().cpu().numpy()
    X0 = np.zeros((Np, N, N))
    for n in need:
        X0[n] = C.initial_object(C.amplitudes(scan["I"][n]), seed, n)
        assert rel_l2(w0[n], X0[n]) <= 1e-6, n

    banner("noisy polyhedron: first iteration (coupling of W_0 across the seam, HIO)")
    _state_step_check(torch, plan, scan, X0, sample, HIO, 0.9, boundary=True, estimate=False, tol=1e-5)

    for k, algo, beta in ((9, HIO, 0.9), (10, HIO, 0.9), (100, HIO, 0.9), (499, HIO, 0.9), (500, ER, 0.0)):
        plan.iterate(k - plan.k, HIO, 0.9)
        assert plan.k == k
        torch.cuda.synchronize()
        X = plan.objects().cpu().numpy().astype(np.float64)
        banner(f"noisy polyhedron: step from the GPU state at k={k} algo={algo}")
        _state_step_check(torch, plan, scan, X, sample, algo, beta, boundary=k % 10 == 0,
                          estimate=(k + 1) % 10 == 0, tol=1e-5)


@pytest.mark.parametrize("real", [F32, F64])
def test_polyhedron_poisson_runs(torch, real):
    """Whole runs on 16 angles of the noisy polyhedron (N = 256, the seam between the last and the
    first angle): 20 ER iterations from W_0 in FP32 (1e-4); 12 HIO then 8 ER in FP64 (1e-9)."""
    scan = noisy_scan(2, Np=16)
    diff, _, diff_cols, _ = asymmetry_counts(scan["I"])
    assert diff > 0 and diff_cols > 0
    sched = [(20, ER, 0.0)] if real == F32 else [(12, HIO, 0.9), (8, ER, 0.0)]
    banner(f"noisy polyhedron run real={real} {sched}")
    _, obj, errs = run_gpu(scan, sched, real=real)
    o, oerrs = run_oracle(scan, sched)
    tol = 1e-4 if real == F32 else 1e-9
    r = scan_rel(obj, o.g)
    print(f"run real={real}: {r:.2e}")
    assert r <= tol
    for a, b in zip(errs, oerrs):
        assert rel_l2(a, b) <= tol


@pytest.mark.parametrize("real", [F32, F64])
@pytest.mark.parametrize("N,Np", [(64, 5), (512, 3), (1024, 3)])
def test_one_sided_beamstop(torch, N, Np, real):
    """Poisson noise plus a beamstop that is not point-symmetric (interior block, rows of the u = 0
    and u = -N/2 columns on one side of w = 0 only): pairs with exactly one measured member take
    the measured member's projection and keep G for the other.  One coupled HIO iteration from
    W_0, then (N <= 512, FP64) a short run through an estimate and a second boundary (n_ei = 3).
    N = 64 takes the one-lane column pass, 512 the two-lane and 1024 the four-lane step 2."""
    scan = noisy_scan(1, N=N, Np=Np, beamstop=True)
    diff, one, diff_cols, one_cols = asymmetry_counts(scan["I"])
    print(f"N={N}: asymmetric pixels {diff}, one-sided pairs {one} (columns u = 0, -N/2: {diff_cols}, {one_cols})")
    assert diff > 0 and one > 0 and diff_cols > 0 and one_cols > 0
    banner(f"one-sided beamstop N={N} real={real}")
    kw = dict(alpha=(0.1, 0.6, 0.3), n_ei=3)
    _, obj, errs = run_gpu(scan, [(1, HIO, 0.9)], real=real, **kw)
    o, oerrs = run_oracle(scan, [(1, HIO, 0.9)], **kw)
    tol = 1e-5 if real == F32 else 1e-12
    r, namb, valid, flips = last_step_parity(obj, o, algo=HIO, beta=0.9, estimate=False,
                                             amb=1e-5 if real == F32 else 1e-12)
    print(f"  one iteration: rel {r:.2e}, ambiguous {namb}, flips {flips}")
    assert valid and namb <= obj.size * 1e-4
    assert r <= tol
    assert rel_l2(errs[0], oerrs[0]) <= tol
    if real == F64 and N <= 512:
        sched = [(7, HIO, 0.9)]
        banner(f"one-sided beamstop N={N} real={real}: 7 iterations")
        _, obj7, errs7 = run_gpu(scan, sched, real=real, **kw)
        o7, oerrs7 = run_oracle(scan, sched, **kw)
        r7 = scan_rel(obj7, o7.g)
        print(f"  7 iterations: {r7:.2e}")
        assert r7 <= 1e-10
        assert rel_l2(errs7[0], oerrs7[0]) <= 1e-10


def test_fp16_amplitudes_noisy_n512(torch):
    """FP16 amplitudes on noisy data at N = 512: eight consecutive angles of the 512^3 cell scan with
    Poisson noise at 1e6 photons, one coupled HIO iteration and one ER episode, FP16 amplitudes and
    FP32 amplitudes against the FP64 oracle.  Bounds: FP32 1e-5 / 1e-4, FP16 1e-2 / 2e-2 (binary16
    rounds each amplitude by up to 2^-11 relative)."""
    import paper_2402_05283_amd as cp
    banner("fp16 amplitudes, noisy N=512")
    scan = noisy_scan(4, angle_subset=list(range(100, 108)))
    diff, _, diff_cols, _ = asymmetry_counts(scan["I"])
    assert diff > 0 and diff_cols > 0
    res = {}
    for name, sched in (("hio1", [(1, HIO, 0.9)]), ("er10", [(10, ER, 0.0)])):
        o, _ = run_oracle(scan, sched)
        for amp in (cp.AMP_F32, cp.AMP_F16):
            _, obj, _ = run_gpu(scan, sched, real=F32, amp=amp)
            res[(name, amp)] = scan_rel(obj, o.g)
    print("noisy N=512, 8 angles, relative L2 vs FP64 oracle:",
          {f"{k[0]}/{'fp16' if k[1] else 'fp32'}": f"{v:.2e}" for k, v in res.items()})
    assert res[("hio1", cp.AMP_F32)] <= 1e-5 and res[("er10", cp.AMP_F32)] <= 1e-4
    assert res[("hio1", cp.AMP_F16)] <= 1e-2 and res[("er10", cp.AMP_F16)] <= 2e-2
