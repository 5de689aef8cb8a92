"""The cell scan at its full size, in the launch configuration the benchmark times (N = 512,
N_p = 360, FP32, HIO beta 0.9 with the Eq. 4 coupling every 10 iterations, 200 iterations, then
step D), checked on sampled angles and voxels that the oracle computes one by one, and by
properties that hold at any size (needs an MI355X).

Sampled angles: both angles at the 180-degree seam (their coupling takes the t-mirrored
neighbour), their ring neighbours, and two inside the ring."""
from types import SimpleNamespace

import numpy as np
import pytest

from gpu_util import banner, last_step_parity, rel_l2, require_gpu
from synth import make_scan

pytestmark = pytest.mark.gpu

SAMPLE = (0, 1, 117, 180, 358, 359)
ALPHA = (0.2, 0.6, 0.2)


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def test_full_size_workload(torch):
    import paper_2402_05283_amd as cp
    from oracle import cpra as C
    from oracle import stepd as D
    banner("full size: generating the N=512 Np=360 cell scan")
    scan = make_scan(4)
    N, Np, seed = scan["N"], scan["Np"], scan["phase_seed"]
    assert (N, Np) == (512, 360)
    assert np.allclose(scan["theta"], np.pi * np.arange(Np) / Np)     # the plan's default angles

    banner("full size: plan, submit, initial objects")
    plan = cp.Plan(N, Np, n_ei=10, seed=seed)                           # the benchmark's plan
    plan.submit(0, torch.from_numpy(scan["I"]).cuda(), torch.from_numpy(scan["support"]).cuda())
    torch.cuda.synchronize()
    w0 = plan.objects().cpu().numpy()
    need = sorted({(n + d) % Np for n in SAMPLE for d in (-1, 0, 1)})
    A = {n: C.amplitudes(scan["I"][n]) for n in need}
    S = {n: scan["support"][n] != 0 for n in need}
    X0 = {n: C.initial_object(A[n], seed, n) for n in need}
    for n in need:
        assert rel_l2(w0[n], X0[n]) <= 1e-6, n

    banner("full size: first iteration (coupling of W_0 across the seam, HIO)")
    err = plan.iterate(1, cp.HIO, 0.9, errors=True)
    torch.cuda.synchronize()
    g1 = plan.objects().cpu().numpy()
    weights = C.coupling_weights(Np, np.ones(Np, bool), ALPHA, C.WRAP_MIRROR)
    g_prev = {}
    for n in SAMPLE:
        (l, wl, ml), w0n, (r, wr, mr) = weights[n]
        xl = C.mirror_t(X0[l]) if ml else X0[l]
        xr = C.mirror_t(X0[r]) if mr else X0[r]
        g_prev[n] = wl * xl + w0n * X0[n] + wr * xr
    assert weights[0][0][2] and weights[Np - 1][2][2]                   # the seam is exercised
    orc = SimpleNamespace(g_prev=g_prev, A=A, S=S, positivity=True)
    rel, namb, valid, flips = last_step_parity(g1, orc, algo=C.HIO, beta=0.9, estimate=False, amb=1e-5,
                                               angles=SAMPLE)
    print(f"first iteration: rel {rel:.2e}, ambiguous pixels {namb}, sign-ambiguous frequencies {flips}")
    assert valid and namb <= len(SAMPLE) * N * N * 1e-4
    assert rel <= 1e-5
    for n in SAMPLE:
        ref = C.fourier_error(C.forward(g_prev[n]), A[n])
        assert abs(err[0, n] - ref) <= 1e-5 * ref, n
    del g1, w0

    banner("full size: 199 more iterations, step D")
    plan.iterate(199, cp.HIO, 0.9)
    vol = torch.empty((N, N, N), dtype=torch.float32, device="cuda")
    plan.assemble_volume(vol)
    torch.cuda.synchronize()
    assert plan.k == 200
    obj = plan.objects().cpu().numpy()
    # iteration 200 ends an episode: the objects are the estimates g' 1_gamma
    assert np.all(np.isfinite(obj))
    assert np.all(obj[scan["support"] == 0] == 0)
    assert obj.min() >= 0

    banner("full size: step D at sampled voxels")
    rng = np.random.default_rng(512)
    pts = np.concatenate([rng.integers(N // 4, 3 * N // 4, size=(16, 3)), rng.integers(0, N, size=(6, 3)),
                          np.array([[N // 2] * 3, [0, 0, 0], [N - 1, N // 2, 3]])])
    idx = torch.from_numpy(pts).long().cuda()
    got = vol[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
    del vol
    ref = D.volume_at(obj.astype(np.float64), scan["theta"], pts)
    assert np.all(np.isfinite(got))
    assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max()
