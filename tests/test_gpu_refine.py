"""3D refinement after step D on the GPU against the refinement oracle (needs an MI355X).  The
oracle iterates in plain 3D with its own FFT; the GPU works per z-plane in the (z, k_y, k_x)
domain, so agreement also checks that factorisation.  The oracle starts from the GPU's own
estimates (error reduction contracts, so the comparison is tight)."""
import numpy as np
import pytest

from gpu_util import banner, rel_l2, require_gpu
from synth import make_scan

pytestmark = pytest.mark.gpu

F32, F64 = 0, 1


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.mark.parametrize("real", [F64, F32])
@pytest.mark.parametrize("shrink", [0, 3])
def test_refine_volume(torch, real, shrink):
    import paper_2402_05283_amd as cp
    from oracle import refine as RF
    from oracle import stepd as D
    scan = make_scan(1, Np=8)
    banner(f"refine volume real={real} shrink={shrink}")
    plan = cp.Plan(64, 8, theta=scan["theta"], n_ei=5, real=real, seed=scan["phase_seed"])
    plan.submit(0, scan["I"], scan["support"])
    plan.iterate(10, cp.HIO, 0.9)
    torch.cuda.synchronize()
    obj = plan.objects().cpu().numpy().astype(np.float64)
    vol = plan.refine_volume(6, shrink_every=shrink, sigma=1.0, threshold=0.1)
    torch.cuda.synchronize()
    got = vol.cpu().numpy()
    E3, sampled = RF.measured_grid(obj, scan["theta"])
    V0 = D.assemble_volume(obj, scan["theta"])
    S3 = RF.support3d(scan["support"].astype(bool), scan["theta"])
    ref, _ = RF.refine(V0, E3, sampled, S3, 6, positivity=True, shrink_every=shrink, sigma=1.0, threshold=0.1)
    assert np.abs(ref).max() > 0
    tol = (1e-4 if real == F32 else 1e-10) * (10 if shrink and real == F32 else 1)
    assert rel_l2(got, ref) <= tol
    # zero outside the back-projected support (no shrinking: the support is fixed)
    if not shrink:
        assert np.all(got[~S3] == 0)


def test_refine_volume_n128(torch):
    """N = 128 (a different transform decomposition), FP32, three iterations."""
    import paper_2402_05283_amd as cp
    from oracle import refine as RF
    from oracle import stepd as D
    scan = make_scan(1, N=128, Np=6)
    banner("refine volume N=128")
    plan = cp.Plan(128, 6, theta=scan["theta"], n_ei=2, seed=scan["phase_seed"])
    plan.submit(0, scan["I"], scan["support"])
    plan.iterate(2, cp.HIO, 0.9)
    torch.cuda.synchronize()
    obj = plan.objects().cpu().numpy().astype(np.float64)
    got = plan.refine_volume(3).cpu().numpy()
    E3, sampled = RF.measured_grid(obj, scan["theta"])
    S3 = RF.support3d(scan["support"].astype(bool), scan["theta"])
    ref, _ = RF.refine(D.assemble_volume(obj, scan["theta"]), E3, sampled, S3, 3)
    assert rel_l2(got, ref) <= 1e-4


def test_refine_needs_an_episode_end(torch):
    import paper_2402_05283_amd as cp
    scan = make_scan(1, Np=4)
    banner("refine state check")
    plan = cp.Plan(64, 4, theta=scan["theta"], n_ei=5)
    plan.submit(0, scan["I"], scan["support"])
    plan.iterate(3)
    with pytest.raises(cp.CpraError) as e:
        plan.refine_volume(2)
    assert e.value.status == -4
