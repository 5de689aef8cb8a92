"""cpra_refine_volume_noalloc (the refinement with its scratch in a fixed device array, for callers
that cannot allocate) against cpra_refine_volume with a caller workspace, through the C ABI (needs
an MI355X).  Two calls in a row, the second on a smaller plan, so the shared scratch holds the
first call's contents when the second starts; an F64 plan; and the size limit."""
import numpy as np
import pytest

from gpu_util import banner, require_gpu
from synth import make_scan

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _plan(cp, torch, N, Np, real=0):
    scan = make_scan(1, N=N, Np=Np)
    plan = cp.Plan(N, Np, theta=scan["theta"], n_ei=2, real=real, seed=scan["phase_seed"])
    plan.submit(0, torch.from_numpy(scan["I"]).cuda(), torch.from_numpy(scan["support"]).cuda())
    plan.iterate(4, cp.HIO, 0.9)
    return plan


def test_noalloc_matches_workspace_entry_point(torch):
    import paper_2402_05283_amd as cp
    for N, Np, real, shrink in ((128, 6, 0, 2), (64, 4, 0, 0), (64, 5, 1, 2)):
        banner(f"refine noalloc N={N} Np={Np} real={real} shrink={shrink}")
        plan = _plan(cp, torch, N, Np, real)
        ref = plan.refine_volume(3, shrink_every=shrink, sigma=1.0, threshold=0.1)
        out = torch.full((N, N, N), float("nan"), dtype=ref.dtype, device=ref.device)
        plan.refine_volume_noalloc(3, out, shrink_every=shrink, sigma=1.0, threshold=0.1)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.abs(b).max() > 0
        assert np.array_equal(a, b)


def test_noalloc_rejects_plans_beyond_the_scratch(torch):
    import paper_2402_05283_amd as cp
    banner("refine noalloc size limit")
    plan = _plan(cp, torch, 256, 3)
    out = torch.empty((256, 256, 256), dtype=torch.float32, device="cuda")
    with pytest.raises(cp.CpraError) as e:
        plan.refine_volume_noalloc(1, out)
    assert e.value.status == -5 and "fixed refinement scratch" in str(e.value)
