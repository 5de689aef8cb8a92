"""Serving loop on the GPU: each scan's volume is the same alone and in the mix (bit-exact: the
schedule is logical, and cpra_iterate_batch runs each plan's own kernels in its own order), and
equals the plain sequential schedule run through one plan."""
import numpy as np
import pytest

from gpu_util import banner, require_gpu
from synth import make_scan

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _jobs(torch, serve, scans, fps, starts, seeds):
    jobs = []
    for sc, t0, seed in zip(scans, starts, seeds):
        I = torch.from_numpy(sc["I"]).cuda()
        S = torch.from_numpy(sc["support"]).cuda()
        jobs.append(serve.Job(t0, sc["N"], sc["Np"], (lambda n, I=I, S=S: (I[n:n + 1], S[n:n + 1])), fps,
                              seed=seed, theta=sc["theta"]))
    torch.cuda.synchronize()
    return jobs


def test_served_volumes_same_alone_and_in_the_mix(torch):
    import paper_2402_05283_amd as cp
    from paper_2402_05283_amd import serve
    scans = [make_scan(1, N=64, Np=8), make_scan(1, N=128, Np=6), make_scan(1, N=64, Np=5)]
    kw = dict(n_ei=5, r_frame=10, r_final=20)
    seeds = [sc["phase_seed"] + i for i, sc in enumerate(scans)]

    banner("serve: sequential reference through one plan")
    ref = []
    for i, sc in enumerate(scans):
        p = cp.Plan(sc["N"], sc["Np"], theta=sc["theta"], n_ei=5, seed=seeds[i])
        I = torch.from_numpy(sc["I"]).cuda()
        S = torch.from_numpy(sc["support"]).cuda()
        for n in range(sc["Np"]):
            p.submit(n, I[n:n + 1], S[n:n + 1])
            p.iterate(10 + (20 if n == sc["Np"] - 1 else 0), cp.HIO, 0.9)
        ref.append(p.assemble_volume().cpu().numpy())

    banner("serve: each scan alone")
    for i, sc in enumerate(scans):
        srv = serve.Server(1 << 34, **kw)
        (done,) = serve.replay(srv, _jobs(torch, serve, [sc], 400.0, [0.0], [seeds[i]]))
        torch.cuda.synchronize()
        assert np.array_equal(done.volume.cpu().numpy(), ref[i])

    banner("serve: all three together, budget for two at a time")
    fps = [serve.Server.footprint(sc["N"], sc["Np"], n_ei=5) for sc in scans]
    srv = serve.Server(sorted(fps)[-1] + sorted(fps)[-2], **kw)
    done = serve.replay(srv, _jobs(torch, serve, scans, 400.0, [0.0, 0.002, 0.004], seeds))
    torch.cuda.synchronize()
    for i, d in enumerate(done):
        assert d.latency_s is not None and d.latency_s >= 0
        assert np.array_equal(d.volume.cpu().numpy(), ref[i])
    assert srv.used == 0 and not srv.busy()
