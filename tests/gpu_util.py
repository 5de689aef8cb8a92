"""Helpers shared by the GPU parity tests (no test functions here)."""
from __future__ import annotations

import sys

import numpy as np


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm device (torch.cuda.is_available() is False)")
    return torch


def banner(msg):
    """Name the case before each GPU step (flushed, so it survives a crash)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def per_angle_rel(a, b):
    """Relative L2 of every plane of a stack of N x N planes (leading axes: guesses, angles); a
    plane whose reference is zero (an absent angle) is measured by its absolute norm."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    a2 = a.reshape(-1, a.shape[-2] * a.shape[-1])
    b2 = b.reshape(-1, b.shape[-2] * b.shape[-1])
    nb = np.linalg.norm(b2, axis=1)
    return np.linalg.norm(a2 - b2, axis=1) / np.where(nb > 0, nb, 1.0)


def scan_rel(a, b):
    """Error of a whole scan of objects, checked against a tolerance `tol`: the larger of the
    relative L2 over all angles and half the largest per-angle relative L2.  So the whole scan must
    be within tol and every single angle within 2 tol: one bad angle is not diluted by the others,
    while the FP32 rounding of a run of several iterations, which concentrates on the angles whose
    support-edge decisions it perturbs, gets a factor of two per angle."""
    return max(rel_l2(a, b), 0.5 * float(per_angle_rel(a, b).max()))


def run_gpu(scan, n_iter_schedule, *, real, amp=0, alpha=(0.2, 0.6, 0.2), n_ei=10, wrap=0, positivity=True,
            seed=None, errors=True, device_inputs=True, plan=None):
    """Submit a scan and run [(n_iter, algo, beta), ...]; returns (plan, objects (np), errors list)."""
    torch = require_gpu()
    import paper_2402_05283_amd as cp
    N, Np = scan["N"], scan["Np"]
    seed = scan["phase_seed"] if seed is None else seed
    if plan is None:
        plan = cp.Plan(N, Np, theta=scan["theta"], alpha=alpha, n_ei=n_ei, wrap=wrap, positivity=positivity,
                       real=real, amp=amp, seed=seed)
        if device_inputs:
            I = torch.from_numpy(scan["I"]).cuda()
            S = torch.from_numpy(scan["support"]).cuda()
        else:
            I, S = scan["I"], scan["support"]
        plan.submit(0, I, S)
    errs = []
    for n_iter, algo, beta in n_iter_schedule:
        errs.append(plan.iterate(n_iter, algo, beta, errors=errors))
    torch.cuda.synchronize()
    obj = plan.objects().cpu().numpy()
    return plan, obj, errs


def run_oracle(scan, n_iter_schedule, *, alpha=(0.2, 0.6, 0.2), n_ei=10, wrap=0, positivity=True, seed=None):
    from oracle import cpra as C
    N, Np = scan["N"], scan["Np"]
    seed = scan["phase_seed"] if seed is None else seed
    o = C.Oracle(N, Np, theta=scan["theta"], alpha=alpha, n_ei=n_ei, wrap=wrap, positivity=positivity, seed=seed)
    o.submit(0, scan["I"], scan["support"])
    errs = [o.iterate(n, a, b) for n, a, b in n_iter_schedule]
    return o, errs


SELF_CONJ = lambda N: [(0, 0), (0, N // 2), (N // 2, 0), (N // 2, N // 2)]


def reference_step(g_prev, A, S, *, algo, beta, positivity, estimate, flips=()):
    """One oracle iteration of one angle from its (coupled) iterate g_prev, optionally with the
    sign of the projected value flipped at the given self-conjugate frequencies."""
    from oracle import cpra as C
    G = C.forward(g_prev)
    Gp = C.modulus_projection(G, A)
    for q in flips:
        Gp[q] = -Gp[q]
    gp = C.inverse_real(Gp)
    return C.real_space_update(g_prev, gp, S, algo, beta, positivity, estimate), gp, G


def last_step_parity(gpu_obj, orc, *, algo, beta, estimate, amb=1e-5, ampF=None, angles=None):
    """Relative L2 of one iteration's result against the oracle, accepting the two kinds of
    legitimately ambiguous decisions:
      * a self-conjugate frequency (G real there) whose |G| is within `ampF` of the angle's RMS |G|
        may take either sign of the projected value;
      * a pixel whose g' is within `amb` of the angle's RMS g' may take either HIO branch.
    `orc` provides g_prev (iterate entering the step), A, S, positivity.
    Returns (relative L2 over decided pixels: the larger of the whole-scan value and the largest
    per-angle value; ambiguous pixel count; all ambiguous pixels valid; flips used)."""
    import itertools
    ampF = amb if ampF is None else ampF
    gpu_obj = np.asarray(gpu_obj, dtype=np.float64)
    angles = range(gpu_obj.shape[0]) if angles is None else angles
    num = den = 0.0
    worst = 0.0
    namb = 0
    valid = True
    used = []
    for n in angles:
        N = gpu_obj.shape[-1]
        kw = dict(algo=algo, beta=beta, positivity=orc.positivity, estimate=estimate)
        ref, gp, G = reference_step(orc.g_prev[n], orc.A[n], orc.S[n], **kw)
        rmsG = np.sqrt(np.mean(np.abs(G) ** 2))
        amb_q = [q for q in SELF_CONJ(N) if abs(G[q]) <= ampF * rmsG and orc.A[n][q] >= 0]
        best = (np.linalg.norm(gpu_obj[n] - ref), ref, gp, ())
        for r in range(1, len(amb_q) + 1):
            for fl in itertools.combinations(amb_q, r):
                alt, agp, _ = reference_step(orc.g_prev[n], orc.A[n], orc.S[n], flips=fl, **kw)
                d = np.linalg.norm(gpu_obj[n] - alt)
                if d < best[0]:
                    best = (d, alt, agp, fl)
        _, ref, gp, fl = best
        if fl:
            used.append((n, fl))
        rms = np.sqrt(np.mean(gp ** 2))
        ambiguous = (np.abs(gp) <= amb * max(rms, 1e-300)) & orc.S[n]
        if estimate or algo == 1:
            other = np.where(gp >= 0, 0.0, gp)
        else:
            other = np.where(gp >= 0, orc.g_prev[n] - beta * gp, gp)
        ok = np.isclose(gpu_obj[n], ref, rtol=1e-3, atol=1e-3 * rms) | np.isclose(gpu_obj[n], other, rtol=1e-3,
                                                                              atol=1e-3 * rms)
        valid = valid and bool(np.all(ok[ambiguous]))
        keep = ~ambiguous
        dn = float(np.sum((gpu_obj[n][keep] - ref[keep]) ** 2))
        rn = float(np.sum(ref[keep] ** 2))
        worst = max(worst, float(np.sqrt(dn / max(rn, 1e-300))))
        num += dn
        den += rn
        namb += int(ambiguous.sum())
    return max(float(np.sqrt(num / max(den, 1e-300))), worst), namb, valid, used
