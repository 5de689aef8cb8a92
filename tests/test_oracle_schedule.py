"""Pins of the schedule oracle (steps A-C with N_r guesses) against closed forms, the single-guess
oracle and constructed cases (CPU only)."""
import numpy as np
import pytest

from oracle import cpra as C
from oracle import schedule as SC


def test_central_inversion_maps_r_to_minus_r():
    N = 16
    x = np.zeros((N, N))
    x[N // 2 + 3, N // 2 - 5] = 1.0                   # r = (3, -5)
    y = SC.central_inversion(x)
    assert y[N // 2 - 3, N // 2 + 5] == 1.0 and y.sum() == 1.0
    rng = np.random.default_rng(0)
    z = rng.standard_normal((N, N))
    assert np.array_equal(SC.central_inversion(SC.central_inversion(z)), z)
    # same intensities: |F2 X(-r)| = |F2 X|
    assert np.allclose(np.abs(np.fft.fft2(SC.central_inversion(z))), np.abs(np.fft.fft2(z)), atol=1e-12)


def test_mass_centre_and_shift():
    N = 32
    x = np.zeros((N, N))
    x[N // 2 + 3, N // 2 - 5] = 2.0
    assert SC.mass_centre(x) == (3.0, -5.0)
    s = SC.centre_shift(x)
    assert s == (-3, 5)
    assert SC.shift(x, s)[N // 2, N // 2] == 2.0
    # half-integer centre: floor(-c + 1/2) rounds -2.5 up to -2
    y = np.zeros((N, N))
    y[N // 2 + 2, N // 2] = 1.0
    y[N // 2 + 3, N // 2] = 1.0
    assert SC.mass_centre(y) == (2.5, 0.0)
    assert SC.centre_shift(y) == (-2, 0)


def _noop_sets(Np, alpha, wrap, monkeypatch):
    """A GuessSet whose per-PO iterations do nothing, so a sweep is the coupling recurrence alone."""
    gs = SC.GuessSet(8, Np, 1, alpha=alpha, wrap=wrap, n_ei=1)
    monkeypatch.setattr(gs, "iterate_po", lambda r, n, k, a, b: np.zeros(k))
    return gs


def test_sweep_propagates_round_the_ring_in_one_episode(monkeypatch):
    """alpha = (a, 1-a, 0), plain wrap, X_0 = 1 and X_n = 0 elsewhere: the consecutive sweep gives
    X_0 = 1-a, X_n = a^n (1-a) (each PO takes its left neighbour's new value); the data-parallel
    form gives X_1 = a and zero beyond."""
    Np, a = 6, 0.3
    gs = _noop_sets(Np, (a, 1 - a, 0.0), C.WRAP_PLAIN, monkeypatch)
    gs.g[0] = 0.0
    gs.g[0, 0] = 1.0
    gs.sweep(1)
    got = gs.g[0, :, 0, 0]
    assert np.allclose(got, [(1 - a) * a ** n for n in range(Np)], rtol=0, atol=1e-15)
    gj = _noop_sets(Np, (a, 1 - a, 0.0), C.WRAP_PLAIN, monkeypatch)
    gj.g[0] = 0.0
    gj.g[0, 0] = 1.0
    gj.jacobi(1)
    assert np.allclose(gj.g[0, :, 0, 0], [1 - a, a, 0, 0, 0, 0], atol=1e-15)


def test_sweep_uses_new_right_neighbour_at_the_end_and_mirror_at_the_seam(monkeypatch):
    """alpha = (0, 1-b, b): PO Np-1 takes PO 0's value from this same episode, mirrored in t
    across the 180-degree seam.  With X_0 = e (a t-asymmetric profile), X_n = 0 otherwise:
    X_0 -> (1-b) e, X_1..X_{Np-2} -> 0, X_{Np-1} -> b M((1-b) e)."""
    Np, b = 5, 0.25
    gs = _noop_sets(Np, (0.0, 1 - b, b), C.WRAP_MIRROR, monkeypatch)
    e = np.zeros((8, 8))
    e[:, 5] = 1.0                                   # t = +1 from the centre
    gs.g[0] = 0.0
    gs.g[0, 0] = e
    gs.sweep(1)
    assert np.allclose(gs.g[0, 0], (1 - b) * e)
    assert np.all(gs.g[0, 1:Np - 1] == 0)
    want = b * (1 - b) * C.mirror_t(e)
    assert np.allclose(gs.g[0, Np - 1], want)
    assert gs.g[0, Np - 1][:, 3].sum() > 0 and gs.g[0, Np - 1][:, 5].sum() == 0   # t = -1 after the mirror


def test_no_coupling_sweep_and_prereconstruction_match_the_single_guess_oracle(scan_c1):
    """alpha = (0, 1, 0): the sweep is plain per-PO phase retrieval, the same as the data-parallel
    oracle; step A equals a one-angle oracle run; guess 0 starts from the oracle's W_0."""
    Np = 3
    I, S, th = scan_c1["I"][:Np], scan_c1["support"][:Np], scan_c1["theta"][:Np]
    seed = scan_c1["phase_seed"]
    gs = SC.GuessSet(64, Np, 2, theta=th, alpha=(0.0, 1.0, 0.0), n_ei=4, wrap=C.WRAP_PLAIN, seed=seed)
    gs.submit(I, S)
    o = C.Oracle(64, Np, theta=th, alpha=(0.0, 1.0, 0.0), n_ei=4, wrap=C.WRAP_PLAIN, seed=seed)
    o.submit(0, I, S)
    assert np.array_equal(gs.g[0], o.g)
    assert not np.allclose(gs.g[1], gs.g[0])        # other guesses start elsewhere
    gs.sweep(2)
    o.iterate(8)
    assert np.allclose(gs.g[0], o.g, rtol=0, atol=1e-12 * np.abs(o.g).max())
    # step A: 6 iterations of PO 0 alone, estimate last
    gp = SC.GuessSet(64, Np, 1, theta=th, n_ei=4, seed=seed)
    gp.submit(I, S)
    gp.prereconstruct(6)
    o1 = C.Oracle(64, 1, theta=th[:1], alpha=(0.0, 1.0, 0.0), n_ei=6, wrap=C.WRAP_PLAIN, seed=seed)
    o1.submit(0, I[:1], S[:1])
    o1.iterate(6)
    assert np.allclose(gp.g[0, 0], o1.g[0], rtol=0, atol=1e-12 * np.abs(o1.g).max())
    w0 = SC.GuessSet(64, Np, 1, theta=th, seed=seed)
    w0.submit(I, S)
    assert np.array_equal(gp.g[0, 1:], w0.g[0, 1:])


def test_episode_error_is_zero_on_the_true_projections():
    from synth import make_scan
    sc = make_scan(1, Np=3, keep_po=True)
    gs = SC.GuessSet(64, 3, 2, theta=sc["theta"])
    gs.submit(sc["I"], sc["support"])
    gs.g[0] = sc["po"]
    e = gs.episode_errors()
    assert e[0] < 1e-6 < e[1]


def test_merge_undoes_shift_and_inversion_and_drops_the_worst():
    """Guess 1 = guess 0 shifted and centrally inverted (same intensities, same error): the merge
    undoes both and returns guess 0 centred.  Guess 2 is noise (largest error) and is dropped."""
    from synth import make_scan
    sc = make_scan(1, Np=4, keep_po=True)
    po = sc["po"]
    gs = SC.GuessSet(64, 4, 3, theta=sc["theta"])
    gs.submit(sc["I"], sc["support"])
    gs.g[0] = po
    gs.g[1] = np.array([SC.shift(SC.central_inversion(p), (2, -3)) for p in po])
    gs.g[2] = np.random.default_rng(1).random(po.shape)
    merged, keep, inverted = gs.merge(2)
    assert sorted(keep) == [0, 1] and 2 not in keep
    assert inverted[1] is True
    want = np.array([SC.shift(p, SC.centre_shift(p)) for p in po])
    if keep[0] == 1:                                 # the twin may rank first: then guess 0 is inverted
        want = SC.central_inversion(want)
    # the mass centres end within half a pixel of the origin
    for n in range(4):
        c = SC.mass_centre(merged[n])
        assert abs(c[0]) <= 0.5 + 1e-9 and abs(c[1]) <= 0.5 + 1e-9
    assert np.allclose(merged, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_sweep_with_taps_propagates_two_steps(monkeypatch):
    """Five taps (0, a, 1-a-b, 0, b) with no-op iterations: PO 1 takes PO 0's new value and PO 2's
    old one (b); checks that the K-tap sweep reads the most recent objects two slots away."""
    Np, a, b = 6, 0.3, 0.2
    gs = SC.GuessSet(8, Np, 1, taps=(0.0, a, 1 - a - b, 0.0, b), wrap=C.WRAP_PLAIN, n_ei=1)
    monkeypatch.setattr(gs, "iterate_po", lambda r, n, k, al, be: np.zeros(k))
    gs.g[0] = 0.0
    gs.g[0, 2] = 1.0
    gs.sweep(1)
    # PO 0 takes b X_2 (old 1); PO 1 takes a X_0(new) = a b; PO 2 takes a X_1(new) + (1-a-b) = ...
    x0 = b * 1.0
    x1 = a * x0
    x2 = a * x1 + (1 - a - b) * 1.0
    assert np.allclose(gs.g[0, :3, 0, 0], [x0, x1, x2], atol=1e-15)
