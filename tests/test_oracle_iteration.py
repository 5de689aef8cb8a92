"""Pins of the oracle's iteration: closed-form HIO/ER steps, fixed points, monotone ER."""
import numpy as np
import pytest

from oracle import cpra as C
from synth import objects as SO


def _oracle_with_state(g, A, S, alpha=(0.0, 1.0, 0.0), n_ei=1000, positivity=True):
    Np, N, _ = g.shape
    o = C.Oracle(N, Np, alpha=alpha, n_ei=n_ei, positivity=positivity, seed=1)
    o.A[:] = A
    o.S[:] = S
    o.g[:] = g
    o.landed[:] = True
    o.present[:] = True
    return o


def test_modulus_projection_closed_forms():
    rng = np.random.default_rng(0)
    G = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    assert np.abs(C.modulus_projection(G, 3 * np.abs(G)) - 3 * G).max() <= 1e-14
    assert np.array_equal(C.modulus_projection(G, -np.ones((8, 8))), G)
    Z = np.zeros((2, 2), complex)
    assert np.array_equal(C.modulus_projection(Z, np.full((2, 2), 2.0)), np.full((2, 2), 2.0 + 0j))


@pytest.mark.parametrize("algo", [C.HIO, C.ER])
def test_one_step_closed_form(algo):
    """A = 2|F2 g| makes the projection return exactly g' = 2g."""
    rng = np.random.default_rng(1)
    Np, N, beta = 3, 16, 0.9
    g = rng.standard_normal((Np, N, N))
    S = rng.uniform(size=(Np, N, N)) < 0.5
    A = np.stack([2 * np.abs(C.forward(x)) for x in g])
    o = _oracle_with_state(g, A, S)
    err = o.iterate(1, algo, beta)
    gamma = S & (g >= 0)
    if algo == C.HIO:
        exp = np.where(gamma, 2 * g, (1 - 2 * beta) * g)
    else:
        exp = np.where(gamma, 2 * g, 0.0)
    assert np.abs(o.g - exp).max() <= 1e-12
    assert np.abs(err - 0.5).max() <= 1e-12          # sqrt(sum(|G|-2|G|)^2 / sum 4|G|^2)


def test_estimate_at_episode_end_and_positivity_flag():
    rng = np.random.default_rng(2)
    g = rng.standard_normal((2, 8, 8))
    S = rng.uniform(size=(2, 8, 8)) < 0.6
    A = np.stack([np.abs(C.forward(x)) for x in g])
    o = _oracle_with_state(g, A, S, n_ei=1)
    err = o.iterate(1, C.HIO, 0.9)
    assert np.abs(o.g - np.where(S & (g >= 0), g, 0)).max() <= 1e-12
    assert np.abs(err).max() <= 1e-12
    o2 = _oracle_with_state(g, A, S, positivity=False)
    o2.iterate(1, C.HIO, 0.5)
    assert np.abs(o2.g - np.where(S, g, 0.5 * g)).max() <= 1e-12


def test_unmeasured_pixels_leave_spectrum_free():
    rng = np.random.default_rng(3)
    g = rng.standard_normal((1, 8, 8))
    S = np.ones((1, 8, 8), bool)
    o = _oracle_with_state(g, -np.ones((1, 8, 8)), S, positivity=False)
    o.iterate(1, C.HIO, 0.9)
    assert np.abs(o.g - g).max() <= 1e-12


def test_true_object_is_fixed_point(scan_c1):
    """A true PO with its own moduli and a support containing it is unchanged."""
    po = scan_c1["po"][:4]
    S = scan_c1["support"][:4].astype(bool)
    assert np.all(po[~S] == 0) and po.min() >= 0
    A = np.stack([np.abs(C.forward(x)) for x in po])
    o = _oracle_with_state(po, A, S)
    o.iterate(3, C.HIO, 0.9)
    assert np.abs(o.g - po).max() <= 1e-12 * po.max()


def test_axisymmetric_object_fixed_through_coupling():
    """All POs of a z-axisymmetric object are equal and mirror-symmetric: coupling keeps them."""
    N, Np = 32, 6
    ell = SO.Ellipsoids([np.zeros(3)], [np.eye(3)], [np.array([7.0, 7.0, 10.0])], [1.0])
    po = np.stack([ell.project(N, t) for t in np.pi * np.arange(Np) / Np])
    assert np.abs(po - po[0]).max() <= 1e-6 * po.max()
    # exact copies of one exactly mirror-symmetric PO
    p0 = 0.5 * (po[0] + C.mirror_t(po[0]))
    po = np.repeat(p0[None], Np, axis=0)
    S = po > 0
    A = np.stack([np.abs(C.forward(x)) for x in po])
    o = _oracle_with_state(po, A, S, alpha=(0.2, 0.6, 0.2), n_ei=2)
    o.iterate(4, C.HIO, 0.9)
    assert np.abs(o.g - po).max() <= 1e-9 * po.max()


def test_er_error_is_non_increasing(scan_c1):
    I = scan_c1["I"][:3].astype(np.float64)
    S = scan_c1["support"][:3]
    o = C.Oracle(64, 3, alpha=(0.0, 1.0, 0.0), n_ei=10, seed=5)
    o.submit(0, I, S)
    err = o.iterate(40, C.ER)
    # once the iterate has been projected onto the object constraints (after
    # the first step) the Fourier error can only fall (Fienup 1982)
    assert np.all(np.diff(err[1:], axis=0) <= 1e-12)


def test_oracle_reconstructs_c1_reasonably(scan_c1):
    """Sanity only (parity unpinned against the paper, which prints no values)."""
    o = C.Oracle(64, 16, seed=scan_c1["phase_seed"])
    o.submit(0, scan_c1["I"], scan_c1["support"])
    err = o.iterate(200, C.HIO, 0.9)
    assert np.nanmean(err[-1]) < np.nanmean(err[0])


def test_raar_closed_form_step():
    """A = 2|F2 g| makes g' = 2g; RAAR's reflection is then 2g' - g = 3g, so per pixel the step is
    2g where 3g meets the constraints (support, >= 0) and beta g + (1 - 2 beta) 2g elsewhere."""
    rng = np.random.default_rng(4)
    Np, N, beta = 2, 16, 0.9
    g = rng.standard_normal((Np, N, N))
    S = rng.uniform(size=(Np, N, N)) < 0.5
    A = np.stack([2 * np.abs(C.forward(x)) for x in g])
    o = _oracle_with_state(g, A, S)
    o.iterate(1, C.RAAR, beta)
    inside = S & (3 * g >= 0)
    exp = np.where(inside, 2 * g, beta * g + (1 - 2 * beta) * 2 * g)
    assert np.abs(o.g - exp).max() <= 1e-12


def test_raar_with_beta_one_is_hio_without_positivity():
    """Douglas-Rachford (RAAR at beta = 1) and HIO with beta = 1 coincide when the only real-space
    constraint is the support (Bauschke, Combettes and Luke 2002)."""
    rng = np.random.default_rng(5)
    g = rng.standard_normal((2, 16, 16))
    S = rng.uniform(size=(2, 16, 16)) < 0.4
    A = np.stack([np.abs(C.forward(x)) * rng.uniform(0.5, 1.5, (16, 16)) for x in g])
    a = _oracle_with_state(g, A, S, positivity=False)
    b = _oracle_with_state(g, A, S, positivity=False)
    a.iterate(5, C.RAAR, 1.0)
    b.iterate(5, C.HIO, 1.0)
    assert np.abs(a.g - b.g).max() <= 1e-12 * np.abs(b.g).max()


def test_true_object_is_fixed_point_of_raar(scan_c1):
    po = scan_c1["po"][:3]
    S = scan_c1["support"][:3].astype(bool)
    A = np.stack([np.abs(C.forward(x)) for x in po])
    o = _oracle_with_state(po, A, S)
    o.iterate(3, C.RAAR, 0.9)
    assert np.abs(o.g - po).max() <= 1e-12 * po.max()


def test_shrinkwrap_window_and_delta_closed_form():
    """A delta at (z0, t0) blurs to k(z - z0) k(t - t0), so the support kept at a fraction f of the
    maximum is the disc exp(-r^2 / 2 sigma^2) >= f (periodic distance r, inside the window)."""
    k = C.gaussian_window(1.5)
    assert len(k) == 2 * 6 + 1 and abs(k.sum() - 1) < 1e-15 and np.all(np.diff(k[:7]) > 0)
    N, sigma, f = 32, 2.0, 0.3
    g = np.zeros((N, N))
    g[1, N - 2] = 5.0                                  # near a corner: the blur wraps
    S = C.shrinkwrap_support(g, sigma, f)
    dz = np.minimum(np.abs(np.arange(N) - 1), N - np.abs(np.arange(N) - 1))
    dt = np.minimum(np.abs(np.arange(N) - (N - 2)), N - np.abs(np.arange(N) - (N - 2)))
    r2 = dz[:, None] ** 2 + dt[None, :] ** 2
    inside = (dz[:, None] <= 8) & (dt[None, :] <= 8)
    want = inside & (np.exp(-r2 / (2 * sigma ** 2)) >= f - 1e-12)
    assert np.array_equal(S, want)


def test_shrinkwrap_small_sigma_is_a_plain_threshold():
    """sigma -> 0: the window is a single tap, the blur is the identity."""
    rng = np.random.default_rng(6)
    g = rng.uniform(size=(16, 16))
    assert len(C.gaussian_window(0.2)) == 3
    k = C.gaussian_window(0.05)
    assert k[1] == 1.0 and k[0] < 1e-80
    assert np.array_equal(C.shrinkwrap_support(g, 0.05, 0.5), g >= 0.5 * g.max())
