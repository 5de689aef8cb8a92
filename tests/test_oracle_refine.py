"""Pins of the 3D refinement oracle: back-projected support closed forms, the error-reduction step
as a projection (idempotent on the step-D volume), the exact object as a fixed point, and the 3D
shrinkwrap of a delta."""
import numpy as np

from oracle import cpra as C
from oracle import geometry as G
from oracle import refine as RF
from oracle import stepd as D


def test_support3d_axis_angles():
    rng = np.random.default_rng(0)
    N = 16
    S2 = rng.uniform(size=(2, N, N)) < 0.6
    S3 = RF.support3d(S2[:1], [0.0])
    assert np.array_equal(S3, np.broadcast_to(S2[0][:, :, None], (N, N, N)))     # t = y at 0 deg
    S3b = RF.support3d(S2[1:], [np.pi / 2])
    x = np.arange(N)
    t = (N // 2 - (x - N // 2))                                                  # t = -x at 90 deg
    want = np.zeros((N, N, N), bool)
    ok = (t >= 0) & (t < N)
    want[:, :, ok] = S2[1][:, t[ok]][:, None, :]
    assert np.array_equal(S3b, want)
    both = RF.support3d(S2, [0.0, np.pi / 2])
    assert np.array_equal(both, S3 & S3b)


def test_refinement_step_is_a_projection():
    """With no real-space constraint the step is the Fourier projection: the step-D volume already
    satisfies it, so one step returns it unchanged."""
    rng = np.random.default_rng(1)
    N, Np = 16, 5
    th = np.pi * np.arange(Np) / Np
    obj = rng.uniform(size=(Np, N, N))
    E3, sampled = RF.measured_grid(obj, th)
    V0 = D.assemble_volume(obj, th)
    V1, _ = RF.refine(V0, E3, sampled, np.ones((N, N, N), bool), 1, positivity=False)
    assert np.abs(V1 - V0).max() <= 1e-12 * np.abs(V0).max()


def test_exact_object_is_a_fixed_point():
    N = 16
    rng = np.random.default_rng(2)
    O = np.zeros((N, N, N))
    O[5:11, 4:12, 6:10] = rng.uniform(0.2, 1.0, size=(6, 8, 4))
    po = np.stack([G.project_right_angle(O, 0), G.project_right_angle(O, 1)])
    th = [0.0, np.pi / 2]
    E3, sampled = RF.measured_grid(po, th)
    S3 = RF.support3d(po > 0, th)
    assert np.all(S3[O > 0])
    V, _ = RF.refine(O, E3, sampled, S3, 3)
    assert np.abs(V - O).max() <= 1e-12


def test_shrinkwrap3d_delta_is_a_ball():
    N, sigma, f = 24, 1.5, 0.25
    V = np.zeros((N, N, N))
    V[3, N - 2, 10] = 1.0
    S = RF.shrinkwrap3d(V, sigma, f)
    d = lambda a, c: np.minimum(np.abs(a - c), N - np.abs(a - c))
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    dz, dy, dx = d(z, 3), d(y, N - 2), d(x, 10)
    W = int(np.ceil(4 * sigma))
    want = (dz <= W) & (dy <= W) & (dx <= W) & (np.exp(-(dz ** 2 + dy ** 2 + dx ** 2) / (2 * sigma ** 2)) >= f - 1e-12)
    assert np.array_equal(S, want)
