"""Seeded synthetic 3D objects and their exact line-integral projections.

This module makes INPUT DATA only.  It models the experiment's forward side
(the object is rotated about z and projected along the beam, Eq. 2-3 of the
paper) and holds none of the reconstruction method's arithmetic.  Both the
CPU oracle and the GPU path receive what it produces.

Geometry (shared convention of the whole project):
  * voxel / pixel index i maps to the coordinate i - N/2 (arrays are centred);
  * angle theta rotates about z: beam direction d = (cos t, sin t, 0),
    transverse axis e_t = (-sin t, cos t, 0);
  * a projected object (PO) is stored as [z][t]: row z is the rotation axis
    coordinate, column t the transverse coordinate;
  * the PO pixel (z, t) is the line integral of the density along
    r(s) = t*e_t + z*e_z + s*d.

Objects are unions of analytic bodies (ellipsoids, balls, a convex
polyhedron), so every projection is an exact sum of chord lengths and the
whole angle set is consistent with one 3D object without voxelising N^3.
"""
from __future__ import annotations

import numpy as np


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly random 3x3 rotation (QR of a Gaussian matrix, sign-fixed)."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def ray_grid(N: int, theta: float):
    """Origins (N*N, 3) and direction (3,) of the rays of one PO, row-major [z][t]."""
    c = np.arange(N, dtype=np.float64) - N / 2
    zz, tt = np.meshgrid(c, c, indexing="ij")
    et = np.array([-np.sin(theta), np.cos(theta), 0.0])
    d = np.array([np.cos(theta), np.sin(theta), 0.0])
    o = tt.reshape(-1, 1) * et[None, :] + zz.reshape(-1, 1) * np.array([0.0, 0.0, 1.0])[None, :]
    return o, d


def ellipsoid_interval(o, d, centre, rot, semi):
    """Entry/exit parameters of rays o + s d through an ellipsoid.

    The ellipsoid is {r : |diag(1/semi) rot^T (r - centre)| <= 1}.  Returns
    (s0, s1, hit) with s1 - s0 the chord length where hit is True.
    """
    m = rot @ np.diag(1.0 / np.asarray(semi, dtype=np.float64) ** 2) @ rot.T
    p = o - centre[None, :]
    a = float(d @ m @ d)
    b = p @ (m @ d)
    c = np.einsum("ij,jk,ik->i", p, m, p) - 1.0
    disc = b * b - a * c
    hit = disc > 0
    sq = np.sqrt(np.where(hit, disc, 0.0))
    s0 = (-b - sq) / a
    s1 = (-b + sq) / a
    return s0, s1, hit


def ball_interval(o, d, centre, radius):
    return ellipsoid_interval(o, d, centre, np.eye(3), (radius, radius, radius))


def halfspace_interval(o, d, centre, normals, dist):
    """Parameters where rays lie inside {r : n_i . (r - centre) <= dist_i for all i}."""
    p = o - centre[None, :]
    nd = normals @ d                      # (F,)
    npv = p @ normals.T                   # (M, F)
    lo = np.full(o.shape[0], -np.inf)
    hi = np.full(o.shape[0], np.inf)
    for f in range(normals.shape[0]):
        lim = dist[f] - npv[:, f]
        if nd[f] > 1e-15:
            hi = np.minimum(hi, lim / nd[f])
        elif nd[f] < -1e-15:
            lo = np.maximum(lo, lim / nd[f])
        else:
            inside = lim >= 0
            lo = np.where(inside, lo, np.inf)
    return lo, hi


class Ellipsoids:
    """Sum of uniform ellipsoids (overlapping densities add)."""

    def __init__(self, centres, rots, semis, dens):
        self.centres = [np.asarray(c, dtype=np.float64) for c in centres]
        self.rots = rots
        self.semis = semis
        self.dens = dens

    def project(self, N: int, theta: float) -> np.ndarray:
        o, d = ray_grid(N, theta)
        out = np.zeros(o.shape[0])
        for c, r, s, rho in zip(self.centres, self.rots, self.semis, self.dens):
            s0, s1, hit = ellipsoid_interval(o, d, c, r, s)
            out += np.where(hit, rho * (s1 - s0), 0.0)
        return out.reshape(N, N)


class PlaneWaveTexture:
    """Smooth random density modulation tau(r) = amp*sqrt(2/K)*sum_k cos(kappa_k.r + phi_k).

    A sum of K random plane waves is close to a Gaussian random field with
    standard deviation `amp`; its line integral over a segment is analytic,
    so textured bodies still project exactly.
    """

    def __init__(self, rng, amp=0.05, K=24, kmin=0.5, kmax=2.0):
        v = rng.standard_normal((K, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        self.kappa = v * rng.uniform(kmin, kmax, size=(K, 1))
        self.phi = rng.uniform(0, 2 * np.pi, size=K)
        self.scale = amp * np.sqrt(2.0 / K)

    def segment_integral(self, o, d, s0, s1):
        """Integral of tau along o + s d for s in [s0, s1] (zero where s1 <= s0)."""
        ln = np.maximum(s1 - s0, 0.0)
        mid = 0.5 * (s0 + s1)
        mid = np.where(np.isfinite(mid), mid, 0.0)
        acc = np.zeros(o.shape[0])
        for kap, ph in zip(self.kappa, self.phi):
            a = o @ kap + ph
            b = float(kap @ d)
            # integral of cos(a + b s) over [s0, s1] = len * cos(a + b*mid) * sinc(b*len/2)
            acc += ln * np.cos(a + b * mid) * np.sinc(b * ln / (2 * np.pi))
        return self.scale * acc


class Polyhedron:
    """Convex polyhedron (clipped by a bounding ball) with spherical voids and texture."""

    def __init__(self, centre, normals, dist, rmax, voids, texture):
        self.centre = np.asarray(centre, dtype=np.float64)
        self.normals = normals
        self.dist = dist
        self.rmax = rmax
        self.voids = voids            # list of (centre, radius)
        self.texture = texture

    def _body_interval(self, o, d, scale=1.0):
        lo, hi = halfspace_interval(o, d, self.centre, self.normals, self.dist * scale)
        b0, b1, hit = ball_interval(o, d, self.centre, self.rmax * scale)
        lo = np.where(hit, np.maximum(lo, b0), np.inf)
        hi = np.where(hit, np.minimum(hi, b1), -np.inf)
        return lo, hi

    def project(self, N: int, theta: float) -> np.ndarray:
        o, d = ray_grid(N, theta)
        s0, s1 = self._body_interval(o, d)
        inside = s1 > s0
        out = np.where(inside, s1 - s0, 0.0)
        if self.texture is not None:
            out += np.where(inside, self.texture.segment_integral(o, d, np.where(inside, s0, 0), np.where(inside, s1, 0)), 0.0)
        for vc, vr in self.voids:
            v0, v1, vh = ball_interval(o, d, np.asarray(vc), vr)
            out -= np.where(vh, v1 - v0, 0.0)
            if self.texture is not None:
                out -= np.where(vh, self.texture.segment_integral(o, d, np.where(vh, v0, 0), np.where(vh, v1, 0)), 0.0)
        return out.reshape(N, N)

    def support(self, N: int, theta: float, dilate: float = 1.2) -> np.ndarray:
        o, d = ray_grid(N, theta)
        s0, s1 = self._body_interval(o, d, scale=dilate)
        return (s1 > s0).reshape(N, N)


class Cell:
    """Ellipsoidal shell with non-overlapping interior granules."""

    def __init__(self, centre, rot, outer, thickness, shell_density, granules):
        self.centre = np.asarray(centre, dtype=np.float64)
        self.rot = rot
        self.outer = np.asarray(outer, dtype=np.float64)
        self.inner = self.outer - thickness
        self.rho = shell_density
        self.granules = granules      # list of (centre, radius, density)

    def project(self, N: int, theta: float) -> np.ndarray:
        o, d = ray_grid(N, theta)
        a0, a1, ah = ellipsoid_interval(o, d, self.centre, self.rot, self.outer)
        b0, b1, bh = ellipsoid_interval(o, d, self.centre, self.rot, self.inner)
        out = self.rho * (np.where(ah, a1 - a0, 0.0) - np.where(bh, b1 - b0, 0.0))
        out = out.reshape(N, N)
        # granules only touch the pixels of their projected disc
        et = np.array([-np.sin(theta), np.cos(theta), 0.0])
        for gc, gr, gd in self.granules:
            gc = np.asarray(gc, dtype=np.float64)
            tc = gc @ et + N / 2
            zc = gc[2] + N / 2
            t0, t1 = max(int(np.floor(tc - gr)) - 1, 0), min(int(np.ceil(tc + gr)) + 2, N)
            z0, z1 = max(int(np.floor(zc - gr)) - 1, 0), min(int(np.ceil(zc + gr)) + 2, N)
            zz, tt = np.meshgrid(np.arange(z0, z1) - N / 2, np.arange(t0, t1) - N / 2, indexing="ij")
            dz = zz - gc[2]
            dt = tt - gc @ et
            r2 = gr * gr - dz * dz - dt * dt
            out[z0:z1, t0:t1] += gd * 2.0 * np.sqrt(np.maximum(r2, 0.0))
        return out

    def support(self, N: int, theta: float, dilate: float = 1.2) -> np.ndarray:
        o, d = ray_grid(N, theta)
        _, _, hit = ellipsoid_interval(o, d, self.centre, self.rot, self.outer * dilate)
        return hit.reshape(N, N)


def make_ellipsoids(rng, n=5, centre_radius=20.0, semi=(3.0, 10.0), support_radius=24.0, dens=(0.5, 1.0)):
    """Random ellipsoids with centres within `centre_radius` that fit in the support ball."""
    centres, rots, semis, rhos = [], [], [], []
    while len(centres) < n:
        s = rng.uniform(semi[0], semi[1], size=3)
        c = rng.uniform(-centre_radius, centre_radius, size=3)
        if np.linalg.norm(c) > centre_radius or np.linalg.norm(c) + s.max() > support_radius:
            continue
        centres.append(c)
        rots.append(random_rotation(rng))
        semis.append(s)
        rhos.append(rng.uniform(dens[0], dens[1]))
    return Ellipsoids(centres, rots, semis, rhos)


def make_polyhedron(rng, N, texture=True):
    """Convex polyhedron of 12-20 faces at distance 0.2N*U[0.85,1], 3-8 voids, textured."""
    centre = np.zeros(3)
    F = int(rng.integers(12, 21))
    while True:
        normals = rng.standard_normal((F, 3))
        normals /= np.linalg.norm(normals, axis=1, keepdims=True)
        probe = rng.standard_normal((2000, 3))
        probe /= np.linalg.norm(probe, axis=1, keepdims=True)
        if (probe @ normals.T).max(axis=1).min() > 0.2:
            break
    dist = 0.2 * N * rng.uniform(0.85, 1.0, size=F)
    rmax = 0.24 * N
    voids = []
    nv = int(rng.integers(3, 9))
    tries = 0
    while len(voids) < nv and tries < 10000:
        tries += 1
        r = rng.uniform(0.03, 0.08) * N
        c = rng.uniform(-0.2 * N, 0.2 * N, size=3)
        margin = dist - normals @ c
        if margin.min() < r + 2 or np.linalg.norm(c) + r + 2 > rmax:
            continue
        if any(np.linalg.norm(c - vc) < r + vr + 1 for vc, vr in voids):
            continue
        voids.append((c, r))
    tex = PlaneWaveTexture(rng) if texture else None
    return Polyhedron(centre, normals, dist, rmax, voids, tex)


def make_cell(rng, N):
    """Ellipsoidal shell (thickness 6-10) with 50-200 granules of radius 2-6, densities 0.2-1."""
    outer = rng.uniform(0.18, 0.24, size=3) * N
    thick = rng.uniform(6.0, 10.0)
    rot = random_rotation(rng)
    rho = rng.uniform(0.2, 1.0)
    inner = outer - thick
    ng = int(rng.integers(50, 201))
    granules = []
    tries = 0
    while len(granules) < ng and tries < 200000:
        tries += 1
        r = rng.uniform(2.0, 6.0)
        u = rng.uniform(-1, 1, size=3)
        if u @ u > 1:
            continue
        # inside the inner ellipsoid with a margin of r
        local = u * np.maximum(inner - r - 1, 1.0)
        c = rot @ local
        if any(np.linalg.norm(c - gc) < r + gr + 0.5 for gc, gr, _ in granules):
            continue
        granules.append((c, r, rng.uniform(0.2, 1.0)))
    return Cell(np.zeros(3), rot, outer, thick, rho, granules)
