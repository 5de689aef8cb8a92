"""FP64 oracle of the carousel phase retrieval (CPRA) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call
this module; only the tests, the smoke check and the benchmark's CPU
baseline do.  It shares no code with the GPU library.

What it computes, in the paper's order (Ai, Lomakin, Shpyrko, "Real time 3D
coherent X-ray diffraction imaging"):

* Forward model: each measured map is I_n = |E_n|^2 with E_n the 2D Fourier
  transform of the projected object O'_n (Eq. 1-3, Fourier slice theorem).
* Input preparation: amplitudes A_n = sqrt(I_n) in FFT-native order;
  I < 0 marks an unmeasured pixel (beamstop), where the modulus constraint is
  not applied.
* Step A / episode W_0: every PO starts from a random guess (no
  pre-reconstruction, N_i^pre = 0): X_n = Re F2^-1(A_n exp(i phi_n)) with
  seeded uniform phases phi_n (counter-based SplitMix64, see rng.py).
* Step B, Eq. 4 with the example weights of the paper read as a 3-tap offset
  sum: at the start of every episode each PO is re-initialised from the
  previous episode's objects, O_n <- a_-1 X_{n-1} + a_0 X_n + a_+1 X_{n+1},
  indices periodic over the angle ring ("carousel"); all angles use the
  previous episode only (Jacobi form).  Across the 180-degree seam the
  wrapped neighbour is the t-mirror of the PO at the other end, because the
  projection at theta + pi is the mirror image of the one at theta.
* Within an episode each PO runs N_ei iterations of 2D phase retrieval:
  G = F2(g); Fourier-modulus projection G' = A G/|G|; g' = Re F2^-1(G');
  gamma = support AND (g' >= 0); HIO: g <- g' on gamma, g - beta g' off it;
  ER: g <- g' on gamma, 0 off it.  The last iteration of an episode writes
  the estimate g' 1_gamma, which is the object X_n of that episode.
* Reconstruction error per angle and iteration (the paper ranks episodes by
  it without defining it): E_F = sqrt(sum_meas (|G| - A)^2 / sum_meas A^2),
  evaluated on G before the projection.
* Step D lives in stepd.py.

Real-space arrays are centred (origin at index N/2), [z][t]; Fourier arrays
are FFT-native [w][u].  F2 is the oracle's own FFT (fft.py).
"""
from __future__ import annotations

import numpy as np

from . import fft as F
from .rng import initial_phases

HIO, ER, RAAR = 0, 1, 2
WRAP_MIRROR, WRAP_PLAIN = 0, 1


def amplitudes(intensity_centred: np.ndarray) -> np.ndarray:
    """A = sqrt(I) moved to native order; unmeasured pixels (I < 0) become -1."""
    I = np.asarray(intensity_centred, dtype=np.float64)
    if not np.all(np.isfinite(I)):
        raise ValueError("intensity contains NaN or Inf")
    A = np.where(I >= 0, np.sqrt(np.maximum(I, 0.0)), -1.0)
    return F.shift_to_native(A, (-2, -1))


def mirror_t(x: np.ndarray) -> np.ndarray:
    """(M x)[z][t] = x[z][(N - t) mod N]: the geometric mirror t -> -t of a centred PO."""
    N = x.shape[-1]
    return x[..., (N - np.arange(N)) % N]


def forward(g_centred: np.ndarray) -> np.ndarray:
    return F.fft2(F.shift_to_native(g_centred, (-2, -1)))


def inverse_real(G: np.ndarray) -> np.ndarray:
    return np.real(F.shift_to_centred(F.ifft2(G), (-2, -1)))


def modulus_projection(G: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Replace |G| by A and keep the phase; A = 0 phase where |G| = 0; G kept where A < 0."""
    mag = np.abs(G)
    safe = np.where(mag > 0, mag, 1.0)
    proj = np.where(mag > 0, A * G / safe, A + 0j)
    return np.where(A >= 0, proj, G)


def fourier_error(G: np.ndarray, A: np.ndarray) -> float:
    meas = A >= 0
    num = np.sum(np.where(meas, (np.abs(G) - A) ** 2, 0.0))
    den = np.sum(np.where(meas, A * A, 0.0))
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))


def support_projection(x, support, positivity):
    """P_S: keep x on the support (and where x >= 0 with positivity), zero elsewhere."""
    keep = support.astype(bool)
    if positivity:
        keep = keep & (x >= 0)
    return np.where(keep, x, 0.0)


def real_space_update(g, gp, support, algo, beta, positivity, estimate):
    """gp = g' = P_M g (the modulus-projected iterate)."""
    gamma = support.astype(bool)
    if positivity:
        gamma = gamma & (gp >= 0)
    if estimate or algo == ER:
        return np.where(gamma, gp, 0.0)
    if algo == HIO:
        return np.where(gamma, gp, g - beta * gp)
    if algo == RAAR:
        # Luke's relaxed averaged alternating reflections in operator form:
        # g+ = beta/2 (R_S R_M + I) g + (1 - beta) P_M g, with R = 2P - I
        rm = 2.0 * gp - g
        rs_rm = 2.0 * support_projection(rm, support, positivity) - rm
        return 0.5 * beta * (rs_rm + g) + (1.0 - beta) * gp
    raise ValueError("algo must be HIO, ER or RAAR")


def gaussian_window(sigma: float) -> np.ndarray:
    """Sampled 1D Gaussian exp(-d^2 / (2 sigma^2)), d = -W..W with W = ceil(4 sigma), normalised
    to sum 1 (the window of the shrinkwrap blur)."""
    W = int(np.ceil(4.0 * sigma))
    d = np.arange(-W, W + 1, dtype=np.float64)
    k = np.exp(-d * d / (2.0 * sigma * sigma))
    return k / k.sum()


def shrinkwrap_support(g: np.ndarray, sigma: float, threshold: float) -> np.ndarray:
    """Shrinkwrap support update (the conventional 2D shrinkwrap step the paper runs at the end
    of each episode): blur the object with the periodic 2D Gaussian K(dz, dt) = k(dz) k(dt) of
    gaussian_window, b[z][t] = sum K(dz, dt) g[z - dz][t - dt] (indices mod N), and keep the pixels
    where b >= threshold * max(b)."""
    b = shrinkwrap_blur(g, sigma)
    return b >= threshold * b.max()


def shrinkwrap_blur(g: np.ndarray, sigma: float) -> np.ndarray:
    """b[z][t] = sum_{dz, dt} k(dz) k(dt) g[z - dz][t - dt], indices mod N."""
    k = gaussian_window(sigma)
    W = (len(k) - 1) // 2
    b = np.zeros_like(g, dtype=np.float64)
    for dz in range(-W, W + 1):
        for dt in range(-W, W + 1):
            b += k[dz + W] * k[dt + W] * np.roll(g, (dz, dt), axis=(0, 1))
    return b


def coupling_weights(Np, present, alpha, wrap):
    """Per angle: ((left, w_left, mirror_left), w_self, (right, w_right, mirror_right)).

    Neighbours are n-1 and n+1 on the periodic ring; an absent neighbour gets
    weight 0 and the remaining weights are rescaled to sum to 1.  With the
    mirror seam rule the neighbour reached by wrapping round the ring is
    t-mirrored.
    """
    out = []
    for n in range(Np):
        l, r = (n - 1) % Np, (n + 1) % Np
        ml = wrap == WRAP_MIRROR and n == 0
        mr = wrap == WRAP_MIRROR and n == Np - 1
        wl = alpha[0] if present[l] else 0.0
        wr = alpha[2] if present[r] else 0.0
        w0 = alpha[1]
        s = wl + w0 + wr
        out.append(((l, wl / s, ml), w0 / s, (r, wr / s, mr)))
    return out


def couple(X: np.ndarray, present, alpha, wrap) -> np.ndarray:
    """Eq. 4 (3 taps): new initial guesses from the previous episode's objects X."""
    Np = X.shape[0]
    out = np.zeros_like(X)
    for n, ((l, wl, ml), w0, (r, wr, mr)) in enumerate(coupling_weights(Np, present, alpha, wrap)):
        if not present[n]:
            out[n] = X[n]
            continue
        xl = mirror_t(X[l]) if ml else X[l]
        xr = mirror_t(X[r]) if mr else X[r]
        out[n] = wl * xl + w0 * X[n] + wr * xr
    return out


def couple_taps(X: np.ndarray, present, taps, wrap) -> np.ndarray:
    """Eq. 4 with 2K+1 taps alpha_{-K..K} (taps[k + K] = alpha_k): new initial guesses
    O_n <- sum_k alpha_k X_{n+k} over the periodic ring; a neighbour reached by wrapping round the
    ring is t-mirrored under the mirror seam rule; absent neighbours drop out and the remaining
    weights are rescaled to sum to 1.  Needs 2K+1 <= Np (each neighbour taken once)."""
    Np = X.shape[0]
    K = (len(taps) - 1) // 2
    out = np.zeros_like(X)
    for n in range(Np):
        if not present[n]:
            out[n] = X[n]
            continue
        terms = []
        for k in range(-K, K + 1):
            m = n + k
            wrapped = m < 0 or m >= Np
            m %= Np
            if k != 0 and not present[m]:
                continue
            x = mirror_t(X[m]) if (wrapped and wrap == WRAP_MIRROR) else X[m]
            terms.append((taps[k + K], x))
        s = sum(w for w, _ in terms)
        out[n] = sum((w / s) * x for w, x in terms)
    return out


def initial_object(A: np.ndarray, seed: int, n: int) -> np.ndarray:
    """W_0 object of angle n: Re F2^-1(A exp(i phi)), unmeasured pixels with amplitude 0."""
    N = A.shape[-1]
    phi = initial_phases(seed, n, N)
    amp = np.where(A >= 0, A, 0.0)
    return inverse_real(amp * (np.cos(phi) + 1j * np.sin(phi)))


class Oracle:
    """Plain FP64 CPRA over one scan of Np angles (mirrors the C-ABI plan semantics)."""

    def __init__(self, N, Np, theta=None, alpha=(0.2, 0.6, 0.2), n_ei=10, wrap=WRAP_MIRROR,
                 positivity=True, seed=0, taps=None):
        self.N, self.Np = int(N), int(Np)
        self.taps = None if taps is None else tuple(float(a) for a in taps)   # 2K+1 taps, else alpha
        self.theta = (np.pi * np.arange(Np) / Np) if theta is None else np.asarray(theta, dtype=np.float64)
        self.alpha = tuple(float(a) for a in alpha)
        self.n_ei = int(n_ei)
        self.wrap = int(wrap)
        self.positivity = bool(positivity)
        self.seed = int(seed)
        self.A = np.zeros((Np, N, N))
        self.S = np.zeros((Np, N, N), dtype=bool)
        self.g = np.zeros((Np, N, N))
        # kept for tests: the iterate entering and the g' of the last iteration
        # (a pixel with g' within rounding of 0 may take either HIO branch)
        self.g_prev = np.zeros((Np, N, N))
        self.last_gp = np.zeros((Np, N, N))
        self.landed = np.zeros(Np, dtype=bool)
        self.present = np.zeros(Np, dtype=bool)
        self.k = 0

    def submit(self, first, intensity, support):
        intensity = np.asarray(intensity)
        cnt = intensity.shape[0]
        for i in range(cnt):
            n = first + i
            self.A[n] = amplitudes(intensity[i])
            self.S[n] = np.asarray(support[i]) != 0
            self.g[n] = initial_object(self.A[n], self.seed, n)
            self.landed[n] = True
        if self.k % self.n_ei == 0:
            self.present = self.landed.copy()

    def iterate(self, n_iter, algo=HIO, beta=0.9):
        """Run n_iter iterations over the present angles; returns E_F history (n_iter, Np)."""
        err = np.full((n_iter, self.Np), np.nan)
        for i in range(n_iter):
            if self.k % self.n_ei == 0:
                self.present = self.landed.copy()
                if self.taps is None:
                    self.g = couple(self.g, self.present, self.alpha, self.wrap)
                else:
                    self.g = couple_taps(self.g, self.present, self.taps, self.wrap)
            estimate = (self.k + 1) % self.n_ei == 0
            for n in np.flatnonzero(self.present):
                G = forward(self.g[n])
                err[i, n] = fourier_error(G, self.A[n])
                gp = inverse_real(modulus_projection(G, self.A[n]))
                self.g_prev[n] = self.g[n]
                self.last_gp[n] = gp
                self.g[n] = real_space_update(self.g[n], gp, self.S[n], algo, beta, self.positivity, estimate)
            self.k += 1
        return err

    def shrinkwrap(self, sigma, threshold):
        """Replace the support of every present angle by the shrinkwrap of its current object."""
        for n in np.flatnonzero(self.present):
            self.S[n] = shrinkwrap_support(self.g[n], sigma, threshold)

    def objects(self):
        return self.g.copy()
