"""FP64 oracle of the paper's own schedule around the hot path: steps A-C with N_r guesses.

TEST INFRASTRUCTURE ONLY (see cpra.py).  Nothing in the product path may import or call this
module; it shares no code with the GPU library.

What it computes (paper, steps A, B and C of CPRA):

* N_r independent reconstructions ("random guesses") of the same scan.  Guess r, angle n starts
  from the random object of cpra.initial_object with RNG stream index r * Np + n, so guess 0 is
  the single-guess oracle's W_0.
* Step A, pre-reconstruction: PO 1 (index 0) of every guess runs N_i^pre iterations of plain 2D
  phase retrieval with no coupling; its last iteration writes the estimate g' 1_gamma.
* Step B, consecutive sweep (reading of "from n = 1 to n = N_p consecutively"): in each episode
  the POs are taken in order n = 0 .. Np-1; PO n is re-initialised from Eq. 4 with its
  neighbours' most recent objects (n-1 already from this episode, n+1 still from the previous
  one; the ring wraps, with the t-mirror across the 180-degree seam), then runs N_ei iterations,
  the last writing its estimate.  The data-parallel alternative (all POs from the previous
  episode, Jacobi) is `jacobi`.
* Episode error of a guess (the paper ranks episodes by "reconstruction error" without defining
  it): E = sqrt(sum_n sum_q (|F2 X_n| - A_n)^2 / sum_n sum_q A_n^2) over measured q, on the
  current objects X_n.
* Step C, merge: keep the N_l guesses of lowest episode error; move every PO's mass centre to
  the origin (shift by -c rounded with floor(x + 1/2), c = sum X r / sum X, the normalised form
  of the paper's -integral O' r dv); take the guess of lowest error as reference and, for every
  other kept guess, compare PO 1 with the reference's PO 1 and with its central inversion
  X(-r); if the inversion is nearer, invert every PO of that guess; average the kept guesses.
"""
from __future__ import annotations

import numpy as np

from . import cpra as C


def central_inversion(x: np.ndarray) -> np.ndarray:
    """X(-r) of a centred [z][t] array: index i -> (N - i) mod N on both axes."""
    N = x.shape[-1]
    idx = (N - np.arange(N)) % N
    return x[..., idx, :][..., :, idx]


def mass_centre(x: np.ndarray) -> tuple[float, float]:
    """(c_z, c_t) = sum x r / sum x with r measured from the centre index N/2."""
    N = x.shape[-1]
    r = np.arange(N, dtype=np.float64) - N // 2
    m = float(np.sum(x))
    if m == 0.0:
        return 0.0, 0.0
    return float(np.sum(x.sum(axis=1) * r) / m), float(np.sum(x.sum(axis=0) * r) / m)


def centre_shift(x: np.ndarray) -> tuple[int, int]:
    """Integer shift that moves the mass centre to the origin: floor(-c + 1/2) per axis."""
    cz, ct = mass_centre(x)
    return int(np.floor(-cz + 0.5)), int(np.floor(-ct + 0.5))


def shift(x: np.ndarray, s: tuple[int, int]) -> np.ndarray:
    """Cyclic shift of a [z][t] array: out[z][t] = x[z - s_z][t - s_t]."""
    return np.roll(x, s, axis=(-2, -1))


class GuessSet:
    """N_r reconstructions of one scan under the paper's schedule."""

    def __init__(self, N, Np, n_guess, theta=None, alpha=(0.2, 0.6, 0.2), n_ei=10, wrap=C.WRAP_MIRROR,
                 positivity=True, seed=0, taps=None):
        self.N, self.Np, self.R = int(N), int(Np), int(n_guess)
        self.theta = (np.pi * np.arange(Np) / Np) if theta is None else np.asarray(theta, dtype=np.float64)
        self.alpha = tuple(float(a) for a in alpha)
        self.n_ei, self.wrap, self.positivity, self.seed = int(n_ei), int(wrap), bool(positivity), int(seed)
        self.taps = None if taps is None else tuple(float(a) for a in taps)    # 2K+1 taps, else alpha
        self.A = np.zeros((Np, N, N))
        self.S = np.zeros((Np, N, N), dtype=bool)
        self.g = np.zeros((self.R, Np, N, N))

    def submit(self, intensity, support):
        for n in range(self.Np):
            self.A[n] = C.amplitudes(intensity[n])
            self.S[n] = np.asarray(support[n]) != 0
        for r in range(self.R):
            for n in range(self.Np):
                self.g[r, n] = C.initial_object(self.A[n], self.seed, r * self.Np + n)

    # ------------------------------------------------------------ building blocks
    def iterate_po(self, r, n, n_iter, algo, beta):
        """Plain 2D phase retrieval of one PO, no coupling; the last iteration writes the estimate.
        Returns E_F per iteration."""
        err = np.zeros(n_iter)
        for i in range(n_iter):
            G = C.forward(self.g[r, n])
            err[i] = C.fourier_error(G, self.A[n])
            gp = C.inverse_real(C.modulus_projection(G, self.A[n]))
            self.g[r, n] = C.real_space_update(self.g[r, n], gp, self.S[n], algo, beta, self.positivity,
                                               i == n_iter - 1)
        return err

    def couple_one(self, r, n):
        """Eq. 4 for PO n of guess r from the current objects (all angles present)."""
        if self.taps is not None:
            self.g[r, n] = C.couple_taps(self.g[r], np.ones(self.Np, bool), self.taps, self.wrap)[n]
            return
        (l, wl, ml), w0, (rr, wr, mr) = C.coupling_weights(self.Np, np.ones(self.Np, bool), self.alpha,
                                                           self.wrap)[n]
        X = self.g[r]
        xl = C.mirror_t(X[l]) if ml else X[l]
        xr = C.mirror_t(X[rr]) if mr else X[rr]
        self.g[r, n] = wl * xl + w0 * X[n] + wr * xr

    # ------------------------------------------------------------ steps
    def prereconstruct(self, n_iter, algo=C.HIO, beta=0.9):
        """Step A on PO 1 (index 0) of every guess."""
        return np.array([self.iterate_po(r, 0, n_iter, algo, beta) for r in range(self.R)])

    def sweep(self, n_episodes, algo=C.HIO, beta=0.9):
        """Step B, consecutive form.  Returns E_F as (n_episodes, R, Np, n_ei)."""
        err = np.zeros((n_episodes, self.R, self.Np, self.n_ei))
        for m in range(n_episodes):
            for n in range(self.Np):
                for r in range(self.R):
                    self.couple_one(r, n)
                    err[m, r, n] = self.iterate_po(r, n, self.n_ei, algo, beta)
        return err

    def jacobi(self, n_episodes, algo=C.HIO, beta=0.9):
        """Step B, data-parallel form: every PO re-initialised from the previous episode."""
        for _ in range(n_episodes):
            for r in range(self.R):
                if self.taps is None:
                    self.g[r] = C.couple(self.g[r], np.ones(self.Np, bool), self.alpha, self.wrap)
                else:
                    self.g[r] = C.couple_taps(self.g[r], np.ones(self.Np, bool), self.taps, self.wrap)
                for n in range(self.Np):
                    self.iterate_po(r, n, self.n_ei, algo, beta)

    def episode_errors(self):
        """Pooled E_F of each guess's current objects."""
        out = np.zeros(self.R)
        meas = self.A >= 0
        den = float(np.sum(np.where(meas, self.A ** 2, 0.0)))
        for r in range(self.R):
            num = 0.0
            for n in range(self.Np):
                G = C.forward(self.g[r, n])
                num += float(np.sum(np.where(meas[n], (np.abs(G) - self.A[n]) ** 2, 0.0)))
            out[r] = np.sqrt(num / den)
        return out

    def merge(self, n_best):
        """Step C: the final episode (Np, N, N) from the n_best guesses of lowest episode error.
        Also returns (kept guess indices in rank order, inverted flags)."""
        e = self.episode_errors()
        keep = [int(i) for i in np.argsort(e, kind="stable")[:n_best]]
        centred = np.array([[shift(self.g[r, n], centre_shift(self.g[r, n])) for n in range(self.Np)]
                            for r in keep])
        ref = centred[0, 0]
        inverted = [False]
        for j in range(1, len(keep)):
            d_same = np.linalg.norm(centred[j, 0] - ref)
            d_inv = np.linalg.norm(central_inversion(centred[j, 0]) - ref)
            inverted.append(bool(d_inv < d_same))
            if inverted[-1]:
                centred[j] = central_inversion(centred[j])
        return centred.mean(axis=0), keep, inverted
