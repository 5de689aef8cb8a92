"""Counter-based SplitMix64 for the random initial phases (oracle side).

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the state advances by the golden-ratio increment
0x9E3779B97F4A7C15 and each output is the state passed through the
"mix64variant13" finaliser (xor-shift 30, multiply 0xBF58476D1CE4E5B9,
xor-shift 27, multiply 0x94D049BB133111EB, xor-shift 31).  The c-th output
(c = 0, 1, ...) of a generator seeded with `seed` is therefore
mix(seed + (c + 1) * increment), which is what `splitmix64_at` evaluates.

Initial phase of pixel (w, u) (native frequency order) of angle n:
counter c = (n*N + w)*N + u, u24 = top 24 bits of the output,
phi = 2*pi*u24 / 2^24.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * M1
    z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def splitmix64_at(seed: int, counter) -> np.ndarray:
    """c-th output (0-based) of SplitMix64 seeded with `seed`, for each c in `counter`."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed % (1 << 64)) + (c + np.uint64(1)) * GOLDEN
        return _mix(z)


def splitmix64_stream(seed: int, count: int) -> np.ndarray:
    """First `count` outputs of the sequential generator (state += increment; out = mix(state))."""
    out = np.empty(count, dtype=np.uint64)
    state = np.uint64(seed % (1 << 64))
    with np.errstate(over="ignore"):
        for i in range(count):
            state = state + GOLDEN
            out[i] = _mix(np.array([state], dtype=np.uint64))[0]
    return out


def initial_phases(seed: int, n: int, N: int) -> np.ndarray:
    """(N, N) float64 phases phi[w][u] of angle n, native frequency order."""
    w = np.arange(N, dtype=np.uint64)[:, None]
    u = np.arange(N, dtype=np.uint64)[None, :]
    c = (np.uint64(n) * np.uint64(N) + w) * np.uint64(N) + u
    u24 = splitmix64_at(seed, c) >> np.uint64(40)
    return (2.0 * np.pi / float(1 << 24)) * u24.astype(np.float64)
