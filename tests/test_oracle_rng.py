"""Pins of the oracle's SplitMix64 against published outputs."""
import os

import numpy as np

from oracle import rng as R

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def _golden():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        rows.append((int(parts[0]), [int(h, 16) for h in parts[1:]]))
    return rows


def test_published_outputs():
    for seed, outs in _golden():
        got = R.splitmix64_stream(seed, len(outs))
        assert [int(v) for v in got] == outs
        got_c = R.splitmix64_at(seed, np.arange(len(outs)))
        assert [int(v) for v in got_c] == outs


def test_counter_form_equals_stream():
    s = R.splitmix64_stream(987654321, 50)
    c = R.splitmix64_at(987654321, np.arange(50))
    assert np.array_equal(s, c)


def test_initial_phase_layout_and_range():
    N = 16
    phi = R.initial_phases(7, 3, N)
    assert phi.shape == (N, N)
    assert phi.min() >= 0 and phi.max() < 2 * np.pi
    # pixel (w, u) of angle n uses counter (n*N + w)*N + u
    w, u = 5, 9
    c = (3 * N + w) * N + u
    u24 = int(R.splitmix64_at(7, [c])[0]) >> 40
    assert phi[w, u] == 2 * np.pi * u24 / 2 ** 24
    big = R.initial_phases(11, 0, 256)
    assert abs(big.mean() - np.pi) < 0.02
