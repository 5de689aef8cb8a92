"""The bench's roofline arithmetic (host only): per-launch bytes and times for full-width and
chunk-major launches, and the fused-iteration figure."""
import pytest

import bench


def _model():
    col_b, row_b = bench.algorithmic_bytes(bench.N, bench.NP, bench.N_EI)
    return col_b, row_b


def test_full_width_launches():
    col_b, row_b = _model()
    n_it = 400                                   # two steps of 200 iterations, one launch per pass each
    r, it_ms = bench.roofline_of(0.29 * n_it, n_it, 0.30 * n_it, n_it, n_it)
    assert it_ms == pytest.approx(0.59)
    assert r["kernel"] == "k_row" and r["launches_per_iteration"] == 1.0
    assert r["bytes_per_launch"] == int(row_b)
    assert r["achieved"] == pytest.approx(row_b / 0.30e-3 / 1e9, rel=1e-4)
    assert r["other"]["achieved"] == pytest.approx(col_b / 0.29e-3 / 1e9, rel=1e-4)
    assert r["fused_iteration"]["frac"] == pytest.approx((col_b + row_b) / 0.59e-3 / 1e9 / bench.HBM_PEAK_GBS,
                                                         rel=1e-3)


def test_chunk_major_launches_cover_part_of_the_angles():
    """Two launches per pass per iteration (half the angles each): the same work as one full-width
    launch of twice the time gives the same achieved bandwidth and iteration time."""
    col_b, row_b = _model()
    n_it = 200
    full, it_full = bench.roofline_of(0.29 * n_it, n_it, 0.30 * n_it, n_it, n_it)
    half, it_half = bench.roofline_of(0.29 * n_it, 2 * n_it, 0.30 * n_it, 2 * n_it, n_it)
    assert it_half == pytest.approx(it_full)
    assert half["launches_per_iteration"] == 2.0
    assert half["avg_launch_ms"] == pytest.approx(full["avg_launch_ms"] / 2, rel=1e-4)
    assert half["bytes_per_launch"] == pytest.approx(full["bytes_per_launch"] / 2, rel=1e-6)
    assert half["achieved"] == pytest.approx(full["achieved"], rel=1e-4)
    assert half["fused_iteration"]["frac"] == pytest.approx(full["fused_iteration"]["frac"])


def test_traffic_scales_with_the_launch():
    tr = {"k_col": {"traffic_bytes": 1.2e9}, "k_row": {"traffic_bytes": 1.5e9}}
    full, _ = bench.roofline_of(58.0, 200, 60.0, 200, 200, traffic=tr)
    half, _ = bench.roofline_of(58.0, 400, 60.0, 400, 200, traffic=tr)
    assert full["traffic"] == 1500000000 and half["traffic"] == 750000000
    assert bench.roofline_of(58.0, 200, 60.0, 200, 200)[0]["traffic"] is None
