"""Pins of the edge placement error reading (oracle/metrics.py) on
rectangles with known displacements (no GPU)."""
import numpy as np

from oracle import metrics


def _rect(shape, y0, y1, x0, x1):
    Z = np.zeros(shape, dtype=np.uint8)
    Z[y0:y1, x0:x1] = 1
    return Z


def test_exact_print_has_zero_epe_and_known_sample_count():
    Z = _rect((64, 96), 20, 40, 30, 70)
    v = metrics.epe(Z, Z, 1.0)
    # 40 nm edges: samples at 5, 15, 25, 35 nm; 20 nm edges: 5, 15 nm
    assert v.size == 2 * 4 + 2 * 2
    assert np.all(v == 0.0)


def test_shifted_edges():
    Z = _rect((64, 96), 20, 40, 30, 70)
    grown = _rect((64, 96), 20, 43, 30, 70)      # bottom edge 3 px outward
    v = metrics.epe(Z, grown, 1.0)
    assert sorted(v.tolist()) == [0.0] * 8 + [3.0] * 4
    shrunk = _rect((64, 96), 20, 40, 32, 70)     # left edge 2 px inward
    v = metrics.epe(Z, shrunk, 1.0)
    assert sorted(v.tolist()) == [-2.0] * 2 + [0.0] * 10
    s = metrics.epe_summary(Z, shrunk, 1.0)
    assert s["samples"] == 12 and abs(s["mean_abs_nm"] - 4.0 / 12) < 1e-12 and s["max_abs_nm"] == 2.0


def test_pitch_scaling_and_search_limit():
    Z = _rect((64, 64), 16, 48, 16, 48)          # 32 px = 128 nm at 4 nm/px
    grown = _rect((64, 64), 16, 48, 16, 50)      # right edge 2 px = 8 nm outward
    v = metrics.epe(Z, grown, 4.0)
    # 128 nm edges: samples at 5, 15, ..., 115, 125? -> up to 123 nm: 5..115 (12 samples)
    assert v.size == 4 * 12
    assert sorted(set(v.tolist())) == [0.0, 8.0] and np.count_nonzero(v == 8.0) == 12
    empty = np.zeros_like(Z)
    assert np.all(metrics.epe(Z, empty, 4.0) == -40.0)
    s = metrics.epe_summary(Z, empty, 4.0)
    assert s["over_limit"] == s["samples"] == 48


def test_l_shape_edges_are_split_at_corners():
    Z = _rect((64, 64), 10, 50, 10, 20) | _rect((64, 64), 40, 50, 10, 50)
    edges = metrics._edges(Z)
    lengths = sorted(b - a for _, _, a, b, _ in edges)
    # an L has six straight edges: outer 40 and 40, inner 30 and 30, ends 10 and 10 px
    assert lengths == [10, 10, 30, 30, 40, 40]


def test_edges_on_the_image_border_are_sampled():
    # a rectangle touching the last row and the last column: its bottom and
    # right edges lie on the image border and are target edges like the rest
    Z = _rect((32, 48), 12, 32, 20, 48)
    edges = metrics._edges(Z)
    assert sorted((o, line, a, b, s) for o, line, a, b, s in edges) == sorted([
        ("h", 12, 20, 48, -1), ("h", 32, 20, 48, +1), ("v", 20, 12, 32, -1), ("v", 48, 12, 32, +1)])
    v = metrics.epe(Z, Z, 1.0)
    # 28 px edges: samples at 5, 15 nm (the last at most 23); 20 px edges: 5, 15
    assert v.size == 2 * 2 + 2 * 2 and np.all(v == 0.0)
    # nothing printed beyond the border: outward search finds the boundary at once
    assert np.all(metrics.epe(Z, np.zeros_like(Z), 1.0) == -40.0)
