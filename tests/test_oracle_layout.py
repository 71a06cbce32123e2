"""Pins of the layout tiling and the shot count (oracle/layout.py)."""
import itertools

import numpy as np
import pytest

from oracle import layout


CASES = [(64, 64, 32, 4), (50, 77, 32, 6), (33, 17, 16, 0), (100, 40, 24, 11), (5, 3, 16, 2)]


@pytest.mark.parametrize("H,W,N,halo", CASES)
def test_cores_partition_the_layout(H, W, N, halo):
    C = N - 2 * halo
    cover = np.zeros((H, W), dtype=int)
    for i, j, y0, x0 in layout.tile_grid(H, W, N, halo):
        assert (y0, x0) == (i * C - halo, j * C - halo)
        cover[max(y0 + halo, 0):min(y0 + halo + C, H), max(x0 + halo, 0):min(x0 + halo + C, W)] += 1
    assert np.all(cover == 1)


@pytest.mark.parametrize("H,W,N,halo", CASES)
def test_extract_against_padding_and_round_trip(H, W, N, halo):
    rng = np.random.default_rng(H * 1000 + W)
    L = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    tiles = layout.extract_tiles(L, N, halo)
    # independent formulation: zero-pad the layout and slice
    pad = np.zeros((H + 2 * N + halo, W + 2 * N + halo), dtype=np.uint8)
    pad[halo:halo + H, halo:halo + W] = L
    for t, (_, _, y0, x0) in enumerate(layout.tile_grid(H, W, N, halo)):
        assert np.array_equal(tiles[t], pad[y0 + halo:y0 + halo + N, x0 + halo:x0 + halo + N])
    assert np.array_equal(layout.stitch(tiles, H, W, N, halo), L)


def test_tile_grid_rejects_bad_halo():
    with pytest.raises(ValueError):
        layout.tile_grid(10, 10, 16, 8)


def _partition_ok(M, rects):
    cover = np.zeros(M.shape, dtype=int)
    for y0, y1, x0, x1 in rects:
        assert y0 < y1 and x0 < x1
        cover[y0:y1, x0:x1] += 1
    return np.array_equal(cover, M.astype(int))


def _shape(rows):
    return np.array([[c == "#" for c in r] for r in rows], dtype=bool)


SHAPES = {
    "empty": (_shape(["....", "...."]), 0),
    "full": (_shape(["###", "###"]), 1),
    "rectangle": (_shape([".....", ".###.", ".###.", "....."]), 1),
    "L": (_shape(["#..", "#..", "###"]), 2),
    "plus": (_shape([".#.", "###", ".#."]), 3),
    "ring": (_shape(["####", "#..#", "#..#", "####"]), 4),
    "checker": (_shape(["#.#.", ".#.#", "#.#."]), 6),
    "stairs": (_shape(["#...", "##..", "###.", "####"]), 4),
}


@pytest.mark.parametrize("name", sorted(SHAPES))
def test_shot_count_of_known_shapes(name):
    M, want = SHAPES[name]
    assert layout.shot_count(M) == want
    assert _partition_ok(M, layout.fracture_rows(M))


def test_row_and_column_fracturings_differ_and_min_is_taken():
    # a comb: one horizontal bar with three teeth hanging below
    M = _shape(["#######", "#.#.#.#", "#.#.#.#"])
    rows = len(layout.fracture_rows(M))
    cols = len(layout.fracture_rows(M.T))
    assert (rows, cols) == (5, 7)
    assert layout.shot_count(M) == 5


def _min_partition(M):
    """Exact minimum number of rectangles partitioning M (exhaustive; tiny M).
    The first uncovered one in row-major order is the top-left corner of its
    rectangle, so branching over the rectangles it can start is complete."""
    M = M.astype(bool)
    H, W = M.shape
    best = [H * W + 1]

    def rec(rem, used):
        if used >= best[0]:
            return
        idx = np.flatnonzero(rem)
        if idx.size == 0:
            best[0] = used
            return
        y, x = divmod(int(idx[0]), W)
        xmax = x
        while xmax < W and rem[y, xmax]:
            xmax += 1
        for x1 in range(xmax, x, -1):
            y1 = y
            while y1 < H and rem[y1, x:x1].all():
                y1 += 1
            for yy in range(y1, y, -1):
                r2 = rem.copy()
                r2[y:yy, x:x1] = False
                rec(r2, used + 1)

    rec(M.copy(), 0)
    return best[0]


def test_shot_count_bounds_the_minimum_partition():
    rng = np.random.default_rng(5)
    hits = 0
    for trial in range(60):
        M = rng.uniform(size=(4, 5)) < 0.6
        m = _min_partition(M)
        s = layout.shot_count(M)
        assert _partition_ok(M, layout.fracture_rows(M))
        assert _partition_ok(M.T, layout.fracture_rows(M.T))
        assert s >= m
        hits += s == m
    assert hits >= 30                     # the estimate is often exact on small masks


def test_exhaustive_3x3_masks():
    """Every 3 x 3 mask: both fracturings are exact partitions and the count
    never falls below the minimum."""
    for bits in itertools.product([0, 1], repeat=9):
        M = np.array(bits, dtype=bool).reshape(3, 3)
        assert _partition_ok(M, layout.fracture_rows(M))
        assert layout.shot_count(M) >= _min_partition(M)
