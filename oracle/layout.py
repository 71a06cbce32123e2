"""Full-layout tiling and the mask-fracturing shot count (test oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Tiling.  The paper optimises fixed-size clips (Sec. IV uses 2048 x 2048);
a layout larger than one clip is covered here by N x N tiles whose cores,
C = N - 2 h pixels square, tile the layout at stride C; tile (i, j) spans
layout rows [i C - h, i C - h + N) and columns [j C - h, j C - h + N), so
every core carries a halo of h pixels of optical context on each side.
Tile pixels outside the layout are empty (0).  Each tile is solved as a clip
on its own and the layout result takes, for every layout pixel, the value of
the tile whose core holds it.

Shot count (Sec. II-C).  The paper counts the rectangles of a fracturing of
the mask that reproduces it exactly, with scripts it does not give.  The
estimate here: fracture into maximal horizontal runs and merge a run with
the identical run (same first and last column) of the row above into one
rectangle; count the rectangles; do the same with the roles of rows and
columns exchanged and take the smaller count.  Both fracturings are exact
partitions of the mask, so the result bounds the minimum partition from
above.
"""
from __future__ import annotations

import numpy as np


def tile_grid(H: int, W: int, N: int, halo: int):
    """[(i, j, y0, x0)]: tile (i, j) covers rows [y0, y0 + N), columns
    [x0, x0 + N); its core starts at (y0 + halo, x0 + halo)."""
    C = N - 2 * halo
    if halo < 0 or C < 1:
        raise ValueError("need 0 <= halo < N / 2")
    rows = -(-H // C)
    cols = -(-W // C)
    return [(i, j, i * C - halo, j * C - halo) for i in range(rows) for j in range(cols)]


def extract_tiles(layout, N: int, halo: int):
    """[T, N, N] tiles of `layout` (zero outside it), in tile_grid order."""
    layout = np.asarray(layout)
    H, W = layout.shape
    grid = tile_grid(H, W, N, halo)
    out = np.zeros((len(grid), N, N), dtype=layout.dtype)
    for t, (_, _, y0, x0) in enumerate(grid):
        for r in range(N):
            y = y0 + r
            if not 0 <= y < H:
                continue
            a, b = max(x0, 0), min(x0 + N, W)
            if a < b:
                out[t, r, a - x0:b - x0] = layout[y, a:b]
    return out


def stitch(tiles, H: int, W: int, N: int, halo: int):
    """Layout [H, W] from per-tile results: each pixel from the tile whose
    core holds it."""
    tiles = np.asarray(tiles)
    C = N - 2 * halo
    out = np.empty((H, W), dtype=tiles.dtype)
    grid = tile_grid(H, W, N, halo)
    for t, (i, j, y0, x0) in enumerate(grid):
        for y in range(i * C, min((i + 1) * C, H)):
            xa, xb = j * C, min((j + 1) * C, W)
            out[y, xa:xb] = tiles[t, y - y0, xa - x0:xb - x0]
    return out


def _runs(row):
    """Maximal runs of ones in a 1-D 0/1 array: [(start, end)] half-open."""
    runs = []
    x = 0
    n = len(row)
    while x < n:
        if row[x]:
            s = x
            while x < n and row[x]:
                x += 1
            runs.append((s, x))
        else:
            x += 1
    return runs


def fracture_rows(M):
    """Rectangles (y0, y1, x0, x1), half-open, of the run-merging fracturing:
    each maximal run of a row extends the rectangle of the identical run
    directly above it, or starts a new one."""
    M = np.asarray(M).astype(bool)
    open_rects = {}                     # (x0, x1) -> y0 of the rectangle ending at the previous row
    done = []
    for y in range(M.shape[0]):
        runs = _runs(M[y])
        nxt = {}
        for run in runs:
            nxt[run] = open_rects.pop(run, y)
        for (x0, x1), y0 in open_rects.items():
            done.append((y0, y, x0, x1))
        open_rects = nxt
    for (x0, x1), y0 in open_rects.items():
        done.append((y0, M.shape[0], x0, x1))
    return done


def shot_count(M) -> int:
    """min(rectangles of the row fracturing, of the column fracturing)."""
    M = np.asarray(M).astype(bool)
    return min(len(fracture_rows(M)), len(fracture_rows(M.T)))
