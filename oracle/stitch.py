"""Tiling a field of view and stitching restored tiles (Methods, "Cell-scale
optical pooled screen data": a grid of tiles with 20 % overlap; "Organelle-scale
optical pooled screen data": a 5 x 5 grid with 25 pixels of overlap, stitched by
linearly weighted Euclidean-distance-transform blending).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Reading R16: each tile's blending weight at a pixel is its Euclidean distance
transform there -- the distance to the nearest pixel outside the tile -- used
linearly; for an axis-aligned rectangle that is min(u + 1, T_y - u, v + 1,
T_x - v) at tile pixel (u, v).  The stitched value is the weighted mean of the
tiles covering the pixel.  Tiles are evenly spaced, the first at 0 and the last
flush with the far edge; the tile size is the smallest even {2, 3, 5}-smooth
length that gives at least the requested overlap.
"""

from __future__ import annotations

import math

import numpy as np


def smooth_even(n: int) -> int:
    """Smallest even m >= n whose prime factors are 2, 3 and 5."""
    m = max(2, n + (n % 2))
    while True:
        k = m
        for f in (2, 3, 5):
            while k % f == 0:
                k //= f
        if k == 1:
            return m
        m += 2


def tile_grid(length: int, count: int, overlap: int):
    """(tile size, start of every tile) along one axis."""
    if count < 1 or length < 2:
        raise ValueError("need at least one tile and two pixels")
    T = smooth_even(math.ceil((length + (count - 1) * overlap) / count))
    if T > length:
        raise ValueError("tiles larger than the field of view")
    if count == 1:
        return T, [(length - T) // 2]
    return T, [(i * (length - T)) // (count - 1) for i in range(count)]


def edt_weight(ty: int, tx: int) -> np.ndarray:
    """Distance from each tile pixel to the nearest pixel outside the tile (R16)."""
    u = np.arange(ty)[:, None]
    v = np.arange(tx)[None, :]
    return np.minimum(np.minimum(u + 1, ty - u), np.minimum(v + 1, tx - v)).astype(np.float64)


def stitch(tiles: np.ndarray, ys, xs, H: int, W: int) -> np.ndarray:
    """Weighted mean of tiles (n_y * n_x, P, T_y, T_x), row-major over the grid of
    starts ys x xs, into a (P, H, W) field."""
    n, P, ty, tx = tiles.shape
    if n != len(ys) * len(xs):
        raise ValueError("tile count does not match the grid")
    w = edt_weight(ty, tx)
    num = np.zeros((P, H, W))
    den = np.zeros((H, W))
    for iy, y0 in enumerate(ys):
        for ix, x0 in enumerate(xs):
            t = tiles[iy * len(xs) + ix]
            num[:, y0:y0 + ty, x0:x0 + tx] += w * t
            den[y0:y0 + ty, x0:x0 + tx] += w
    return num / den
