"""Pins of the tiling/stitching oracle (CPU only)."""

import numpy as np
import pytest
from scipy import ndimage

from oracle import stitch


@pytest.mark.parametrize("ty,tx", [(6, 9), (16, 16), (1, 5)])
def test_edt_weight_is_the_euclidean_distance_transform(ty, tx):
    # distance to the nearest pixel outside the tile: the library EDT of the tile
    # mask padded with one ring of background
    mask = np.zeros((ty + 2, tx + 2), bool)
    mask[1:-1, 1:-1] = True
    ref = ndimage.distance_transform_edt(mask)[1:-1, 1:-1]
    assert np.array_equal(stitch.edt_weight(ty, tx), ref)


@pytest.mark.parametrize("length,count,overlap", [(2048, 6, 410), (1000, 5, 25), (300, 1, 0), (130, 2, 0)])
def test_tile_grid_covers_the_field_with_the_overlap(length, count, overlap):
    T, starts = stitch.tile_grid(length, count, overlap)
    k = T
    for f in (2, 3, 5):
        while k % f == 0:
            k //= f
    assert k == 1 and T % 2 == 0 and T <= length
    cover = np.zeros(length, int)
    for s in starts:
        cover[s:s + T] += 1
    assert np.all(cover >= 1)
    if count > 1:
        assert starts[0] == 0 and starts[-1] == length - T
        assert min(starts[i] + T - starts[i + 1] for i in range(count - 1)) >= overlap


def test_stitching_tiles_of_one_image_returns_the_image():
    rng = np.random.default_rng(0)
    H, W, P = 90, 110, 2
    img = rng.standard_normal((P, H, W))
    Ty, ys = stitch.tile_grid(H, 3, 10)
    Tx, xs = stitch.tile_grid(W, 4, 8)
    tiles = np.stack([img[:, y:y + Ty, x:x + Tx] for y in ys for x in xs])
    assert np.allclose(stitch.stitch(tiles, ys, xs, H, W), img, rtol=0, atol=1e-13)


def test_two_constant_tiles_blend_linearly_in_the_overlap():
    """Tiles of values a and b overlapping by k columns: the stitched value in the
    overlap is the EDT-weighted mean, a ramp between a and b."""
    a, b, T, k = 1.0, 3.0, 12, 6
    W = 2 * T - k
    tiles = np.stack([np.full((1, 40, T), a), np.full((1, 40, T), b)])
    out = stitch.stitch(tiles, [0], [0, T - k], 40, W)[0, 20]  # row 20: its distance (20) exceeds k
    for j, x in enumerate(range(T - k, T)):
        wa, wb = T - x, j + 1                                   # distances to each tile's near edge
        assert abs(out[x] - (wa * a + wb * b) / (wa + wb)) < 1e-14
    assert np.all(out[:T - k] == a) and np.all(out[T:] == b)
