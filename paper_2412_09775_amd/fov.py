"""Shift-variant restoration of a field of view: overlapping tiles, each auto-tuned
and reconstructed with its own parameters in one batched call, then blended back
with EDT weights (Methods, "Cell-scale optical pooled screen data" and
"Organelle-scale optical pooled screen data").  Every step runs in the library:
``wo_tile_grid``, ``wo_crop_stacks``, the learned initialiser (optional),
``wo_restore_tiles`` and ``wo_stitch_tiles``."""

from __future__ import annotations

import copy

import numpy as np

from . import api


def tile_stacks(stack, ys, xs, ty, tx, out=None):
    """The (n_y * n_x, Z, ty, tx) tiles of a (Z, H, W) stack, row-major over the grid."""
    import torch
    Z, H, W = stack.shape
    n = len(ys) * len(xs)
    if out is None:
        out = torch.empty((n, Z, ty, tx), dtype=torch.float32, device=stack.device)
    src = stack.contiguous().reshape(1, Z, H, W)
    for iy, y0 in enumerate(ys):
        for ix, x0 in enumerate(xs):
            t = iy * len(xs) + ix
            api.crop_stacks(src, (Z, ty, tx), (0, y0, x0), out=out[t:t + 1])
    return out


def restore_fov(stack, template, grid=(6, 6), overlap=(0, 0), eta=1e-2, net=None, theta0=None,
                iters=20, mask=0b0101, lr=api.PAPER_LR, lo=(-1e300,) * 4, hi=(1e300,) * 4,
                nu_c=None, use_graph=2, branches=8):
    """Restore a (Z, H, W) defocus stack.  `template` gives the thin-model optics of
    a tile (its ny, nx are replaced by the tile size); `theta0` (n_tiles, 4) or the
    network `net` or, by default, the template's parameters start every tile.
    Returns (field (2, H, W), tuned optics per tile, loss per tile, (ys, xs, ty, tx))."""
    Z, H, W = stack.shape
    ty, ys = api.tile_grid(H, grid[0], overlap[0])
    tx, xs = api.tile_grid(W, grid[1], overlap[1])
    tiles = tile_stacks(stack, ys, xs, ty, tx)
    n = tiles.shape[0]
    opts = []
    for _ in range(n):
        o = copy.copy(template)
        o.nz, o.ny, o.nx = Z, ty, tx
        opts.append(o)
    th0 = None
    if theta0 is not None:
        th0 = np.asarray(theta0, dtype=np.float64).reshape(n, 1, 4)
    elif net is not None:   # the library's CNN start (centre windows, network, prior)
        pred = api.cnn_init_theta(net.params, opts, tiles)
        th0 = np.zeros((n, 1, 4))
        th0[:, 0, :3] = np.clip(pred[:, :3], np.asarray(lo[:3]), np.asarray(hi[:3]))
        th0[:, 0, 3] = template.tilt_azimuth
    out, loss, _, _, f = api.restore_tiles(opts, tiles, np.broadcast_to(eta, (n,)), iters=iters, lr=lr,
                                           lo=lo, hi=hi, mask=mask, theta0=th0, nu_c=nu_c,
                                           use_graph=use_graph, branches=branches)
    import torch
    packed = torch.stack(f)                       # (n, 2, ty, tx) views of one buffer
    field = api.stitch_tiles(packed, ys, xs, H, W)
    return field, out, loss, (ys, xs, ty, tx)
