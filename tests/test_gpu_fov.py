"""Field of view: tiling, stitching and the whole shift-variant restoration vs the oracle.

* the stitch kernel against the oracle's EDT-weighted blend (relative L2 1e-6)
  and the exact partition of unity on tiles cut from one image;
* the pipeline at fixed per-tile parameters (no iterations): tiles cropped,
  reconstructed with their own optics and blended, against the oracle doing
  the same steps (relative L2 1e-4, the reconstruction tolerance).
"""

import numpy as np
import pytest

import synth
from oracle import linear
from oracle import optics as op
from oracle import stitch
from oracle import tf as tfm

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("H,W,gy,gx,oy,ox", [(90, 110, 3, 4, 10, 8), (256, 200, 2, 5, 25, 12),
                                             (64, 64, 1, 1, 0, 0)])
def test_stitch_matches_oracle(gpu_lib, H, W, gy, gx, oy, ox):
    import torch
    print(f"[case] stitch {H}x{W} grid {gy}x{gx}", flush=True)
    ty, ys = gpu_lib.tile_grid(H, gy, oy)
    tx, xs = gpu_lib.tile_grid(W, gx, ox)
    rng = np.random.default_rng(H + W)
    tiles = rng.standard_normal((gy * gx, 2, ty, tx)).astype(np.float32)
    got = gpu_lib.stitch_tiles(torch.from_numpy(tiles).cuda(), ys, xs, H, W).cpu().numpy()
    ref = stitch.stitch(tiles.astype(np.float64), ys, xs, H, W)
    assert rel(got, ref) < 1e-6
    img = rng.standard_normal((2, H, W)).astype(np.float32)
    cut = np.stack([img[:, y:y + ty, x:x + tx] for y in ys for x in xs])
    got = gpu_lib.stitch_tiles(torch.from_numpy(cut).cuda(), ys, xs, H, W).cpu().numpy()
    assert np.max(np.abs(got - img)) < 1e-5


def test_fov_restoration_at_fixed_parameters_matches_oracle(gpu_lib):
    import torch
    from paper_2412_09775_amd import fov
    Z, H, W, grid, ovl = 8, 120, 150, (2, 3), (20, 16)
    print(f"[case] fov {Z}x{H}x{W} grid {grid}", flush=True)
    base = op.Optics(model=op.LABELFREE_THIN, nz=Z, ny=H, nx=W, dz=0.3, dy=0.1, dx=0.1, wavelength=0.532,
                     na_ill=0.5, na_det=1.15, n_medium=1.33, edge_width=0.5)
    f = synth.thin_cells((H, W), 0.1, 12, seed=31)
    d = (linear.forward(tfm.labelfree_thin(base.replace(defocus=0.3)), f)
         + synth.gaussian_noise((Z, H, W), 2e-3, 32)).astype(np.float32)
    ty, ys = stitch.tile_grid(H, grid[0], ovl[0])
    tx, xs = stitch.tile_grid(W, grid[1], ovl[1])
    n = len(ys) * len(xs)
    theta = np.array([[0.1 * i - 0.2, 1.1 + 0.02 * i, 0.05 * i, 0.0] for i in range(n)])
    tile_o = base.replace(ny=ty, nx=tx)
    eta = 1e-2 * linear.max_singular_value_sq(tfm.labelfree_thin(tile_o))
    tmpl = gpu_lib.Optics(model=2, nz=Z, ny=ty, nx=tx, dz=0.3, dy=0.1, dx=0.1, wavelength=0.532,
                          na_ill=0.5, na_det=1.15, n_medium=1.33, edge_width=0.5)
    field, _, _, geom = fov.restore_fov(torch.from_numpy(d).cuda(), tmpl, grid=grid, overlap=ovl, eta=eta,
                                        theta0=theta, iters=0)
    assert geom == (ys, xs, ty, tx)
    recs = []
    for iy, y0 in enumerate(ys):
        for ix, x0 in enumerate(xs):
            t = iy * len(xs) + ix
            o = tile_o.replace(defocus=theta[t, 0], na_det=theta[t, 1], tilt_zenith=theta[t, 2])
            recs.append(linear.reconstruct(tfm.labelfree_thin(o), d[:, y0:y0 + ty, x0:x0 + tx].astype(np.float64),
                                           eta=eta))
    ref = stitch.stitch(np.stack(recs), ys, xs, H, W)
    e = rel(field.cpu().numpy(), ref)
    print(f"  fov rel L2 {e:.2e}")
    assert e < 1e-4
