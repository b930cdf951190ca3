"""Uneven tiles: batched loss/gradient, auto-tune and thin restoration vs the FP64 oracle.

Tiles of different shapes (and a shape that repeats at non-adjacent positions,
so one launch group reads non-contiguous stacks) go through one call:

* loss and dL/dtheta of every tile against the oracle (loss 1e-4, gradient 1e-3);
* restoration without iterations: the best of two starts (by loss) and the
  thin Tikhonov reconstruction at it, against the oracle's choice and its
  reconstruction (relative L2 <= 1e-4, the reconstruction tolerance);
* restoration after Adam iterations: theta against the oracle's Adam, the
  reconstruction against wo_transfer_function + wo_reconstruct at the
  returned theta;
* plain launches, one iteration replayed as a graph, and the whole call as one
  graph launch (1 and 4 branches) give bitwise equal results.
"""

import numpy as np
import pytest

import synth
from oracle import autotune as at
from oracle import linear
from oracle import optics as op
from oracle import tf as tfm

pytestmark = pytest.mark.gpu

LR = (0.02, 0.005, 0.005, 0.001)
LO = (-2.0, 1.0, 0.0, -1.0)
HI = (2.0, 1.3, 0.5, 1.0)

# (nz, ny, nx) per tile; shape 0 repeats at tile 3
SHAPES = [(12, 64, 64), (8, 48, 80), (16, 80, 60), (12, 64, 64)]
TRUTHS = [dict(defocus=0.4, na_det=1.1, tilt_zenith=0.25),
          dict(defocus=-0.6, na_det=1.2, tilt_zenith=0.1),
          dict(defocus=0.2, na_det=1.05, tilt_zenith=0.35),
          dict(defocus=-0.2, na_det=1.15, tilt_zenith=0.2)]
STARTS = [dict(defocus=0.2, na_det=1.1, tilt_zenith=0.2),
          dict(defocus=-0.4, na_det=1.2, tilt_zenith=0.15),
          dict(defocus=0.1, na_det=1.05, tilt_zenith=0.3),
          dict(defocus=-0.1, na_det=1.15, tilt_zenith=0.25)]


def tile_optics(shape, **kw):
    nz, ny, nx = shape
    return op.Optics(model=op.LABELFREE_THIN, nz=nz, ny=ny, nx=nx, dz=0.3, dy=0.1, dx=0.1,
                     wavelength=0.532, na_ill=0.5, na_det=1.15, n_medium=1.33, edge_width=0.5).replace(**kw)


@pytest.fixture(scope="module")
def tiles():
    stacks, etas, nucs, starts = [], [], [], []
    for i, (shape, tr, s0) in enumerate(zip(SHAPES, TRUTHS, STARTS)):
        o = tile_optics(shape, **tr)
        f = synth.thin_cells((o.ny, o.nx), o.dx, 8, seed=70 + i)
        d = linear.forward(tfm.labelfree_thin(o), f) + synth.gaussian_noise(shape, 2e-3, 80 + i)
        nominal = tile_optics(shape)
        stacks.append(d.astype(np.float32))
        etas.append(1e-2 * linear.max_singular_value_sq(tfm.labelfree_thin(nominal)))
        nucs.append(at.nominal_cutoff(nominal))
        starts.append(tile_optics(shape, **s0))
    return starts, stacks, np.array(etas), np.array(nucs)


def dev(stacks):
    import torch
    return [torch.from_numpy(s).cuda() for s in stacks]


def test_uneven_loss_and_gradient_match_oracle(gpu_lib, tiles):
    starts, stacks, etas, nucs = tiles
    print(f"[case] uneven loss/grad shapes {SHAPES}", flush=True)
    loss, grad = gpu_lib.midband_loss_grad(starts, dev(stacks), etas, nucs)
    for i, o in enumerate(starts):
        L, g = at.loss_and_gradient(o, stacks[i].astype(np.float64), etas[i], nucs[i])
        el = abs(loss[i] - L) / abs(L)
        eg = np.max(np.abs(grad[i] - g)) / np.max(np.abs(g))
        print(f"  tile {i} {SHAPES[i]}: loss rel {el:.2e} grad rel {eg:.2e}")
        assert el < 1e-4 and eg < 1e-3


def test_restore_without_iterations_matches_oracle(gpu_lib, tiles):
    """Two starts per tile: the given one and one 1 um further out of focus; the
    restoration picks the lower loss and reconstructs there."""
    starts, stacks, etas, nucs = tiles
    print(f"[case] restore iters=0 shapes {SHAPES}", flush=True)
    n, M = len(starts), 2
    theta0 = np.zeros((n, M, 4))
    for i, o in enumerate(starts):
        theta0[i, 0] = at.theta_of(o)
        theta0[i, 1] = at.theta_of(o) + np.array([1.0, 0.0, 0.0, 0.0])
    out, loss, _, all_loss, f = gpu_lib.restore_tiles(starts, dev(stacks), etas, iters=0, multistart=M,
                                                      theta0=theta0, nu_c=nucs, lr=LR, lo=LO, hi=HI)
    for i, o in enumerate(starts):
        d64 = stacks[i].astype(np.float64)
        L = [at.loss(at.with_theta(o, theta0[i, s]), d64, etas[i], nucs[i]) for s in range(M)]
        best = int(np.argmin(L))
        assert int(np.argmin(all_loss[i])) == best
        assert np.allclose(all_loss[i], L, rtol=1e-4, atol=0)
        ob = at.with_theta(o, theta0[i, best])
        ref = linear.reconstruct(tfm.labelfree_thin(ob), d64, eta=etas[i])
        got = f[i].cpu().numpy()
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"  tile {i} {SHAPES[i]}: start {best} losses {all_loss[i]} recon rel {e:.2e}")
        assert e < 1e-4


def test_restore_after_adam_matches_oracle(gpu_lib, tiles):
    import torch
    starts, stacks, etas, nucs = tiles
    print(f"[case] restore iters=5 shapes {SHAPES}", flush=True)
    iters, mask = 5, 0b0101
    out, loss, _, _, f = gpu_lib.restore_tiles(starts, dev(stacks), etas, iters=iters, mask=mask,
                                               nu_c=nucs, lr=LR, lo=LO, hi=HI)
    for i, o in enumerate(starts):
        th, L = at.autotune(o, stacks[i].astype(np.float64), etas[i], nucs[i], iters, np.array(LR),
                            np.array(LO), np.array(HI), mask=(1, 0, 1, 0))
        got = np.array([out[i].defocus, out[i].na_det, out[i].tilt_zenith, out[i].tilt_azimuth])
        print(f"  tile {i}: gpu {got}\n          ora {th}")
        assert np.all(np.abs(got - th) <= 0.02 * np.array(LR) * iters + 1e-12)
        assert abs(loss[i] - L) / abs(L) < 1e-3
        # the restoration equals the plain calls at the returned theta
        tf = gpu_lib.transfer_function([out[i]])
        rec = gpu_lib.reconstruct([out[i]], tf, torch.from_numpy(stacks[i][None]).cuda(), float(etas[i]))
        a, b = f[i].cpu().numpy(), rec[0].cpu().numpy()
        assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(b)


@pytest.mark.parametrize("mode,branches", [(1, 0), (2, 1), (2, 4)])
def test_graph_modes_equal_plain_launches(gpu_lib, tiles, mode, branches):
    starts, stacks, etas, nucs = tiles
    print(f"[case] graph mode {mode} branches {branches}", flush=True)
    kw = dict(iters=3, nu_c=nucs, lr=LR, lo=LO, hi=HI, multistart=2,
              theta0=np.stack([[at.theta_of(o), at.theta_of(o) + [0.3, 0, 0, 0]] for o in starts]))
    a = gpu_lib.restore_tiles(starts, dev(stacks), etas, use_graph=0, **kw)
    b = gpu_lib.restore_tiles(starts, dev(stacks), etas, use_graph=mode, branches=branches, **kw)
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])
    for x, y in zip(a[4], b[4]):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())


@pytest.mark.parametrize("mode", [1, 2])
def test_reused_graph_takes_new_parameters(gpu_lib, tiles, mode):
    """A repeated call with the same buffers reuses its graph; the new starting
    parameters still take effect (they live in the workspace, not in the graph)."""
    import torch
    starts, stacks, etas, nucs = tiles
    print(f"[case] graph reuse mode {mode}", flush=True)
    d = gpu_lib.pack_stacks(dev(stacks))
    ws = torch.empty(gpu_lib.tune_workspace_size(starts, 1), dtype=torch.uint8, device="cuda")
    fo = torch.empty(sum(2 * o.ny * o.nx for o in starts), dtype=torch.float32, device="cuda")
    kw = dict(iters=3, nu_c=nucs, lr=LR, lo=LO, hi=HI, ws=ws, f_out=fo)
    th_a = np.stack([[at.theta_of(o)] for o in starts])
    th_b = th_a + np.array([0.25, 0.0, 0.05, 0.0])
    gpu_lib.restore_tiles(starts, d, etas, use_graph=mode, theta0=th_a, **kw)
    b1 = gpu_lib.restore_tiles(starts, d, etas, use_graph=mode, theta0=th_b, **kw)
    f1 = [x.cpu().numpy() for x in b1[4]]
    ref = gpu_lib.restore_tiles(starts, d, etas, use_graph=0, theta0=th_b, iters=3, nu_c=nucs, lr=LR,
                                lo=LO, hi=HI)
    assert np.array_equal(b1[2], ref[2]) and np.array_equal(b1[1], ref[1])
    for x, y in zip(f1, ref[4]):
        assert np.array_equal(x, y.cpu().numpy())


def test_graph_with_aberration_tuning_is_not_reused_for_plain_theta(gpu_lib, tiles):
    """A whole-call graph captured for theta-only tuning is not replayed for a call
    that tunes the aberration coefficients with the same shapes and buffers (the
    aberration-aware kernels differ); both equal their plain-launch results."""
    import torch
    starts, stacks, etas, nucs = tiles
    print("[case] graph keys with aberration tuning", flush=True)
    d = gpu_lib.pack_stacks(dev(stacks))
    ws = torch.empty(gpu_lib.tune_workspace_size(starts, 1), dtype=torch.uint8, device="cuda")
    fo = torch.empty(sum(2 * o.ny * o.nx for o in starts), dtype=torch.float32, device="cuda")
    kw = dict(iters=3, nu_c=nucs, lr=LR, lo=LO, hi=HI, ws=ws, f_out=fo)
    zkw = dict(mask=0b0101 | (0x7F << 4), lr_zernike=0.01, zernike_bound=0.3)
    res = {}
    for name, extra in (("theta", dict(mask=0b0101)), ("zern", zkw)):
        for mode in (2, 0):
            r = gpu_lib.restore_tiles(starts, d, etas, use_graph=mode, **kw, **extra)
            res[(name, mode)] = (r[1].copy(), [np.array(o.zernike) for o in r[0]],
                                 [x.cpu().numpy() for x in r[4]])
    for name in ("theta", "zern"):
        a, b = res[(name, 2)], res[(name, 0)]
        assert np.array_equal(a[0], b[0])
        for x, y in zip(a[2], b[2]):
            assert np.array_equal(x, y)
    # the aberration call moved the coefficients, the theta-only call did not
    assert all(np.any(z != 0) for z in res[("zern", 0)][1])
    assert all(len(z) == 0 or not np.any(z) for z in res[("theta", 0)][1])
