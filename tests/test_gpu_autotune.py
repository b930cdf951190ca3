"""GPU auto-tune path vs the FP64 oracle (thin phase-from-defocus model).

* mid-band loss: relative error <= 1e-4;
* dL/dtheta (hand-written reverse mode through the solve and the transfer
  function): relative error <= 1e-3 against the oracle's analytic gradient and
  against central finite differences of the oracle loss;
* Adam trajectory over a few iterations against the oracle's Adam;
* HIP-graph replay bitwise equal to eager launches;
* multistart keeps the lowest loss.
"""

import copy

import numpy as np
import pytest

import synth
from oracle import autotune as at
from oracle import linear
from oracle import optics as op
from oracle import tf as tfm

pytestmark = pytest.mark.gpu

TOL_LOSS = 1e-4
TOL_GRAD = 1e-3


def base_optics(**kw):
    o = op.Optics(model=op.LABELFREE_THIN, nz=12, ny=64, nx=64, dz=0.3, dy=0.1, dx=0.1,
                  wavelength=0.532, na_ill=0.5, na_det=1.15, n_medium=1.33, edge_width=0.5)
    return o.replace(**kw)


TRUTHS = [dict(defocus=0.4, na_det=1.1, tilt_zenith=0.25, tilt_azimuth=0.0),
          dict(defocus=-0.7, na_det=1.25, tilt_zenith=0.1, tilt_azimuth=0.0),
          dict(defocus=0.0, na_det=1.05, tilt_zenith=0.4, tilt_azimuth=0.0)]
STARTS = [dict(defocus=0.1, na_det=1.15, tilt_zenith=0.15, tilt_azimuth=0.0),
          dict(defocus=-0.3, na_det=1.2, tilt_zenith=0.2, tilt_azimuth=0.0),
          dict(defocus=0.2, na_det=1.1, tilt_zenith=0.3, tilt_azimuth=0.0)]


@pytest.fixture(scope="module")
def problem():
    """Three patches: thin cells imaged with their own true optics, plus noise."""
    stacks, etas = [], []
    nominal = base_optics()
    eta_abs = 1e-2 * linear.max_singular_value_sq(tfm.labelfree_thin(nominal))
    for i, tr in enumerate(TRUTHS):
        o = base_optics(**tr)
        f = synth.thin_cells((o.ny, o.nx), o.dx, 10, seed=50 + i)
        d = linear.forward(tfm.labelfree_thin(o), f) + synth.gaussian_noise((o.nz, o.ny, o.nx), 2e-3, 60 + i)
        stacks.append(d.astype(np.float32))
        etas.append(eta_abs)
    starts = [base_optics(**s) for s in STARTS]
    return starts, np.stack(stacks), np.array(etas), at.nominal_cutoff(nominal)


def test_loss_and_gradient_match_oracle(gpu_lib, problem):
    import torch
    starts, d, etas, nu_c = problem
    print(f"[case] loss/grad thin {d.shape}", flush=True)
    loss, grad = gpu_lib.midband_loss_grad(starts, torch.from_numpy(d).cuda(), etas, nu_c)
    for i, o in enumerate(starts):
        L, g = at.loss_and_gradient(o, d[i].astype(np.float64), etas[i], nu_c)
        el = abs(loss[i] - L) / abs(L)
        eg = np.max(np.abs(grad[i] - g)) / np.max(np.abs(g))
        print(f"  patch {i}: loss {loss[i]:.6e} vs {L:.6e} (rel {el:.2e}); grad rel {eg:.2e}")
        print(f"    gpu {grad[i]}\n    ora {g}")
        assert el < TOL_LOSS
        assert eg < TOL_GRAD


def test_gradient_matches_finite_differences(gpu_lib, problem):
    import torch
    starts, d, etas, nu_c = problem
    _, grad = gpu_lib.midband_loss_grad(starts[:1], torch.from_numpy(d[:1]).cuda(), etas[:1], nu_c)
    fd = at.fd_gradient(starts[0], d[0].astype(np.float64), etas[0], nu_c,
                        steps=[1e-3, 1e-4, 1e-3, 1e-3], which=(0, 1, 2))
    err = np.max(np.abs(grad[0][:3] - fd[:3])) / np.max(np.abs(fd[:3]))
    print(f"  gpu {grad[0]}\n  fd  {fd}\n  rel {err:.2e}")
    assert err < TOL_GRAD


def test_autograd_wrapper_gives_the_hand_gradient(gpu_lib, problem):
    import torch
    starts, d, etas, nu_c = problem
    theta = torch.tensor([[o.defocus, o.na_det, o.tilt_zenith, o.tilt_azimuth] for o in starts],
                         dtype=torch.float64, requires_grad=True)
    loss = gpu_lib.midband_loss_fn(theta, starts, torch.from_numpy(d).cuda(), etas, nu_c)
    loss.sum().backward()
    _, grad = gpu_lib.midband_loss_grad(starts, torch.from_numpy(d).cuda(), etas, nu_c)
    assert np.allclose(theta.grad.numpy(), grad, rtol=0, atol=0)


LR = (0.02, 0.005, 0.005, 0.001)
LO = (-2.0, 1.0, 0.0, -1.0)
HI = (2.0, 1.3, 0.5, 1.0)


@pytest.mark.parametrize("mask,patches", [(0b0101, (0, 1, 2)), (0b0111, (2,))])
def test_adam_trajectory_matches_oracle(gpu_lib, problem, mask, patches):
    """Adam normalises each gradient component, so a component whose gradient is
    ~0 (FP32 noise against an FP64 zero) takes steps of arbitrary sign; the
    trajectory is compared only on components with well-conditioned gradients
    (patches 0 and 1 have a vanishing NA gradient at their start)."""
    import torch
    starts, d, etas, nu_c = problem
    sel = list(patches)
    opts = [starts[i] for i in sel]
    iters = 5
    out, loss, _, _ = gpu_lib.autotune(opts, torch.from_numpy(d[sel]).cuda(), etas[sel], iters=iters,
                                       lr=LR, lo=LO, hi=HI, mask=mask, nu_c=nu_c)
    bits = tuple((mask >> j) & 1 for j in range(4))
    for k, i in enumerate(sel):
        th, L = at.autotune(starts[i], d[i].astype(np.float64), etas[i], nu_c, iters, np.array(LR),
                            np.array(LO), np.array(HI), mask=bits)
        got = np.array([out[k].defocus, out[k].na_det, out[k].tilt_zenith, out[k].tilt_azimuth])
        print(f"  patch {i}: gpu {got} loss {loss[k]:.6e}\n           ora {th} loss {L:.6e}")
        # Adam moves each parameter by about lr per step; agree to 2 % of that
        assert np.all(np.abs(got - th) <= 0.02 * np.array(LR) * iters + 1e-12)
        assert abs(loss[k] - L) / abs(L) < 1e-3


@pytest.mark.parametrize("iters", [1, 3])
def test_graph_replay_equals_eager(gpu_lib, problem, iters):
    import torch
    starts, d, etas, nu_c = problem
    dd = torch.from_numpy(d).cuda()
    a = gpu_lib.autotune(starts, dd, etas, iters=iters, lr=LR, lo=LO, hi=HI, nu_c=nu_c, use_graph=False)
    b = gpu_lib.autotune(starts, dd, etas, iters=iters, lr=LR, lo=LO, hi=HI, nu_c=nu_c, use_graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[1], b[1])


def test_multistart_keeps_the_lowest_loss(gpu_lib, problem):
    import torch
    starts, d, etas, nu_c = problem
    M = 3
    theta0 = np.zeros((len(starts), M, 4))
    for i, o in enumerate(starts):
        for s in range(M):
            theta0[i, s] = [o.defocus + 0.4 * (s - 1), o.na_det, o.tilt_zenith, 0.0]
    out, loss, all_theta, all_loss = gpu_lib.autotune(starts, torch.from_numpy(d).cuda(), etas, iters=4,
                                                      lr=LR, lo=LO, hi=HI, multistart=M, theta0=theta0,
                                                      nu_c=nu_c)
    for i in range(len(starts)):
        best = int(np.argmin(all_loss[i]))
        assert loss[i] == all_loss[i, best]
        assert out[i].defocus == all_theta[i, best, 0]


def test_linear_forward_autograd_uses_the_adjoint(gpu_lib):
    import torch
    o = op.Optics(model=op.LABELFREE_3D, nz=16, ny=48, nx=40, dz=0.2, dy=0.1, dx=0.1,
                  wavelength=0.532, na_ill=0.5, na_det=1.2, n_medium=1.33)
    bank = tfm.transfer_function(o)
    tf = gpu_lib.transfer_function([o])
    f = torch.from_numpy(synth.gaussian_noise((1, 2, 16, 48, 40), 1.0, 5)).cuda().requires_grad_(True)
    r = synth.gaussian_noise((1, 1, 16, 48, 40), 1.0, 6)
    d = gpu_lib.linear_forward_fn(f, [o], tf)
    (d * torch.from_numpy(r).cuda()).sum().backward()
    ref = linear.adjoint(bank, r[0])
    err = np.linalg.norm(f.grad.cpu().numpy()[0] - ref) / np.linalg.norm(ref)
    assert err < 1e-5


def test_gradients_at_tile_shape_match_finite_differences(gpu_lib):
    """Tile shape 32x128x128 with per-patch truth drawn from the auto-tune prior
    (defocus U(-2, 2) um, NA_det U(1.0, 1.3), zenith tilt U(0, 30 deg)): the GPU
    gradient of 8 patches x (defocus, NA, tilt) against central finite
    differences of the FP64 oracle loss, relative error <= 1e-3 per patch."""
    import math

    import torch
    rng = np.random.default_rng(77)
    nominal = op.Optics(model=op.LABELFREE_THIN, nz=32, ny=128, nx=128, dz=0.2, dy=0.1, dx=0.1,
                        wavelength=0.532, na_ill=0.5, na_det=1.15, n_medium=1.33, edge_width=0.5)
    eta = 1e-2 * linear.max_singular_value_sq(tfm.labelfree_thin(nominal))
    nu_c = at.nominal_cutoff(nominal)
    starts, stacks = [], []
    for i in range(8):
        tr = nominal.replace(defocus=rng.uniform(-2, 2), na_det=rng.uniform(1.0, 1.3),
                             tilt_zenith=rng.uniform(0, math.radians(30)))
        f = synth.thin_cells((128, 128), 0.1, 20, seed=700 + i)
        d = linear.forward(tfm.labelfree_thin(tr), f) + synth.gaussian_noise((32, 128, 128), 2e-3, 800 + i)
        stacks.append(d.astype(np.float32))
        starts.append(nominal.replace(defocus=tr.defocus + rng.uniform(-0.5, 0.5),
                                      na_det=float(np.clip(tr.na_det + rng.uniform(-0.05, 0.05), 1.0, 1.3)),
                                      tilt_zenith=float(np.clip(tr.tilt_zenith + rng.uniform(-0.1, 0.1), 0, 0.52))))
    stacks = np.stack(stacks)
    print("[case] tile-shape FD gradients, 8 patches", flush=True)
    _, grad = gpu_lib.midband_loss_grad(starts, torch.from_numpy(stacks).cuda(), np.full(8, eta), nu_c)
    for i, o in enumerate(starts):
        # small steps: the C1 smoothstep pupil edge has a discontinuous second
        # derivative, so Richardson-extrapolated differences need h well below
        # the edge width (a 1e-3 rad tilt step leaves ~1e-3 truncation error here)
        fd = at.fd_gradient(o, stacks[i].astype(np.float64), eta, nu_c, steps=[1e-4, 1e-5, 1e-5, 1e-5],
                            which=(0, 1, 2))
        err = np.max(np.abs(grad[i][:3] - fd[:3])) / np.max(np.abs(fd[:3]))
        print(f"  patch {i}: gpu {grad[i][:3]} fd {fd[:3]} rel {err:.2e}", flush=True)
        assert err < TOL_GRAD


ABER = (0.08, -0.05, 0.06, 0.04, -0.03, 0.02, 0.05)


@pytest.mark.parametrize("coeffs", [ABER, (0.0,) * 7])
def test_aberration_gradient_matches_finite_differences(gpu_lib, problem, coeffs):
    """dL/d(defocus, NA, tilt) of aberrated optics and dL/d(Zernike 5..11) (also at
    zero coefficients) against central differences of the FP64 oracle loss."""
    import torch
    starts, d, etas, nu_c = problem
    o = starts[0].replace(zernike=coeffs)
    print(f"[case] aberration gradient {coeffs}", flush=True)
    dd = torch.from_numpy(d[:1]).cuda()
    loss, grad = gpu_lib.midband_loss_grad([o], dd, etas[:1], nu_c, aberration=True)
    L = at.loss(o, d[0].astype(np.float64), etas[0], nu_c)
    assert abs(loss[0] - L) / abs(L) < TOL_LOSS
    fd_t = at.fd_gradient(o, d[0].astype(np.float64), etas[0], nu_c, steps=[1e-3, 1e-4, 1e-3, 1e-3],
                          which=(0, 1, 2))
    fd_c = at.fd_gradient_aberration(o, d[0].astype(np.float64), etas[0], nu_c, h=1e-3)
    et = np.max(np.abs(grad[0][:3] - fd_t[:3])) / np.max(np.abs(fd_t[:3]))
    ec = np.max(np.abs(grad[0][4:] - fd_c)) / np.max(np.abs(fd_c))
    print(f"  theta gpu {grad[0][:3]} fd {fd_t[:3]} rel {et:.2e}\n  zern gpu {grad[0][4:]}\n"
          f"       fd  {fd_c} rel {ec:.2e}")
    assert et < TOL_GRAD and ec < TOL_GRAD
    # the theta-only call on the same optics gives the same first four components
    _, g4 = gpu_lib.midband_loss_grad([o], dd, etas[:1], nu_c)
    if any(coeffs):
        assert np.array_equal(g4[0], grad[0][:4])


def test_adam_on_aberration_coefficients_matches_oracle(gpu_lib, problem):
    """Mask bits 4..10: Adam on the Zernike coefficients (theta held) against the
    oracle's Adam driven by central differences of its loss."""
    import torch
    starts, d, etas, nu_c = problem
    o = starts[2].replace(zernike=ABER)
    iters, lr_z, bound = 4, 0.01, 0.3
    print("[case] Adam on aberration coefficients", flush=True)
    out, loss, _, _ = gpu_lib.autotune([o], torch.from_numpy(d[2:3]).cuda(), etas[2:3], iters=iters,
                                       lr=LR, lo=LO, hi=HI, mask=0x7F << 4, nu_c=nu_c,
                                       lr_zernike=lr_z, zernike_bound=bound)
    c, L = at.autotune_aberration(o, d[2].astype(np.float64), etas[2], nu_c, iters, lr_z, bound)
    got = np.array(out[0].zernike)
    print(f"  gpu {got}\n  ora {c}")
    # theta held, every coefficient moved by about lr per step, as the oracle's
    assert out[0].defocus == o.defocus and out[0].na_det == o.na_det
    assert np.all(np.abs(got - c) <= 0.02 * lr_z * iters + 1e-6)
    assert abs(loss[0] - L) / abs(L) < 1e-3


@pytest.mark.parametrize("use_graph", [0, 1])
def test_nonfinite_patch_is_reported_and_does_not_fail_the_batch(gpu_lib, problem, use_graph):
    """A patch whose data hold a NaN (a condition forced from the host: every kernel
    still runs to its end, the NaN only propagates through arithmetic) ends with
    status WO_DIVERGED, keeps its starting optics and a NaN loss; the other patches
    tune exactly as in a batch without it."""
    import torch
    starts, d, etas, nu_c = problem
    bad = d.copy()
    bad[1, 3, 10, 20] = np.nan
    status = np.full(len(starts), 99, dtype=np.int32)
    out, loss, _, _ = gpu_lib.autotune(starts, torch.from_numpy(bad).cuda(), etas, iters=5, lr=LR, lo=LO,
                                       hi=HI, nu_c=nu_c, use_graph=use_graph, status=status)
    ref, ref_loss, _, _ = gpu_lib.autotune(starts, torch.from_numpy(d).cuda(), etas, iters=5, lr=LR, lo=LO,
                                           hi=HI, nu_c=nu_c, use_graph=use_graph)
    assert list(status) == [0, gpu_lib.DIVERGED, 0]
    assert np.isnan(loss[1])
    assert out[1].defocus == starts[1].defocus and out[1].tilt_zenith == starts[1].tilt_zenith
    for i in (0, 2):
        assert loss[i] == ref_loss[i]
        assert out[i].defocus == ref[i].defocus and out[i].tilt_zenith == ref[i].tilt_zenith
