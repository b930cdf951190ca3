"""Gradient of a loss of the 3D reconstruction (wo_reconstruct_grad) against the
FP64 oracle's reverse mode and central finite differences of the oracle's plain
definition L = <w, R_eta(theta) d> (Ext. Data Fig. 3: backpropagation through the
Tikhonov inverse into the transfer-function synthesis).

Tolerance: relative error 1e-3 (max over components / max |gradient|) for
dL/dtheta (defocus, NA, illumination tilt and azimuth, detection tilt and
azimuth), relative L2 1e-4 for dL/dd.  Inputs: oracle forward model of a
seeded specimen plus noise; w a seeded Gaussian field.
"""

import numpy as np
import pytest

import synth
from oracle import autotune as at
from oracle import linear
from oracle import optics as op
from oracle import tf as tfm

pytestmark = pytest.mark.gpu

TOL_THETA = 1e-3
TOL_DATA = 1e-4


def labelfree(**kw):
    base = dict(model=op.LABELFREE_3D, nz=16, ny=64, nx=48, dz=0.2, dy=0.1, dx=0.1, wavelength=0.532,
                na_ill=0.5, na_det=1.1, n_medium=1.33, defocus=0.25, tilt_zenith=0.2, tilt_azimuth=0.6,
                edge_width=0.5)
    base.update(kw)
    return op.Optics(**base)


def pol5(**kw):
    base = dict(model=op.POL5_3D, nz=12, ny=48, nx=64, dz=0.25, dy=0.1, dx=0.1, wavelength=0.532,
                na_ill=0.5, na_det=0.75, n_medium=1.33, defocus=-0.3, tilt_zenith=0.15, tilt_azimuth=1.1,
                edge_width=0.5, swing=0.1)
    base.update(kw)
    return op.Optics(**base)


CASES = {
    "labelfree": [labelfree()],
    "labelfree_batch2": [labelfree(nz=12, ny=40, nx=50), labelfree(nz=12, ny=40, nx=50, defocus=-0.4,
                                                                   na_det=1.0, tilt_zenith=0.05)],
    "labelfree_compiled_96": [labelfree(nz=8, ny=96, nx=96, defocus=0.1, tilt_zenith=0.3, tilt_azimuth=-0.5)],
    "pol5": [pol5()],
    # oblique detection: the gradient also along the detection axis's tilt and azimuth
    "labelfree_oblique": [labelfree(nz=12, ny=48, nx=48, na_det=0.9, det_tilt=0.3, det_azimuth=0.7)],
    "pol5_oblique": [pol5(det_tilt=0.25, det_azimuth=-0.5)],
}


def inputs(opts, seed):
    ds, ws = [], []
    for i, o in enumerate(opts):
        C, P, _ = tfm.bank_shape(o)
        bank = tfm.transfer_function(o)
        if o.model == op.POL5_3D:
            f = synth.fibres((o.nz, o.ny, o.nx), (o.dz, o.dy, o.dx), 4, seed + i)
        else:
            f = synth.ellipsoids((o.nz, o.ny, o.nx), (o.dz, o.dy, o.dx), 6, seed + i, semi_axes=(0.4, 1.0))
        d = linear.forward(bank, f) + synth.gaussian_noise((C, o.nz, o.ny, o.nx), 1e-3, seed + 10 + i)
        ds.append(d.astype(np.float32))
        ws.append(synth.gaussian_noise((P, o.nz, o.ny, o.nx), 1.0, seed + 20 + i).astype(np.float32))
    eta = 1e-2 * linear.max_singular_value_sq(tfm.transfer_function(opts[0]))
    return np.stack(ds), np.stack(ws), eta


def rel_vec(got, ref):
    return float(np.max(np.abs(np.asarray(got) - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("name", list(CASES))
def test_theta_and_data_gradients_match_the_oracle(gpu_lib, name):
    import torch
    opts = CASES[name]
    print(f"[case] reconstruct grad {name} shape={(opts[0].nz, opts[0].ny, opts[0].nx)} n={len(opts)}",
          flush=True)
    d, w, eta = inputs(opts, 100)
    C = d.shape[1]
    b = np.linspace(0.05, 0.15, len(opts) * C).reshape(len(opts), C).astype(np.float32)
    gth, gd = gpu_lib.reconstruct_grad(opts, torch.from_numpy(d).cuda(), eta, torch.from_numpy(w).cuda(),
                                       b=torch.from_numpy(b).cuda())
    gd = gd.cpu().numpy()
    for i, o in enumerate(opts):
        ref_th, ref_dd = at.recon_gradient(o, d[i], eta, w[i], b=b[i])
        e_th = rel_vec(gth[i], ref_th)
        e_dd = float(np.linalg.norm(gd[i] - ref_dd) / np.linalg.norm(ref_dd))
        print(f"  patch {i}: dL/dtheta gpu {gth[i]} oracle {ref_th} rel {e_th:.2e}; dL/dd rel L2 {e_dd:.2e}")
        assert e_th < TOL_THETA
        assert e_dd < TOL_DATA


@pytest.mark.parametrize("name", ["labelfree", "pol5", "labelfree_oblique"])
def test_theta_gradient_matches_central_differences(gpu_lib, name):
    """Against central differences (Richardson) of the oracle's plain definition."""
    import torch
    opts = CASES[name]
    print(f"[case] reconstruct grad vs FD {name}", flush=True)
    d, w, eta = inputs(opts, 200)
    gth, _ = gpu_lib.reconstruct_grad(opts, torch.from_numpy(d).cuda(), eta, torch.from_numpy(w).cuda(),
                                      want_data=False)
    fd = at.recon_fd_gradient(opts[0], d[0], eta, w[0], steps=(1e-5,) * 6)
    e = rel_vec(gth[0], fd)
    print(f"  gpu {gth[0]} fd {fd} rel {e:.2e}")
    assert e < TOL_THETA


def test_aberrated_optics_gradient_matches_central_differences(gpu_lib):
    import torch
    o = labelfree(nz=12, ny=48, nx=48, zernike=(0.1, -0.05, 0.08, 0.0, 0.04, 0.0, 0.06))
    print("[case] reconstruct grad aberrated", flush=True)
    d, w, eta = inputs([o], 300)
    gth, _ = gpu_lib.reconstruct_grad([o], torch.from_numpy(d).cuda(), eta, torch.from_numpy(w).cuda(),
                                      want_data=False)
    # aberrations are defined on the untilted pupil: the detection axis stays fixed
    fd = at.recon_fd_gradient(o, d[0], eta, w[0], steps=(1e-5,) * 6, which=(0, 1, 2, 3))[:4]
    e = rel_vec(gth[0][:4], fd)
    print(f"  gpu {gth[0][:4]} fd {fd} rel {e:.2e}")
    assert e < TOL_THETA


def test_autograd_reconstruction_gives_both_gradients(gpu_lib):
    """torch.autograd through reconstruct_fn: a quadratic loss of f; the gradients
    wrt the data and theta equal the oracle's reverse mode with w = dL/df."""
    import torch
    o = labelfree(nz=12, ny=48, nx=40)
    print("[case] autograd reconstruction", flush=True)
    d, _, eta = inputs([o], 400)
    target = synth.gaussian_noise((2, o.nz, o.ny, o.nx), 0.05, 401).astype(np.float32)
    dt = torch.from_numpy(d).cuda().requires_grad_(True)
    th = torch.tensor([[o.defocus, o.na_det, o.tilt_zenith, o.tilt_azimuth]], dtype=torch.float64,
                      requires_grad=True)
    f = gpu_lib.reconstruct_fn(dt, th, [o], eta)
    tt = torch.from_numpy(target[None]).cuda()
    loss = 0.5 * ((f - tt) ** 2).sum()
    loss.backward()
    w = (f - tt).detach().cpu().numpy()[0].astype(np.float64)      # dL/df
    ref_th, ref_dd = at.recon_gradient(o, d[0], eta, w)
    e_th = rel_vec(th.grad.numpy()[0], ref_th[:4])
    e_dd = float(np.linalg.norm(dt.grad.cpu().numpy()[0] - ref_dd) / np.linalg.norm(ref_dd))
    print(f"  theta rel {e_th:.2e}, data rel L2 {e_dd:.2e}")
    assert e_th < TOL_THETA and e_dd < TOL_DATA


def test_unsupported_models_are_rejected_on_the_host(gpu_lib):
    import ctypes
    lib = gpu_lib.load()
    o = op.Optics(model=op.FLUOR_3D, nz=16, ny=32, nx=32, dz=0.25, dy=0.1, dx=0.1, wavelength=0.52,
                  na_ill=0.0, na_det=1.2, n_medium=1.33)
    arr = gpu_lib.optics_array([o])
    assert lib.wo_reconstruct_grad_workspace_size(arr, 1) == 0
    one = ctypes.c_void_p(1)
    out = (ctypes.c_double * 6)()
    assert lib.wo_reconstruct_grad(arr, 1, one, None, ctypes.c_double(1e-3), one, out, None, one, 1 << 40,
                                   None) == -2
