"""wo_reconstruct_noalloc (static library scratch, no workspace) against
wo_reconstruct (caller workspace) and the FP64 oracle, through the C ABI.

Two calls in a row on one GPU: the second with a smaller input, so a call that
read scratch values left behind by the previous one would differ from the
workspace call.  Both entry points run the same kernels with the same
schedules, so their outputs are compared bit for bit; each is also within the
reconstruction tolerance (relative L2 1e-4) of the oracle.
"""

import numpy as np
import pytest

import synth
from oracle import linear
from oracle import optics as op
from oracle import tf as tfm

pytestmark = pytest.mark.gpu

TOL_REC = 1e-4


def _case(o, n_obj, seed, b=None):
    """Oracle bank and data (oracle forward model + noise) of one patch."""
    bank = tfm.transfer_function(o)
    C, P = bank.shape[:2]
    if P == 1:   # fluorescence: point beads
        f = synth.beads((o.nz, o.ny, o.nx), 10 * n_obj, seed)[None]
    else:        # label-free: [phase, absorption] of random ellipsoids
        f = synth.ellipsoids((o.nz, o.ny, o.nx), (o.dz, o.dy, o.dx), n_obj, seed=seed,
                             semi_axes=(0.4, 1.0))
    d = linear.forward(bank, f, b) + synth.gaussian_noise((C, o.nz, o.ny, o.nx), 1e-3, seed + 10)
    return bank, d.astype(np.float32)


def _rel(got, ref):
    return float(np.linalg.norm(got.astype(np.float64) - ref) / np.linalg.norm(ref))


def test_noalloc_matches_workspace_call_twice_shrinking(gpu_lib):
    import torch
    api = gpu_lib
    dev = "cuda:0"
    big = op.Optics(model=op.LABELFREE_3D, nz=24, ny=96, nx=80, dz=0.2, dy=0.1, dx=0.1,
                    wavelength=0.532, na_ill=0.5, na_det=1.2, n_medium=1.33, defocus=0.2,
                    tilt_zenith=0.15, edge_width=0.5)
    small = op.Optics(model=op.FLUOR_3D, nz=16, ny=64, nx=48, dz=0.25, dy=0.1, dx=0.1,
                      wavelength=0.52, na_ill=0.0, na_det=1.2, n_medium=1.33, defocus=0.1)
    calls = [
        ([big, big.replace(defocus=-0.3)], 8, 1, None),
        ([small], 5, 3, np.array([[0.05]])),
    ]
    ws_sizes = []
    for optics, n_obj, seed, b in calls:
        print(f"noalloc case: model {optics[0].model} shape {optics[0].nz}x{optics[0].ny}x"
              f"{optics[0].nx} n={len(optics)}", flush=True)
        cases = [_case(o, n_obj, seed + 20 * i, None if b is None else b[i]) for i, o in enumerate(optics)]
        d = torch.from_numpy(np.stack([c[1] for c in cases])).to(dev)
        eta = 1e-3 * linear.max_singular_value_sq(cases[0][0])   # one eta per call
        tf = api.transfer_function(optics, device=dev)
        bt = None if b is None else torch.from_numpy(b.astype(np.float32)).to(dev)
        ws_sizes.append(api.workspace_size(optics, api.OP_RECONSTRUCT))
        assert ws_sizes[-1] <= api.NOALLOC_SCRATCH_BYTES
        f_ws = api.reconstruct(optics, tf, d, eta, b=bt)
        f_na = api.reconstruct_noalloc(optics, tf, d, eta, b=bt)
        torch.cuda.synchronize()
        got_ws, got_na = f_ws.cpu().numpy(), f_na.cpu().numpy()
        assert np.array_equal(got_na, got_ws)
        for i, (bank, di) in enumerate(cases):
            ref = linear.reconstruct(bank, di, None if b is None else b[i], eta)
            assert _rel(got_na[i], ref) < TOL_REC
    assert ws_sizes[1] < ws_sizes[0]


def test_noalloc_rejects_inputs_beyond_the_scratch(gpu_lib):
    import ctypes
    api = gpu_lib
    o = op.Optics(model=op.LABELFREE_3D, nz=96, ny=512, nx=512, dz=0.2, dy=0.1, dx=0.1,
                  wavelength=0.532, na_ill=0.5, na_det=1.2, n_medium=1.33)
    assert api.workspace_size([o], api.OP_RECONSTRUCT) > api.NOALLOC_SCRATCH_BYTES
    arr = api.optics_array([o])
    lib = api.load()
    st = lib.wo_reconstruct_noalloc(arr, 1, ctypes.c_void_p(1), ctypes.c_void_p(1), None,
                                    ctypes.c_double(1e-3), ctypes.c_void_p(1), None)
    assert st == -3
