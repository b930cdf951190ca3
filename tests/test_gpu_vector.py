"""Vector label-free bank on the GPU against the FP64 oracle (Table 1, vector column).

* Every spherical-harmonic coefficient (18 property codes over three calls),
  both channel sets, element by element on ragged grids with tilt, defocus,
  aberrations and soft edges (the forward model, reconstruction and adjoint
  with vector banks run in the shared parity suite).
* The bench's volume (Stokes 4 x 4, 64 x 512 x 512): the bank at sampled
  frequencies against the oracle's direct source sum.
* The GPU vector bank of the five swing states approaches the GPU
  polarisation bank (paraxial Jones reduction) as the apertures shrink, and
  differs from it at high NA.
"""

import numpy as np
import pytest

from oracle import optics as op
from oracle import tf as tfm
from oracle import vector as vec

pytestmark = pytest.mark.gpu


def vopt(**kw):
    base = dict(model=op.VECTOR_3D, nz=10, ny=40, nx=50, dz=0.25, dy=0.1, dx=0.1, wavelength=0.532,
                na_ill=0.5, na_det=1.2, n_medium=1.33)
    base.update(kw)
    return op.Optics(**base)


@pytest.mark.parametrize("chans", [vec.STOKES, vec.POL_STATES])
def test_every_property_code_elementwise(gpu_lib, chans):
    kw = dict(vec_channels=chans, tilt_zenith=0.25, tilt_azimuth=-0.9, defocus=0.1, edge_width=0.5,
              zernike=(0.05, -0.05, 0.1), ill_jones=(0.8, 0.6j * np.exp(0.4j)), swing=0.11)
    for codes in (tuple(range(8)), tuple(range(8, 16)), (16, 17)):
        o = vopt(vec_props=codes, **kw)
        print(f"[case] vector tf codes {codes} channels {chans}", flush=True)
        got = gpu_lib.transfer_function([o]).cpu().numpy()[0]
        ref = vec.vector_3d(o)[..., : o.nx // 2 + 1]
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"  max abs err / max = {err:.3e}", flush=True)
        assert err < 1e-5


def test_bench_volume_at_sampled_frequencies(gpu_lib):
    o = vopt(nz=64, ny=512, nx=512, vec_props=(0, 16, 8, 1))
    assert op.hard_edge_margin(o) > 1e-9
    print("[case] vector tf 64x512x512 sampled", flush=True)
    tf = gpu_lib.transfer_function([o])
    rng = np.random.default_rng(5)
    samples = [(0, 0, 0), (1, 3, 5), (63, 500, 20), (10, 40, 60), (32, 256, 100)]
    samples += [(int(rng.integers(64)), int(rng.integers(512)), int(rng.integers(60))) for _ in range(7)]
    got = np.stack([tf[0, :, :, k[0], k[1], k[2]].cpu().numpy() for k in samples])
    ref = np.stack([vec.vector_3d_at(o, *k) for k in samples])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"  rel L2 over {len(samples)} frequencies = {err:.3e}", flush=True)
    assert err < 1e-5


def test_vector_bank_approaches_the_polarisation_bank_at_low_na(gpu_lib):
    """Two GPU paths: the vector bank of the swing states and the polarisation bank;
    relative difference O(NA^2) (below 2 % at NA 0.1 / 0.05) and large at NA 1.2."""
    diffs = []
    for s in (1.0, 0.1):
        kw = dict(nz=12, ny=64, nx=64, dy=0.1 / s, dx=0.1 / s, dz=0.25 / s ** 2, na_det=1.2 * s, na_ill=0.5 * s,
                  swing=0.1)
        v = gpu_lib.transfer_function([vopt(vec_channels=vec.POL_STATES, vec_props=(0, 16, 8, 1), **kw)])
        p = gpu_lib.transfer_function([vopt(**kw).replace(model=op.POL5_3D)])
        d = float((v - p).abs().square().sum().sqrt() / p.abs().square().sum().sqrt())
        print(f"  scale {s}: rel diff {d:.3e}", flush=True)
        diffs.append(d)
    assert diffs[0] > 0.05 and diffs[1] < 0.02


def test_tuned_schedules_keep_the_vector_bank_and_reconstruction(gpu_lib):
    """The FFT tuner on the vector synthesis and on a reconstruction with the vector
    bank (band layout): the tuned calls still match the oracle."""
    import torch
    from oracle import linear
    o = vopt(nz=12, ny=96, nx=128, na_det=0.8, na_ill=0.4, vec_channels=vec.POL_STATES, vec_props=(0, 16, 8, 1),
             tilt_zenith=0.1, edge_width=0.5)
    print("[case] vector tf + reconstruction, tuned schedules", flush=True)
    bank = vec.vector_3d(o)
    rng = np.random.default_rng(9)
    f = rng.standard_normal((4, o.nz, o.ny, o.nx)) * 0.1
    d = linear.forward(bank, f).astype(np.float32)
    eta = 1e-3 * linear.max_singular_value_sq(bank)
    dt = torch.from_numpy(d[None]).cuda()
    try:
        tfb = gpu_lib.transfer_function_band([o])
        gpu_lib.fft_tune(gpu_lib.OP_TRANSFER_FUNCTION, [o], out=tfb, reps=2, band=True)
        out = torch.empty((1, 4, o.nz, o.ny, o.nx), dtype=torch.float32, device="cuda")
        gpu_lib.fft_tune(gpu_lib.OP_RECONSTRUCT, [o], tf=tfb, x=dt, out=out, eta=eta, reps=2, band=True)
        tf = gpu_lib.transfer_function([o]).cpu().numpy()[0]
        tfb = gpu_lib.transfer_function_band([o])
        rec = gpu_lib.linear_band(gpu_lib.OP_RECONSTRUCT, [o], tfb, dt, eta).cpu().numpy()[0]
    finally:
        gpu_lib.fft_plans_clear()
    half = bank[..., : o.nx // 2 + 1]
    e_tf = np.linalg.norm(tf - half) / np.linalg.norm(half)
    ref = linear.reconstruct(bank, d, None, eta)
    e_rec = np.linalg.norm(rec - ref) / np.linalg.norm(ref)
    print(f"  tf {e_tf:.2e}  reconstruct {e_rec:.2e}", flush=True)
    assert e_tf < 1e-5 and e_rec < 1e-4
