"""Parity at the workloads' full sizes, in the bench's launch configuration.

* Label-free 96x512x512 (1 channel -> 2 properties): the FP64 oracle runs the
  whole volume (TF synthesis, forward model, reconstruction); comparison is
  element by element.
* Polarisation 64x1024x1024 (5 channels -> 4 properties): too large for the
  dense oracle solve.  The GPU bank is checked at sampled frequencies against
  the oracle's direct source sum (no FFT), and the reconstruction of a
  plane-wave input (plus a per-channel background) is checked at every voxel
  of every fourth plane against its closed form
  f_p(r) = sum_w Re[F_p(nu_w) exp(i 2 pi nu_w . r)],
  F(nu_w) = (H^H H + eta I)^-1 H^H (a_w e^{i phi_w}), H from the direct sum.

Each workload runs twice: through the full-layout calls with the default FFT
schedules, and through the calls the bench times -- the bank in the band
layout (the polarisation bank in its reduced form) with the schedules the
tuner picks at that size.
"""

import math
import os

import numpy as np
import pytest

import synth
from oracle import linear
from oracle import optics as op
from oracle import tf as tfm

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, dtype=np.result_type(a, np.float64)) - b) / np.linalg.norm(b))


LF = dict(model=op.LABELFREE_3D, nz=96, ny=512, nx=512, dz=0.2, dy=0.1, dx=0.1, wavelength=0.532,
          na_ill=0.5, na_det=1.2, n_medium=1.33)


@pytest.fixture(scope="module")
def labelfree_case():
    """The oracle's bank, specimen, data and reconstruction of the 96x512x512 volume."""
    import scipy.fft as sfft
    o = op.Optics(**LF)
    assert op.hard_edge_margin(o) > 1e-9
    with sfft.set_workers(len(os.sched_getaffinity(0))):
        bank = tfm.transfer_function(o)
        obj = synth.ellipsoids((96, 512, 512), (0.2, 0.1, 0.1), 200, seed=2001)
        clean = linear.forward(bank, obj)
        d = synth.poisson_gaussian(clean, seed=2002)
        eta = 1e-3 * linear.max_singular_value_sq(bank)
        ref_rec = linear.reconstruct(bank, d, None, eta)
    return o, bank, obj, clean, d, eta, ref_rec


def test_labelfree_96x512x512_full_volume(gpu_lib, labelfree_case):
    import torch
    o, bank, obj, clean, d, eta, ref_rec = labelfree_case
    print("[case] label-free 96x512x512 full volume", flush=True)
    tf = gpu_lib.transfer_function([o])
    e_tf = rel(tf[0].cpu().numpy(), bank[..., :257])
    fwd = gpu_lib.forward([o], tf, torch.from_numpy(obj[None]).cuda())
    e_fwd = rel(fwd[0].cpu().numpy(), clean)
    rec = gpu_lib.reconstruct([o], tf, torch.from_numpy(d[None]).cuda(), eta)
    e_rec = rel(rec[0].cpu().numpy(), ref_rec)
    print(f"  tf {e_tf:.2e}  forward {e_fwd:.2e}  reconstruct {e_rec:.2e}", flush=True)
    assert e_tf < 1e-5 and e_fwd < 1e-5 and e_rec < 1e-4


def test_labelfree_96x512x512_band_path_with_tuned_schedules(gpu_lib, labelfree_case):
    """The bench's step: band-layout synthesis + band reconstruction, schedules tuned
    at this size, against the oracle's reconstruction of the whole volume."""
    import torch
    o, bank, obj, clean, d, eta, ref_rec = labelfree_case
    print("[case] label-free 96x512x512 band path, tuned schedules", flush=True)
    dt = torch.from_numpy(d[None]).cuda()
    try:
        tfb = gpu_lib.transfer_function_band([o])
        gpu_lib.fft_tune(gpu_lib.OP_TRANSFER_FUNCTION, [o], out=tfb, reps=3, band=True)
        out = torch.empty((1, 2) + d.shape, dtype=torch.float32, device="cuda")
        gpu_lib.fft_tune(gpu_lib.OP_RECONSTRUCT, [o], tf=tfb, x=dt, out=out, eta=eta, reps=3, band=True)
        table = gpu_lib.fft_plans_export()
        tfb = gpu_lib.transfer_function_band([o])
        rec = gpu_lib.linear_band(gpu_lib.OP_RECONSTRUCT, [o], tfb, dt, eta)
    finally:
        gpu_lib.fft_plans_clear()
    e_rec = rel(rec[0].cpu().numpy(), ref_rec)
    print(f"  schedules: {table.splitlines()}\n  reconstruct {e_rec:.2e}", flush=True)
    assert e_rec < 1e-4


WAVES = [((1, 10, 20), 0.8, 0.3), ((3, -40, 15), 0.5, -1.1), ((-2, 25, -30), 0.6, 2.0),
         ((0, 60, 7), 0.4, 0.7), ((5, -3, 41), 0.3, -0.4), ((-6, -70, 33), 0.2, 1.5)]


POL5 = dict(model=op.POL5_3D, nz=64, ny=1024, nx=1024, dz=0.25, dy=0.1, dx=0.1, wavelength=0.532,
            na_ill=0.5, na_det=0.75, n_medium=1.33, swing=0.1)


@pytest.fixture(scope="module")
def pol5_case():
    """Plane-wave data (plus a background per channel) on the 64x1024x1024 grid,
    the oracle's bank at the waves' and at random frequencies, and the closed-form
    reconstruction coefficients F(nu_w)."""
    import torch
    Z, Y, X = POL5["nz"], POL5["ny"], POL5["nx"]
    o = op.Optics(**POL5)
    assert op.hard_edge_margin(o) > 1e-9
    rng = np.random.default_rng(12)
    samples = [(w[0][0] % Z, w[0][1] % Y, w[0][2] % X) for w in WAVES]
    samples += [(int(rng.integers(Z)), int(rng.integers(Y)), int(rng.integers(X // 2 + 1))) for _ in range(24)]
    Hs = {k: tfm.pol5_3d_at(o, *k) for k in samples}        # (5, 4) each, pinned against the Jones sum
    b = np.array([0.0, 0.1, 0.2, 0.3, 0.4])
    amps = rng.uniform(0.5, 1.5, (5, len(WAVES)))
    phs = rng.uniform(-math.pi, math.pi, (5, len(WAVES)))
    # each wave's lateral pattern once; every (channel, z) plane is a weighted sum of them
    yy = np.exp(2j * math.pi * np.outer([w[0][1] for w in WAVES], np.arange(Y)) / Y)   # (W, Y)
    xx = np.exp(2j * math.pi * np.outer([w[0][2] for w in WAVES], np.arange(X)) / X)   # (W, X)
    E = (yy[:, :, None] * xx[:, None, :]).reshape(len(WAVES), -1)                      # (W, Y*X)
    kz = np.array([w[0][0] for w in WAVES])
    a0 = np.array([w[1] for w in WAVES])
    p0 = np.array([w[2] for w in WAVES])
    d = torch.empty((1, 5, Z, Y, X), dtype=torch.float32, device="cuda")
    for c in range(5):
        coef = (a0 * amps[c])[None, :] * np.exp(1j * (2 * math.pi * np.outer(np.arange(Z), kz) / Z
                                                     + (p0 + phs[c])[None, :]))            # (Z, W)
        planes = b[c] + np.real(coef @ E).reshape(Z, Y, X)
        d[0, c] = torch.from_numpy(planes.astype(np.float32))
    eta = 1e-3 * max(np.linalg.svd(H, compute_uv=False)[0] ** 2 for H in Hs.values())
    # closed form: F(nu_w) from the direct-sum bank at nu_w
    Fw = []
    for w, (k, aw, pw) in enumerate(WAVES):
        H = Hs[(k[0] % Z, k[1] % Y, k[2] % X)]
        Dw = aw * amps[:, w] * np.exp(1j * (pw + phs[:, w]))
        Fw.append(np.linalg.solve(H.conj().T @ H + eta * np.eye(4), H.conj().T @ Dw))
    Fm = np.stack(Fw, 1)                                                                 # (4, W)
    bt = torch.from_numpy(b[None].astype(np.float32)).cuda()
    return o, Hs, d, bt, eta, Fm, E, kz


def pol5_reconstruction_error(rec, case):
    """Relative L2 over every fourth plane and all 4 properties against the closed form."""
    o, _, _, _, _, Fm, E, kz = case
    Z, Y, X = o.nz, o.ny, o.nx
    errs = []
    for z in range(0, Z, 4):
        got = rec[0, :, z].cpu().numpy().astype(np.float64)
        coef = Fm * np.exp(2j * math.pi * kz * z / Z)[None, :]
        ref = np.real(coef @ E).reshape(4, Y, X)
        errs.append((np.linalg.norm(got - ref) ** 2, np.linalg.norm(ref) ** 2))
    return math.sqrt(sum(a for a, _ in errs) / sum(r for _, r in errs))


def test_pol5_64x1024x1024_sampled_and_plane_waves(gpu_lib, pol5_case):
    o, Hs, d, bt, eta = pol5_case[:5]
    X = o.nx
    print("[case] pol5 64x1024x1024: TF at sampled frequencies", flush=True)
    tf = gpu_lib.transfer_function([o])          # (1, 5, 4, Z, Y, Xh)
    errs = []
    for (kz, ky, kx), H in Hs.items():
        if kx <= X // 2:
            got = tf[0, :, :, kz, ky, kx].cpu().numpy()
            errs.append((np.abs(got - H).max(), np.abs(H).max()))
    scale = max(s for _, s in errs)
    worst = max(e for e, _ in errs) / scale
    print(f"  sampled TF max error / max |H| = {worst:.2e}", flush=True)
    assert worst < 1e-5
    print("[case] pol5 64x1024x1024: plane-wave reconstruction", flush=True)
    rec = gpu_lib.reconstruct([o], tf, d, eta, b=bt)
    e_rec = pol5_reconstruction_error(rec, pol5_case)
    print(f"  reconstruction rel L2 over 16 planes x 4 properties = {e_rec:.2e}", flush=True)
    assert e_rec < 1e-4


def test_pol5_64x1024x1024_reduced_band_path_with_tuned_schedules(gpu_lib, pol5_case):
    """The bench's step: the reduced bank (label-free pair on its support) and the
    band reconstruction, schedules tuned at this size, against the closed form; the
    reduced pair expanded with the library's coupling against the sampled oracle bank."""
    import torch
    o, Hs, d, bt, eta = pol5_case[:5]
    print("[case] pol5 64x1024x1024 reduced band path, tuned schedules", flush=True)
    sup = gpu_lib.lateral_support([o])
    try:
        tfb = gpu_lib.transfer_function_band([o])
        gpu_lib.fft_tune(gpu_lib.OP_TRANSFER_FUNCTION, [o], out=tfb, reps=3, band=True)
        out = torch.empty((1, 4) + tuple(d.shape[2:]), dtype=torch.float32, device="cuda")
        gpu_lib.fft_tune(gpu_lib.OP_RECONSTRUCT, [o], tf=tfb, x=d, out=out, eta=eta, reps=3, band=True)
        table = gpu_lib.fft_plans_export()
        tfb = gpu_lib.transfer_function_band([o])
        rec = gpu_lib.linear_band(gpu_lib.OP_RECONSTRUCT, [o], tfb, d, eta, b=bt)
    finally:
        gpu_lib.fft_plans_clear()
    print(f"  schedules: {table.splitlines()}", flush=True)
    # the reduced pair at the sampled frequencies, expanded with the library's kappa:
    # row b of the band holds y = b (b <= h) or y = ny - band_rows + b, h = band_rows // 2
    kappa = gpu_lib.pol5_coupling(o.swing).astype(np.complex128)
    nb, kt, h = sup["band_rows"], sup["tf_cols"], sup["band_rows"] // 2
    pair = tfb[0, 0].cpu().numpy().astype(np.complex128)                # (2, Z, nb, kt)
    scale = max(np.abs(H).max() for H in Hs.values())
    worst, inside = 0.0, 0
    for (kz, ky, kx), H in Hs.items():
        row = ky if ky <= h else (ky - (o.ny - nb) if ky >= o.ny - nb + h + 1 else None)
        if kx > o.nx // 2:
            continue
        if row is None or kx >= kt:
            worst = max(worst, np.abs(H).max() / scale)                # off the support: zero
            continue
        hp, ha = pair[0, kz, row, kx], pair[1, kz, row, kx]
        got = kappa.real * hp + kappa.imag * ha
        worst = max(worst, np.abs(got - H).max() / scale)
        inside += 1
    print(f"  reduced pair x kappa vs oracle at {inside} sampled frequencies on the support: {worst:.2e}",
          flush=True)
    assert inside >= 6 and worst < 1e-5
    e_rec = pol5_reconstruction_error(rec, pol5_case)
    print(f"  reconstruction rel L2 over 16 planes x 4 properties = {e_rec:.2e}", flush=True)
    assert e_rec < 1e-4
