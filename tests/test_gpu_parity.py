"""GPU (HIP, FP32) vs FP64 oracle, element by element, through the C ABI.

Tolerances (relative L2 over all elements): transfer functions and the
forward model 1e-5, reconstruction 1e-4, adjoint 1e-5.  Inputs are seeded
synthetic specimens from ``synth``; data come from the oracle's forward model.
Shapes span several LDS tiles with ragged tails (Xh = X/2 + 1 columns, row
counts that do not fill the last workgroup).
"""

import math

import numpy as np
import pytest

import synth
from oracle import linear
from oracle import optics as op
from oracle import tf as tfm

pytestmark = pytest.mark.gpu

TOL_TF = 1e-5
TOL_FWD = 1e-5
TOL_REC = 1e-4
TOL_ADJ = 1e-5


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.complex128 if np.iscomplexobj(got) else np.float64)
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def half(bank):
    """Oracle full-spectrum bank -> the half spectrum along X the ABI stores."""
    return bank[..., : bank.shape[-1] // 2 + 1]


def fluor(nz=32, ny=64, nx=64, **kw):
    o = op.Optics(model=op.FLUOR_3D, nz=nz, ny=ny, nx=nx, dz=0.25, dy=0.1, dx=0.1,
                  wavelength=0.52, na_ill=0.0, na_det=1.2, n_medium=1.33)
    return o.replace(**kw)


def labelfree(nz=24, ny=96, nx=80, **kw):
    o = op.Optics(model=op.LABELFREE_3D, nz=nz, ny=ny, nx=nx, dz=0.2, dy=0.1, dx=0.1,
                  wavelength=0.532, na_ill=0.5, na_det=1.2, n_medium=1.33)
    return o.replace(**kw)


def pol5(nz=16, ny=64, nx=64, **kw):
    o = op.Optics(model=op.POL5_3D, nz=nz, ny=ny, nx=nx, dz=0.25, dy=0.1, dx=0.1,
                  wavelength=0.532, na_ill=0.5, na_det=0.75, n_medium=1.33, swing=0.1)
    return o.replace(**kw)


def sectors(nz=16, ny=64, nx=64, **kw):
    o = op.Optics(model=op.SECTORS9_3D, nz=nz, ny=ny, nx=nx, dz=0.2, dy=0.1, dx=0.1,
                  wavelength=0.532, na_ill=0.5, na_det=1.2, n_medium=1.33)
    return o.replace(**kw)


def vector(nz=12, ny=48, nx=40, **kw):
    o = op.Optics(model=op.VECTOR_3D, nz=nz, ny=ny, nx=nx, dz=0.25, dy=0.1, dx=0.1,
                  wavelength=0.532, na_ill=0.5, na_det=1.2, n_medium=1.33)
    return o.replace(**kw)


def thin(nz=32, ny=128, nx=128, **kw):
    o = op.Optics(model=op.LABELFREE_THIN, nz=nz, ny=ny, nx=nx, dz=0.2, dy=0.1, dx=0.1,
                  wavelength=0.532, na_ill=0.5, na_det=1.2, n_medium=1.33, edge_width=0.5)
    return o.replace(**kw)


CASES = {
    "fluor_cfg1": [fluor()],
    "fluor_defocus_odd": [fluor(nz=15, ny=48, nx=40, defocus=0.3)],
    "labelfree_3d": [labelfree()],
    "labelfree_3d_tilt_soft": [labelfree(nz=30, ny=48, nx=64, defocus=-0.25, tilt_zenith=0.3,
                                         tilt_azimuth=0.8, edge_width=0.5)],
    "pol5": [pol5()],
    "thin_batch3": [thin(defocus=0.4, na_det=1.05, tilt_zenith=0.2),
                    thin(defocus=-1.1, na_det=1.25, tilt_zenith=0.45, tilt_azimuth=0.3),
                    thin(defocus=0.0, na_det=1.15)],
    # degenerate and extreme cases: coherent point source (NA_ill = 0) with odd Z and
    # lengths without compiled stages; the smallest volume; the longest rows and the
    # deepest stack the ABI accepts (4096, runtime plans, one column per Z tile)
    "labelfree_coherent_odd": [labelfree(nz=9, ny=40, nx=50, na_ill=0.0, defocus=0.1)],
    "labelfree_tiny": [labelfree(nz=2, ny=8, nx=8)],
    "labelfree_rows_4096": [labelfree(nz=2, ny=8, nx=4096)],
    "fluor_depth_4096": [fluor(nz=4096, ny=8, nx=8, dz=0.25)],
    "pol5_ragged": [pol5(nz=12, ny=40, nx=50, tilt_zenith=0.1)],
    # 9 apertures (8 azimuthal sectors + the full disc) x phase; a tilted, soft-edged
    # batch of two with uncompiled lengths
    "sectors9": [sectors()],
    "sectors9_tilt_soft_batch2": [sectors(nz=12, ny=48, nx=40, defocus=0.2, tilt_zenith=0.2,
                                          tilt_azimuth=0.5, edge_width=0.5),
                                  sectors(nz=12, ny=48, nx=40, na_det=1.1, tilt_zenith=0.05,
                                          edge_width=0.5)],
    # detection aberrations (Noll 5..11, waves): every model, compiled and runtime lengths
    "labelfree_3d_aberrated": [labelfree(zernike=(0.15, -0.1, 0.08, 0.05, -0.04, 0.03, 0.12),
                                         tilt_zenith=0.2, edge_width=0.5)],
    "labelfree_aberrated_runtime": [labelfree(nz=9, ny=40, nx=50, zernike=(0.1,) * 7)],
    "fluor_aberrated": [fluor(zernike=(0.1, 0.0, 0.0, 0.2, 0.0, 0.0, -0.15), defocus=0.2)],
    "thin_aberrated_batch2": [thin(zernike=(0.1,)), thin(zernike=(0.0,) * 6 + (0.2,), defocus=0.5)],
    "pol5_aberrated": [pol5(zernike=(0.0, 0.0, 0.1))],
    "sectors9_aberrated": [sectors(zernike=(0.05, 0.05, 0.1))],
    # lateral band limits well inside the grid: the fields are kept on the
    # detection pupil's columns and the transfer function on its support until
    # the Z pass; a batch of two with different pupils (the support is their union)
    "labelfree_3d_band_batch2": [labelfree(nz=16, ny=96, nx=128, defocus=0.3, tilt_zenith=0.35,
                                           tilt_azimuth=2.0, edge_width=0.5),
                                 labelfree(nz=16, ny=96, nx=128, na_det=1.0, na_ill=0.3,
                                           edge_width=0.25)],
    "sectors9_band": [sectors(nz=12, ny=96, nx=128, tilt_zenith=0.2, tilt_azimuth=-0.7,
                              edge_width=0.5)],
    # the correlation's extent well below the grid: the synthesis runs on
    # shorter transforms (192 x 240 here) than the 256 x 256 grid
    "labelfree_3d_short_transforms": [labelfree(nz=8, ny=256, nx=256, defocus=-0.2, tilt_zenith=0.2,
                                                edge_width=0.5)],
    "sectors9_short_transforms": [sectors(nz=6, ny=256, nx=256, tilt_zenith=0.15, tilt_azimuth=1.1)],
    # polarisation bank on a support well inside the grid: synthesised on shortened
    # transforms as the label-free pair, then mixed by each patch's coupling
    "pol5_band": [pol5(nz=16, ny=96, nx=128, tilt_zenith=0.2, tilt_azimuth=0.6, edge_width=0.5)],
    "pol5_band_batch2_swings": [pol5(nz=12, ny=96, nx=96, swing=0.1),
                                pol5(nz=12, ny=96, nx=96, swing=0.05, defocus=0.3, na_ill=0.3)],
    # oblique detection: the detection pupil is the cap about a tilted axis (every
    # model; soft and hard edges; a batch with tilted and straight detection)
    "labelfree_3d_oblique": [labelfree(nz=16, ny=96, nx=80, na_det=0.9, det_tilt=0.35, det_azimuth=0.6,
                                       defocus=0.2, edge_width=0.5)],
    "labelfree_3d_oblique_hard_batch2": [labelfree(nz=12, ny=64, nx=64, na_det=0.8, det_tilt=0.3,
                                                   det_azimuth=-1.0),
                                         labelfree(nz=12, ny=64, nx=64, na_det=0.8)],
    "fluor_oblique": [fluor(nz=24, ny=64, nx=64, na_det=0.8, det_tilt=0.4, det_azimuth=2.0, edge_width=0.5)],
    "pol5_oblique": [pol5(nz=12, ny=96, nx=96, det_tilt=0.3, det_azimuth=0.4, edge_width=0.5)],
    "thin_oblique": [thin(nz=16, ny=64, nx=64, na_det=0.9, det_tilt=0.3, det_azimuth=1.2)],
    # vector (non-paraxial) label-free bank: Stokes channels under circular or
    # elliptical illumination, the five swing states, 2 or 4 spherical-harmonic
    # coefficients (phase, transverse birefringence, absorption; a z-coupled
    # quadrupole); tilted, defocused, aberrated and soft-edged patches
    "vector_stokes": [vector(tilt_zenith=0.2, tilt_azimuth=0.7, edge_width=0.5)],
    "vector_stokes_p2_batch2": [vector(nz=8, ny=64, nx=64, vec_props=(0, 14), ill_jones=(1.0, 0.0)),
                                vector(nz=8, ny=64, nx=64, vec_props=(0, 14), defocus=0.2,
                                       ill_jones=(0.6, 0.8j), edge_width=0.5, zernike=(0.1, 0.0, 0.05))],
    "vector_pol_states": [vector(nz=12, ny=64, nx=48, vec_channels=1, swing=0.08, defocus=-0.15,
                                 edge_width=0.5)],
    # the vector bank's support well inside the grid (band layout, compact spectra)
    "vector_band_batch2": [vector(nz=12, ny=96, nx=128, na_det=0.8, na_ill=0.4, vec_channels=1,
                                  tilt_zenith=0.15, edge_width=0.5),
                           vector(nz=12, ny=96, nx=128, na_det=0.8, na_ill=0.4, vec_channels=1, swing=0.05,
                                  defocus=0.2, edge_width=0.5)],
}


def oracle_bank(o):
    return tfm.transfer_function(o)


def specimen(o, seed):
    """A specimen with the structure of the workload, (P, *vol) float32."""
    C, P, dims = tfm.bank_shape(o)
    if o.model == op.FLUOR_3D:
        return synth.beads((o.nz, o.ny, o.nx), 50, seed)[None]
    if o.model == op.LABELFREE_3D:
        return synth.ellipsoids((o.nz, o.ny, o.nx), (o.dz, o.dy, o.dx), 12, seed, semi_axes=(0.5, 1.5))
    if o.model == op.POL5_3D:
        return synth.fibres((o.nz, o.ny, o.nx), (o.dz, o.dy, o.dx), 6, seed)
    if o.model == op.SECTORS9_3D:
        return synth.ellipsoids((o.nz, o.ny, o.nx), (o.dz, o.dy, o.dx), 12, seed, semi_axes=(0.5, 1.5))[:1]
    if o.model == op.VECTOR_3D:
        if P == 4:
            return synth.fibres((o.nz, o.ny, o.nx), (o.dz, o.dy, o.dx), 6, seed)
        return synth.ellipsoids((o.nz, o.ny, o.nx), (o.dz, o.dy, o.dx), 12, seed, semi_axes=(0.5, 1.5))[:P]
    return synth.thin_cells((o.ny, o.nx), o.dx, 8, seed)


def eta_for(o, bank):
    if o.model == op.FLUOR_3D:
        return 1e-3
    return 1e-3 * linear.max_singular_value_sq(bank)


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


@pytest.mark.parametrize("name", list(CASES))
def test_edges_are_decided_identically(name):
    for o in CASES[name]:
        if o.edge_width == 0:
            assert op.hard_edge_margin(o) > 1e-9
        if o.model == op.SECTORS9_3D and o.tilt_zenith != 0:
            # lattice points sit on a sector boundary (an axis or diagonal through the
            # tilted centre) exactly -- decided alike everywhere -- or keep away from it,
            # so FP64 rounding of the centre cannot flip a decision
            fy, fx = op.lateral_frequencies(o)
            cy, cx = op.source_centre(o)
            dy, dx = fy - cy, fx - cx
            r = np.hypot(dy, dx) + 1e-300
            inside = r <= o.na_ill / o.wavelength + o.edge_width * o.dnu
            for g in (dy, dx, dy - dx, dy + dx):
                m = np.abs(g[inside]) / r[inside]
                assert np.all((g[inside] == 0) | (m > 1e-9))


@pytest.mark.parametrize("name", list(CASES))
def test_transfer_function_matches_oracle(gpu_lib, torch, name):
    opts = CASES[name]
    print(f"[case] tf {name} shape={(opts[0].nz, opts[0].ny, opts[0].nx)} n={len(opts)}", flush=True)
    got = gpu_lib.transfer_function(opts).cpu().numpy()
    for i, o in enumerate(opts):
        ref = half(oracle_bank(o))
        err = rel_l2(got[i], ref)
        print(f"  patch {i}: rel L2 = {err:.3e}")
        assert err < TOL_TF


@pytest.mark.parametrize("name", list(CASES))
def test_forward_matches_oracle(gpu_lib, torch, name):
    opts = CASES[name]
    print(f"[case] forward {name}", flush=True)
    tf = gpu_lib.transfer_function(opts)
    fs = np.stack([specimen(o, 100 + i) for i, o in enumerate(opts)])
    C = tfm.bank_shape(opts[0])[0]
    b = np.linspace(0.1, 0.3, C * len(opts)).reshape(len(opts), C).astype(np.float32)
    d = gpu_lib.forward(opts, tf, torch.from_numpy(fs).cuda(), b=torch.from_numpy(b).cuda()).cpu().numpy()
    # the same kernels fed the oracle's bank isolate the FFT passes from TF synthesis
    tf_or = torch.from_numpy(np.stack([half(oracle_bank(o)) for o in opts]).astype(np.complex64)).cuda()
    d2 = gpu_lib.forward(opts, tf_or, torch.from_numpy(fs).cuda(), b=torch.from_numpy(b).cuda()).cpu().numpy()
    for i, o in enumerate(opts):
        ref = linear.forward(oracle_bank(o), fs[i], b[i])
        e1, e2 = rel_l2(d[i], ref), rel_l2(d2[i], ref)
        print(f"  patch {i}: gpu TF {e1:.3e}, oracle TF {e2:.3e}")
        assert e1 < TOL_FWD and e2 < TOL_FWD


@pytest.mark.parametrize("name", list(CASES))
def test_reconstruct_matches_oracle(gpu_lib, torch, name):
    opts = CASES[name]
    print(f"[case] reconstruct {name}", flush=True)
    tf = gpu_lib.transfer_function(opts)
    banks = [oracle_bank(o) for o in opts]
    C = banks[0].shape[0]
    ds, bs = [], []
    for i, o in enumerate(opts):
        f = specimen(o, 200 + i)
        b = np.full(C, 0.05 * (i + 1))
        d = linear.forward(banks[i], f, b) + synth.gaussian_noise((C,) + banks[i].shape[2:], 1e-3, 300 + i)
        ds.append(d.astype(np.float32))
        bs.append(b.astype(np.float32))
    ds, bs = np.stack(ds), np.stack(bs)
    etas = [eta_for(o, bk) for o, bk in zip(opts, banks)]
    eta = etas[0]
    got = gpu_lib.reconstruct(opts, tf, torch.from_numpy(ds).cuda(), eta,
                              b=torch.from_numpy(bs).cuda()).cpu().numpy()
    for i, o in enumerate(opts):
        ref = linear.reconstruct(banks[i], ds[i], bs[i], eta)
        err = rel_l2(got[i], ref)
        print(f"  patch {i}: rel L2 = {err:.3e}")
        assert err < TOL_REC


@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_matches_oracle(gpu_lib, torch, name):
    opts = CASES[name]
    print(f"[case] adjoint {name}", flush=True)
    tf = gpu_lib.transfer_function(opts)
    banks = [oracle_bank(o) for o in opts]
    C = banks[0].shape[0]
    rs = np.stack([synth.gaussian_noise((C,) + bk.shape[2:], 1.0, 400 + i) for i, bk in enumerate(banks)])
    got = gpu_lib.adjoint(opts, tf, torch.from_numpy(rs).cuda()).cpu().numpy()
    for i in range(len(opts)):
        ref = linear.adjoint(banks[i], rs[i])
        err = rel_l2(got[i], ref)
        print(f"  patch {i}: rel L2 = {err:.3e}")
        assert err < TOL_ADJ


@pytest.mark.parametrize("name", ["labelfree_3d_band_batch2", "sectors9_band", "labelfree_3d_tilt_soft",
                                  "labelfree_3d_short_transforms", "sectors9_short_transforms"])
def test_transfer_function_elementwise_at_support_edge(gpu_lib, torch, name):
    """Every value, including the faint ring at the edge of the support, within
    1e-5 of the largest (a support bound one column short fails this)."""
    opts = CASES[name]
    print(f"[case] tf elementwise {name}", flush=True)
    got = gpu_lib.transfer_function(opts).cpu().numpy()
    for i, o in enumerate(opts):
        ref = half(oracle_bank(o))
        err = np.max(np.abs(got[i] - ref)) / np.max(np.abs(ref))
        print(f"  patch {i}: max abs err / max = {err:.3e}")
        assert err < 1e-5


def test_fluorescence_eta_zero_is_pseudo_inverse(gpu_lib, torch):
    """P = 1 at eta = 0: F = D / H where H != 0 and 0 where H = 0."""
    o = fluor()
    bank = oracle_bank(o)
    f = specimen(o, 7)
    d = linear.forward(bank, f).astype(np.float32)
    tf = gpu_lib.transfer_function([o])
    got = gpu_lib.reconstruct([o], tf, torch.from_numpy(d[None]).cuda(), 0.0).cpu().numpy()[0]
    ref = linear.reconstruct(bank, d, None, 0.0)
    # only the well-conditioned band is comparable in FP32; compare in Fourier space there
    G, R = np.fft.fftn(got[0]), np.fft.fftn(ref[0])
    band = np.abs(bank[0, 0]) > 1e-2
    assert np.linalg.norm((G - R)[band]) / np.linalg.norm(R[band]) < 1e-4


def band_slice(torch, full, sup, ny):
    """The band layout cut from a full-layout bank (n, C, P, Z, Y, Xh)."""
    nb, kt = sup["band_rows"], sup["tf_cols"]
    ky = (nb - 1) // 2
    rows = list(range(ky + 1)) + list(range(ny - ky, ny)) if nb < ny else list(range(ny))
    return full[..., rows, :kt].contiguous(), rows


@pytest.mark.parametrize("name", ["labelfree_3d", "labelfree_3d_band_batch2", "labelfree_3d_short_transforms",
                                  "sectors9_band", "labelfree_3d_aberrated", "vector_band_batch2", "vector_stokes"])
def test_band_bank_is_the_full_bank_on_its_support(gpu_lib, torch, name):
    """wo_transfer_function_band writes bit for bit the values of the full bank on
    the support; the full bank is exactly zero off it."""
    opts = CASES[name]
    print(f"[case] band bank {name}", flush=True)
    sup = gpu_lib.lateral_support(opts)
    full = gpu_lib.transfer_function(opts)
    band = gpu_lib.transfer_function_band(opts)
    cut, rows = band_slice(torch, full, sup, opts[0].ny)
    assert tuple(band.shape) == tuple(cut.shape)
    assert torch.equal(band, cut)
    rest = full.clone()
    rest[..., rows, :sup["tf_cols"]] = 0
    assert int(torch.count_nonzero(rest)) == 0


@pytest.mark.parametrize("name", ["labelfree_3d_band_batch2", "labelfree_3d_short_transforms", "sectors9_band",
                                  "fluor_cfg1", "vector_band_batch2"])
def test_linear_calls_with_the_band_bank_equal_the_full_bank(gpu_lib, torch, name):
    """wo_linear_band (forward, reconstruction, adjoint) with the band layout cut from
    the full bank gives bit for bit the full-layout calls' results."""
    opts = CASES[name]
    print(f"[case] linear band {name}", flush=True)
    sup = gpu_lib.lateral_support(opts)
    full = gpu_lib.transfer_function(opts)
    band, _ = band_slice(torch, full, sup, opts[0].ny)
    C, P, _, _ = gpu_lib.bank_shape(opts)
    vol = (opts[0].nz, opts[0].ny, opts[0].nx)
    g = torch.Generator(device="cuda").manual_seed(7)
    f = torch.randn((len(opts), P) + vol, device="cuda", generator=g)
    d = torch.randn((len(opts), C) + vol, device="cuda", generator=g)
    b = torch.linspace(0.1, 0.2, len(opts) * C, device="cuda").reshape(len(opts), C)
    eta = 1e-2
    assert torch.equal(gpu_lib.linear_band(gpu_lib.OP_FORWARD, opts, band, f, b=b),
                       gpu_lib.forward(opts, full, f, b=b))
    assert torch.equal(gpu_lib.linear_band(gpu_lib.OP_RECONSTRUCT, opts, band, d, eta=eta, b=b),
                       gpu_lib.reconstruct(opts, full, d, eta, b=b))
    assert torch.equal(gpu_lib.linear_band(gpu_lib.OP_ADJOINT, opts, band, d),
                       gpu_lib.adjoint(opts, full, d))


POL5_BAND = ["pol5", "pol5_ragged", "pol5_band", "pol5_band_batch2_swings", "pol5_aberrated"]


def pol5_expand(gpu_lib, opts, red):
    """The 5 x 4 bank on the support from its reduced form, in plain FP32 on the host:
    Re(kappa) * H_phase + Im(kappa) * H_abs, each product and the sum rounded alone."""
    out = []
    for i, o in enumerate(opts):
        k = gpu_lib.pol5_coupling(o.swing)
        u, v = red[i, 0, 0], red[i, 0, 1]
        kr = k.real.astype(np.float32)[:, :, None, None, None]
        ki = k.imag.astype(np.float32)[:, :, None, None, None]
        re = kr * u.real[None, None] + ki * v.real[None, None]
        im = kr * u.imag[None, None] + ki * v.imag[None, None]
        out.append((re + 1j * im).astype(np.complex64))
    return np.stack(out)


@pytest.mark.parametrize("name", POL5_BAND)
def test_pol5_full_bank_is_the_expansion_of_its_reduced_form(gpu_lib, torch, name):
    """wo_transfer_function_band of the polarisation model is the label-free pair on
    the support; the full 5 x 4 bank is bit for bit its FP32 expansion there and
    exactly zero elsewhere; the pair is the oracle's label-free pair."""
    opts = CASES[name]
    print(f"[case] pol5 reduced bank {name}", flush=True)
    sup = gpu_lib.lateral_support(opts)
    red = gpu_lib.transfer_function_band(opts)
    assert tuple(red.shape) == (len(opts), 1, 2, opts[0].nz, sup["band_rows"], sup["tf_cols"])
    full = gpu_lib.transfer_function(opts)
    cut, rows = band_slice(torch, full, sup, opts[0].ny)
    redh = red.cpu().numpy()
    assert np.array_equal(cut.cpu().numpy(), pol5_expand(gpu_lib, opts, redh))
    rest = full.clone()
    rest[..., rows, :sup["tf_cols"]] = 0
    assert int(torch.count_nonzero(rest)) == 0
    for i, o in enumerate(opts):
        pair = tfm.labelfree_3d(o)[..., : o.nx // 2 + 1][..., rows, : sup["tf_cols"]]
        err = rel_l2(redh[i, 0], pair)
        print(f"  patch {i}: pair rel L2 = {err:.3e}")
        assert err < TOL_TF


@pytest.mark.parametrize("name", POL5_BAND)
def test_pol5_linear_calls_with_the_reduced_bank_equal_the_full_bank(gpu_lib, torch, name):
    """wo_linear_band with the reduced polarisation bank: the forward model and the
    adjoint (entries formed per frequency in the fused Z pass) give bit for bit the
    full-layout calls' results; the reconstruction (its Gram matrix formed from the
    pair and constants of the coupling, a different rounding order) is within 1e-4
    of the oracle's, and within 2e-5 of the full-layout call: two FP32 solves of
    one system differ by rounding (6e-8) amplified by cond(M + eta I) <= 1 + 1e3
    at eta = 1e-3 sigma_max^2."""
    opts = CASES[name]
    print(f"[case] pol5 reduced linear {name}", flush=True)
    red = gpu_lib.transfer_function_band(opts)
    full = gpu_lib.transfer_function(opts)
    C, P, _, _ = gpu_lib.bank_shape(opts)
    vol = (opts[0].nz, opts[0].ny, opts[0].nx)
    g = torch.Generator(device="cuda").manual_seed(11)
    f = torch.randn((len(opts), P) + vol, device="cuda", generator=g)
    r = torch.randn((len(opts), C) + vol, device="cuda", generator=g)
    b = torch.linspace(0.1, 0.2, len(opts) * C, device="cuda").reshape(len(opts), C)
    assert torch.equal(gpu_lib.linear_band(gpu_lib.OP_FORWARD, opts, red, f, b=b),
                       gpu_lib.forward(opts, full, f, b=b))
    assert torch.equal(gpu_lib.linear_band(gpu_lib.OP_ADJOINT, opts, red, r),
                       gpu_lib.adjoint(opts, full, r))
    banks = [oracle_bank(o) for o in opts]
    ds = []
    for i, o in enumerate(opts):
        d = linear.forward(banks[i], specimen(o, 500 + i), b[i].cpu().numpy())
        ds.append((d + synth.gaussian_noise((C,) + vol, 1e-3, 600 + i)).astype(np.float32))
    dt = torch.from_numpy(np.stack(ds)).cuda()
    eta = eta_for(opts[0], banks[0])
    got = gpu_lib.linear_band(gpu_lib.OP_RECONSTRUCT, opts, red, dt, eta=eta, b=b)
    ref_full = gpu_lib.reconstruct(opts, full, dt, eta, b=b)
    e_full = float(torch.linalg.vector_norm(got - ref_full) / torch.linalg.vector_norm(ref_full))
    print(f"  reduced vs full-layout reconstruction rel L2 = {e_full:.3e}")
    assert e_full < 2e-5
    for i in range(len(opts)):
        ref = linear.reconstruct(banks[i], ds[i], b[i].cpu().numpy().astype(np.float64), eta)
        err = rel_l2(got[i].cpu().numpy(), ref)
        print(f"  patch {i}: reconstruction rel L2 = {err:.3e}")
        assert err < TOL_REC
