"""Pins of the oracle's vector label-free bank (Table 1, vector column), CPU only.

The bank is checked against computations that do not use its correlation of
fields or its angle-free pupil mapping:

* the brute-force source sum of the detected intensities behind each channel's
  analyser for a weak point dipole, with plane-wave sums written out and the
  polarisation bases built from the polar angles (the unified-framework
  section: label-free contrast is the direct-scatter interference summed over
  the source);
* the zero-frequency value from Parseval's theorem;
* the exact reduction to the paraxial polarisation bank (itself pinned against
  Jones intensities) and the second-order approach to it as the apertures
  shrink;
* covariance under a 90-degree rotation of microscope, polarisations and
  object about the optical axis.
"""

import math

import numpy as np
import pytest

from oracle import optics as op
from oracle import tf as tfm
from oracle import vector as vec


def vec_optics(**kw):
    base = dict(model=op.VECTOR_3D, nz=3, ny=8, nx=8, dz=0.3, dy=0.13, dx=0.13, wavelength=0.532,
                na_ill=0.45, na_det=0.8, n_medium=1.33)
    base.update(kw)
    return op.Optics(**base)


def polar_bases(o):
    """k^, t^, f^ (3-vectors) and r^, f^_t (pupil 2-vectors) from the polar angles
    t = asin(|p| / k_m), f = atan2(p_y, p_x) on the lateral grid (f = 0 at p = 0)."""
    fy, fx = op.lateral_frequencies(o)
    km = o.k_medium
    t = np.arcsin(np.minimum(np.hypot(fy, fx) / km, 1.0))
    f = np.arctan2(fy, fx)
    kh = np.stack([np.sin(t) * np.cos(f), np.sin(t) * np.sin(f), np.cos(t)], -1)
    th = np.stack([np.cos(t) * np.cos(f), np.cos(t) * np.sin(f), -np.sin(t)], -1)
    fh = np.stack([-np.sin(f), np.cos(f), np.zeros_like(f)], -1)
    rh = np.stack([np.cos(f), np.sin(f)], -1)
    fth = np.stack([-np.sin(f), np.cos(f)], -1)
    return kh, th, fh, rh, fth


def abbe_vector_response(o, J, M, T, eps=1e-3):
    """First-order response of the channel (J, M) to a point dipole tensor eps T at
    the origin by brute force: I(eps) = sum_q S(q) E^H M E, E = direct + scattered,
    direct = P(q) E(q) [r^ (t^ . e) + f^_t (f^ . e)] exp(i 2 pi (q . x + kz (z - dz0)))
    with e = r^.J t^ + f^_t.J f^ at q, scattered = 1/(Y X) sum_p P E g [r^ (t^ . d) +
    f^_t (f^ . d)] exp(...) with the dipole d = eps T e(q) and the transverse
    projection of d at p taken explicitly; returns (I(eps) - I(-eps)) / (2 eps I_bg)."""
    S = op.illumination_pupil(o)
    P = op.detection_pupil(o)
    E = op.aberration(o)
    fy, fx = op.lateral_frequencies(o)
    kz = op.axial_wavenumber(o)
    g = op.greens_spectrum(o)
    kh, th, fh, rh, fth = polar_bases(o)
    ys = np.arange(o.ny)[:, None] * o.dy
    xs = np.arange(o.nx)[None, :] * o.dx
    ibg = np.sum(S * P * P)
    J = np.asarray(J, dtype=np.complex128)

    def detect(v, p):
        """Pupil-plane 2-vector of the 3D field v travelling along p."""
        return rh[p] * (th[p] @ v) + fth[p] * (fh[p] @ v)

    out = np.zeros((o.nz, o.ny, o.nx))
    pidx = [tuple(p) for p in np.argwhere(P > 0)]
    for zi, z in enumerate(op.z_planes_3d(o)):
        waves = {p: np.exp(2j * np.pi * (fy[p] * ys + fx[p] * xs + kz[p] * (z - o.defocus))) for p in pidx}
        for q in map(tuple, np.argwhere(S * P > 0)):
            e = (rh[q] @ J) * th[q] + (fth[q] @ J) * fh[q]
            d = T @ e
            direct = [P[q] * E[q] * detect(e, q)[i] * waves[q] for i in range(2)]
            scat = [np.zeros((o.ny, o.nx), dtype=np.complex128) for _ in range(2)]
            for p in pidx:
                dt = d - kh[p] * (kh[p] @ d)                 # field radiated along p: transverse part
                a = P[p] * E[p] * g[p] * detect(dt, p) / (o.ny * o.nx)
                for i in range(2):
                    scat[i] += a[i] * waves[p]
            inten = []
            for sg in (eps, -eps):
                fld = [direct[i] + sg * scat[i] for i in range(2)]
                inten.append(np.real(sum(np.conj(fld[i]) * M[i, j] * fld[j] for i in range(2) for j in range(2))))
            out[zi] += S[q] * (inten[0] - inten[1]) / (2 * eps)
    return out / ibg


CASES = [dict(),
         dict(defocus=0.15, tilt_zenith=0.25, tilt_azimuth=0.7),
         dict(na_det=1.1, na_ill=0.3, tilt_zenith=0.2, tilt_azimuth=-2.0, zernike=(0.1, 0.0, -0.15))]


@pytest.mark.parametrize("kw", CASES)
def test_stokes_bank_is_the_abbe_sum_of_a_weak_point_dipole(kw):
    """Every Stokes channel and every spherical-harmonic tensor (real and imaginary
    coefficients) against the brute-force vector source sum."""
    o = vec_optics(vec_props=tuple(range(18)), ill_jones=(0.6, 0.8j * np.exp(0.3j)), **kw)
    bank = vec.vector_3d(o)
    scale = np.abs(bank).max()
    for c, (J, M) in enumerate(vec.channels(o)):
        for p, code in enumerate(o.vec_props):
            ref = np.fft.fftn(abbe_vector_response(o, J, M, vec.property_tensor(code)))
            assert np.max(np.abs(bank[c, p] - ref)) < 1e-10 * scale, (c, code)


def test_polarisation_state_bank_is_the_abbe_sum():
    o = vec_optics(vec_channels=vec.POL_STATES, vec_props=(0, 16, 8, 1, 14, 3), swing=0.12,
                   tilt_zenith=0.2, tilt_azimuth=0.4, defocus=-0.1)
    bank = vec.vector_3d(o)
    scale = np.abs(bank).max()
    for c, (J, M) in enumerate(vec.channels(o)):
        for p, code in enumerate(o.vec_props):
            ref = np.fft.fftn(abbe_vector_response(o, J, M, vec.property_tensor(code)))
            assert np.max(np.abs(bank[c, p] - ref)) < 1e-10 * scale, (c, code)


def test_mistakes_in_the_tensors_fail_the_abbe_sum():
    """What the brute force guards against: a conjugated, transposed object tensor
    and a flipped longitudinal row of the pupil map both fail it; dropping the
    Green's tensor's projector changes nothing, because the detection map already
    removes the longitudinal component (Q^T k^ = 0)."""
    o = vec_optics(tilt_zenith=0.25, tilt_azimuth=0.7, na_det=1.1)
    J, M = vec.channels(o)[1]
    T = vec.property_tensor(14)            # (xz + zx)/2: couples the z component
    ref = np.fft.fftn(abbe_vector_response(o, J, M, T))
    good = np.fft.fftn(2 * vec.point_response(o, J, M, T).real)
    scale = np.abs(good).max()
    assert np.max(np.abs(good - ref)) < 1e-10 * scale
    Q = vec.pupil_map(o)
    bad_T = np.fft.fftn(2 * vec.point_response(o, J, M, T.T.conj() * 1j).real)
    assert np.max(np.abs(bad_T - ref)) > 1e-3 * scale
    orig = vec.pupil_map
    try:
        vec.pupil_map = lambda o_, paraxial=False: Q * np.array([1.0, 1.0, -1.0])[:, None]
        flipped = np.fft.fftn(2 * vec.point_response(o, J, M, T).real)
    finally:
        vec.pupil_map = orig
    assert np.max(np.abs(flipped - ref)) > 1e-3 * scale
    origG = vec.greens_tensor
    try:
        vec.greens_tensor = lambda o_, paraxial=False: origG(o_, paraxial=True)
        unprojected = np.fft.fftn(2 * vec.point_response(o, J, M, T).real)
    finally:
        vec.greens_tensor = origG
    # the detection map already drops the longitudinal component (Q^T k^ = 0), so
    # the projection of G only matters through the pupil map; both must agree
    assert np.max(np.abs(unprojected - ref)) < 1e-10 * scale


@pytest.mark.parametrize("code", [0, 1, 6, 9, 12, 14, 17])
def test_zero_frequency_is_parseval(code):
    """H_cp(0) = nz 2 Re[(1 / I_bg) sum_p S P^2 g (J^H M Q^T T Q J)] (Parseval over
    each plane: the propagators cancel), with Q built from the polar angles."""
    o = vec_optics(vec_props=(code,), tilt_zenith=0.2, tilt_azimuth=1.1, ill_jones=(0.8, 0.6j))
    bank = vec.vector_3d(o)
    S, P = op.illumination_pupil(o), op.detection_pupil(o)
    g = op.greens_spectrum(o)
    _, th, fh, rh, fth = polar_bases(o)
    Q = th[..., :, None] * rh[..., None, :] + fh[..., :, None] * fth[..., None, :]
    T = vec.property_tensor(code)
    ibg = np.sum(S * P * P)
    for c, (J, M) in enumerate(vec.channels(o)):
        e = Q @ J
        w = np.einsum("i,ij,yxnj,nk,yxk->yx", np.conj(J), M, Q, T, e)
        ref = o.nz * 2 * np.real(np.sum(S * P * P * g * w) / ibg)
        assert abs(bank[c, 0, 0, 0, 0] - ref) < 1e-12 * max(1.0, abs(ref)), c


def test_paraxial_map_gives_the_polarisation_bank_exactly():
    """With Q = [I; 0] and G = g I the vector bank is the Jones reduction: the
    polarisation bank H = Re(kappa) H_phase + Im(kappa) H_abs."""
    for kw in (dict(), dict(defocus=0.2, tilt_zenith=0.2, tilt_azimuth=2.5, zernike=(0.1, -0.1))):
        o = vec_optics(vec_channels=vec.POL_STATES, vec_props=(0, 16, 8, 1), swing=0.09, **kw)
        got = vec.vector_3d(o, paraxial=True)
        ref = tfm.pol5_3d(o.replace(model=op.POL5_3D))
        assert np.max(np.abs(got - ref)) < 1e-12 * np.abs(ref).max()


def test_vector_bank_approaches_the_paraxial_bank_quadratically():
    """Scaling all lateral frequencies by s (apertures NA s, voxels / s, axial
    voxels / s^2 keep the lattice) the vector corrections are O(s^2)."""
    errs = []
    for s in (0.2, 0.1, 0.05):
        o = vec_optics(vec_channels=vec.POL_STATES, vec_props=(0, 16, 8, 1), na_det=0.8 * s,
                       na_ill=0.45 * s, dy=0.13 / s, dx=0.13 / s, dz=0.3 / s ** 2, tilt_zenith=0.2 * s)
        v = vec.vector_3d(o)
        p = tfm.pol5_3d(o.replace(model=op.POL5_3D))
        errs.append(np.linalg.norm(v - p) / np.linalg.norm(p))
    assert errs[0] < 0.05
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.5, errs


def _rot2(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s], [s, c]])


def test_rotating_microscope_and_object_rotates_the_bank():
    """Rotate everything by 90 degrees about z: source tilt azimuth + pi/2, Jones
    vector R J, analyser R M R^T, object tensor R3 T R3^T.  Each channel's
    response is then the old one on the rotated grid, H'(R nu) = H(nu)."""
    o = vec_optics(ny=8, nx=8, dy=0.13, dx=0.13, tilt_zenith=0.25, tilt_azimuth=0.4, defocus=0.1)
    R2 = _rot2(math.pi / 2)
    R3 = np.eye(3)
    R3[:2, :2] = R2
    o2 = o.replace(tilt_azimuth=o.tilt_azimuth + math.pi / 2)
    rng = np.random.default_rng(3)
    T = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    J = np.array([0.6, 0.8j])
    M = np.array([[0.3, 0.2 - 0.5j], [0.2 + 0.5j, -0.7]])
    h = np.fft.fftn(2 * vec.point_response(o, J, M, T).real)
    h2 = np.fft.fftn(2 * vec.point_response(o2, R2 @ J, R2 @ M @ R2.T, R3 @ T @ R3.T).real)
    # rotation by +90 degrees maps (kx, ky) -> (-ky, kx): H2[kz, ky', kx'] = H[kz, ky, kx]
    n = o.nx
    ky, kx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    moved = np.empty_like(h)
    moved[:, kx % n, (-ky) % n] = h[:, ky, kx]
    assert np.max(np.abs(h2 - moved)) < 1e-10 * np.abs(h).max()
    # and not without rotating the object tensor
    h3 = np.fft.fftn(2 * vec.point_response(o2, R2 @ J, R2 @ M @ R2.T, T).real)
    assert np.max(np.abs(h3 - moved)) > 1e-3 * np.abs(h).max()


def test_stokes_background_and_s0_of_unpolarised_average():
    """Backgrounds are J^H sigma_c J; averaging the S0 channel over two orthogonal
    illumination states gives a response that no longer depends on the pair."""
    o = vec_optics(ill_jones=(0.6, 0.8j))
    assert np.allclose(vec.channel_background(o), [1.0, 0.36 - 0.64, 0.0, 2 * 0.6 * 0.8])
    T = vec.property_tensor(0)
    M = vec.stokes_matrices()[0]
    pairs = [((1, 0), (0, 1)), ((2 ** -0.5, 2 ** -0.5), (2 ** -0.5, -(2 ** -0.5))),
             ((2 ** -0.5, 1j * 2 ** -0.5), (2 ** -0.5, -1j * 2 ** -0.5))]
    avg = [sum(vec.point_response(o, np.array(J, dtype=complex), M, T) for J in pr) for pr in pairs]
    for a in avg[1:]:
        assert np.allclose(a, avg[0], atol=1e-12 * np.abs(avg[0]).max())


def test_model_validity():
    with pytest.raises(ValueError):
        op.check_optics(vec_optics(det_tilt=0.1))
    with pytest.raises(ValueError):
        vec.property_tensor(18)
    assert tfm.bank_shape(vec_optics(vec_props=(0, 1))) == (4, 2, 3)
    assert tfm.bank_shape(vec_optics(vec_channels=1)) == (5, 4, 3)


def test_spherical_harmonic_tensors_are_the_stated_basis():
    """R25: Y_0 = I; Y_1..Y_3 antisymmetric, Y_4..Y_8 symmetric and traceless; all
    mutually orthogonal (Frobenius), |Y_b|^2 = 1/2 for b >= 1; the transverse
    blocks of Y_8 and Y_4 are the polarisation bank's diag(1, -1)/2 and
    [[0, 1], [1, 0]]/2; Y_6 is the m = 0 quadrupole (2 zz - xx - yy) / (2 sqrt 3)."""
    Y = [vec.sh_tensor(b) for b in range(9)]
    G = np.array([[np.sum(np.conj(a) * b) for b in Y] for a in Y])
    assert np.allclose(G, np.diag([3.0] + [0.5] * 8))
    assert np.allclose(Y[0], np.eye(3))
    for b in (1, 2, 3):
        assert np.allclose(Y[b], -Y[b].T)
    for b in range(4, 9):
        assert np.allclose(Y[b], Y[b].T) and abs(np.trace(Y[b])) < 1e-15
    assert np.allclose(Y[8][:2, :2], tfm.pol5_property_matrices()[1])
    assert np.allclose(Y[4][:2, :2], tfm.pol5_property_matrices()[2])
    assert np.allclose(Y[6], np.diag([-1.0, -1.0, 2.0]) / (2 * math.sqrt(3.0)))
    assert np.allclose(vec.property_tensor(1), 1j * np.eye(3))


def test_bank_at_one_frequency_is_the_bank():
    """The direct source sum at one frequency equals the FFT-based bank there."""
    o = vec_optics(nz=4, ny=8, nx=10, vec_props=(0, 16, 8, 1, 14, 7), tilt_zenith=0.15, defocus=0.1,
                   zernike=(0.05, 0.0, -0.1), ill_jones=(0.6, 0.8j))
    for chans in (vec.STOKES, vec.POL_STATES):
        oc = o.replace(vec_channels=chans, swing=0.07)
        bank = vec.vector_3d(oc)
        for k in [(0, 0, 0), (1, 2, 3), (3, 7, 9), (2, 5, 1)]:
            got = vec.vector_3d_at(oc, *k)
            assert np.allclose(got, bank[(slice(None), slice(None)) + k], atol=1e-12 * np.abs(bank).max())
