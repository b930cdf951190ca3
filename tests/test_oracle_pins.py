"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test names the passage of the paper (or the mathematics) it pins.  The
checks are chosen so that a plausible mistake -- a dropped term, a wrong sign,
a conjugate on the wrong factor, a transposed operand, a lost normalisation --
fails at least one of them.
"""

import math

import numpy as np
import pytest

from oracle import autotune as at
from oracle import linear
from oracle import optics as op
from oracle import tf as tfm


def direct_dft(x, inverse=False):
    """O(N^2) DFT along every axis, written out from the definition."""
    out = np.asarray(x, dtype=np.complex128)
    for ax in range(out.ndim):
        n = out.shape[ax]
        k = np.arange(n)
        sgn = 1.0 if inverse else -1.0
        W = np.exp(sgn * 2j * np.pi * np.outer(k, k) / n)
        out = np.moveaxis(np.tensordot(W, np.moveaxis(out, ax, 0), axes=(1, 0)), 0, ax)
        if inverse:
            out = out / n
    return out


def lf_optics(**kw):
    base = dict(model=op.LABELFREE_3D, nz=5, ny=16, nx=16, dz=0.25, dy=0.1, dx=0.1,
                wavelength=0.532, na_ill=0.4, na_det=0.9, n_medium=1.33)
    base.update(kw)
    return op.Optics(**base)


def fl_optics(**kw):
    base = dict(model=op.FLUOR_3D, nz=6, ny=16, nx=16, dz=0.25, dy=0.1, dx=0.1,
                wavelength=0.52, na_ill=0.0, na_det=1.2, n_medium=1.33)
    base.update(kw)
    return op.Optics(**base)


# ---------------------------------------------------------------- FFT conventions

@pytest.mark.parametrize("shape", [(4, 6, 8), (3, 5, 7), (5, 8, 6), (16, 12, 10)])
def test_fft_matches_direct_dft(shape):
    import scipy.fft as sfft
    rng = np.random.default_rng(1)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    assert np.allclose(sfft.fftn(x), direct_dft(x), atol=1e-11)
    assert np.allclose(sfft.ifftn(x), direct_dft(x, inverse=True), atol=1e-12)


# ---------------------------------------------------------------- linear operators

def _random_bank(C, P, shape, seed):
    """A bank whose PSFs are random real arrays (H Hermitian by construction)."""
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((C, P) + shape)
    return h, np.fft.fftn(h, axes=tuple(range(2, 2 + len(shape))))


def _circulant_matrix(h, shape):
    """Dense real matrix A with (A f)_c(r) = sum_p sum_r' h_cp(r - r') f_p(r')."""
    C, P = h.shape[:2]
    N = int(np.prod(shape))
    idx = np.array(np.unravel_index(np.arange(N), shape)).T
    A = np.zeros((C * N, P * N))
    for i, r in enumerate(idx):
        diff = (r[None, :] - idx) % np.array(shape)
        lin = np.ravel_multi_index(diff.T, shape)
        for c in range(C):
            for p in range(P):
                A[c * N + i, p * N:(p + 1) * N] = h[c, p].reshape(-1)[lin]
    return A


@pytest.mark.parametrize("C,P,shape", [(1, 1, (3, 4, 5)), (2, 3, (2, 3, 4)), (3, 2, (4, 5))])
def test_forward_is_brute_force_circular_convolution(C, P, shape):
    """Convolution form of the shift-invariant model equals the Fourier form."""
    h, bank = _random_bank(C, P, shape, 2)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((P,) + shape)
    b = rng.standard_normal(C)
    N = int(np.prod(shape))
    idx = np.array(np.unravel_index(np.arange(N), shape)).T
    hf = h.reshape(C, P, -1)
    ff = f.reshape(P, -1)
    ref = np.zeros((C, N))
    for i, r in enumerate(idx):
        for j, rp in enumerate(idx):
            lin = np.ravel_multi_index(tuple((r - rp) % np.array(shape)), shape)
            ref[:, i] += hf[:, :, lin] @ ff[:, j]
    ref += b[:, None]
    got = linear.forward(bank, f, b)
    assert np.allclose(got.reshape(C, N), ref, atol=1e-11)
    assert linear.forward_imag_residual(bank, f) < 1e-13


@pytest.mark.parametrize("C,P,shape,eta", [(1, 1, (3, 4, 4), 0.3), (2, 3, (2, 3, 4), 0.05),
                                          (5, 4, (2, 2, 3), 1e-3), (4, 2, (3, 4), 0.2)])
def test_reconstruct_matches_dense_normal_equations_and_svd(C, P, shape, eta):
    """Tikhonov minimiser (Reconstructing object properties) and Eq. tls_solution via a dense SVD."""
    h, bank = _random_bank(C, P, shape, 4)
    A = _circulant_matrix(h, shape)
    rng = np.random.default_rng(5)
    d = rng.standard_normal((C,) + shape)
    b = rng.standard_normal(C)
    rhs = (d - b.reshape((C,) + (1,) * len(shape))).reshape(-1)
    dense = np.linalg.solve(A.T @ A + eta * np.eye(A.shape[1]), A.T @ rhs)
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    svd = Vt.T @ ((s / (s * s + eta)) * (U.T @ rhs))
    got = linear.reconstruct(bank, d, b, eta).reshape(-1)
    assert np.allclose(got, dense, atol=1e-10 * max(1, np.abs(dense).max()))
    assert np.allclose(got, svd, atol=1e-10 * max(1, np.abs(svd).max()))


def test_reconstruct_eta_zero_is_minimum_norm_least_squares():
    """eta -> 0 limit: the pseudo-inverse (SVD sum over the rank R), zero where H vanishes."""
    shape = (3, 4)
    h, bank = _random_bank(2, 2, shape, 6)
    bank[:, :, 1, 1] = 0.0          # a frequency and its mirror carry nothing
    bank[:, :, 2, 3] = 0.0
    h = np.fft.ifftn(bank, axes=(2, 3)).real
    A = _circulant_matrix(h, shape)
    d = np.random.default_rng(7).standard_normal((2,) + shape)
    ref = np.linalg.pinv(A, rcond=1e-10) @ d.reshape(-1)
    got = linear.reconstruct(bank, d, None, 0.0).reshape(-1)
    assert np.allclose(got, ref, atol=1e-9)


def test_noiseless_in_band_recovery_error_is_exactly_minus_eta_Minv_F():
    """With D = H F the per-frequency error is -eta (H^H H + eta)^-1 F -> 0 as eta -> 0."""
    shape = (4, 6)
    _, bank = _random_bank(3, 2, shape, 8)
    f = np.random.default_rng(9).standard_normal((2,) + shape)
    d = linear.forward(bank, f)
    F = np.fft.fftn(f, axes=(1, 2))
    Hn = np.moveaxis(bank.reshape(3, 2, -1), 2, 0)
    Fn = np.moveaxis(F.reshape(2, -1), 1, 0)
    errs = []
    for eta in (1e-1, 1e-3, 1e-6):
        got = np.moveaxis(linear.reconstruct_spectrum(bank, d, None, eta).reshape(2, -1), 1, 0)
        M = np.conj(np.swapaxes(Hn, 1, 2)) @ Hn + eta * np.eye(2)
        pred = -eta * np.linalg.solve(M, Fn[..., None])[..., 0]
        assert np.allclose(got - Fn, pred, atol=1e-9 * np.abs(Fn).max())
        errs.append(np.linalg.norm(linear.reconstruct(bank, d, None, eta) - f))
    assert errs[2] < 1e-4 * errs[0]


@pytest.mark.parametrize("C,P,shape", [(2, 3, (3, 4, 5)), (4, 2, (5, 6))])
def test_adjoint_is_transpose(C, P, shape):
    h, bank = _random_bank(C, P, shape, 10)
    A = _circulant_matrix(h, shape)
    r = np.random.default_rng(11).standard_normal((C,) + shape)
    assert np.allclose(linear.adjoint(bank, r).reshape(-1), A.T @ r.reshape(-1), atol=1e-10)
    f = np.random.default_rng(12).standard_normal((P,) + shape)
    lhs = np.vdot(linear.forward(bank, f), r)
    rhs = np.vdot(f, linear.adjoint(bank, r))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


# ---------------------------------------------------------------- fluorescence OTF

def test_fluorescence_otf_is_discrete_pupil_autocorrelation():
    """Table 1, scalar fluorescence row: H = [P * P] (correlation of the 3D pupil)."""
    o = fl_optics(nz=4, ny=8, nx=8, dx=0.13, dy=0.13, na_det=1.0, defocus=0.1)
    P = op.detection_pupil(o)
    h = np.stack([np.fft.ifft2(P * op.propagator(o, z)) for z in op.z_planes_3d(o)])
    P3 = direct_dft(h)
    N = h.size
    shape = h.shape
    ref = np.zeros(shape, dtype=np.complex128)
    for nu in np.ndindex(shape):
        shifted = np.roll(P3, shift=nu, axis=(0, 1, 2))     # P3(kappa - nu)
        ref[nu] = np.sum(P3 * np.conj(shifted)) / N
    ref /= ref[0, 0, 0]
    got = tfm.fluorescence_3d(o)
    assert np.allclose(got, ref, atol=1e-12)


def test_fluorescence_otf_normalisation_symmetry_support():
    o = fl_optics()
    H = tfm.fluorescence_3d(o)
    assert abs(H[0, 0, 0] - 1.0) < 1e-13
    # Hermitian; real and even for zero defocus
    mirror = np.conj(np.roll(np.flip(H), 1, axis=(0, 1, 2)))
    assert np.allclose(H, mirror, atol=1e-13)
    assert np.max(np.abs(H.imag)) < 1e-13
    # lateral support |nu_perp| <= 2 NA / lambda
    fy, fx = op.lateral_frequencies(o)
    out = np.sqrt(fy ** 2 + fx ** 2) > 2 * o.na_det / o.wavelength + 1e-9
    assert np.max(np.abs(H[:, out])) < 1e-13
    # projection-slice: sum over nu_z equals Z * FFT2 of the in-focus PSF plane
    P = op.detection_pupil(o)
    psf = np.stack([np.abs(np.fft.ifft2(P * op.propagator(o, z))) ** 2 for z in op.z_planes_3d(o)])
    psf /= psf.sum()
    assert np.allclose(H.sum(axis=0), o.nz * np.fft.fft2(psf[0]), atol=1e-13)


def test_fluorescence_infocus_otf_is_close_to_airy():
    """In-focus 2D OTF of a disc pupil -> (2/pi)(acos s - s sqrt(1 - s^2)), s = |nu| lambda/(2 NA)."""
    o = fl_optics(nz=1, ny=256, nx=256, dx=0.1, dy=0.1, na_det=0.9)
    P = op.detection_pupil(o)
    psf = np.abs(np.fft.ifft2(P)) ** 2
    otf = np.fft.fft2(psf).real / psf.sum()
    fy, fx = op.lateral_frequencies(o)
    s = np.sqrt(fy ** 2 + fx ** 2) * o.wavelength / (2 * o.na_det)
    sc = np.clip(s, 0, 1)
    airy = np.where(s < 1, (2 / np.pi) * (np.arccos(sc) - sc * np.sqrt(1 - sc ** 2)), 0.0)
    assert np.max(np.abs(otf - airy)) < 0.02


# ---------------------------------------------------------------- label-free TFs

def abbe_point_response(o, S=None):
    """Brute-force 'summing over the source': c(x, z) from the double sum over q and p."""
    if S is None:
        S = op.illumination_pupil(o)
    P = op.detection_pupil(o)
    E = op.aberration(o)            # detection aberration phase on the pupil (1 without)
    fy, fx = op.lateral_frequencies(o)
    kz = op.axial_wavenumber(o)
    km = o.k_medium
    ys = np.arange(o.ny)[:, None] * o.dy
    xs = np.arange(o.nx)[None, :] * o.dx
    zs = op.z_planes_thin(o) if o.model == op.LABELFREE_THIN else op.z_planes_3d(o)
    ibg = np.sum(S * P * P)
    out = np.zeros((o.nz, o.ny, o.nx), dtype=np.complex128)
    pidx = np.argwhere(P > 0)
    for qi in np.argwhere(S * P > 0):
        q = tuple(qi)
        for zi, z in enumerate(zs):
            acc = np.zeros((o.ny, o.nx), dtype=np.complex128)
            for pi in pidx:
                p = tuple(pi)
                # direct plane wave q through the aberrated pupil (conjugated in
                # b conj(a)), scattered plane wave p through it
                amp = S[q] * P[q] * np.conj(E[q]) * P[p] * E[p] * (1j * km / kz[p])
                ph = (fy[p] - fy[q]) * ys + (fx[p] - fx[q]) * xs + (kz[p] - kz[q]) * (z - o.defocus)
                acc += amp * np.exp(2j * np.pi * ph)
            out[zi] += acc
    return out / (o.ny * o.nx * ibg)


@pytest.mark.parametrize("kw", [dict(), dict(defocus=0.3, tilt_zenith=0.2, tilt_azimuth=0.7),
                                dict(model=op.LABELFREE_THIN, nz=3, defocus=-0.2, edge_width=0.5),
                                dict(defocus=0.1, tilt_zenith=0.1, zernike=(0.2, -0.1, 0.15, 0.0, 0.1, 0, 0.2))])
def test_labelfree_point_response_is_abbe_source_sum(kw):
    """Label-free contrast summed over source points (unified-framework section)."""
    o = lf_optics(ny=8, nx=8, dx=0.13, dy=0.13, na_det=0.8, na_ill=0.45, **kw)
    got = tfm.labelfree_point_response(o)
    ref = abbe_point_response(o)
    assert np.allclose(got, ref, atol=1e-12 * np.abs(ref).max())


def test_labelfree_3d_symmetries_and_dc():
    """Hermitian (Summary of TFs); on-axis in-focus: H_abs real-even, H_phase imaginary-odd in nu_z."""
    o = lf_optics()
    Hp, Ha = tfm.labelfree_3d(o)
    for H in (Hp, Ha):
        mirror = np.conj(np.roll(np.flip(H), 1, axis=(0, 1, 2)))
        assert np.allclose(H, mirror, atol=1e-12)
    assert np.max(np.abs(Ha.imag)) < 1e-12
    assert np.max(np.abs(Hp.real)) < 1e-12
    zflip = np.roll(np.flip(Hp, axis=0), 1, axis=0)
    assert np.allclose(Hp, -zflip, atol=1e-12)
    assert np.max(np.abs(Hp[0])) < 1e-12            # phase vanishes on the nu_z = 0 plane (odd Z)
    # DC: H_phase(0) = 0, H_abs(0) = -2 Z sum S P^2/cos / sum S P^2
    S, P = op.illumination_pupil(o), op.detection_pupil(o)
    cos = op.axial_wavenumber(o) / o.k_medium
    ratio = np.sum(S * P * P / np.where(cos > 0, cos, 1)) / np.sum(S * P * P)
    assert abs(Hp[0, 0, 0]) < 1e-12
    assert abs(Ha[0, 0, 0] - (-2 * o.nz * ratio)) < 1e-12


def test_labelfree_dc_holds_with_tilt_and_defocus():
    o = lf_optics(nz=6, defocus=0.4, tilt_zenith=0.3, tilt_azimuth=1.1)
    Hp, Ha = tfm.labelfree_3d(o)
    S, P = op.illumination_pupil(o), op.detection_pupil(o)
    cos = op.axial_wavenumber(o) / o.k_medium
    ratio = np.sum(S * P * P / np.where(cos > 0, cos, 1)) / np.sum(S * P * P)
    assert abs(Hp[0, 0, 0]) < 1e-12
    assert abs(Ha[0, 0, 0] + 2 * o.nz * ratio) < 1e-12
    # lateral support inside (NA_det + NA_ill)/lambda + |q0|
    fy, fx = op.lateral_frequencies(o)
    cy, cx = op.source_centre(o)
    rad = (o.na_det + o.na_ill) / o.wavelength + math.hypot(cy, cx)
    out = np.sqrt(fy ** 2 + fx ** 2) > rad + 1e-9
    assert np.max(np.abs(Hp[:, out])) < 1e-12 and np.max(np.abs(Ha[:, out])) < 1e-12


def test_labelfree_dc_ratio_continuum_limit():
    """<1/cos> over an on-axis disc -> 2 / (1 + cos alpha_ill) (continuum closed form)."""
    o = lf_optics(nz=1, ny=512, nx=512, dx=0.1, dy=0.1, na_ill=0.5, na_det=1.2)
    Hp, Ha = tfm.labelfree_3d(o)
    cos_a = math.sqrt(1 - (o.na_ill / o.n_medium) ** 2)
    assert abs(Ha[0, 0, 0] / (-2.0) - 2 / (1 + cos_a)) < 2e-3


@pytest.mark.parametrize("defocus", [0.0, 0.35])
def test_thin_coherent_limit_is_textbook_weak_object_tf(defocus):
    """Single on-axis source point: H_phase = -2 P sin(psi)/cos, H_abs = -2 P cos(psi)/cos,
    psi = 2 pi (kz - k_m)(z - defocus) (classical weak-object transfer functions)."""
    o = lf_optics(model=op.LABELFREE_THIN, nz=4, na_ill=0.02, defocus=defocus)
    assert np.sum(op.illumination_pupil(o)) == 1.0
    bank = tfm.labelfree_thin(o)
    P = op.detection_pupil(o)
    kz = op.axial_wavenumber(o)
    cos = np.where(kz > 0, kz / o.k_medium, 1.0)
    for k, z in enumerate(op.z_planes_thin(o)):
        psi = 2 * np.pi * (kz - o.k_medium) * (z - defocus)
        assert np.allclose(bank[k, 0], -2 * P * np.sin(psi) / cos, atol=1e-12)
        assert np.allclose(bank[k, 1], -2 * P * np.cos(psi) / cos, atol=1e-12)


def test_thin_phase_vanishes_in_focus():
    """Phase contrast disappears in focus (Results: in-focus disappearance)."""
    o = lf_optics(model=op.LABELFREE_THIN, nz=5, defocus=0.0)
    bank = tfm.labelfree_thin(o)
    assert np.max(np.abs(bank[2, 0])) < 1e-12          # z_2 = 0 plane
    assert np.max(np.abs(bank[0, 0])) > 1e-2


# ---------------------------------------------------------------- polarisation bank

def test_pol5_coupling_against_jones_intensities():
    """kappa from finite perturbations of the channel intensity |a^H J e_c|^2."""
    swing = 0.1
    k = tfm.pol5_coupling(swing)
    states, a = tfm.pol5_states(swing)
    Bs = tfm.pol5_property_matrices()
    eps = 1e-6
    for c, e in enumerate(states):
        for p, B in enumerate(Bs):
            def inten(J):
                return abs(np.conj(a) @ (J @ e)) ** 2
            dre = (inten(np.eye(2) + eps * B) - inten(np.eye(2) - eps * B)) / (2 * eps)
            dim = (inten(np.eye(2) + 1j * eps * B) - inten(np.eye(2) - 1j * eps * B)) / (2 * eps)
            assert abs(dre - 2 * k[c, p].real) < 1e-8
            assert abs(dim + 2 * k[c, p].imag) < 1e-8
    assert np.max(np.abs(k[0])) < 1e-15                 # extinction channel carries nothing
    assert np.allclose(k[:, 3], 1j * k[:, 0])            # absorption = i * phase coupling
    # as the swing goes to zero the retardance couplings vanish linearly and the
    # isotropic ones (phase, absorption) quadratically, as sin^2(pi swing)
    k1, k2 = tfm.pol5_coupling(1e-4), tfm.pol5_coupling(2e-4)
    assert np.allclose(k2[:, 1:3], 2 * k1[:, 1:3], rtol=1e-3, atol=1e-14)
    assert np.allclose(k2[:, [0, 3]], 4 * k1[:, [0, 3]], rtol=1e-3, atol=1e-14)
    # per frequency the 5x4 system has rank 3: phase and absorption share the isotropic response
    h1, h2 = 0.3 + 0.2j, -0.7 + 0.1j
    assert np.linalg.matrix_rank(k.real * h1 + k.imag * h2, tol=1e-9) == 3


def test_pol5_background():
    bg = tfm.pol5_background(0.1)
    assert bg[0] < 1e-15 and np.all(bg[1:] > 0)
    assert np.allclose(bg[1:], math.sin(math.pi * 0.1) ** 2)


def jones_abbe_channel_response(o, e, a, B, eps=1e-3):
    """First-order channel response of a weak point scatterer with Jones
    perturbation eps * B at the origin, by brute force over source points:
    I(eps) = sum_q S(q) |a^H (e d_q + eps B e s)|^2 with the direct plane wave
    d_q = P(q) E(q) exp(i 2 pi (q.x + kz(q)(z - dz0))) carrying the illumination
    state e through the pupil, and the scattered field
    s = (1 / (Y X)) sum_p P(p) E(p) g(p) exp(i 2 pi (p.x + kz(p)(z - dz0)))
    carrying B e; returns (I(eps) - I(-eps)) / (2 eps I_bg) on the (Z, Y, X) grid
    (exact: I is quadratic in eps).  Jones vectors throughout; the
    kappa-composition of the bank is not used."""
    S = op.illumination_pupil(o)
    P = op.detection_pupil(o)
    E = op.aberration(o)
    fy, fx = op.lateral_frequencies(o)
    kz = op.axial_wavenumber(o)
    ys = np.arange(o.ny)[:, None] * o.dy
    xs = np.arange(o.nx)[None, :] * o.dx
    ibg = np.sum(S * P * P)
    g = np.where(P > 0, 1j * o.k_medium / np.where(kz > 0, kz, 1.0), 0.0)
    pidx = np.argwhere(P > 0)
    ah = np.conj(a)
    out = np.zeros((o.nz, o.ny, o.nx))
    for zi, z in enumerate(op.z_planes_3d(o)):
        s = np.zeros((o.ny, o.nx), dtype=np.complex128)
        for p in map(tuple, pidx):
            s += P[p] * E[p] * g[p] * np.exp(2j * np.pi * (fy[p] * ys + fx[p] * xs + kz[p] * (z - o.defocus)))
        s /= o.ny * o.nx
        scat = B @ e                                   # Jones vector of the scattered wave
        for q in map(tuple, np.argwhere(S * P > 0)):
            d = P[q] * E[q] * np.exp(2j * np.pi * (fy[q] * ys + fx[q] * xs + kz[q] * (z - o.defocus)))
            inten = []
            for sg in (eps, -eps):
                field = [e[j] * d + sg * scat[j] * s for j in range(2)]     # (Ex, Ey) on the grid
                inten.append(np.abs(ah[0] * field[0] + ah[1] * field[1]) ** 2)
            out[zi] += S[q] * (inten[0] - inten[1]) / (2 * eps)
    return out / ibg


def test_pol5_bank_is_the_jones_abbe_response_of_a_weak_point_scatterer():
    """The 5 x 4 bank against the brute-force channel intensities of a point scatterer
    with each property's Jones perturbation (Table 1 vector row, paraxial reading R9):
    FFT3 of the first-order response of channel c to property p equals H_cp.  A sign
    slip on the Im(kappa) term or swapped phase/absorption columns fails here."""
    o = lf_optics(model=op.POL5_3D, nz=3, ny=8, nx=8, dx=0.13, dy=0.13, na_det=0.8, na_ill=0.45,
                  defocus=0.15, tilt_zenith=0.2, tilt_azimuth=0.7, swing=0.1)
    bank = tfm.pol5_3d(o)
    states, a = tfm.pol5_states(o.swing)
    Bs = tfm.pol5_property_matrices()
    scale = np.abs(bank).max()
    for c, e in enumerate(states):
        for p, B in enumerate(Bs):
            ref = np.fft.fftn(jones_abbe_channel_response(o, e, a, B))
            assert np.max(np.abs(bank[c, p] - ref)) < 1e-10 * scale, (c, p)
    # the flipped compositions are far off (what this test guards against)
    hp, ha = tfm.labelfree_3d(o)
    k = tfm.pol5_coupling(o.swing)
    ref = np.fft.fftn(jones_abbe_channel_response(o, states[1], a, Bs[1]))
    for wrong in (k[1, 1].real * hp - k[1, 1].imag * ha, k[1, 1].real * ha + k[1, 1].imag * hp):
        assert np.max(np.abs(wrong - ref)) > 1e-3 * scale


def test_pol5_bank_at_one_frequency_is_the_bank():
    """The one-frequency polarisation bank (direct source sum) equals pol5_3d there."""
    o = lf_optics(model=op.POL5_3D, nz=4, ny=8, nx=10, dx=0.13, dy=0.13, na_det=0.8, na_ill=0.45,
                  defocus=0.1, tilt_zenith=0.15, swing=0.08)
    bank = tfm.pol5_3d(o)
    for k in [(0, 0, 0), (1, 2, 3), (3, 7, 9), (2, 5, 1)]:
        assert np.allclose(tfm.pol5_3d_at(o, *k), bank[(slice(None), slice(None)) + k],
                           atol=1e-12 * np.abs(bank).max())


def test_jones_abbe_response_reduces_to_the_scalar_phase_response():
    """Scalar limit of the brute force: an analyser that passes the illumination
    state entirely and an isotropic perturbation (B = I, B = i I) give the scalar
    label-free phase and absorption point responses 2 Re c and -2 Im c."""
    o = lf_optics(nz=3, ny=8, nx=8, dx=0.13, dy=0.13, na_det=0.8, na_ill=0.45, defocus=0.15,
                  tilt_zenith=0.2, tilt_azimuth=0.7)
    c = abbe_point_response(o)
    e = np.array([1.0, 1.0j]) / math.sqrt(2.0)
    ph = jones_abbe_channel_response(o, e, e, np.eye(2))
    ab = jones_abbe_channel_response(o, e, e, 1j * np.eye(2))
    assert np.allclose(ph, 2 * c.real, atol=1e-11 * np.abs(c).max())
    assert np.allclose(ab, -2 * c.imag, atol=1e-11 * np.abs(c).max())


# ---------------------------------------------------------------- auto-tune pieces

def test_analytic_gradient_matches_finite_differences():
    """Backpropagated dL/dtheta (Ext. Data Fig. 3) vs central FD with Richardson."""
    from synth import thin_cells
    o = op.Optics(model=op.LABELFREE_THIN, nz=5, ny=32, nx=32, dz=0.3, dy=0.1, dx=0.1,
                  wavelength=0.532, na_ill=0.5, na_det=1.1, n_medium=1.33,
                  defocus=0.25, tilt_zenith=0.2, tilt_azimuth=0.4, edge_width=0.5)
    truth = o.replace(defocus=0.1, na_det=1.15, tilt_zenith=0.3)
    f = thin_cells((32, 32), 0.1, 6, seed=3).astype(np.float64)
    d = linear.forward(tfm.labelfree_thin(truth), f)
    eta = 1e-2 * linear.max_singular_value_sq(tfm.labelfree_thin(o))
    nu_c = at.nominal_cutoff(o)
    L, g = at.loss_and_gradient(o, d, eta, nu_c)
    assert abs(L - at.loss(o, d, eta, nu_c)) < 1e-12 * abs(L)
    fd = at.fd_gradient(o, d, eta, nu_c, steps=[1e-3, 1e-4, 1e-3, 1e-3])
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-7 * np.abs(fd).max())


def test_adam_first_step_is_signed_learning_rate():
    """Adam's bias correction makes the first step lr * g / (|g| + eps)."""
    st = at.AdamState(np.zeros(4), np.zeros(4), np.zeros(4))
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    lr = np.array([0.02, 0.005, 0.005, 0.001])
    at.adam_step(st, g, lr, -np.inf, np.inf)
    assert np.allclose(st.theta, -lr * g / (np.abs(g) + 1e-8))


def test_hard_edges_of_test_optics_are_not_on_lattice_points():
    for o in (lf_optics(), fl_optics()):
        assert op.hard_edge_margin(o) > 1e-6


@pytest.mark.parametrize("zern", [(), (0.1, 0.0, -0.12, 0.05, 0.0, 0.08, 0.1)])
def test_direct_frequency_sum_equals_the_bank(zern):
    """One-frequency evaluation by the direct source sum (no FFT) equals the FFT-route bank."""
    o = lf_optics(nz=8, ny=32, nx=32, defocus=0.1, tilt_zenith=0.1, tilt_azimuth=0.4, zernike=zern)
    hp, ha = tfm.labelfree_3d(o)
    for kz, ky, kx in [(0, 0, 0), (1, 2, 3), (7, 31, 5), (3, 10, 30), (4, 16, 16)]:
        a, b = tfm.labelfree_3d_at(o, kz, ky, kx)
        assert abs(a - hp[kz, ky, kx]) < 1e-12 and abs(b - ha[kz, ky, kx]) < 1e-12


# ---------------------------------------------------------------- 9-aperture bank

def test_octant_is_the_azimuth_sector():
    rng = np.random.default_rng(5)
    dy, dx = rng.standard_normal((2, 2000))
    ang = np.mod(np.arctan2(dy, dx), 2 * np.pi)
    assert np.array_equal(op.octant(dy, dx), np.floor(ang / (np.pi / 4)).astype(int))
    # boundaries belong to the sector they open; the origin to sector 0
    pts = [(0, 1, 0), (1, 1, 1), (1, 0, 2), (1, -1, 3), (0, -1, 4), (-1, -1, 5), (-1, 0, 6), (-1, 1, 7),
           (0, 0, 0)]
    for y, x, k in pts:
        assert int(op.octant(float(y), float(x))) == k


def test_sectors_partition_the_source_and_their_tfs_add_up():
    o = lf_optics(model=op.SECTORS9_3D, nz=8, ny=32, nx=32, tilt_zenith=0.15, tilt_azimuth=0.4)
    S = op.illumination_pupil(o)
    parts = [op.sector_pupil(o, c) for c in range(8)]
    assert np.array_equal(np.sum(parts, axis=0), S) and np.array_equal(op.sector_pupil(o, 8), S)
    P = op.detection_pupil(o)
    bank = tfm.sectors9_3d(o)
    ib = [np.sum(Sc * P * P) for Sc in parts]
    # the unnormalised responses are linear in S: sum_c I_bg,c H_c = I_bg H_full
    lhs = sum(ib[c] * bank[c, 0] for c in range(8))
    rhs = np.sum(S * P * P) * bank[8, 0]
    assert np.allclose(lhs, rhs, atol=1e-12 * np.abs(rhs).max())
    assert np.allclose(bank[8, 0], tfm.labelfree_3d(o.replace(model=op.LABELFREE_3D))[0],
                       atol=1e-13 * np.abs(bank[8, 0]).max())
    # Hermitian: H(-nu) = conj H(nu) for every aperture
    for c in range(9):
        H = bank[c, 0]
        Hm = np.roll(np.flip(H, axis=(0, 1, 2)), 1, axis=(0, 1, 2))
        assert np.allclose(Hm, np.conj(H), atol=1e-12 * np.abs(H).max())


def test_sector_point_response_is_abbe_source_sum():
    o = lf_optics(model=op.SECTORS9_3D, nz=3, ny=24, nx=24, na_det=0.8, na_ill=0.45,
                  defocus=0.2, tilt_zenith=0.1, tilt_azimuth=0.3)
    for c in (0, 3, 6):
        Sc = op.sector_pupil(o, c)
        assert np.count_nonzero(Sc) >= 1
        got = tfm.labelfree_point_response(o, Sc)
        ref = abbe_point_response(o, Sc)
        assert np.allclose(got, ref, atol=1e-12 * np.abs(ref).max())


# ---------------------------------------------------------------- gradient of the 3D reconstruction

def _recon_case(model, seed=0, **kw):
    import synth
    base = dict(model=model, nz=6, ny=16, nx=16, dz=0.25, dy=0.13, dx=0.13, wavelength=0.532,
                na_ill=0.4, na_det=0.9, n_medium=1.33, defocus=0.12, tilt_zenith=0.15, tilt_azimuth=0.4,
                edge_width=0.5, swing=0.1)
    base.update(kw)
    o = op.Optics(**base)
    C, P, _ = tfm.bank_shape(o)
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(C, o.nz, o.ny, o.nx))
    w = rng.normal(size=(P, o.nz, o.ny, o.nx))
    eta = 1e-2 * linear.max_singular_value_sq(tfm.transfer_function(o))
    return o, d, w, eta


@pytest.mark.parametrize("model", [op.LABELFREE_3D, op.POL5_3D])
def test_recon_gradient_matches_finite_differences(model):
    """Reverse mode through the Tikhonov inverse and the 3D synthesis (Ext. Data
    Fig. 3) against central differences of the plain definition L = <w, R_eta d>."""
    o, d, w, eta = _recon_case(model)
    grad, _ = at.recon_gradient(o, d, eta, w)
    fd = at.recon_fd_gradient(o, d, eta, w, steps=(1e-5,) * 6)
    scale = np.max(np.abs(fd))
    assert np.max(np.abs(grad - fd)) < 1e-6 * scale, (grad, fd)


def test_recon_gradient_with_a_background_and_odd_depth():
    o, d, w, eta = _recon_case(op.LABELFREE_3D, seed=3, nz=5, defocus=-0.2, tilt_zenith=0.05)
    b = np.array([0.3])
    grad, _ = at.recon_gradient(o, d, eta, w, b=b)
    fd = at.recon_fd_gradient(o, d, eta, w, steps=(1e-5,) * 6, b=b)
    assert np.max(np.abs(grad - fd)) < 1e-6 * np.max(np.abs(fd))


@pytest.mark.parametrize("model", [op.LABELFREE_3D, op.POL5_3D])
def test_recon_data_gradient_is_the_transpose_of_the_reconstruction(model):
    """dL/dd = R_eta^T w: <dL/dd, e> = <w, R_eta e> for any e (dot-product test)."""
    o, d, w, eta = _recon_case(model, seed=5)
    _, dd = at.recon_gradient(o, d, eta, w)
    e = np.random.default_rng(9).normal(size=d.shape)
    lhs = float(np.sum(dd * e))
    rhs = float(np.sum(w * linear.reconstruct(tfm.transfer_function(o), e, None, eta)))
    assert abs(lhs - rhs) < 1e-10 * abs(rhs)


# ---------------------------------------------------------------- oblique detection (R20)

def test_untilted_detection_is_the_disc_for_every_azimuth():
    for az in (0.0, 0.7, -2.1):
        o = lf_optics(det_azimuth=az, edge_width=0.5)
        fy, fx = op.lateral_frequencies(o)
        assert np.array_equal(op.detection_pupil(o),
                              op.radius_disc(fy, fx, o.na_det / o.wavelength, o.edge_width * o.dnu))


def test_tilted_detection_cap_is_the_cone_about_the_axis():
    """Hard cap: a shell point is inside exactly when the angle between k = (p, kz)
    and the tilted axis is at most asin(NA_det / n) (the angle computed directly)."""
    o = lf_optics(ny=32, nx=32, na_det=0.7, det_tilt=0.35, det_azimuth=0.9)
    P = op.detection_pupil(o)
    fy, fx = op.lateral_frequencies(o)
    kz = op.axial_wavenumber(o)
    ay, ax, az = op.detection_axis(o)
    cosang = np.clip((fy * ay + fx * ax + kz * az) / o.k_medium, -1.0, 1.0)
    ang = np.arccos(cosang)
    alpha = math.asin(o.na_det / o.n_medium)
    on = fy * fy + fx * fx < o.k_medium ** 2
    assert np.all(ang[on & (P > 0)] <= alpha + 1e-9)
    assert np.all(ang[on & (P == 0)] > alpha - 1e-9)
    assert P.sum() > 10
    # the cap is displaced towards the tilt: its centroid lies along (sin az, cos az)
    cy, cx = np.sum(P * fy) / P.sum(), np.sum(P * fx) / P.sum()
    assert cy * math.cos(o.det_azimuth) - cx * math.sin(o.det_azimuth) == pytest.approx(0.0, abs=0.06)
    assert cy * math.sin(o.det_azimuth) + cx * math.cos(o.det_azimuth) > 0.5


def test_detection_tilt_azimuth_rotates_the_bank():
    """On a square grid, turning the detection azimuth by pi/2 turns the transfer
    function by pi/2 (odd grid sizes: every frequency has its rotated partner)."""
    base = dict(model=op.LABELFREE_3D, nz=5, ny=15, nx=15, dz=0.25, dy=0.13, dx=0.13, wavelength=0.532,
                na_ill=0.0, na_det=0.8, n_medium=1.33, det_tilt=0.3, det_azimuth=0.2, edge_width=0.5)
    o1 = op.Optics(**base)
    o2 = o1.replace(det_azimuth=0.2 + math.pi / 2)
    h1, h2 = tfm.labelfree_3d(o1), tfm.labelfree_3d(o2)
    # a = (sin t sin az, sin t cos az) in (y, x): az + pi/2 turns a by R: (y, x) -> (x, -y),
    # so H2(f) = H1(R^-1 f) with R^-1 (y, x) = (-x, y)
    n = o1.ny
    iy, ix = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for k in range(2):
        rot = h1[k][:, (-ix) % n, iy]
        assert np.allclose(h2[k], rot, atol=1e-10 * np.abs(h1[k]).max())


def test_tilted_detection_point_response_is_abbe_source_sum():
    o = lf_optics(ny=8, nx=8, dx=0.13, dy=0.13, na_det=0.7, na_ill=0.4, defocus=0.1, det_tilt=0.3,
                  det_azimuth=0.6, edge_width=0.5)
    got = tfm.labelfree_point_response(o)
    ref = abbe_point_response(o)
    assert np.allclose(got, ref, atol=1e-12 * np.abs(ref).max())


def test_tilted_detection_fluorescence_otf_is_pupil_autocorrelation():
    o = fl_optics(nz=4, ny=8, nx=8, dx=0.13, dy=0.13, na_det=0.8, defocus=0.1, det_tilt=0.3, det_azimuth=-0.4)
    P = op.detection_pupil(o)
    h = np.stack([np.fft.ifft2(P * op.propagator(o, z)) for z in op.z_planes_3d(o)])
    P3 = direct_dft(h)
    ref = np.zeros(h.shape, dtype=np.complex128)
    for nu in np.ndindex(h.shape):
        ref[nu] = np.sum(P3 * np.conj(np.roll(P3, shift=nu, axis=(0, 1, 2)))) / h.size
    ref /= ref[0, 0, 0]
    assert np.allclose(tfm.fluorescence_3d(o), ref, atol=1e-12)


@pytest.mark.parametrize("model", [op.LABELFREE_3D, op.POL5_3D])
def test_recon_gradient_with_tilted_detection_matches_finite_differences(model):
    o, d, w, eta = _recon_case(model, seed=7, det_tilt=0.25, det_azimuth=0.8, na_det=0.7)
    grad, _ = at.recon_gradient(o, d, eta, w)
    fd = at.recon_fd_gradient(o, d, eta, w, steps=(1e-5,) * 6)
    assert np.max(np.abs(grad - fd)) < 1e-6 * np.max(np.abs(fd)), (grad, fd)
    assert abs(fd[4]) > 1e-3 * np.max(np.abs(fd)) and abs(fd[5]) > 1e-3 * np.max(np.abs(fd))


def test_detection_cap_must_stay_inside_the_shell():
    o = lf_optics(na_det=1.0, det_tilt=0.9)          # asin(1/1.33) + 0.9 > pi/2
    with pytest.raises(ValueError):
        op.check_optics(o)
    with pytest.raises(ValueError):
        op.check_optics(lf_optics(det_tilt=0.2, zernike=(0.1,)))
