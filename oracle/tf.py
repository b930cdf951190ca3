"""Transfer functions of the oracle (Table 1, scalar column; polarisation bank).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Table 1 writes every transfer function as an autocorrelation of pupils.  The
oracle evaluates each autocorrelation through the correlation theorem on the
lateral FFT grid, one z plane at a time, and then transforms along z:

* fluorescence (scatter-scatter term, "summing over the sample"):
  H = [P * P], i.e. the 3D Fourier transform of the intensity PSF |h_z|^2,
  h_z = IFFT2(P exp(i 2 pi kz (z - dz0))), normalised to H(0) = 1;
* label-free (direct-scatter interference, "summing over the source"):
  the complex point response c_z = (X Y / I_bg) IFFT2(B_z) conj(IFFT2(A_z)) with
  A_z = S P exp(i 2 pi kz (z - dz0)) (direct light through the pupil) and
  B_z = P g exp(i 2 pi kz (z - dz0)) (scattered light through the pupil).
  Table 1's [[1, 1], [i, -i]] pair then reads h_re = 2 Re c (phase) and
  h_im = -2 Im c (absorption), whose transforms are the phase and absorption
  transfer functions.

Units (reading R2): properties are radians per voxel -- phase 2 pi dn dz /
lambda0 and absorption 2 pi dkappa dz / lambda0 -- and label-free data are the
relative contrast I / I_bg - 1.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft

from . import optics as op


def _planes(o: op.Optics) -> np.ndarray:
    return op.z_planes_thin(o) if o.model == op.LABELFREE_THIN else op.z_planes_3d(o)


def labelfree_point_response(o: op.Optics, S: np.ndarray | None = None) -> np.ndarray:
    """c_z(x) for every plane: (Z, Y, X) complex (Table 1 scalar label-free row),
    for the illumination pupil S (default: the optics' disc).

    The phase PSF is 2 Re c and the absorption PSF is -2 Im c.
    """
    if S is None:
        S = op.illumination_pupil(o)
    P = op.detection_pupil(o)
    E = op.aberration(o)       # detection aberration phase (R18)
    g = op.greens_spectrum(o)
    ibg = float(np.sum(S * P * P))
    if ibg <= 0:
        raise ValueError("no direct light reaches the detector")
    out = np.empty((o.nz, o.ny, o.nx), dtype=np.complex128)
    for k, z in enumerate(_planes(o)):
        prop = op.propagator(o, z)
        a = sfft.ifft2(S * P * E * prop)
        b = sfft.ifft2(P * E * g * prop)
        out[k] = (o.ny * o.nx / ibg) * b * np.conj(a)
    return out


def labelfree_3d(o: op.Optics) -> np.ndarray:
    """[H_phase, H_abs] of the 3D scalar label-free model: (2, Z, Y, X) complex."""
    c = labelfree_point_response(o)
    return np.stack([sfft.fftn(2.0 * c.real), sfft.fftn(-2.0 * c.imag)])


def labelfree_thin(o: op.Optics) -> np.ndarray:
    """Thin (phase-from-defocus) model: one 2D TF pair per plane, (Z, 2, Y, X).

    Channel k is the image of a thin object at the nominal plane taken with the
    focus at z_k; it is the 2D transform of plane k of the 3D point response.
    """
    c = labelfree_point_response(o)
    return np.stack([sfft.fft2(2.0 * c.real), sfft.fft2(-2.0 * c.imag)], axis=1)


def fluorescence_3d(o: op.Optics) -> np.ndarray:
    """Scalar fluorescence OTF [P * P]: (Z, Y, X) complex, H(0) = 1 (Table 1)."""
    P = op.detection_pupil(o) * op.aberration(o)
    psf = np.empty((o.nz, o.ny, o.nx))
    for k, z in enumerate(op.z_planes_3d(o)):
        h = sfft.ifft2(P * op.propagator(o, z))
        psf[k] = np.abs(h) ** 2
    psf /= psf.sum()
    return sfft.fftn(psf)


# --- polarisation-resolved bank (paraxial Jones reduction of Table 1's vector row)

def _rot(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, s], [-s, c]], dtype=np.complex128)


def _retarder(delta: float, axis: float) -> np.ndarray:
    """Jones matrix of a linear retarder of retardance delta with its fast axis at ``axis``."""
    d = np.diag([np.exp(-0.5j * delta), np.exp(0.5j * delta)])
    return _rot(-axis) @ d @ _rot(axis)


def pol5_states(swing: float):
    """Illumination Jones vectors e_0..e_4 and the circular analyser a (reading R9).

    e_0 = (1, i)/sqrt2 is the extinction state; e_c = J(2 pi swing, alpha_c) e_0
    with alpha_c in {0, pi/4, pi/2, 3pi/4}; a = (1, -i)/sqrt2.
    """
    e0 = np.array([1.0, 1.0j]) / math.sqrt(2.0)
    states = [e0]
    for alpha in (0.0, math.pi / 4, math.pi / 2, 3 * math.pi / 4):
        states.append(_retarder(2 * math.pi * swing, alpha) @ e0)
    a = np.array([1.0, -1.0j]) / math.sqrt(2.0)
    return states, a


def pol5_property_matrices():
    """Jones scattering matrices B_p of the four properties (reading R9).

    phase: I; rho cos 2w: diag(1, -1)/2; rho sin 2w: [[0, 1], [1, 0]]/2;
    absorption: i I.
    """
    return [
        np.eye(2, dtype=np.complex128),
        0.5 * np.array([[1, 0], [0, -1]], dtype=np.complex128),
        0.5 * np.array([[0, 1], [1, 0]], dtype=np.complex128),
        1j * np.eye(2, dtype=np.complex128),
    ]


def pol5_coupling(swing: float) -> np.ndarray:
    """kappa_cp = conj(a^H e_c) (a^H B_p e_c): (5, 4) complex.

    The interference of the direct field a^H e_c with the scattered field
    a^H B_p e_c g gives the channel response Re(kappa) h_phase + Im(kappa) h_abs.
    """
    states, a = pol5_states(swing)
    ah = np.conj(a)
    k = np.empty((5, 4), dtype=np.complex128)
    for c, e in enumerate(states):
        direct = ah @ e
        for p, B in enumerate(pol5_property_matrices()):
            k[c, p] = np.conj(direct) * (ah @ (B @ e))
    return k


def pol5_background(swing: float) -> np.ndarray:
    """Direct-direct background of each channel relative to I_bg: |a^H e_c|^2."""
    states, a = pol5_states(swing)
    return np.array([abs(np.conj(a) @ e) ** 2 for e in states])


def pol5_3d(o: op.Optics) -> np.ndarray:
    """(5, 4, Z, Y, X) bank H_cp = Re(kappa_cp) H_phase + Im(kappa_cp) H_abs."""
    hp, ha = labelfree_3d(o)
    k = pol5_coupling(o.swing)
    return k.real[:, :, None, None, None] * hp + k.imag[:, :, None, None, None] * ha


def sectors9_3d(o: op.Optics) -> np.ndarray:
    """(9, 1, Z, Y, X) phase bank of the 9-aperture scheme: channel c is the 3D phase
    TF of the label-free model under aperture c (8 sectors, then the full disc),
    each normalised by its own background sum_q S_c P^2 (Fig. 4c: a 9 x 1 column)."""
    out = np.empty((9, 1, o.nz, o.ny, o.nx), dtype=np.complex128)
    for c in range(9):
        cz = labelfree_point_response(o, op.sector_pupil(o, c))
        out[c, 0] = sfft.fftn(2.0 * cz.real)
    return out


def transfer_function(o: op.Optics) -> np.ndarray:
    """TF bank of the model: (C, P, Z, Y, X) for 3D models, (C=Z, P=2, Y, X) for thin."""
    op.check_optics(o)
    if o.model == op.FLUOR_3D:
        return fluorescence_3d(o)[None, None]
    if o.model == op.LABELFREE_3D:
        return labelfree_3d(o)[None]
    if o.model == op.LABELFREE_THIN:
        return labelfree_thin(o)
    if o.model == op.POL5_3D:
        return pol5_3d(o)
    if o.model == op.SECTORS9_3D:
        return sectors9_3d(o)
    if o.model == op.VECTOR_3D:
        from . import vector
        return vector.vector_3d(o)
    raise ValueError(f"unknown model {o.model}")


def bank_shape(o: op.Optics):
    """(C, P, spectral dims) of the model's bank."""
    if o.model == op.FLUOR_3D:
        return 1, 1, 3
    if o.model == op.LABELFREE_3D:
        return 1, 2, 3
    if o.model == op.LABELFREE_THIN:
        return o.nz, 2, 2
    if o.model == op.POL5_3D:
        return 5, 4, 3
    if o.model == op.SECTORS9_3D:
        return 9, 1, 3
    if o.model == op.VECTOR_3D:
        return (4 if o.vec_channels == 0 else 5), len(o.vec_props), 3
    raise ValueError(o.model)


def labelfree_response_at(o: op.Optics, ky: int, kx: int) -> np.ndarray:
    """C_z(nu_perp) for every plane at one lateral frequency index (ky, kx), by the
    direct sum over source points q (Table 1, [P * PS] as a correlation):

        C_z(nu) = sum_q S(q) P(q) P(q + nu) g(q + nu) e^{i 2 pi (kz(q + nu) - kz(q)) (z - dz0)} / I_bg

    (times conj(E(q)) E(q + nu) with the aberration phase E of R18).

    Independent of any FFT; used to check full-size banks frequency by frequency.
    Returns (Z,) complex.
    """
    S = op.illumination_pupil(o)
    P = op.detection_pupil(o)
    E = op.aberration(o)
    g = op.greens_spectrum(o)
    kzz = op.axial_wavenumber(o)
    ibg = float(np.sum(S * P * P))
    qy, qx = np.nonzero(S * P)
    py, px = (qy + ky) % o.ny, (qx + kx) % o.nx        # q + nu on the periodic grid
    w = S[qy, qx] * P[qy, qx] * np.conj(E[qy, qx]) * P[py, px] * E[py, px] * g[py, px]
    dk = kzz[py, px] - kzz[qy, qx]
    zs = _planes(o) - o.defocus
    return np.exp(2j * np.pi * np.outer(zs, dk)) @ w / ibg


def labelfree_3d_at(o: op.Optics, kz: int, ky: int, kx: int):
    """(H_phase, H_abs) of the 3D label-free model at one frequency index, from
    labelfree_response_at at nu and -nu and a direct DFT along z."""
    cp = labelfree_response_at(o, ky, kx)
    cm = labelfree_response_at(o, (-ky) % o.ny, (-kx) % o.nx)
    ez = np.exp(-2j * np.pi * kz * np.arange(o.nz) / o.nz)
    hp = np.sum(ez * (cp + np.conj(cm)))
    ha = np.sum(ez * 1j * (cp - np.conj(cm)))
    return hp, ha


def pol5_3d_at(o: op.Optics, kz: int, ky: int, kx: int) -> np.ndarray:
    """(5, 4) polarisation bank at one frequency index: pol5_3d's composition applied
    to labelfree_3d_at (the direct source sum, no FFT)."""
    hp, ha = labelfree_3d_at(o, kz, ky, kx)
    k = pol5_coupling(o.swing)
    return k.real * hp + k.imag * ha
