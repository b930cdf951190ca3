"""Vector label-free transfer functions (Table 1, vector column, label-free row).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Table 1 writes the vector label-free bank as

    [H_re; H_im]_cp = sigma_c^{ii'} [[1, 1], [i, -i]]
                      [ [P_ij G_jn (star) P_i'k' S_k' S*_k] ; [swapped] ] Y_p^{nk},

the correlation of the detected scattered field of a dipole (detection pupil P
times the Green's tensor spectrum G) with the detected direct field of each
source point times the conjugate incident field that drives the dipole, summed
over data-space (sigma) and object-space (Y) indices.  The supplement that
fixes the conventions is not available; the readings used here are:

R21 Directions: the plane wave of lateral frequency p = (p_x, p_y) travels along
    k^(p) = (p_x, p_y, kz(p)) / k_m (x, y, z order).  With p = k_m sin(t)
    (cos f, sin f): t^ = (cos t cos f, cos t sin f, -sin t), f^ = (-sin f,
    cos f, 0), and in the pupil plane r^ = (cos f, sin f), f^_t = (-sin f,
    cos f).  Q(p) = t^ r^T + f^ f^_t^T (3 x 2) is written without angles:
    Q = [[1 - px^2 w, -px py w], [-px py w, 1 - py^2 w], [-px/k_m, -py/k_m]],
    w = 1 / (k_m (k_m + kz)); Q(0) = [I; 0].
R22 Vector source pupil: source point q of the disc S(q) with Jones vector J in
    the condenser's pupil illuminates the sample with the plane wave of
    polarisation e(q) = Q(q) J (aplanatic condenser; like the scalar model, no
    apodisation factor).
R23 Green's tensor spectrum: G_jn(p) = (delta_jn - k^_j k^_n) g(p), g the scalar
    factor of R2: a dipole radiates the field transverse to each direction.
R24 Tensor detection pupil: P_ij(p) = P(p) E(p) Q(p)^T (2 x 3; E the aberration
    phase of R18): the objective maps a plane wave's t^ and f^ components to
    the radial and azimuthal directions of its pupil.  Since Q^T Q = I, the
    direct light of source point q reaches the detector as P(q) E(q) J, the
    paraxial Jones field.  Oblique detection is not combined with this model.
R25 Object: the scattering-potential tensor f_nk = sum_p F_p T_p^{nk} with real
    coefficients F_p of complex 3 x 3 tensors; property code 2 b + part takes
    T = Y_b (part 0) or i Y_b (part 1) of the spherical-harmonic tensors
    (``sh_tensor``): b = 0 the isotropic tensor I (real part phase, imaginary
    part absorption, as in the scalar model), b = 1..3 the antisymmetric
    (l = 1) tensors, b = 4..8 the symmetric traceless (l = 2) tensors of
    m = -2..2, scaled so that their transverse blocks are the polarisation
    bank's property matrices (Y_4 = (xy + yx)/2, Y_8 = (xx - yy)/2).  A
    dipole induced by the field e is f e.
R26 Data space: channel c has an illumination Jones state J_c and a Hermitian
    analyser M_c; the channel records E^H M_c E of the detected field E,
    relative to I_bg = sum_q S P^2.  Stokes channels: one state and M =
    sigma_0..sigma_3 (sigma_0 = I, sigma_1 = diag(1, -1), sigma_2 = [[0, 1],
    [1, 0]], sigma_3 = [[0, -i], [i, 0]], so S3 = 2 Im(conj(Ex) Ey)); the
    polarisation states: the five swing states through the analyser a,
    M = a a^H.  The first-order response of channel c to property p is 2 Re
    R_cp with
        R_cp(x, z) = 1 / (Y X I_bg) sum M_c^{ii'} conj(v_ik) u_i'n T_p^{nk},
        u_i'n = IFFT2u[P_i'j G_jn prop],  v_ik = IFFT2u[S P_ik' e_k' conj(e_k) prop]
    (IFFT2u the unnormalised inverse DFT, prop the propagator of R1/R8), so
    H_cp = FFT3(2 Re R_cp): Table 1's pair with the [[1, 1], [i, -i]] rows is
    (FFT3 R)(nu) + conj((FFT3 R)(-nu)) and i times their difference, i.e. the
    properties T and i T.  The channel background is J_c^H M_c J_c.

Pins (tests/test_oracle_vector.py): the brute-force source sum of the detected
intensities of a weak point dipole (the unified-framework section's "summing
over the source" with vector fields); the exact reduction to the paraxial
polarisation bank when Q is replaced by [I; 0]; the approach to that bank as
the apertures shrink; Hermitian symmetry; and covariance under a rotation of
the whole microscope and object by 90 degrees about z.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft

from . import optics as op
from . import tf as tfm

STOKES = 0
POL_STATES = 1


def sh_tensor(b: int) -> np.ndarray:
    """Spherical-harmonic tensor Y_b (R25), complex 3 x 3 in (x, y, z)."""
    e = np.eye(3)
    x, y, z = e[0], e[1], e[2]

    def sym(a, c):
        return 0.5 * (np.outer(a, c) + np.outer(c, a))

    def asym(a, c):
        return 0.5 * (np.outer(a, c) - np.outer(c, a))

    table = [
        np.eye(3),                                          # l = 0
        asym(y, z), asym(z, x), asym(x, y),                 # l = 1
        sym(x, y),                                          # l = 2, m = -2
        sym(y, z),                                          # m = -1
        (2 * np.outer(z, z) - np.outer(x, x) - np.outer(y, y)) / (2 * math.sqrt(3.0)),   # m = 0
        sym(x, z),                                          # m = 1
        0.5 * (np.outer(x, x) - np.outer(y, y)),            # m = 2
    ]
    return table[b].astype(np.complex128)


def property_tensor(code: int) -> np.ndarray:
    """T of property code 2 b + part (R25)."""
    if not 0 <= code < 18:
        raise ValueError(f"property code {code}")
    t = sh_tensor(code // 2)
    return 1j * t if code % 2 else t


def stokes_matrices():
    """sigma_0..sigma_3 (R26)."""
    return [np.eye(2, dtype=np.complex128),
            np.array([[1, 0], [0, -1]], dtype=np.complex128),
            np.array([[0, 1], [1, 0]], dtype=np.complex128),
            np.array([[0, -1j], [1j, 0]], dtype=np.complex128)]


def channels(o: op.Optics):
    """[(J_c, M_c)] of the model's channel set (R26)."""
    if o.vec_channels == STOKES:
        J = np.asarray(o.ill_jones, dtype=np.complex128)
        return [(J, m) for m in stokes_matrices()]
    if o.vec_channels == POL_STATES:
        states, a = tfm.pol5_states(o.swing)
        M = np.outer(a, np.conj(a))
        return [(e, M) for e in states]
    raise ValueError(f"channel set {o.vec_channels}")


def channel_background(o: op.Optics) -> np.ndarray:
    """Direct-direct term of each channel relative to I_bg: J_c^H M_c J_c (R26)."""
    return np.array([float(np.real(np.conj(J) @ M @ J)) for J, M in channels(o)])


def pupil_map(o: op.Optics, paraxial: bool = False) -> np.ndarray:
    """Q(p) on the lateral grid: (Y, X, 3, 2) (R21); [I; 0] everywhere if paraxial."""
    fy, fx = op.lateral_frequencies(o)
    Q = np.zeros(fy.shape + (3, 2))
    if paraxial:
        Q[..., 0, 0] = Q[..., 1, 1] = 1.0
        return Q
    km = o.k_medium
    kz = op.axial_wavenumber(o)
    w = 1.0 / (km * (km + kz))
    Q[..., 0, 0] = 1.0 - fx * fx * w
    Q[..., 0, 1] = -fx * fy * w
    Q[..., 1, 0] = -fx * fy * w
    Q[..., 1, 1] = 1.0 - fy * fy * w
    Q[..., 2, 0] = -fx / km
    Q[..., 2, 1] = -fy / km
    return Q


def greens_tensor(o: op.Optics, paraxial: bool = False) -> np.ndarray:
    """G_jn(p) = (delta_jn - k^_j k^_n) g(p): (Y, X, 3, 3) (R23); g I if paraxial."""
    g = op.greens_spectrum(o)
    if paraxial:
        return g[..., None, None] * np.eye(3)
    fy, fx = op.lateral_frequencies(o)
    kz = op.axial_wavenumber(o)
    k = np.stack([fx, fy, kz], axis=-1) / o.k_medium
    return g[..., None, None] * (np.eye(3) - k[..., :, None] * k[..., None, :])


def detection_tensor(o: op.Optics, paraxial: bool = False) -> np.ndarray:
    """P_ij(p) = P E Q^T: (Y, X, 2, 3) (R24)."""
    PE = op.detection_pupil(o) * op.aberration(o)
    return PE[..., None, None] * np.swapaxes(pupil_map(o, paraxial), -1, -2)


def incident_field(o: op.Optics, J, paraxial: bool = False) -> np.ndarray:
    """e(q) = Q(q) J: (Y, X, 3) (R22)."""
    return pupil_map(o, paraxial) @ np.asarray(J, dtype=np.complex128)


def point_response(o: op.Optics, J, M, T, paraxial: bool = False) -> np.ndarray:
    """R(x, z) of one channel (J, M) and property tensor T: (Z, Y, X) complex (R26)."""
    S = op.illumination_pupil(o)
    Pt = detection_tensor(o, paraxial)
    G = greens_tensor(o, paraxial)
    e = incident_field(o, J, paraxial)
    ibg = op.background(o)
    if ibg <= 0:
        raise ValueError("no direct light reaches the detector")
    PG = np.einsum("yxij,yxjn->yxin", Pt, G)                      # scattered arm, (2, 3)
    Pe = np.einsum("yxij,yxj->yxi", Pt, e)                         # direct field at the detector
    PSS = S[..., None, None] * Pe[..., :, None] * np.conj(e)[..., None, :]   # (2, 3): i, k
    n = o.ny * o.nx
    out = np.empty((o.nz, o.ny, o.nx), dtype=np.complex128)
    for zi, z in enumerate(op.z_planes_3d(o)):
        prop = op.propagator(o, z)[..., None, None]
        u = sfft.ifft2(PG * prop, axes=(0, 1)) * n
        v = sfft.ifft2(PSS * prop, axes=(0, 1)) * n
        out[zi] = np.einsum("ab,yxak,yxbn,nk->yx", M, np.conj(v), u, T) / (n * ibg)
    return out


def vector_3d(o: op.Optics, paraxial: bool = False) -> np.ndarray:
    """(C, P, Z, Y, X) bank H_cp = FFT3(2 Re R_cp) over the model's channels and
    properties (Table 1 vector label-free row, R21-R26)."""
    chans = channels(o)
    props = [property_tensor(c) for c in o.vec_props]
    out = np.empty((len(chans), len(props), o.nz, o.ny, o.nx), dtype=np.complex128)
    for c, (J, M) in enumerate(chans):
        for p, T in enumerate(props):
            out[c, p] = sfft.fftn(2.0 * point_response(o, J, M, T, paraxial).real)
    return out


def vector_3d_at(o: op.Optics, kz: int, ky: int, kx: int) -> np.ndarray:
    """(C, P) bank at one frequency index by the direct sum over source points q
    (no FFT): the lateral spectrum of R_cp at nu is
        C_cp(nu, z) = (1 / I_bg) sum_q sum M_c^{ii'} conj(V_ik(q)) U_i'n(q + nu) T_p^{nk}
    with V = S (P e)_i conj(e_k) prop and U = P_i'j G_jn prop (the correlation
    theorem applied to R26), and H_cp = sum_z e^{-i 2 pi kz z / Z}
    (C_cp(nu, z) + conj(C_cp(-nu, z)))."""
    S = op.illumination_pupil(o)
    Pt = detection_tensor(o)
    G = greens_tensor(o)
    ibg = op.background(o)
    chans = channels(o)
    props = [property_tensor(c) for c in o.vec_props]
    PG = np.einsum("yxij,yxjn->yxin", Pt, G)
    qy, qx = np.nonzero(S * op.detection_pupil(o))
    kzz = op.axial_wavenumber(o)
    zs = op.z_planes_3d(o) - o.defocus

    Q = pupil_map(o)[qy, qx]                                                             # (q, 3, 2)
    # scattered arm at q + nu and q - nu, and the z phases of the two correlations
    arms = []
    for ny_, nx_ in ((ky, kx), ((-ky) % o.ny, (-kx) % o.nx)):
        py, px = (qy + ny_) % o.ny, (qx + nx_) % o.nx
        dk = kzz[py, px] - kzz[qy, qx]
        arms.append((PG[py, px], np.exp(2j * np.pi * np.outer(zs, dk)) / ibg))          # (q, i', n), (Z, q)

    def lateral(V, M, T, arm):
        U, ph = arm
        w = np.einsum("ab,qak,qbn,nk->q", M, np.conj(V), U, T, optimize=True)
        return ph @ w                                                                    # (Z,)

    ez = np.exp(-2j * np.pi * kz * np.arange(o.nz) / o.nz)
    out = np.empty((len(chans), len(props)), dtype=np.complex128)
    for c, (J, M) in enumerate(chans):
        e = Q @ np.asarray(J, dtype=np.complex128)                                       # e(q) = Q J
        Pe = np.einsum("qij,qj->qi", Pt[qy, qx], e)
        V = S[qy, qx, None, None] * Pe[:, :, None] * np.conj(e[:, None, :])              # (q, i, k)
        for p, T in enumerate(props):
            cp = lateral(V, M, T, arms[0])
            cm = lateral(V, M, T, arms[1])
            out[c, p] = np.sum(ez * (cp + np.conj(cm)))
    return out
