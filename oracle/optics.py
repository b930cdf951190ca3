"""Optics submodels of the oracle: grids, pupils, Green's spectrum, propagators.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper: Methods, "Summary of transfer functions" -- every transfer function is
built from an illumination model (source pupil S), a scattering model (Green's
spectrum G) and a detection model (detection pupil P), each a function on the
spherical shell of radius 1/lambda (lambda in the medium).  Ext. Data Fig. 3
gives the parameters: the illumination pupil depends on NA_ill and a tilt
(zenith, azimuth) and is (Y, X); the detection pupil depends on NA_det and a
defocus offset and is (Z, Y, X).

Readings (the paper's derivations are in a supplement that is not available):

R1  The shell is sampled as a 2D pupil on the lateral FFT grid times the
    angular-spectrum propagator exp(i 2 pi kz(p) (z - dz0)), kz(p) =
    sqrt(k_m^2 - |p|^2), k_m = n / lambda0, with signed z (forward hemisphere).
R2  Scalar scattered arm: P(p) * g(p) with g(p) = i / cos(theta(p)),
    cos(theta) = kz(p) / k_m -- the Weyl spectrum of the Helmholtz Green's
    function scaled so that a laterally uniform slab of phase phi scatters
    i*phi at normal incidence.
R6  Pupil edge: hard disc with the boundary included, or a compact C1
    smoothstep of half-width ``edge_width`` frequency pixels.
R7  Tilt shifts the source disc to q0 = (n sin(zenith)/lambda0) (cos az,
    sin az); the tilted disc must stay inside k_m.
R8  Defocus shifts every plane, z -> z - defocus.
R18 Detection aberrations (Ext. Data Fig. 3b: Zernike coefficients enter
    calc_det_pupil): the detection pupil becomes P(p) exp(i 2 pi W(p)), W in
    waves, W = sum_j c_j Z_j(rho, phi) over Noll's unit-RMS Zernike
    polynomials j = 5..11, rho = |p| / (NA_det / lambda0), phi = atan2(p_y,
    p_x).  The phase multiplies the pupil wherever it appears (direct and
    scattered arms, fluorescence); the polynomials continue past rho = 1 into
    a soft edge.  I_bg = sum S |P|^2 is unchanged.
R20 Oblique detection (Ext. Data Fig. light paths, panel b: the oblique
    detection path; Results, neuromasts imaged with oblique and straight
    detection): the detection objective's axis a is tilted from the sample's z
    axis by the zenith angle det_tilt in the azimuth det_azimuth, a =
    (sin t sin az, sin t cos az, cos t) in (y, x, z) (the source tilt's azimuth
    convention).  The detection pupil is the cap of the shell within the
    detection NA about a: P(p) = edge(NA_det/lambda0 - |p'|) with |p'|^2 =
    k_m^2 - (k . a)^2 the lateral distance in the tilted frame, k = (p,
    kz(p)), and k . a > 0; at det_tilt = 0 this is the disc.  The cap must
    stay inside the shell: k_m sin(det_tilt + asin(NA_det/n)) plus the soft
    edge below k_m.  The reconstruction stays on the sample grid (re-slicing
    an oblique acquisition onto it is not part of the method's arithmetic).
    The aberration polynomials are defined on the untilted pupil, so detection
    tilt and aberrations are not combined.
All arithmetic is float64 / complex128.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

FLUOR_3D = 0
LABELFREE_3D = 1
LABELFREE_THIN = 2
POL5_3D = 3
SECTORS9_3D = 4
VECTOR_3D = 5


@dataclasses.dataclass
class Optics:
    """Microscope and sampling parameters of one volume or patch (units: um, rad)."""

    model: int
    nz: int
    ny: int
    nx: int
    dz: float
    dy: float
    dx: float
    wavelength: float          # vacuum wavelength (emission wavelength for fluorescence)
    na_ill: float
    na_det: float
    n_medium: float
    defocus: float = 0.0
    tilt_zenith: float = 0.0
    tilt_azimuth: float = 0.0
    edge_width: float = 0.0    # soft pupil edge half-width in frequency pixels; 0 = hard
    swing: float = 0.1         # polarisation bank only
    zernike: tuple = ()        # detection aberration, waves, Noll j = 5, 6, ... (R18)
    det_tilt: float = 0.0      # detection axis zenith angle, rad (R20)
    det_azimuth: float = 0.0   # and its azimuth, rad
    # vector label-free model only (R21-R26, oracle.vector): channel set (0: Stokes
    # S0..S3 under the illumination Jones state ill_jones; 1: the five swing states
    # through the circular analyser) and property codes 2 b + part
    vec_channels: int = 0
    vec_props: tuple = (0, 16, 8, 1)
    ill_jones: tuple = (2 ** -0.5, 1j * 2 ** -0.5)

    def replace(self, **kw) -> "Optics":
        return dataclasses.replace(self, **kw)

    @property
    def k_medium(self) -> float:
        """Shell radius n / lambda0 in cycles/um (Summary of transfer functions)."""
        return self.n_medium / self.wavelength

    @property
    def dnu(self) -> float:
        """Lateral frequency pixel used to scale the soft pupil edge."""
        return min(1.0 / (self.nx * self.dx), 1.0 / (self.ny * self.dy))


def lateral_frequencies(o: Optics):
    """(fy, fx) lateral frequency grids in cycles/um, FFT order (numpy fftfreq)."""
    fy = np.fft.fftfreq(o.ny, o.dy)
    fx = np.fft.fftfreq(o.nx, o.dx)
    return np.meshgrid(fy, fx, indexing="ij")


def z_planes_3d(o: Optics) -> np.ndarray:
    """Axial PSF coordinates of the 3D models, FFT order: 0, dz, ..., -dz."""
    return np.fft.fftfreq(o.nz) * o.nz * o.dz


def z_planes_thin(o: Optics) -> np.ndarray:
    """Physical planes of a defocus stack, centred on the nominal focus."""
    return o.dz * (np.arange(o.nz) - (o.nz - 1) / 2.0)


def edge(inside: np.ndarray, halfwidth: float) -> np.ndarray:
    """Pupil edge profile of a signed distance ``inside`` (positive inside).

    Hard edge (halfwidth == 0): 1 where inside >= 0, else 0.
    Soft edge: t = clip((inside/halfwidth + 1)/2, 0, 1), value 3 t^2 - 2 t^3.
    """
    inside = np.asarray(inside, dtype=np.float64)
    if halfwidth == 0.0:
        return (inside >= 0.0).astype(np.float64)
    t = np.clip((inside / halfwidth + 1.0) * 0.5, 0.0, 1.0)
    return t * t * (3.0 - 2.0 * t)


def radius_disc(fy, fx, radius: float, halfwidth: float, cy=0.0, cx=0.0):
    """Disc of the given radius centred on (cy, cx).

    The hard disc is decided on squared distances (no square root), the soft
    disc on the signed radial distance.
    """
    r2 = (fy - cy) ** 2 + (fx - cx) ** 2
    if halfwidth == 0.0:
        return (r2 <= radius * radius).astype(np.float64)
    return edge(radius - np.sqrt(r2), halfwidth)


def detection_axis(o: Optics):
    """Unit vector (ay, ax, az) of the detection axis (reading R20)."""
    t, az = o.det_tilt, o.det_azimuth
    return math.sin(t) * math.sin(az), math.sin(t) * math.cos(az), math.cos(t)


def detection_lateral_distance_sq(o: Optics):
    """(|p'|^2, k . a) on the lateral grid: the squared lateral distance of the
    shell point k = (p, kz(p)) from the detection axis a, and k . a (R20)."""
    fy, fx = lateral_frequencies(o)
    kz = np.sqrt(np.maximum(o.k_medium ** 2 - fy * fy - fx * fx, 0.0))
    ay, ax, az = detection_axis(o)
    ka = fy * ay + fx * ax + kz * az
    return o.k_medium ** 2 - ka * ka, ka


def detection_pupil(o: Optics) -> np.ndarray:
    """P(p): disc of radius NA_det/lambda0 (Ext. Data Fig. 3b, calc_det_pupil); with
    oblique detection the cap of that NA about the tilted detection axis (R20)."""
    fy, fx = lateral_frequencies(o)
    rd, hw = o.na_det / o.wavelength, o.edge_width * o.dnu
    if o.det_tilt == 0.0:
        return radius_disc(fy, fx, rd, hw)
    pp2, ka = detection_lateral_distance_sq(o)
    on_shell = fy * fy + fx * fx < o.k_medium ** 2
    fwd = (ka > 0.0) & on_shell
    if hw == 0.0:
        return ((pp2 <= rd * rd) & fwd).astype(np.float64)
    return np.where(fwd, edge(rd - np.sqrt(np.maximum(pp2, 0.0)), hw), 0.0)


def detection_radius(o: Optics) -> float:
    """Radius about p = 0 of a disc holding the detection pupil's support (without
    the soft edge): NA_det/lambda0, or k_m sin(det_tilt + asin(NA_det/n)) (R20)."""
    if o.det_tilt == 0.0:
        return o.na_det / o.wavelength
    a = abs(o.det_tilt) + math.asin(min(o.na_det / o.n_medium, 1.0))
    return o.k_medium * (math.sin(a) if a < 0.5 * math.pi else 1.0)


ZERNIKE_FIRST = 5     # Noll index of zernike[0]


def noll_nm(j: int):
    """(n, m) of Noll's index j >= 1: radial order n, azimuthal order m >= 0.
    Within order n the indices run through |m| ascending, each m > 0 twice."""
    n = 0
    while (n + 1) * (n + 2) // 2 < j:
        n += 1
    k = j - n * (n + 1) // 2 - 1
    ms = [m for m in range(n % 2, n + 1, 2) for _ in range(1 if m == 0 else 2)]
    return n, ms[k]


def zernike_noll(j: int, rho, phi):
    """Noll's Zernike polynomial Z_j: unit RMS over the unit disc, sqrt(n + 1)
    R_n^0 for m = 0, else sqrt(2 (n + 1)) R_n^m times cos(m phi) (even j) or
    sin(m phi) (odd j); R_n^m(rho) = sum_s (-1)^s (n - s)! / (s! ((n + m)/2 - s)!
    ((n - m)/2 - s)!) rho^(n - 2s)."""
    n, m = noll_nm(j)
    rho = np.asarray(rho, dtype=np.float64)
    R = np.zeros_like(rho)
    for s_ in range((n - m) // 2 + 1):
        c = ((-1) ** s_ * math.factorial(n - s_)
             / (math.factorial(s_) * math.factorial((n + m) // 2 - s_) * math.factorial((n - m) // 2 - s_)))
        R = R + c * rho ** (n - 2 * s_)
    if m == 0:
        return math.sqrt(n + 1) * R
    ang = np.cos(m * np.asarray(phi)) if j % 2 == 0 else np.sin(m * np.asarray(phi))
    return math.sqrt(2 * (n + 1)) * R * ang


def aberration_waves(o: Optics) -> np.ndarray:
    """W(p) in waves on the lateral grid (R18); zeros without coefficients."""
    fy, fx = lateral_frequencies(o)
    W = np.zeros_like(fy)
    if not any(o.zernike):
        return W
    rho = np.sqrt(fy * fy + fx * fx) / (o.na_det / o.wavelength)
    phi = np.arctan2(fy, fx)
    for k, c in enumerate(o.zernike):
        if c:
            W = W + c * zernike_noll(ZERNIKE_FIRST + k, rho, phi)
    return W


def aberration(o: Optics) -> np.ndarray:
    """exp(i 2 pi W(p)): the phase factor of the aberrated detection pupil (R18)."""
    return np.exp(2j * np.pi * aberration_waves(o))


def source_centre(o: Optics):
    """q0 = (n sin(zenith) / lambda0) (sin az, cos az) as (qy, qx) (reading R7)."""
    r = o.n_medium * math.sin(o.tilt_zenith) / o.wavelength
    return r * math.sin(o.tilt_azimuth), r * math.cos(o.tilt_azimuth)


def illumination_pupil(o: Optics) -> np.ndarray:
    """S(q): disc of radius NA_ill/lambda0 centred at the tilt q0 (calc_ill_pupil)."""
    fy, fx = lateral_frequencies(o)
    cy, cx = source_centre(o)
    return radius_disc(fy, fx, o.na_ill / o.wavelength, o.edge_width * o.dnu, cy, cx)


def octant(dy, dx):
    """Sector index k of the direction (dy, dx): its azimuth lies in [k pi/4, (k+1) pi/4)
    measured from +x towards +y; the origin is in sector 0 (reading R17).  Written
    with comparisons only, so equal inputs give equal decisions on any machine."""
    dy = np.asarray(dy, dtype=np.float64)
    dx = np.asarray(dx, dtype=np.float64)
    k = np.full(np.broadcast(dy, dx).shape, 6, dtype=np.int64)
    q0 = (dy >= 0) & (dx > 0)
    q1 = (dx <= 0) & (dy > 0)
    q2 = (dy <= 0) & (dx < 0)
    q3 = ~(q0 | q1 | q2)                      # dy < 0, dx >= 0, or the origin
    k = np.where(q0, np.where(dy < dx, 0, 1), k)
    k = np.where(q1, np.where(dy > -dx, 2, 3), k)
    k = np.where(q2, np.where(dy > dx, 4, 5), k)
    k = np.where(q3, np.where(dx < -dy, 6, 7), k)
    return np.where((dy == 0) & (dx == 0), 0, k)


def sector_pupil(o: Optics, c: int) -> np.ndarray:
    """Illumination pupil of aperture c of the 9-aperture scheme (Results, cardiomyocytes;
    Methods "Cardiomyocyte reconstructions"): sectors c = 0..7 of the source disc,
    split by azimuth about its centre q0, and the full disc for c = 8 (reading R17)."""
    S = illumination_pupil(o)
    if c == 8:
        return S
    fy, fx = lateral_frequencies(o)
    cy, cx = source_centre(o)
    return S * (octant(fy - cy, fx - cx) == c)


def axial_wavenumber(o: Optics, wavelength: float | None = None) -> np.ndarray:
    """kz(p) = sqrt(k_m^2 - |p|^2), set to 0 outside the shell (evanescent)."""
    lam = o.wavelength if wavelength is None else wavelength
    km = o.n_medium / lam
    fy, fx = lateral_frequencies(o)
    return np.sqrt(np.maximum(km * km - fy * fy - fx * fx, 0.0))


def greens_spectrum(o: Optics) -> np.ndarray:
    """Scalar scattered-field factor g(p) = i / cos(theta(p)) (reading R2).

    Zero where kz = 0 (the pupils vanish there, which ``check_optics`` enforces).
    """
    kz = axial_wavenumber(o)
    g = np.zeros(kz.shape, dtype=np.complex128)
    ok = kz > 0
    g[ok] = 1j * o.k_medium / kz[ok]
    return g


def propagator(o: Optics, z: float) -> np.ndarray:
    """Angular-spectrum propagator exp(i 2 pi kz(p) (z - defocus)) (readings R1, R8)."""
    return np.exp(2j * np.pi * axial_wavenumber(o) * (z - o.defocus))


def background(o: Optics) -> float:
    """Direct-direct intensity I_bg = sum_q S(q) P(q)^2 (unified-framework section)."""
    return float(np.sum(illumination_pupil(o) * detection_pupil(o) ** 2))


def check_optics(o: Optics) -> None:
    """Raise ValueError where the discrete model is not the paper's continuous one.

    * pupils must stay strictly inside the shell (no evanescent support, where
      the Green's factor 1/cos(theta) diverges);
    * the label-free correlation must not wrap laterally: its support radius
      (NA_det + NA_ill)/lambda0 + |q0| must stay below the lateral Nyquist
      frequency; fluorescence needs 2 NA_det/lambda0 below it;
    * the axial support must stay below the axial Nyquist frequency.
    """
    if min(o.nz, o.ny, o.nx) < 1 or min(o.dz, o.dy, o.dx) <= 0 or o.wavelength <= 0:
        raise ValueError("bad sampling")
    if o.na_det < 0 or o.na_ill < 0 or o.n_medium <= 0:
        raise ValueError("bad aperture")
    km = o.k_medium
    hw = o.edge_width * o.dnu
    rdet = detection_radius(o)
    if rdet + hw >= km or abs(o.det_tilt) + math.asin(min(o.na_det / o.n_medium, 1.0)) >= 0.5 * math.pi:
        raise ValueError("detection pupil reaches the evanescent boundary")
    if o.det_tilt != 0.0 and any(o.zernike):
        raise ValueError("detection tilt with aberrations is not supported (R20)")
    if o.model == VECTOR_3D and o.det_tilt != 0.0:
        raise ValueError("the vector model's pupil mapping is for the untilted objective (R24)")
    qy, qx = source_centre(o)
    q0 = math.hypot(qy, qx)
    if o.model != FLUOR_3D and o.na_ill / o.wavelength + q0 + hw >= km:
        raise ValueError("illumination pupil reaches the evanescent boundary")
    nyq = min(0.5 / o.dx, 0.5 / o.dy)
    if o.model == FLUOR_3D:
        lat = 2.0 * (rdet + hw)
        ax = km * (1.0 - math.sqrt(1.0 - ((rdet + hw) / km) ** 2))
    else:
        lat = rdet + o.na_ill / o.wavelength + q0 + 2.0 * hw
        kd = min(rdet + hw, km)
        ax = km - math.sqrt(km * km - kd * kd)
    if lat >= nyq:
        raise ValueError("lateral aliasing")
    if o.model != LABELFREE_THIN and ax >= 0.5 / o.dz:
        raise ValueError("axial aliasing")


def hard_edge_margin(o: Optics) -> float:
    """Smallest relative distance of a lattice point's |p|^2 from a hard edge radius^2.

    Used by tests to make sure FP32/FP64 evaluations of the hard disc agree.
    """
    fy, fx = lateral_frequencies(o)
    out = np.inf
    cy, cx = source_centre(o)
    # (squared distance, edge radius): the detection pupil (its tilted cap, R20),
    # then the source disc
    pd2 = detection_lateral_distance_sq(o)[0] if o.det_tilt != 0.0 else fy * fy + fx * fx
    for r2, radius in ((pd2, o.na_det / o.wavelength),
                       ((fy - cy) ** 2 + (fx - cx) ** 2, o.na_ill / o.wavelength)):
        if radius <= 0:
            continue
        out = min(out, float(np.min(np.abs(r2 - radius * radius))) / (radius * radius))
    return out
