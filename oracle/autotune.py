"""Mid-band power loss, its parameter gradient, and the Adam auto-tune loop.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper: Results, "Physics-guided ML auto-tunes multi-contrast blind
deconvolution", and Methods, "Cell-scale optical pooled screen data"; the
computational graph of Ext. Data Fig. 3: parameters -> illumination and
detection pupils -> defocus transfer function -> Tikhonov inverse (phase
image) -> mid-band power -> backpropagation -> Adam step.

Parameter vector theta = (defocus, na_det, tilt_zenith, tilt_azimuth).

Readings (paper silent):
R10 The transverse cutoff nu_c is (NA_det + NA_ill)/lambda0 of the nominal
    optics and is held fixed while theta moves, so the band
    B = {nu_c/8 <= |nu_perp| <= nu_c/4} does not jump with NA_det.
R11 The loss is L = -(1/|B|) sum_{nu in B} |F_phase(nu)|^2 on the unnormalised
    2D DFT of the reconstructed phase; minimising L maximises mid-band power.
R12 Adam uses beta1 = 0.9, beta2 = 0.999, eps = 1e-8; after each step theta is
    clipped to the box given by the caller (the optics must stay valid).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.fft as sfft

from . import linear
from . import optics as op
from . import tf as tfm

PARAMS = ("defocus", "na_det", "tilt_zenith", "tilt_azimuth")


def with_theta(o: op.Optics, theta) -> op.Optics:
    return o.replace(defocus=float(theta[0]), na_det=float(theta[1]),
                     tilt_zenith=float(theta[2]), tilt_azimuth=float(theta[3]))


def theta_of(o: op.Optics) -> np.ndarray:
    return np.array([o.defocus, o.na_det, o.tilt_zenith, o.tilt_azimuth], dtype=np.float64)


def midband_mask(o: op.Optics, nu_c: float) -> np.ndarray:
    """Boolean (Y, X) mask of nu_c/8 <= |nu_perp| <= nu_c/4 (reading R10)."""
    fy, fx = op.lateral_frequencies(o)
    r = np.sqrt(fy * fy + fx * fx)
    return (r >= nu_c / 8.0) & (r <= nu_c / 4.0)


def nominal_cutoff(o: op.Optics) -> float:
    return (o.na_det + o.na_ill) / o.wavelength


def loss(o: op.Optics, d: np.ndarray, eta: float, nu_c: float) -> float:
    """Mid-band loss of the thin phase reconstruction of the stack d (Z, Y, X)."""
    bank = tfm.labelfree_thin(o)
    F = linear.reconstruct_spectrum(bank, d, None, eta)
    m = midband_mask(o, nu_c)
    return float(-np.mean(np.abs(F[0][m]) ** 2))


def fd_gradient(o: op.Optics, d, eta, nu_c, steps, which=(0, 1, 2, 3)) -> np.ndarray:
    """Central finite differences with one Richardson step (h and h/2)."""
    th = theta_of(o)
    g = np.zeros(4)
    for j in which:
        def cd(h):
            tp, tm = th.copy(), th.copy()
            tp[j] += h
            tm[j] -= h
            return (loss(with_theta(o, tp), d, eta, nu_c) - loss(with_theta(o, tm), d, eta, nu_c)) / (2 * h)
        h = steps[j]
        g[j] = (4.0 * cd(h / 2) - cd(h)) / 3.0
    return g


def fd_gradient_aberration(o: op.Optics, d, eta, nu_c, h=1e-3, n=7) -> np.ndarray:
    """dL/d zernike[j] (j < n, per wave) by central differences with one Richardson
    step (h and h/2), the other coefficients and theta held (R18)."""
    c0 = np.zeros(n)
    c0[: len(o.zernike)] = o.zernike[:n]
    g = np.zeros(n)
    for j in range(n):
        def cd(step):
            cp, cm = c0.copy(), c0.copy()
            cp[j] += step
            cm[j] -= step
            return (loss(o.replace(zernike=tuple(cp)), d, eta, nu_c)
                    - loss(o.replace(zernike=tuple(cm)), d, eta, nu_c)) / (2 * step)
        g[j] = (4.0 * cd(h / 2) - cd(h)) / 3.0
    return g


# --- analytic reverse-mode gradient (Ext. Data Fig. 3, dashed arrows)

def _edge_slope(inside: np.ndarray, halfwidth: float) -> np.ndarray:
    """d edge / d inside for the soft edge (0 for the hard edge)."""
    if halfwidth == 0.0:
        return np.zeros_like(inside)
    t = (inside / halfwidth + 1.0) * 0.5
    s = 6.0 * t * (1.0 - t) * (0.5 / halfwidth)
    return np.where((t > 0.0) & (t < 1.0), s, 0.0)


def detection_tilt_derivatives(o: op.Optics):
    """dP/d(det_tilt) and dP/d(det_azimuth) of the tilted detection cap (R20):
    P = edge(NA_det/lambda0 - |p'|), |p'| = sqrt(k_m^2 - (k . a)^2), so
    d|p'| = -(k . a)(k . da)/|p'| (zero for the hard edge)."""
    fy, fx = op.lateral_frequencies(o)
    hw = o.edge_width * o.dnu
    pp2, ka = op.detection_lateral_distance_sq(o)
    pp = np.sqrt(np.maximum(pp2, 0.0))
    kz = np.sqrt(np.maximum(o.k_medium ** 2 - fy * fy - fx * fx, 0.0))
    on = (fy * fy + fx * fx < o.k_medium ** 2) & (ka > 0.0)
    sl = np.where(on, _edge_slope(o.na_det / o.wavelength - pp, hw), 0.0)
    t, az = o.det_tilt, o.det_azimuth
    da_dt = (math.cos(t) * math.sin(az), math.cos(t) * math.cos(az), -math.sin(t))
    da_daz = (math.sin(t) * math.cos(az), -math.sin(t) * math.sin(az), 0.0)
    out = []
    for da in (da_dt, da_daz):
        kda = fy * da[0] + fx * da[1] + kz * da[2]
        with np.errstate(invalid="ignore", divide="ignore"):
            dpp = np.where(pp > 0, -ka * kda / pp, 0.0)
        out.append(-sl * dpp)
    return out[0], out[1]


def pupil_derivatives(o: op.Optics):
    """S, P and their partial derivatives w.r.t. (na_det, tilt_zenith, tilt_azimuth)."""
    fy, fx = op.lateral_frequencies(o)
    hw = o.edge_width * o.dnu
    rp = np.sqrt(fy * fy + fx * fx)
    if o.det_tilt != 0.0:   # the lateral distance in the tilted frame (R20)
        rp = np.sqrt(np.maximum(op.detection_lateral_distance_sq(o)[0], 0.0))
    P = op.detection_pupil(o)
    dP_dna = _edge_slope(o.na_det / o.wavelength - rp, hw) / o.wavelength
    cy, cx = op.source_centre(o)
    dy, dx = fy - cy, fx - cx
    rq = np.sqrt(dy * dy + dx * dx)
    S = op.illumination_pupil(o)
    slope = _edge_slope(o.na_ill / o.wavelength - rq, hw)
    with np.errstate(invalid="ignore", divide="ignore"):
        uy = np.where(rq > 0, dy / rq, 0.0)
        ux = np.where(rq > 0, dx / rq, 0.0)
    # d|q - q0| / d q0 = -(q - q0)/|q - q0|, and d inside = -d|q - q0|
    dS_dcy, dS_dcx = slope * uy, slope * ux
    r = o.n_medium * math.sin(o.tilt_zenith) / o.wavelength
    dr = o.n_medium * math.cos(o.tilt_zenith) / o.wavelength
    sa, ca = math.sin(o.tilt_azimuth), math.cos(o.tilt_azimuth)
    dS_dzen = dS_dcy * dr * sa + dS_dcx * dr * ca
    dS_daz = dS_dcy * r * ca - dS_dcx * r * sa
    return S, P, dP_dna, dS_dzen, dS_daz


def loss_and_gradient(o: op.Optics, d: np.ndarray, eta: float, nu_c: float):
    """Loss and dL/dtheta by hand-written reverse mode through the thin model."""
    Z, Y, X = o.nz, o.ny, o.nx
    N = Y * X
    S, P, dP_dna, dS_dzen, dS_daz = pupil_derivatives(o)
    g = op.greens_spectrum(o)
    kz = op.axial_wavenumber(o)
    ibg = float(np.sum(S * P * P))
    s = N / ibg
    zs = op.z_planes_thin(o)
    a = np.empty((Z, Y, X), np.complex128)
    b = np.empty((Z, Y, X), np.complex128)
    for k, z in enumerate(zs):
        prop = np.exp(2j * np.pi * kz * (z - o.defocus))
        a[k] = sfft.ifft2(S * P * prop)
        b[k] = sfft.ifft2(P * g * prop)
    c = s * b * np.conj(a)
    bank = np.stack([sfft.fft2(2.0 * c.real), sfft.fft2(-2.0 * c.imag)], axis=1)  # (Z, 2, Y, X)
    Dk = sfft.fft2(np.asarray(d, dtype=np.float64))
    Hn = np.moveaxis(bank.reshape(Z, 2, -1), 2, 0)          # (n, C, P)
    Dn = np.moveaxis(Dk.reshape(Z, -1), 1, 0)               # (n, C)
    Hh = np.conj(np.swapaxes(Hn, 1, 2))
    M = Hh @ Hn + eta * np.eye(2)[None]
    Fn = np.linalg.solve(M, np.einsum("npc,nc->np", Hh, Dn)[..., None])[..., 0]
    mask = midband_mask(o, nu_c).reshape(-1)
    nb = int(mask.sum())
    L = float(-np.sum(np.abs(Fn[mask, 0]) ** 2) / nb)
    # dL/dF* on the band, phase component only
    GF = np.zeros_like(Fn)
    GF[mask, 0] = -Fn[mask, 0] / nb
    Yv = np.linalg.solve(M, GF[..., None])[..., 0]          # M^-1 G_F
    r = Dn - np.einsum("ncp,np->nc", Hn, Fn)
    HY = np.einsum("ncp,np->nc", Hn, Yv)
    GH = r[:, :, None] * np.conj(Yv)[:, None, :] - HY[:, :, None] * np.conj(Fn)[:, None, :]
    GH = np.moveaxis(GH, 0, 2).reshape(Z, 2, Y, X)
    return L, _pair_gradient_to_theta(o, zs, GH, a, b)[:4]


def _pair_gradient_to_theta(o: op.Optics, zs, GH: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """dL/dtheta (defocus, na_det, tilt_zenith, tilt_azimuth, det_tilt,
    det_azimuth) from the gradient GH = dL/dH_z* (Z, 2, Y, X) of the per-plane 2D
    label-free pair H_z = [fft2(2 Re c_z), fft2(-2 Im c_z)] at the planes zs,
    c_z = (N / I_bg) b_z conj(a_z), a_z, b_z the inverse 2D transforms of the
    direct and scattered arms (Table 1's label-free row), by reverse mode
    through c, the arms and the pupils."""
    Y, X = o.ny, o.nx
    N = Y * X
    S, P, dP_dna, dS_dzen, dS_daz = pupil_derivatives(o)
    dP_dt, dP_daz = detection_tilt_derivatives(o)
    g = op.greens_spectrum(o)
    kz = op.axial_wavenumber(o)
    ibg = float(np.sum(S * P * P))
    s = N / ibg
    # back through H = fft2(2 Re c), fft2(-2 Im c): Gamma = Re(N ifft2 G_ph) + i Re(N ifft2 G_abs)
    gam = N * sfft.ifft2(GH, axes=(-2, -1))
    Gam = gam[:, 0].real + 1j * gam[:, 1].real              # (Z, Y, X)
    # dL = 4 Re sum_r Gam dc,  c = s b conj(a)
    ds_term = 4.0 * np.real(np.sum(Gam * b * np.conj(a)))
    UB = sfft.ifft2(s * Gam * np.conj(a), axes=(-2, -1))     # dL = 4 Re sum dB * UB
    UA = sfft.ifft2(s * np.conj(Gam * b), axes=(-2, -1))     # dL = 4 Re sum dA * UA
    grad = np.zeros(6)
    for k, z in enumerate(zs):
        prop = np.exp(2j * np.pi * kz * (z - o.defocus))
        A = S * P * prop
        B = P * g * prop
        dprop = -2j * np.pi * kz                               # d prop / d defocus, relative
        grad[0] += 4.0 * np.real(np.sum(UB[k] * B * dprop) + np.sum(UA[k] * A * dprop))
        grad[1] += 4.0 * np.real(np.sum(UB[k] * dP_dna * g * prop) + np.sum(UA[k] * S * dP_dna * prop))
        grad[2] += 4.0 * np.real(np.sum(UA[k] * dS_dzen * P * prop))
        grad[3] += 4.0 * np.real(np.sum(UA[k] * dS_daz * P * prop))
        grad[4] += 4.0 * np.real(np.sum(UB[k] * dP_dt * g * prop) + np.sum(UA[k] * S * dP_dt * prop))
        grad[5] += 4.0 * np.real(np.sum(UB[k] * dP_daz * g * prop) + np.sum(UA[k] * S * dP_daz * prop))
    # s = N / I_bg, I_bg = sum S P^2
    dibg = np.array([0.0, np.sum(2.0 * S * P * dP_dna), np.sum(dS_dzen * P * P), np.sum(dS_daz * P * P),
                     np.sum(2.0 * S * P * dP_dt), np.sum(2.0 * S * P * dP_daz)])
    grad += ds_term * (-s / ibg) * dibg
    return grad


# --- gradient of a loss of the 3D reconstruction (Ext. Data Fig. 3, backpropagation
# through the Tikhonov inverse into the transfer-function synthesis)

def recon_objective(o: op.Optics, d: np.ndarray, eta: float, w: np.ndarray, b=None) -> float:
    """L = sum_r w(r) f(r), f = the Tikhonov reconstruction of d with the bank of o
    (a loss linear in f; any loss enters the reverse mode only through dL/df = w)."""
    f = linear.reconstruct(tfm.transfer_function(o), d, b, eta)
    return float(np.sum(np.asarray(w, dtype=np.float64) * f))


PARAMS6 = PARAMS + ("det_tilt", "det_azimuth")


def with_theta6(o: op.Optics, theta) -> op.Optics:
    return with_theta(o, theta).replace(det_tilt=float(theta[4]), det_azimuth=float(theta[5]))


def recon_fd_gradient(o: op.Optics, d, eta, w, steps, b=None, which=(0, 1, 2, 3, 4, 5)) -> np.ndarray:
    """dL/dtheta (the six components of PARAMS6) of recon_objective by central
    differences with one Richardson step (steps: one per component)."""
    th = np.concatenate([theta_of(o), [o.det_tilt, o.det_azimuth]])
    g = np.zeros(6)
    for j in which:
        def cd(h):
            tp, tm = th.copy(), th.copy()
            tp[j] += h
            tm[j] -= h
            return (recon_objective(with_theta6(o, tp), d, eta, w, b)
                    - recon_objective(with_theta6(o, tm), d, eta, w, b)) / (2 * h)
        h = steps[j]
        g[j] = (4.0 * cd(h / 2) - cd(h)) / 3.0
    return g


def recon_gradient(o: op.Optics, d: np.ndarray, eta: float, w: np.ndarray, b=None):
    """Reverse mode for a loss L of the 3D reconstruction f given w = dL/df
    (P, Z, Y, X): returns (dL/dtheta (6,) over PARAMS6, dL/dd (C, Z, Y, X)).  Label-free 3D and
    the 5 x 4 polarisation bank (whose entries are Re(kappa) H_phase +
    Im(kappa) H_abs of the label-free pair).

    Per 3D frequency, F = M^-1 H^H (D - N b delta), M = H^H H + eta I; with
    dL/dF* = FFT3(w) / (2 N) (f = Re IFFT3 F), Y = M^-1 dL/dF*, R = D - N b delta - H F:
    dL/dH* = R Y^H - H Y F^H and dL/dd = Re IFFT3(2 N H Y).  The 3D pair is the
    axial DFT of the per-plane 2D pair, H(kz) = sum_z e^{-i 2 pi kz z / Z} H_z, so
    dL/dH_z* = sum_kz e^{+i 2 pi kz z / Z} dL/dH(kz)* (the unnormalised inverse
    DFT), after which the chain is the per-plane one of the thin model."""
    if o.model not in (op.LABELFREE_3D, op.POL5_3D):
        raise ValueError("label-free 3D or polarisation models only")
    if any(z != 0 for z in o.zernike):
        raise ValueError("unaberrated optics only (aberrated: recon_fd_gradient)")
    Z, Y, X = o.nz, o.ny, o.nx
    N = Z * Y * X
    zs = op.z_planes_3d(o)
    S = op.illumination_pupil(o)
    P = op.detection_pupil(o)
    g = op.greens_spectrum(o)
    kzz = op.axial_wavenumber(o)
    ibg = float(np.sum(S * P * P))
    a = np.empty((Z, Y, X), np.complex128)
    bb = np.empty((Z, Y, X), np.complex128)
    for k, z in enumerate(zs):
        prop = np.exp(2j * np.pi * kzz * (z - o.defocus))
        a[k] = sfft.ifft2(S * P * prop)
        bb[k] = sfft.ifft2(P * g * prop)
    c = (Y * X / ibg) * bb * np.conj(a)
    hp, ha = sfft.fftn(2.0 * c.real), sfft.fftn(-2.0 * c.imag)
    if o.model == op.POL5_3D:
        kap = tfm.pol5_coupling(o.swing)
        bank = kap.real[:, :, None, None, None] * hp + kap.imag[:, :, None, None, None] * ha
    else:
        kap = None
        bank = np.stack([hp, ha])[None]
    C, Pn = bank.shape[:2]
    D = sfft.fftn(np.asarray(d, dtype=np.float64), axes=(-3, -2, -1))
    if b is not None:
        D[:, 0, 0, 0] -= N * np.asarray(b, dtype=np.float64)
    Gw = sfft.fftn(np.asarray(w, dtype=np.float64), axes=(-3, -2, -1)) / (2.0 * N)
    Hn = np.moveaxis(bank.reshape(C, Pn, -1), 2, 0)            # (n, C, P)
    Dn = np.moveaxis(D.reshape(C, -1), 1, 0)                    # (n, C)
    Gn = np.moveaxis(Gw.reshape(Pn, -1), 1, 0)                  # (n, P)
    Hh = np.conj(np.swapaxes(Hn, 1, 2))
    M = Hh @ Hn + eta * np.eye(Pn)[None]
    Fn = np.linalg.solve(M, np.einsum("npc,nc->np", Hh, Dn)[..., None])[..., 0]
    Yv = np.linalg.solve(M, Gn[..., None])[..., 0]
    r = Dn - np.einsum("ncp,np->nc", Hn, Fn)
    HY = np.einsum("ncp,np->nc", Hn, Yv)
    GH = r[:, :, None] * np.conj(Yv)[:, None, :] - HY[:, :, None] * np.conj(Fn)[:, None, :]   # (n, C, P)
    if kap is None:
        Gpair = GH[:, 0, :]                                      # (n, 2)
    else:
        # dH_cp = Re(kappa_cp) dH_phase + Im(kappa_cp) dH_abs with real coefficients
        Gpair = np.stack([np.einsum("cp,ncp->n", kap.real, GH), np.einsum("cp,ncp->n", kap.imag, GH)], 1)
    G3 = np.moveaxis(Gpair, 0, 1).reshape(2, Z, Y, X)
    Gz = Z * sfft.ifft(G3, axis=1)                               # unnormalised inverse DFT along z
    grad = _pair_gradient_to_theta(o, zs, np.moveaxis(Gz, 0, 1), a, bb)
    dd = sfft.ifftn((2.0 * N) * np.moveaxis(HY, 0, 1).reshape(C, Z, Y, X), axes=(-3, -2, -1)).real
    return grad, dd


# --- optimiser

@dataclasses.dataclass
class AdamState:
    theta: np.ndarray
    m: np.ndarray
    v: np.ndarray
    t: int = 0


def adam_step(st: AdamState, grad, lr, lo, hi, b1=0.9, b2=0.999, eps=1e-8, mask=None):
    """One Adam step (Kingma & Ba), then clip theta to [lo, hi] (reading R12)."""
    grad = np.asarray(grad, dtype=np.float64)
    if mask is not None:
        grad = grad * mask
    st.t += 1
    st.m = b1 * st.m + (1 - b1) * grad
    st.v = b2 * st.v + (1 - b2) * grad * grad
    mh = st.m / (1 - b1 ** st.t)
    vh = st.v / (1 - b2 ** st.t)
    st.theta = np.clip(st.theta - np.asarray(lr) * mh / (np.sqrt(vh) + eps), lo, hi)
    return st


def autotune(o: op.Optics, d, eta, nu_c, iters, lr, lo, hi, mask=(1, 1, 1, 0)):
    """Adam on theta for ``iters`` iterations from o's parameters; returns (theta, loss)."""
    th0 = theta_of(o)
    st = AdamState(th0.copy(), np.zeros(4), np.zeros(4))
    msk = np.asarray(mask, dtype=np.float64)
    for _ in range(iters):
        _, g = loss_and_gradient(with_theta(o, st.theta), d, eta, nu_c)
        adam_step(st, g, lr, lo, hi, mask=msk)
    return st.theta, loss(with_theta(o, st.theta), d, eta, nu_c)


def autotune_aberration(o: op.Optics, d, eta, nu_c, iters, lr, bound, mask=(1,) * 7):
    """Adam on the seven Zernike coefficients (theta held) for ``iters`` iterations from
    o's coefficients, gradients by central differences of the loss, box [-bound,
    bound]; returns (coefficients, loss)."""
    c0 = np.zeros(7)
    c0[: len(o.zernike)] = o.zernike[:7]
    st = AdamState(c0.copy(), np.zeros(7), np.zeros(7))
    msk = np.asarray(mask, dtype=np.float64)
    for _ in range(iters):
        g = fd_gradient_aberration(o.replace(zernike=tuple(st.theta)), d, eta, nu_c)
        adam_step(st, g, lr, -bound, bound, mask=msk)
    return st.theta, loss(o.replace(zernike=tuple(st.theta)), d, eta, nu_c)
