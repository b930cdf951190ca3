"""Seeded specimen and noise generators (float32 outputs).

Specimens mimic the structure of the paper's workloads: point beads for
widefield fluorescence, ellipsoidal cells for label-free phase/absorption,
spline fibres with retardance and orientation for polarisation imaging, and
thin cells at a nominal plane for phase-from-defocus tiles.  Values are in
the property units the model uses (radians per voxel for label-free
properties, arbitrary density for fluorescence).
"""

from __future__ import annotations

import math

import numpy as np


def _rotation(rng) -> np.ndarray:
    """Uniformly random 3D rotation (QR of a Gaussian matrix, sign-fixed)."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def beads(shape, n_beads, seed, amp=(0.5, 1.0)) -> np.ndarray:
    """Point beads at uniform random integer voxels, amplitudes ~U(amp); coincident beads add."""
    rng = np.random.default_rng(seed)
    vol = np.zeros(shape, dtype=np.float64)
    idx = tuple(rng.integers(0, s, n_beads) for s in shape)
    np.add.at(vol, idx, rng.uniform(amp[0], amp[1], n_beads))
    return vol.astype(np.float32)


def ellipsoids(shape, voxel, n, seed, semi_axes=(1.0, 5.0), dn=(0.01, 0.05),
               dkappa=(0.0, 0.005), wavelength=0.532) -> np.ndarray:
    """Randomly oriented ellipsoids; returns (2, Z, Y, X) [phase, absorption] per voxel.

    Each ellipsoid carries an index contrast dn and an absorption dkappa; per
    voxel of axial size dz they contribute 2 pi dn dz / lambda0 radians of phase
    and 2 pi dkappa dz / lambda0 of absorption.  Overlaps add; ellipsoids are
    clipped at the volume boundary.
    """
    rng = np.random.default_rng(seed)
    Z, Y, X = shape
    dz, dy, dx = voxel
    out = np.zeros((2,) + tuple(shape), dtype=np.float64)
    ext = np.array([Z * dz, Y * dy, X * dx])
    for _ in range(n):
        R = _rotation(rng)
        ax = rng.uniform(semi_axes[0], semi_axes[1], 3)
        c = rng.uniform(0.0, 1.0, 3) * ext
        vals = (2 * math.pi * rng.uniform(*dn) * dz / wavelength,
                2 * math.pi * rng.uniform(*dkappa) * dz / wavelength)
        rmax = ax.max()
        lo = np.maximum(np.floor((c - rmax) / np.array(voxel)).astype(int), 0)
        hi = np.minimum(np.ceil((c + rmax) / np.array(voxel)).astype(int) + 1, shape)
        if np.any(hi <= lo):
            continue
        zz, yy, xx = np.meshgrid(*(np.arange(l, h) * v for l, h, v in zip(lo, hi, voxel)),
                                 indexing="ij", sparse=True)
        rel = [zz - c[0], yy - c[1], xx - c[2]]
        u = [R[0, i] * rel[0] + R[1, i] * rel[1] + R[2, i] * rel[2] for i in range(3)]
        inside = (u[0] / ax[0]) ** 2 + (u[1] / ax[1]) ** 2 + (u[2] / ax[2]) ** 2 <= 1.0
        sl = tuple(slice(l, h) for l, h in zip(lo, hi))
        out[0][sl] += vals[0] * inside
        out[1][sl] += vals[1] * inside
    return out.astype(np.float32)


def _catmull_rom(ctrl: np.ndarray, n: int) -> np.ndarray:
    """Points on a cubic Catmull-Rom spline through the control points (end points doubled)."""
    p = np.concatenate([ctrl[:1], ctrl, ctrl[-1:]], axis=0)
    segs = len(ctrl) - 1
    out = []
    for s in range(segs):
        p0, p1, p2, p3 = p[s], p[s + 1], p[s + 2], p[s + 3]
        t = np.linspace(0.0, 1.0, n, endpoint=(s == segs - 1))[:, None]
        out.append(0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t ** 2
                          + (-p0 + 3 * p1 - 3 * p2 + p3) * t ** 3))
    return np.concatenate(out, axis=0)


def fibres(shape, voxel, n, seed, sigma=0.15, retardance_nm=(0.0, 5.0), dn=(0.01, 0.05),
           wavelength=0.532, batch=64) -> np.ndarray:
    """Spline fibres with a Gaussian cross-section; returns (4, Z, Y, X).

    Properties per voxel: [phase, rho cos 2w, rho sin 2w, absorption(=0)], where
    rho = 2 pi retardance / lambda0 and w ~ U(0, pi) is the fibre's orientation;
    the profile is 1 on the fibre axis and falls off as exp(-r^2 / 2 sigma^2).
    Each fibre is a chain of points sigma/2 apart, each point spreading a 3D
    Gaussian (the product of one Gaussian per axis) over the voxels within
    3 sigma of it.
    """
    rng = np.random.default_rng(seed)
    Z, Y, X = shape
    vox = np.asarray(voxel, dtype=np.float64)
    ext = np.array([Z, Y, X]) * vox
    nvox = Z * Y * X
    out = np.zeros((3, nvox), dtype=np.float64)
    step = sigma / 2.0
    half = np.ceil(3 * sigma / vox).astype(int)
    pend_idx, pend_w = [], []

    def flush():
        if not pend_idx:
            return
        idx = np.concatenate(pend_idx)
        w = np.concatenate(pend_w, axis=1)
        for j in range(3):
            np.add.at(out[j], idx, w[j])
        pend_idx.clear()
        pend_w.clear()

    for i in range(n):
        ctrl = rng.uniform(0.0, 1.0, (4, 3)) * ext
        rho = 2 * math.pi * rng.uniform(*retardance_nm) * 1e-3 / wavelength
        w = rng.uniform(0.0, math.pi)
        phase = 2 * math.pi * rng.uniform(*dn) * vox[0] / wavelength
        vals = np.array([phase, rho * math.cos(2 * w), rho * math.sin(2 * w)])
        dense = _catmull_rom(ctrl, 64)
        seg = np.linalg.norm(np.diff(dense, axis=0), axis=1)
        s = np.concatenate([[0.0], np.cumsum(seg)])
        npts = max(int(s[-1] / step), 2)
        si = np.linspace(0.0, s[-1], npts)
        pts = np.stack([np.interp(si, s, dense[:, k]) for k in range(3)], -1)
        ds = s[-1] / (npts - 1)
        base = np.rint(pts / vox).astype(np.int64)
        # per axis: the cells within 3 sigma, their 1D Gaussian factor and validity
        cell, g, ok = [], [], []
        for a in range(3):
            c = base[:, a, None] + np.arange(-half[a], half[a] + 1)[None, :]
            g.append(np.exp(-((c * vox[a] - pts[:, a, None]) ** 2) / (2 * sigma * sigma)))
            cell.append(c)
            ok.append((c >= 0) & (c < shape[a]))
        wgt = (g[0][:, :, None, None] * g[1][:, None, :, None] * g[2][:, None, None, :]
               * (ds / (math.sqrt(2 * math.pi) * sigma)))
        flat = ((cell[0][:, :, None, None] * Y + cell[1][:, None, :, None]) * X + cell[2][:, None, None, :])
        keep = ok[0][:, :, None, None] & ok[1][:, None, :, None] & ok[2][:, None, None, :]
        wk = wgt[keep]
        pend_idx.append(flat[keep])
        pend_w.append(vals[:, None] * wk[None, :])
        if (i + 1) % batch == 0:
            flush()
    flush()
    res = np.zeros((4, nvox), dtype=np.float32)
    res[:3] = out
    return res.reshape((4,) + tuple(shape))


def fibres_on_device(shape, voxel, n, seed, device, sigma=0.15, retardance_nm=(0.0, 5.0),
                     dn=(0.01, 0.05), wavelength=0.532):
    """fibres() rendered with torch on `device` (FP32 accumulation): the same
    random draws and the same point chains and per-axis Gaussian factors, for
    volumes whose host rendering would take minutes.  Returns a (4, Z, Y, X)
    float32 tensor on the device."""
    import torch
    rng = np.random.default_rng(seed)
    Z, Y, X = shape
    vox = np.asarray(voxel, dtype=np.float64)
    ext = np.array([Z, Y, X]) * vox
    out = torch.zeros((4, Z * Y * X), dtype=torch.float32, device=device)
    step = sigma / 2.0
    half = np.ceil(3 * sigma / vox).astype(int)
    rel = [torch.arange(-h, h + 1, device=device) for h in half]
    for _ in range(n):
        ctrl = rng.uniform(0.0, 1.0, (4, 3)) * ext
        rho = 2 * math.pi * rng.uniform(*retardance_nm) * 1e-3 / wavelength
        w = rng.uniform(0.0, math.pi)
        phase = 2 * math.pi * rng.uniform(*dn) * vox[0] / wavelength
        vals = (phase, rho * math.cos(2 * w), rho * math.sin(2 * w))
        dense = _catmull_rom(ctrl, 64)
        seg = np.linalg.norm(np.diff(dense, axis=0), axis=1)
        s = np.concatenate([[0.0], np.cumsum(seg)])
        npts = max(int(s[-1] / step), 2)
        si = np.linspace(0.0, s[-1], npts)
        pts_h = np.stack([np.interp(si, s, dense[:, k]) for k in range(3)], -1)
        ds = s[-1] / (npts - 1)
        pts = torch.from_numpy(pts_h).to(device)
        base = torch.from_numpy(np.rint(pts_h / vox).astype(np.int64)).to(device)
        cell, g, ok = [], [], []
        for a in range(3):
            c = base[:, a, None] + rel[a][None, :]
            g.append(torch.exp(-((c * vox[a] - pts[:, a, None]) ** 2) / (2 * sigma * sigma)))
            cell.append(c)
            ok.append((c >= 0) & (c < shape[a]))
        wgt = (g[0][:, :, None, None] * g[1][:, None, :, None] * g[2][:, None, None, :]
               * (ds / (math.sqrt(2 * math.pi) * sigma)))
        flat = (cell[0][:, :, None, None] * Y + cell[1][:, None, :, None]) * X + cell[2][:, None, None, :]
        keep = ok[0][:, :, None, None] & ok[1][:, None, :, None] & ok[2][:, None, None, :]
        idx, wk = flat[keep], wgt[keep].to(torch.float32)
        for j in range(3):
            out[j].index_add_(0, idx, wk * float(vals[j]))
    return out.reshape((4,) + tuple(shape))


def thin_cells(shape_yx, pixel, n, seed, semi_axes=(0.8, 2.5), phase=(0.1, 0.5),
               absorption=(0.0, 0.02)) -> np.ndarray:
    """Thin 2D cells at the nominal plane; returns (2, Y, X) [phase, absorption].

    Each cell is a randomly oriented ellipse with a dome profile 1 - rho^2/2
    (rho the normalised elliptical radius) scaled by its peak phase and
    absorption; cells add where they overlap and wrap around the tile edges.
    """
    rng = np.random.default_rng(seed)
    Y, X = shape_yx
    yy = np.arange(Y)[:, None] * pixel
    xx = np.arange(X)[None, :] * pixel
    out = np.zeros((2, Y, X))
    for _ in range(n):
        cy, cx = rng.uniform(0, Y * pixel), rng.uniform(0, X * pixel)
        a, b = rng.uniform(*semi_axes, 2)
        t = rng.uniform(0, math.pi)
        ph, ab = rng.uniform(*phase), rng.uniform(*absorption)
        dy = (yy - cy + 0.5 * Y * pixel) % (Y * pixel) - 0.5 * Y * pixel
        dx = (xx - cx + 0.5 * X * pixel) % (X * pixel) - 0.5 * X * pixel
        u = dx * math.cos(t) + dy * math.sin(t)
        v = -dx * math.sin(t) + dy * math.cos(t)
        r2 = (u / a) ** 2 + (v / b) ** 2
        prof = np.where(r2 <= 1.0, 1.0 - 0.5 * r2, 0.0)
        out[0] += ph * prof
        out[1] += ab * prof
    return out.astype(np.float32)


def gaussian_noise(shape, sigma, seed) -> np.ndarray:
    return (np.random.default_rng(seed).standard_normal(shape) * sigma).astype(np.float32)


def poisson_gaussian(contrast, seed, i_bg=1000.0, read_sigma=2.0) -> np.ndarray:
    """Noisy relative contrast: I = Poisson(I_bg (1 + d)) + N(0, read_sigma^2); returns I/I_bg - 1."""
    rng = np.random.default_rng(seed)
    lam = np.clip(i_bg * (1.0 + np.asarray(contrast, dtype=np.float64)), 0.0, None)
    inten = rng.poisson(lam).astype(np.float64) + rng.standard_normal(lam.shape) * read_sigma
    return (inten / i_bg - 1.0).astype(np.float32)


def plane_waves(shape, waves) -> np.ndarray:
    """Sum of real plane waves A cos(2 pi sum_i k_i r_i / N_i + phi) on the grid.

    ``waves`` is a list of (k_tuple, amplitude, phase) with integer frequency
    indices k (one per axis).  Used for full-size checks whose spectra are
    known in closed form.
    """
    out = np.zeros(shape, dtype=np.float64)
    grids = np.meshgrid(*(np.arange(n) / n for n in shape), indexing="ij", sparse=True)
    for k, amp, ph in waves:
        arg = sum(2 * math.pi * ki * g for ki, g in zip(k, grids))
        out += amp * np.cos(arg + ph)
    return out.astype(np.float32)
