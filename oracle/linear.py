"""Forward model, Tikhonov reconstruction and adjoint of the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Forward (Methods, "Linear contrast-separable shift-invariant imaging
  systems"): d_c = sum_p h_cp (*) f_p + b_c, i.e. in Fourier space
  D_c(nu) = sum_p H_cp(nu) F_p(nu) + b_c delta(nu).  Convolutions are circular
  on the sampled grid, so the DFT diagonalises them exactly.
* Reconstruction (Methods, "Reconstructing object properties" and
  "Reconstruction algorithm"): the minimiser of
  ||d - b - H f||^2 + eta ||f||^2.  Because H is block-diagonal in nu, its SVD
  splits into one C x P SVD per frequency and Eq. tls_solution
  R_eta = sum_i s_i / (s_i^2 + eta) v_i u_i^H equals, per frequency,
  F = (H^H H + eta I)^-1 H^H (D - N b delta).  For eta == 0 the oracle uses the
  minimum-norm pseudo-inverse (the SVD sum over the rank R).
* Adjoint: g_p = Re IFFT(sum_c conj(H_cp) R_c).

Array layout: bank (C, P, *spatial), object (P, *spatial), data (C, *spatial),
where *spatial is (Z, Y, X) for the 3D models and (Y, X) for the thin model.
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sfft


def _axes(bank: np.ndarray):
    nd = bank.ndim - 2
    return tuple(range(-nd, 0))


def forward(bank: np.ndarray, f: np.ndarray, b=None) -> np.ndarray:
    """d = H f + b (Eq. fwd), real output (C, *spatial)."""
    ax = _axes(bank)
    F = sfft.fftn(np.asarray(f, dtype=np.float64), axes=ax)
    D = np.einsum("cp...,p...->c...", bank, F)
    if b is not None:
        n = int(np.prod(bank.shape[2:]))
        D[(slice(None),) + (0,) * len(ax)] += n * np.asarray(b, dtype=np.float64)
    return sfft.ifftn(D, axes=ax).real


def forward_imag_residual(bank: np.ndarray, f: np.ndarray) -> float:
    """Relative size of the discarded imaginary part of IFFT(H F) (Hermitian check)."""
    ax = _axes(bank)
    F = sfft.fftn(np.asarray(f, dtype=np.float64), axes=ax)
    d = sfft.ifftn(np.einsum("cp...,p...->c...", bank, F), axes=ax)
    return float(np.linalg.norm(d.imag) / max(np.linalg.norm(d.real), 1e-300))


def solve_per_frequency(H: np.ndarray, D: np.ndarray, eta: float) -> np.ndarray:
    """Per-frequency Tikhonov solve.  H: (n, C, P), D: (n, C) -> F: (n, P)."""
    P = H.shape[2]
    Hh = np.conj(np.swapaxes(H, 1, 2))
    rhs = np.einsum("npc,nc->np", Hh, D)
    if eta > 0:
        M = Hh @ H + eta * np.eye(P)[None]
        return np.linalg.solve(M, rhs[..., None])[..., 0]
    # eta == 0: minimum-norm least squares, zero where H vanishes
    return np.einsum("npc,nc->np", np.linalg.pinv(H), D)


def reconstruct(bank: np.ndarray, d: np.ndarray, b=None, eta: float = 0.0) -> np.ndarray:
    """f = R_eta d (Eq. recon / tls_solution), real output (P, *spatial)."""
    ax = _axes(bank)
    C, P = bank.shape[:2]
    spatial = bank.shape[2:]
    D = sfft.fftn(np.asarray(d, dtype=np.float64), axes=ax)
    if b is not None:
        n = int(np.prod(spatial))
        D[(slice(None),) + (0,) * len(ax)] -= n * np.asarray(b, dtype=np.float64)
    Hn = np.moveaxis(bank.reshape(C, P, -1), 2, 0)
    Dn = np.moveaxis(D.reshape(C, -1), 1, 0)
    Fn = solve_per_frequency(Hn, Dn, eta)
    F = np.moveaxis(Fn, 0, 1).reshape((P,) + spatial)
    return sfft.ifftn(F, axes=ax).real


def reconstruct_spectrum(bank: np.ndarray, d: np.ndarray, b=None, eta: float = 0.0) -> np.ndarray:
    """The reconstructed spectrum F (P, *spatial) before the inverse transform."""
    ax = _axes(bank)
    C, P = bank.shape[:2]
    spatial = bank.shape[2:]
    D = sfft.fftn(np.asarray(d, dtype=np.float64), axes=ax)
    if b is not None:
        D[(slice(None),) + (0,) * len(ax)] -= int(np.prod(spatial)) * np.asarray(b, dtype=np.float64)
    Hn = np.moveaxis(bank.reshape(C, P, -1), 2, 0)
    Dn = np.moveaxis(D.reshape(C, -1), 1, 0)
    return np.moveaxis(solve_per_frequency(Hn, Dn, eta), 0, 1).reshape((P,) + spatial)


def adjoint(bank: np.ndarray, r: np.ndarray) -> np.ndarray:
    """g = H^H r, real output (P, *spatial)."""
    ax = _axes(bank)
    R = sfft.fftn(np.asarray(r, dtype=np.float64), axes=ax)
    G = np.einsum("cp...,c...->p...", np.conj(bank), R)
    return sfft.ifftn(G, axes=ax).real


def max_singular_value_sq(bank: np.ndarray) -> float:
    """max over nu of sigma_max(H(nu))^2, used to scale a relative eta."""
    C, P = bank.shape[:2]
    Hn = np.moveaxis(bank.reshape(C, P, -1), 2, 0)
    if C == 1 or P == 1:
        return float(np.max(np.sum(np.abs(Hn) ** 2, axis=(1, 2))))
    return float(np.max(np.linalg.svd(Hn, compute_uv=False)[:, 0] ** 2))
