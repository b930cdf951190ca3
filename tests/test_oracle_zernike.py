"""Pins of the oracle's detection aberrations (Zernike polynomials on the
detection pupil), independent of the oracle's own formulas:

* Noll's index ordering (n, m) for j = 1..15, his published table;
* unit-RMS orthonormality over the unit disc by Gauss-Legendre x uniform
  quadrature (catches a wrong normalisation, radial polynomial or cos/sin
  assignment);
* textbook closed forms of Z_5..Z_11 at random points (a second formulation
  of the general radial sum);
* zero coefficients give the unaberrated bank; the aberration changes it;
* symmetry: astigmatism cos(2 phi) rotated by 90 degrees is its own negative,
  so on a square grid with an untilted source the bank of +a rotated by 90
  degrees equals the bank of -a; primary spherical aberration keeps the
  x <-> y transpose symmetry;
* the in-focus fluorescence PSF peak falls by |sum_p P e^{i 2 pi W}|^2 /
  |sum_p P|^2 (a direct sum over the pupil), which is close to the Marechal
  value exp(-(2 pi sigma)^2) for sigma^2 = sum c_j^2 waves^2 (unit-RMS terms).
"""

import math

import numpy as np
import pytest

from oracle import optics as op
from oracle import tf as tfm


def test_noll_ordering_matches_the_published_table():
    table = [(0, 0), (1, 1), (1, 1), (2, 0), (2, 2), (2, 2), (3, 1), (3, 1), (3, 3), (3, 3),
             (4, 0), (4, 2), (4, 2), (4, 4), (4, 4)]
    assert [op.noll_nm(j) for j in range(1, 16)] == table


def test_zernike_orthonormal_over_the_unit_disc():
    x, w = np.polynomial.legendre.leggauss(40)
    rho = 0.5 * (x + 1.0)
    wr = 0.5 * w * rho                          # d rho with the Jacobian rho
    phi = np.linspace(0.0, 2.0 * np.pi, 64, endpoint=False)
    R, F = np.meshgrid(rho, phi, indexing="ij")
    Wt = np.outer(wr, np.full(phi.size, 2.0 * np.pi / phi.size))
    js = list(range(1, 12))
    Z = {j: op.zernike_noll(j, R, F) for j in js}
    for a in js:
        for b in js:
            g = np.sum(Wt * Z[a] * Z[b]) / np.pi
            assert abs(g - (1.0 if a == b else 0.0)) < 1e-10, (a, b, g)


def test_zernike_closed_forms():
    rng = np.random.default_rng(3)
    r = rng.uniform(0, 1.2, 50)
    p = rng.uniform(-np.pi, np.pi, 50)
    forms = {
        5: math.sqrt(6) * r ** 2 * np.sin(2 * p),
        6: math.sqrt(6) * r ** 2 * np.cos(2 * p),
        7: math.sqrt(8) * (3 * r ** 3 - 2 * r) * np.sin(p),
        8: math.sqrt(8) * (3 * r ** 3 - 2 * r) * np.cos(p),
        9: math.sqrt(8) * r ** 3 * np.sin(3 * p),
        10: math.sqrt(8) * r ** 3 * np.cos(3 * p),
        11: math.sqrt(5) * (6 * r ** 4 - 6 * r ** 2 + 1),
    }
    for j, ref in forms.items():
        assert np.allclose(op.zernike_noll(j, r, p), ref, rtol=0, atol=1e-12), j


def square(model=op.LABELFREE_3D, **kw):
    o = op.Optics(model=model, nz=8, ny=48, nx=48, dz=0.25, dy=0.1, dx=0.1, wavelength=0.532,
                  na_ill=0.5, na_det=1.1, n_medium=1.33)
    return o.replace(**kw)


def test_zero_coefficients_leave_the_bank_unchanged():
    o = square()
    a = tfm.transfer_function(o)
    b = tfm.transfer_function(o.replace(zernike=(0.0,) * 7))
    c = tfm.transfer_function(o.replace(zernike=(0.1,)))
    assert np.array_equal(a, b)
    assert np.linalg.norm(c - a) > 1e-3 * np.linalg.norm(a)


def rot90(h):
    """H(fy, fx) -> H(fx, -fy) on an FFT-ordered square grid (exact index map)."""
    n = h.shape[-1]
    idx = (-np.arange(n)) % n
    return np.swapaxes(h, -1, -2)[..., idx, :]


@pytest.mark.parametrize("model", [op.LABELFREE_3D, op.FLUOR_3D])
def test_astigmatism_rotated_by_90_degrees_changes_sign(model):
    z6 = (0.0, 0.2)                                     # Noll 6: cos(2 phi)
    hp = tfm.transfer_function(square(model, zernike=z6))
    hm = tfm.transfer_function(square(model, zernike=(0.0, -0.2)))
    assert np.linalg.norm(hp - hm) > 1e-3 * np.linalg.norm(hp)
    err = np.linalg.norm(rot90(hp) - hm) / np.linalg.norm(hm)
    assert err < 1e-12, err


def test_spherical_aberration_keeps_the_transpose_symmetry():
    h = tfm.transfer_function(square(zernike=(0, 0, 0, 0, 0, 0, 0.15)))
    h0 = tfm.transfer_function(square())
    assert np.linalg.norm(h - h0) > 1e-3 * np.linalg.norm(h0)
    assert np.linalg.norm(np.swapaxes(h, -1, -2) - h) < 1e-12 * np.linalg.norm(h)


def test_strehl_ratio_of_the_fluorescence_psf():
    c = (0.03, -0.02, 0.025, 0.0, 0.015, 0.0, 0.02)
    o = op.Optics(model=op.FLUOR_3D, nz=16, ny=96, nx=96, dz=0.25, dy=0.05, dx=0.05,
                  wavelength=0.52, na_ill=0.0, na_det=1.2, n_medium=1.33, defocus=0.0)
    z0 = 0                                              # plane z = 0 (FFT order; defocus 0)
    assert abs(op.z_planes_3d(o)[z0]) < 1e-12
    psf0 = np.fft.ifftn(tfm.transfer_function(o)[0, 0]).real
    psfa = np.fft.ifftn(tfm.transfer_function(o.replace(zernike=c))[0, 0]).real
    P = op.detection_pupil(o)
    W = np.zeros_like(P)
    fy, fx = op.lateral_frequencies(o)
    rho = np.hypot(fy, fx) / (o.na_det / o.wavelength)
    ph = np.arctan2(fy, fx)
    for k, ck in enumerate(c):
        W += ck * op.zernike_noll(5 + k, rho, ph)
    strehl = abs(np.sum(P * np.exp(2j * np.pi * W))) ** 2 / np.sum(P) ** 2
    assert abs(psfa[z0, 0, 0] / psf0[z0, 0, 0] - strehl) < 1e-10
    marechal = math.exp(-(2 * math.pi) ** 2 * sum(x * x for x in c))
    assert abs(strehl - marechal) < 0.01, (strehl, marechal)
