"""Pins of the CNN oracle (CPU only): explicit loops, adjoint identities and
finite differences on tiny shapes."""

import math

import numpy as np
import pytest

from oracle import cnn


def conv_loops(x, w, b):
    """Strided 3x3x3 convolution written out as nested loops."""
    N, D, H, W, Ci = x.shape
    Co = w.shape[0]
    Do, Ho, Wo = cnn.out_size(D), cnn.out_size(H), cnn.out_size(W)
    z = np.zeros((N, Do, Ho, Wo, Co))
    for n in range(N):
        for od in range(Do):
            for oh in range(Ho):
                for ow in range(Wo):
                    for co in range(Co):
                        acc = b[co]
                        for kd in range(3):
                            for kh in range(3):
                                for kw in range(3):
                                    i, j, k = 2 * od + kd - 1, 2 * oh + kh - 1, 2 * ow + kw - 1
                                    if 0 <= i < D and 0 <= j < H and 0 <= k < W:
                                        acc += np.dot(w[co, kd, kh, kw], x[n, i, j, k])
                        z[n, od, oh, ow, co] = acc
    return z


@pytest.mark.parametrize("shape", [(2, 5, 4, 6, 3), (1, 4, 7, 3, 2)])
def test_conv_matches_loops(shape):
    rng = np.random.default_rng(0)
    x = rng.standard_normal(shape)
    w = rng.standard_normal((2, 3, 3, 3, shape[-1]))
    b = rng.standard_normal(2)
    assert np.allclose(cnn.conv3d(x, w, b), conv_loops(x, w, b), atol=1e-12)


def test_dgrad_and_wgrad_are_adjoints():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 6, 5, 4, 3))
    w = rng.standard_normal((4, 3, 3, 3, 3))
    gz = rng.standard_normal(cnn.conv3d(x, w).shape)
    lhs = np.vdot(cnn.conv3d(x, w), gz)
    assert abs(lhs - np.vdot(x, cnn.conv3d_dgrad(gz, w, x.shape))) < 1e-10 * abs(lhs)
    gw, gb = cnn.conv3d_wgrad(x, gz)
    assert abs(lhs - np.vdot(w, gw)) < 1e-10 * abs(lhs)
    assert np.allclose(gb, gz.sum(axis=(0, 1, 2, 3)))


def test_gelu_values_and_derivative():
    assert cnn.gelu(np.array(0.0)) == 0.0
    assert abs(cnn.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (cnn.gelu(z + h) - cnn.gelu(z - h)) / (2 * h)
    assert np.allclose(cnn.gelu_grad(z), fd, atol=1e-9)


def test_network_gradient_matches_finite_differences():
    ch = (1, 4, 8, 8, 8)
    p = cnn.init_params(3, ch)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 8, 16, 16, 1))
    t = rng.standard_normal((2, 3))
    L, g = cnn.loss_and_grad(p, x, t, ch)
    idx = rng.choice(p.size, 24, replace=False)
    for i in idx:
        h = 1e-5
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (cnn.loss_and_grad(pp, x, t, ch)[0] - cnn.loss_and_grad(pm, x, t, ch)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    assert cnn.param_count() == 1163331


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.1415926])
    out = cnn.bf16(v)
    assert out[0] == 1.0
    assert out[1] == 1.0                      # tie rounds to even
    assert out[2] == 1.0 + 2 ** -7
    assert out[3] == -2.5
    assert abs(out[4] - 3.140625) < 1e-12


def test_adamw_first_step():
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -3.0])
    q, _, _ = cnn.adamw_step(p, g, np.zeros(2), np.zeros(2), 1, lr=1e-2, wd=0.1)
    assert np.allclose(q, p - 1e-2 * (np.sign(g) + 0.1 * p), atol=1e-9)
