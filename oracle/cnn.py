"""FP64 oracle of the 3D CNN that regresses auto-tune parameters from a stack.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper has no network: its "learning" is the physics graph of Ext. Data
Fig. 3.  This network is the learned initialiser the build adds in front of
the auto-tune: 4 blocks of [3x3x3 convolution, stride 2, padding 1, bias,
GELU] with channels 1 -> 32 -> 64 -> 128 -> 256, global average pooling and a
linear head to 3 normalised parameters (defocus, NA_det, tilt), trained with a
mean-squared error and AdamW.

Layouts are channels-last: activations (N, D, H, W, C); convolution weights
(Cout, 3, 3, 3, Cin).  ``bf16`` emulates round-to-nearest-even BF16 storage so
parity tests can feed both sides identical operands.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

CHANNELS = (1, 32, 64, 128, 256)
N_OUT = 3


def bf16(x) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = (rounded.astype(np.uint32) << 16).view(np.float32)
    return out.astype(np.float64)


def out_size(n: int) -> int:
    """Output length of a 3-tap, stride-2, padding-1 convolution."""
    return (n - 1) // 2 + 1


def conv3d(x, w, b=None):
    """z[n, o] = b + sum_{tap, ci} w[co, tap, ci] x[n, 2o + tap - 1, ci] (zero padding)."""
    N, D, H, W, Ci = x.shape
    Co = w.shape[0]
    Do, Ho, Wo = out_size(D), out_size(H), out_size(W)
    xp = np.zeros((N, D + 2, H + 2, W + 2, Ci))
    xp[:, 1:D + 1, 1:H + 1, 1:W + 1] = x
    z = np.zeros((N, Do, Ho, Wo, Co))
    for kd in range(3):
        for kh in range(3):
            for kw in range(3):
                patch = xp[:, kd:kd + 2 * Do:2, kh:kh + 2 * Ho:2, kw:kw + 2 * Wo:2, :]
                z += np.einsum("ndhwc,oc->ndhwo", patch, w[:, kd, kh, kw, :])
    if b is not None:
        z += b
    return z


def conv3d_dgrad(gz, w, in_shape):
    """Gradient of the loss wrt the convolution input, given dL/dz."""
    N, D, H, W, Ci = in_shape
    Do, Ho, Wo = gz.shape[1:4]
    gxp = np.zeros((N, D + 2, H + 2, W + 2, Ci))
    for kd in range(3):
        for kh in range(3):
            for kw in range(3):
                gxp[:, kd:kd + 2 * Do:2, kh:kh + 2 * Ho:2, kw:kw + 2 * Wo:2, :] += np.einsum(
                    "ndhwo,oc->ndhwc", gz, w[:, kd, kh, kw, :])
    return gxp[:, 1:D + 1, 1:H + 1, 1:W + 1]


def conv3d_wgrad(x, gz):
    """Gradients of the loss wrt the weights and bias, given the input and dL/dz."""
    N, D, H, W, Ci = x.shape
    Do, Ho, Wo, Co = gz.shape[1:]
    xp = np.zeros((N, D + 2, H + 2, W + 2, Ci))
    xp[:, 1:D + 1, 1:H + 1, 1:W + 1] = x
    gw = np.zeros((Co, 3, 3, 3, Ci))
    for kd in range(3):
        for kh in range(3):
            for kw in range(3):
                patch = xp[:, kd:kd + 2 * Do:2, kh:kh + 2 * Ho:2, kw:kw + 2 * Wo:2, :]
                gw[:, kd, kh, kw, :] = np.einsum("ndhwo,ndhwc->oc", gz, patch)
    return gw, gz.sum(axis=(0, 1, 2, 3))


def gelu(z):
    """Exact GELU, z * Phi(z)."""
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def param_shapes(channels=CHANNELS):
    shapes = []
    for ci, co in zip(channels[:-1], channels[1:]):
        shapes += [("w", (co, 3, 3, 3, ci)), ("b", (co,))]
    shapes += [("w", (N_OUT, channels[-1])), ("b", (N_OUT,))]
    return shapes


def unpack(flat, channels=CHANNELS):
    out, off = [], 0
    for _, shp in param_shapes(channels):
        n = int(np.prod(shp))
        out.append(np.asarray(flat[off:off + n], dtype=np.float64).reshape(shp))
        off += n
    return out


def param_count(channels=CHANNELS) -> int:
    return int(sum(np.prod(s) for _, s in param_shapes(channels)))


def normalise_input(stacks):
    """Per-sample scaling x / std(x) of (N, Z, Y, X) stacks -> (N, Z, Y, X, 1)."""
    s = np.asarray(stacks, dtype=np.float64)
    sd = np.sqrt(np.mean(s * s, axis=(1, 2, 3), keepdims=True))
    return (s / np.where(sd > 0, sd, 1.0))[..., None]


def forward(flat, x, channels=CHANNELS, round_bf16=False):
    """Network output (N, 3) and the cache for backward.

    With round_bf16 the activations and weights entering every convolution are
    rounded to BF16, as the MFMA kernels store them.
    """
    P = unpack(flat, channels)
    r = bf16 if round_bf16 else (lambda v: v)
    a = r(x)
    cache = []
    for layer in range(len(channels) - 1):
        w, b = P[2 * layer], P[2 * layer + 1]
        z = conv3d(a, r(w), b)
        cache.append((a, z))
        a = r(gelu(z))
    feat = a.mean(axis=(1, 2, 3))
    wh, bh = P[-2], P[-1]
    y = feat @ wh.T + bh
    return y, (cache, a, feat)


def loss_and_grad(flat, x, target, channels=CHANNELS, round_bf16=False):
    """MSE loss mean((y - t)^2) and its gradient wrt the flat parameters."""
    P = unpack(flat, channels)
    r = bf16 if round_bf16 else (lambda v: v)
    y, (cache, a_last, feat) = forward(flat, x, channels, round_bf16)
    N = x.shape[0]
    diff = y - target
    loss = float(np.mean(diff * diff))
    dy = 2.0 * diff / diff.size
    grads = [None] * len(P)
    grads[-2] = dy.T @ feat
    grads[-1] = dy.sum(axis=0)
    dfeat = dy @ P[-2]
    npos = np.prod(a_last.shape[1:4])
    ga = np.broadcast_to(dfeat[:, None, None, None, :] / npos, a_last.shape)
    for layer in range(len(channels) - 2, -1, -1):
        a_in, z = cache[layer]
        gz = ga * gelu_grad(z)
        if round_bf16:
            gz = bf16(gz)
        gw, gb = conv3d_wgrad(a_in, gz)
        grads[2 * layer], grads[2 * layer + 1] = gw, gb
        if layer > 0:
            ga = conv3d_dgrad(gz, r(P[2 * layer]), a_in.shape)
    return loss, np.concatenate([g.reshape(-1) for g in grads])


def init_params(seed, channels=CHANNELS):
    """He-normal convolution weights, zero biases, small head."""
    rng = np.random.default_rng(seed)
    out = []
    for kind, shp in param_shapes(channels):
        if kind == "b":
            out.append(np.zeros(shp))
        elif len(shp) == 5:
            fan_in = 27 * shp[-1]
            out.append(rng.standard_normal(shp) * math.sqrt(2.0 / fan_in))
        else:
            out.append(rng.standard_normal(shp) * math.sqrt(1.0 / shp[-1]))
    return np.concatenate([o.reshape(-1) for o in out])


def adamw_step(p, g, m, v, t, lr, wd=1e-4, b1=0.9, b2=0.999, eps=1e-8):
    """AdamW (decoupled weight decay, Loshchilov & Hutter) on flat arrays; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    return p, m, v
