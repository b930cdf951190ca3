"""Learned initialiser of the auto-tune: a CNN trained on forward-model patches.

The network (BF16 MFMA kernels behind ``wo_cnn_*``) regresses the normalised
parameters (defocus, NA_det, illumination zenith tilt) of a thin-model defocus
stack.  Training patches are simulated by the library itself: random thin
cells (``wo_synth_thin_cells``), per-patch transfer functions and the forward
model (``wo_transfer_function``, ``wo_forward``) and Gaussian noise
(``wo_add_gaussian_noise``).  Its predictions start ``wo_autotune``; plain
multistart remains the fallback and the reference for its error.
"""

from __future__ import annotations

import math

import numpy as np

from . import api

# Prior of the auto-tune parameters: defocus (um), NA_det, zenith tilt (rad).
PRIOR_LO = np.array([-2.0, 1.0, 0.0])
PRIOR_HI = np.array([2.0, 1.3, math.radians(30.0)])


def normalise_theta(theta3):
    return 2.0 * (np.asarray(theta3) - PRIOR_LO) / (PRIOR_HI - PRIOR_LO) - 1.0


def denormalise_theta(y):
    return PRIOR_LO + 0.5 * (np.asarray(y) + 1.0) * (PRIOR_HI - PRIOR_LO)


def init_params(seed: int) -> np.ndarray:
    """He-normal convolution weights, zero biases, head scaled by 1/sqrt(fan_in)."""
    rng = np.random.default_rng(seed)
    chans = (1, 32, 64, 128, 256)
    out = []
    for ci, co in zip(chans[:-1], chans[1:]):
        out.append(rng.standard_normal(co * 27 * ci) * math.sqrt(2.0 / (27 * ci)))
        out.append(np.zeros(co))
    out.append(rng.standard_normal(3 * 256) * math.sqrt(1.0 / 256))
    out.append(np.zeros(3))
    p = np.concatenate(out).astype(np.float32)
    assert p.size == api.cnn_param_count()
    return p


def simulate(template, n, seed, device, noise_sigma=0.03, chunk=1024, ncells=8, stream=None):
    """n defocus stacks (n, Z, Y, X) of random thin cells with parameters drawn
    from the prior; returns (stacks, theta (n, 3))."""
    import copy

    import torch
    rng = np.random.default_rng(seed)
    theta = np.stack([rng.uniform(PRIOR_LO[j], PRIOR_HI[j], n) for j in range(3)], 1)
    Z, Y, X = template.nz, template.ny, template.nx
    stacks = torch.empty((n, Z, Y, X), dtype=torch.float32, device=device)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        opts = []
        for i in range(c0, c1):
            o = copy.copy(template)
            o.defocus, o.na_det, o.tilt_zenith, o.tilt_azimuth = (float(theta[i, 0]), float(theta[i, 1]),
                                                                   float(theta[i, 2]), 0.0)
            opts.append(o)
        cells = api.synth_thin_cells(c1 - c0, Y, X, template.dx, ncells, seed * 1000003 + c0, device, stream)
        tf = api.transfer_function(opts, device=device, stream=stream)
        stacks[c0:c1] = api.forward(opts, tf, cells, stream=stream)
        del tf, cells
    api.add_gaussian_noise(stacks, noise_sigma, seed * 7919 + 13, stream)
    return stacks, theta


def clear_outer_planes(stacks, seed, keeps=(16, 24, 32)):
    """In place: each stack keeps only its central k planes, k drawn uniformly from
    `keeps`, so that the network also learns from the zero-padded inputs of tiles
    with fewer planes (see ``network_input``)."""
    rng = np.random.default_rng(seed)
    keep = rng.choice(np.asarray(keeps), stacks.shape[0]).astype(np.int32)
    api.crop_stacks(stacks, tuple(stacks.shape[1:]), keep_z=keep, out=stacks)
    return keep


def network_input(tiles, shape=(32, 64, 64), out=None):
    """The centred (Z, Y, X) = `shape` window of each tile (a list of (Z_i, Y_i, X_i)
    device stacks of any size): central planes of deeper tiles, symmetric zero
    padding of shallower ones.  Returns (n, *shape)."""
    import torch
    oz, oy, ox = shape
    n = len(tiles)
    if out is None:
        out = torch.empty((n, oz, oy, ox), dtype=torch.float32, device=tiles[0].device)
    for i, t in enumerate(tiles):
        Z, Y, X = t.shape
        # centre plane of the window (oz - 1) / 2 on the tile's centre (Z - 1) / 2
        api.crop_stacks(t.reshape(1, Z, Y, X), shape, ((Z - oz) // 2, (Y - oy) // 2, (X - ox) // 2),
                        out=out[i:i + 1])
    return out


class LearnedInit:
    """FP32 master parameters and AdamW moments on the device."""

    def __init__(self, device, seed=0):
        import torch
        self.device = device
        self.params = torch.from_numpy(init_params(seed)).to(device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0

    def train(self, stacks, theta, epochs=20, batch=64, lr=1e-3, weight_decay=1e-4, seed=0,
              log_every=0, stream=None):
        """AdamW with a cosine learning-rate schedule; returns the mean loss of each epoch."""
        import torch
        n = stacks.shape[0] // batch * batch
        target = torch.from_numpy(normalise_theta(theta).astype(np.float32)).to(self.device)
        ws = api.cnn_workspace(batch, stacks.shape[1:], self.device)
        y = torch.empty((batch, 3), dtype=torch.float32, device=self.device)
        losses = torch.zeros(n // batch, dtype=torch.float32, device=self.device)
        total = epochs * (n // batch)
        rng = np.random.default_rng(seed)
        hist = []
        step = 0
        for ep in range(epochs):
            order = rng.permutation(n // batch)
            for j, b in enumerate(order):
                lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * step / total))
                self.t += 1
                step += 1
                xb = stacks[b * batch:(b + 1) * batch]
                tb = target[b * batch:(b + 1) * batch]
                api.cnn_train_step(self.params, self.m, self.v, self.t, lr_t, weight_decay, xb, tb, ws, y,
                                   losses[j:j + 1], stream)
            hist.append(float(losses.mean()))
            if log_every and (ep + 1) % log_every == 0:
                print(f"[learned_init] epoch {ep + 1}/{epochs} loss {hist[-1]:.4f}", flush=True)
        return hist

    def predict(self, stacks, batch=256, stream=None):
        """Parameters (n, 3) in physical units for stacks (n, Z, Y, X)."""
        import torch
        out = []
        ws = api.cnn_workspace(min(batch, stacks.shape[0]), stacks.shape[1:], self.device)
        for c0 in range(0, stacks.shape[0], batch):
            xb = stacks[c0:c0 + batch]
            if xb.shape[0] != min(batch, stacks.shape[0]):
                ws = api.cnn_workspace(xb.shape[0], stacks.shape[1:], self.device)
            out.append(api.cnn_forward(self.params, xb, ws=ws, stream=stream).cpu().numpy())
        return denormalise_theta(np.concatenate(out).astype(np.float64))
