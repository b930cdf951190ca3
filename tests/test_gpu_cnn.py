"""BF16-MFMA CNN kernels vs the FP64 oracle (learned initialiser of the auto-tune).

Single convolutions get identical BF16 operands on both sides, so the only
difference is FP32 vs FP64 accumulation: relative L2 <= 1e-5.  The whole
network (forward + backward) is compared with the oracle emulating the same
BF16 roundings: loss relative error <= 1e-3, gradient relative L2 <= 1e-2.
"""

import numpy as np
import pytest

from oracle import cnn

pytestmark = pytest.mark.gpu


def to_bits(a):
    """float64 array already on the BF16 grid -> int16 bit patterns."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32) >> 16
    return u.astype(np.uint16).view(np.int16)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


# 64 x 64 and 128 x 32 (N <= 32) tiles, scalar and vector operand loads, ragged edges
SHAPES = [(2, 8, 12, 10, 8, 40), (1, 9, 7, 6, 1, 32), (2, 16, 32, 32, 32, 64), (1, 6, 10, 14, 24, 16)]


@pytest.mark.parametrize("N,D,H,W,Ci,Co", SHAPES)
def test_conv_kernels_match_oracle(gpu_lib, N, D, H, W, Ci, Co):
    import torch
    print(f"[case] conv N={N} D={D} H={H} W={W} Cin={Ci} Cout={Co}", flush=True)
    rng = np.random.default_rng(N * 1000 + Ci)
    x = cnn.bf16(rng.standard_normal((N, D, H, W, Ci)))
    w = cnn.bf16(rng.standard_normal((Co, 3, 3, 3, Ci)) / np.sqrt(27 * Ci))
    xb = torch.from_numpy(to_bits(x)).cuda()
    wb = torch.from_numpy(to_bits(w.reshape(Co, -1))).cuda()
    z = gpu_lib.conv3d_forward(xb, wb, Co).cpu().numpy()
    ref = cnn.conv3d(x, w)
    e = rel(z, ref)
    print(f"  forward rel {e:.2e}")
    assert e < 1e-5
    gz = cnn.bf16(rng.standard_normal(ref.shape))
    gzb = torch.from_numpy(to_bits(gz)).cuda()
    gx = gpu_lib.conv3d_input_grad(gzb, wb, x.shape).cpu().numpy()
    e = rel(gx, cnn.conv3d_dgrad(gz, w, x.shape))
    print(f"  input grad rel {e:.2e}")
    assert e < 1e-5
    gw = gpu_lib.conv3d_weight_grad(xb, gzb).cpu().numpy()
    gw_ref, _ = cnn.conv3d_wgrad(x, gz)
    e = rel(gw, gw_ref.reshape(Co, -1))
    print(f"  weight grad rel {e:.2e}")
    assert e < 1e-5


def test_network_gradient_matches_oracle(gpu_lib):
    import torch
    from paper_2412_09775_amd import learned_init
    rng = np.random.default_rng(9)
    p = learned_init.init_params(5)
    p[-3:] = [0.1, -0.2, 0.05]                    # non-zero head bias
    stacks = rng.standard_normal((2, 8, 16, 16)).astype(np.float32)
    target = rng.uniform(-1, 1, (2, 3)).astype(np.float32)
    y, loss, g = gpu_lib.cnn_gradient(torch.from_numpy(p).cuda(), torch.from_numpy(stacks).cuda(),
                                      torch.from_numpy(target).cuda())
    x = cnn.normalise_input(stacks)
    L, gref = cnn.loss_and_grad(p.astype(np.float64), x, target.astype(np.float64), round_bf16=True)
    yref, _ = cnn.forward(p.astype(np.float64), x, round_bf16=True)
    print(f"  loss {float(loss):.6f} vs {L:.6f}; y rel {rel(y.cpu().numpy(), yref):.2e}; "
          f"grad rel {rel(g.cpu().numpy(), gref):.2e}")
    assert abs(float(loss) - L) <= 1e-3 * abs(L)
    assert rel(y.cpu().numpy(), yref) < 1e-3
    assert rel(g.cpu().numpy(), gref) < 1e-2
    # per-layer gradient blocks, so no layer hides behind the norm of another
    off = 0
    for kind, shp in cnn.param_shapes():
        n = int(np.prod(shp))
        e = rel(g.cpu().numpy()[off:off + n], gref[off:off + n]) if np.any(gref[off:off + n]) else 0.0
        assert e < 2e-2, (kind, shp, e)
        off += n


def test_adamw_step_matches_oracle(gpu_lib):
    import torch
    from paper_2412_09775_amd import learned_init
    n = gpu_lib.cnn_param_count()
    rng = np.random.default_rng(3)
    p = learned_init.init_params(1)
    stacks = rng.standard_normal((2, 8, 16, 16)).astype(np.float32)
    target = rng.uniform(-1, 1, (2, 3)).astype(np.float32)
    pt = torch.from_numpy(p).cuda()
    m, v = torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    _, _, g = gpu_lib.cnn_gradient(pt.clone(), torch.from_numpy(stacks).cuda(), torch.from_numpy(target).cuda())
    ws = gpu_lib.cnn_workspace(2, (8, 16, 16), "cuda")
    y = torch.empty((2, 3), device="cuda")
    loss = torch.empty(1, device="cuda")
    gpu_lib.cnn_train_step(pt, m, v, 1, 1e-3, 1e-4, torch.from_numpy(stacks).cuda(),
                           torch.from_numpy(target).cuda(), ws, y, loss)
    ref, _, _ = cnn.adamw_step(p.astype(np.float64), g.cpu().numpy().astype(np.float64), np.zeros(n),
                               np.zeros(n), 1, 1e-3, 1e-4)
    assert np.max(np.abs(pt.cpu().numpy() - ref)) < 1e-6


def test_training_data_is_deterministic(gpu_lib):
    a = gpu_lib.synth_thin_cells(3, 64, 64, 0.1, 8, 42).cpu().numpy()
    b = gpu_lib.synth_thin_cells(3, 64, 64, 0.1, 8, 42).cpu().numpy()
    c = gpu_lib.synth_thin_cells(3, 64, 64, 0.1, 8, 43).cpu().numpy()
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert 0.0 <= a[:, 0].min() and a[:, 0].max() < 8 * 0.5 and a[:, 1].max() < 8 * 0.02
    import torch
    x = torch.zeros(1 << 20, device="cuda")
    gpu_lib.add_gaussian_noise(x, 0.5, 7)
    s = x.cpu().numpy()
    assert abs(s.mean()) < 2e-3 and abs(s.std() - 0.5) < 2e-3


def test_training_reduces_the_loss(gpu_lib):
    import torch
    from paper_2412_09775_amd import learned_init
    # 64x64 patches: a quarter-pixel soft edge has the same absolute width as
    # half a pixel on 128x128 tiles and keeps NA 1.3 inside the shell
    tmpl = gpu_lib.Optics(model=2, nz=32, ny=64, nx=64, dz=0.2, dy=0.1, dx=0.1, wavelength=0.532,
                          na_ill=0.5, na_det=1.15, n_medium=1.33, edge_width=0.25)
    stacks, theta = learned_init.simulate(tmpl, 1024, seed=11, device="cuda")
    net = learned_init.LearnedInit("cuda", seed=2)
    hist = net.train(stacks, theta, epochs=4, batch=64, lr=1e-3)
    torch.cuda.synchronize()
    print(f"  epoch losses {hist}")
    assert hist[-1] < 0.7 * hist[0]


@pytest.mark.parametrize("Z", [16, 24, 32, 48])
def test_network_input_window(gpu_lib, Z):
    """Centred 32x64x64 window of a tile: central planes or symmetric zero padding,
    the same planes a 32-plane stack with its outer planes cleared keeps."""
    import torch
    from paper_2412_09775_amd import learned_init
    rng = np.random.default_rng(Z)
    t = rng.standard_normal((Z, 96, 80)).astype(np.float32)
    got = learned_init.network_input([torch.from_numpy(t).cuda()]).cpu().numpy()[0]
    ref = np.zeros((32, 64, 64), np.float32)
    z0 = (Z - 32) // 2
    for z in range(32):
        if 0 <= z + z0 < Z:
            ref[z] = t[z + z0, 16:80, 8:72]
    assert np.array_equal(got, ref)
    full = rng.standard_normal((2, 32, 8, 8)).astype(np.float32)
    x = torch.from_numpy(full).cuda()
    keep = np.array([Z if Z <= 32 else 32, 32], np.int32)
    gpu_lib.crop_stacks(x, (32, 8, 8), keep_z=keep, out=x)
    kept = x.cpu().numpy()
    for i in range(2):
        lo = (32 - keep[i]) // 2
        ref = np.zeros_like(full[i])
        ref[lo:lo + keep[i]] = full[i, lo:lo + keep[i]]
        assert np.array_equal(kept[i], ref)


def test_trained_network_gains_over_the_start_without_it(gpu_lib):
    """What the learned initialiser buys: on held-out patches drawn from the prior,
    (a) its prediction is much closer to the truth than the start the auto-tune has
    without it (the centre of the prior), and (b) after the same 20 Adam iterations
    (defocus and tilt tuned, NA held at the start) the CNN-started tune ends closer
    to the truth than the centre-started one."""
    import torch
    from paper_2412_09775_amd import learned_init
    tmpl = gpu_lib.Optics(model=2, nz=32, ny=64, nx=64, dz=0.2, dy=0.1, dx=0.1, wavelength=0.532,
                          na_ill=0.5, na_det=1.15, n_medium=1.33, edge_width=0.25)
    train_x, train_t = learned_init.simulate(tmpl, 4096, seed=21, device="cuda")
    net = learned_init.LearnedInit("cuda", seed=4)
    net.train(train_x, train_t, epochs=6, batch=64, lr=1e-3)
    del train_x
    test_x, truth = learned_init.simulate(tmpl, 96, seed=22, device="cuda")
    rng_ = learned_init.PRIOR_HI - learned_init.PRIOR_LO
    centre = 0.5 * (learned_init.PRIOR_LO + learned_init.PRIOR_HI)
    pred = net.predict(test_x)
    e_cnn = np.median(np.abs(pred - truth) / rng_, axis=0)
    e_ctr = np.median(np.abs(centre - truth) / rng_, axis=0)
    print(f"  prediction error (defocus, NA, tilt): cnn {e_cnn}, prior centre {e_ctr}")
    assert np.all(e_cnn < 0.5 * e_ctr)
    # the same short auto-tune from both starts
    n = test_x.shape[0]
    opts = [gpu_lib.Optics(**{**tmpl.__dict__}) for _ in range(n)]
    nominal_tf = gpu_lib.transfer_function([tmpl])
    h0, h1 = nominal_tf[:, :, 0], nominal_tf[:, :, 1]
    a, b = (h0.abs() ** 2).sum(1), (h1.abs() ** 2).sum(1)
    m = (h0.conj() * h1).sum(1).abs()
    eta = 1e-2 * float(((a + b) / 2 + (((a - b) / 2) ** 2 + m ** 2).sqrt()).max())
    lr, lo, hi = (0.02, 0.005, 0.005, 0.001), (-2.5, 1.0, 0.0, -1.0), (2.5, 1.3, 0.56, 1.0)
    errs = {}
    for label, start in (("cnn", pred), ("centre", np.tile(centre, (n, 1)))):
        theta0 = np.zeros((n, 1, 4))
        theta0[:, 0, :3] = np.clip(start, lo[:3], hi[:3])
        out, _, _, _ = gpu_lib.autotune(opts, test_x, eta, iters=20, lr=lr, lo=lo, hi=hi, mask=0b0101,
                                        theta0=theta0, nu_c=(tmpl.na_det + tmpl.na_ill) / tmpl.wavelength,
                                        use_graph=True)
        th = np.array([[o.defocus, o.na_det, o.tilt_zenith] for o in out])
        e = np.abs(th - truth) / rng_
        errs[label] = float(np.median(np.maximum(e[:, 0], e[:, 2])))
    print(f"  after 20 iterations, median max(defocus, tilt) error: {errs}")
    assert errs["cnn"] < 0.5 * errs["centre"]


def test_cnn_start_call_equals_the_python_path(gpu_lib):
    """wo_cnn_init_theta (crop of packed uneven patches, network, denormalisation
    in the library) gives exactly what learned_init's network_input + cnn_forward +
    denormalise_theta give, for patches deeper and shallower, wider and narrower
    (odd sizes: floor offsets) than the network input."""
    import torch
    from paper_2412_09775_amd import learned_init
    shapes = [(16, 128, 192), (17, 63, 65), (48, 64, 64), (33, 200, 90), (32, 64, 64), (5, 31, 129)]
    rng = np.random.default_rng(77)
    tiles = [torch.from_numpy(rng.standard_normal(s).astype(np.float32)).cuda() for s in shapes]
    opts = [gpu_lib.Optics(model=2, nz=s[0], ny=s[1], nx=s[2], dz=0.2, dy=0.1, dx=0.1, wavelength=0.532,
                           na_ill=0.5, na_det=1.15, n_medium=1.33, tilt_azimuth=0.1 * i)
            for i, s in enumerate(shapes)]
    net = learned_init.LearnedInit("cuda", seed=3)
    print("[case] cnn start call vs python path", flush=True)
    got = gpu_lib.cnn_init_theta(net.params, opts, tiles)
    x = learned_init.network_input(tiles)
    y = gpu_lib.cnn_forward(net.params, x).cpu().numpy()
    ref = learned_init.denormalise_theta(y.astype(np.float64))
    assert np.array_equal(got[:, :3], ref)
    assert np.array_equal(got[:, 3], [o.tilt_azimuth for o in opts])
