"""FFT schedule tuner: every schedule the tuner may pick computes the same call.

For each FFT pass of a label-free 3D reconstruction (rows along X = 80, a
length without compiled stages, so three radix orders compete; columns along
Y = 96 and the fused Z = 24 pass, both with compiled stages), every candidate
schedule is imported on its own and the reconstruction and the forward model
are compared with the FP64 oracle at the parity tolerances (1e-4, 1e-5).  The
tuner's own pick is then checked end to end, and a tuned transfer-function
synthesis against the oracle bank.
"""

import numpy as np
import pytest

import synth
from oracle import linear
from oracle import optics as op
from oracle import tf as tfm

pytestmark = pytest.mark.gpu


def labelfree(**kw):
    return op.Optics(model=op.LABELFREE_3D, nz=24, ny=96, nx=80, dz=0.2, dy=0.1, dx=0.1,
                     wavelength=0.532, na_ill=0.5, na_det=1.2, n_medium=1.33).replace(**kw)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def case(gpu_lib):
    import torch
    o = labelfree()
    bank = tfm.transfer_function(o)
    f = synth.ellipsoids((o.nz, o.ny, o.nx), (o.dz, o.dy, o.dx), 12, seed=91)
    d = linear.forward(bank, f) + synth.gaussian_noise((1, o.nz, o.ny, o.nx), 1e-3, 92)
    eta = 1e-3 * linear.max_singular_value_sq(bank)
    ref_rec = linear.reconstruct(bank, d, eta=eta)
    ref_fwd = linear.forward(bank, f)
    tf = gpu_lib.transfer_function([o])
    dd = torch.from_numpy(d[None].astype(np.float32)).cuda()
    ff = torch.from_numpy(f[None].astype(np.float32)).cuda()
    gpu_lib.fft_plans_clear()
    out = torch.empty((1, 2, o.nz, o.ny, o.nx), device="cuda")
    gpu_lib.fft_tune(gpu_lib.OP_RECONSTRUCT, [o], tf=tf, x=dd, out=out, eta=eta)
    keys_rec = [" ".join(ln.split()[:5]) for ln in gpu_lib.fft_plans_export().splitlines()]
    gpu_lib.fft_plans_clear()
    out = torch.empty((1, 1, o.nz, o.ny, o.nx), device="cuda")
    gpu_lib.fft_tune(gpu_lib.OP_FORWARD, [o], tf=tf, x=ff, out=out)
    keys_fwd = [" ".join(ln.split()[:5]) for ln in gpu_lib.fft_plans_export().splitlines()]
    gpu_lib.fft_plans_clear()
    yield dict(o=o, tf=tf, dd=dd, ff=ff, eta=eta, ref_rec=ref_rec, ref_fwd=ref_fwd, keys_rec=keys_rec,
               keys_fwd=keys_fwd, bank=bank)
    gpu_lib.fft_plans_clear()


def test_tuner_records_every_pass(gpu_lib, case):
    kinds = sorted(k.split()[0] for k in case["keys_rec"])
    print(f"  reconstruct passes: {case['keys_rec']}")
    assert kinds == ["cols", "cols", "rows_c2r", "rows_r2c", "zop"]


@pytest.mark.parametrize("which", ["rec", "fwd"])
def test_every_candidate_schedule_matches_oracle(gpu_lib, case, which):
    o = case["o"]
    keys = case["keys_rec"] if which == "rec" else case["keys_fwd"]
    tol = 1e-4 if which == "rec" else 1e-5
    total, worst = 0, 0.0
    for key in keys:
        cands = gpu_lib.fft_candidates(key)
        assert len(cands) >= 2
        print(f"[case] {which} {key}: {len(cands)} schedules", flush=True)
        for line in cands:
            gpu_lib.fft_plans_clear()
            gpu_lib.fft_plans_import(line)
            if which == "rec":
                got = gpu_lib.reconstruct([o], case["tf"], case["dd"], case["eta"])[0].cpu().numpy()
                e = rel(got, case["ref_rec"])
            else:
                got = gpu_lib.forward([o], case["tf"], case["ff"])[0].cpu().numpy()
                e = rel(got, case["ref_fwd"])
            worst = max(worst, e)
            total += 1
            assert e < tol, (line, e)
    gpu_lib.fft_plans_clear()
    print(f"  {total} schedules, worst rel {worst:.2e}")


def test_tuned_calls_match_oracle(gpu_lib, case):
    import torch
    o = case["o"]
    gpu_lib.fft_plans_clear()
    out = torch.empty((1, 2, o.nz, o.ny, o.nx), device="cuda")
    gpu_lib.fft_tune(gpu_lib.OP_RECONSTRUCT, [o], tf=case["tf"], x=case["dd"], out=out, eta=case["eta"])
    tfo = torch.empty_like(case["tf"])
    gpu_lib.fft_tune(gpu_lib.OP_TRANSFER_FUNCTION, [o], out=tfo)
    table = gpu_lib.fft_plans_export()
    print(table)
    got = gpu_lib.reconstruct([o], case["tf"], case["dd"], case["eta"])[0].cpu().numpy()
    assert rel(got, case["ref_rec"]) < 1e-4
    tf2 = gpu_lib.transfer_function([o]).cpu().numpy()[0]
    ref = case["bank"][0][..., : o.nx // 2 + 1]
    assert np.linalg.norm(tf2 - ref) / np.linalg.norm(ref) < 1e-5
    # the exported table imports back unchanged
    gpu_lib.fft_plans_clear()
    gpu_lib.fft_plans_import(table)
    assert gpu_lib.fft_plans_export() == table
    gpu_lib.fft_plans_clear()


def test_every_field_kernel_chunk_gives_the_oracle_bank(gpu_lib, case):
    """The TF synthesis records the field kernel's pass (planes per workgroup,
    kind tf_fields); every candidate chunk gives the oracle's bank."""
    import torch
    o = case["o"]
    gpu_lib.fft_plans_clear()
    tfo = torch.empty_like(case["tf"])
    gpu_lib.fft_tune(gpu_lib.OP_TRANSFER_FUNCTION, [o], out=tfo)
    keys = [" ".join(ln.split()[:5]) for ln in gpu_lib.fft_plans_export().splitlines()]
    fkeys = [k for k in keys if k.split()[0] == "tf_fields"]
    assert len(fkeys) == 1, keys
    ref = case["bank"][0][..., : o.nx // 2 + 1]
    cands = gpu_lib.fft_candidates(fkeys[0])
    print(f"[case] tf_fields {fkeys[0]}: {len(cands)} chunks", flush=True)
    assert len(cands) >= 5
    for line in cands:
        gpu_lib.fft_plans_clear()
        gpu_lib.fft_plans_import(line)
        got = gpu_lib.transfer_function([o]).cpu().numpy()[0]
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5, line
    gpu_lib.fft_plans_clear()


def test_column_tile_loop_over_several_tiles_per_workgroup(gpu_lib):
    """Schedule plan 4 of the column passes: a resident grid of workgroups that
    each transform several tiles in turn (the loads of the next tile in flight
    during the passes of the current one).  At 32×512×576 the 512-point Y
    passes cover more 16-column tiles than the device holds workgroups of 1024
    threads at once; reconstruction and forward model against the oracle."""
    import torch
    o = labelfree(nz=32, ny=512, nx=576)
    bank = tfm.transfer_function(o)
    f = synth.ellipsoids((o.nz, o.ny, o.nx), (o.dz, o.dy, o.dx), 24, seed=93)
    d = linear.forward(bank, f) + synth.gaussian_noise((1, o.nz, o.ny, o.nx), 1e-3, 94)
    eta = 1e-3 * linear.max_singular_value_sq(bank)
    tf = gpu_lib.transfer_function([o])
    dd = torch.from_numpy(d[None].astype(np.float32)).cuda()
    ff = torch.from_numpy(f[None].astype(np.float32)).cuda()
    lines = []
    for op_, x, shape in ((gpu_lib.OP_RECONSTRUCT, dd, (1, 2)), (gpu_lib.OP_FORWARD, ff, (1, 1))):
        gpu_lib.fft_plans_clear()
        out = torch.empty(shape + (o.nz, o.ny, o.nx), device="cuda")
        gpu_lib.fft_tune(op_, [o], tf=tf, x=x, out=out, eta=eta)
        for ln in gpu_lib.fft_plans_export().splitlines():
            key = " ".join(ln.split()[:5])
            if key.startswith("cols 512 "):
                loop = [c for c in gpu_lib.fft_candidates(key) if c.split()[-1] == "4"]
                assert loop, key
                lines.append(loop[0])
    gpu_lib.fft_plans_clear()
    assert len(lines) >= 2
    print(f"[case] tile-loop schedules: {lines}", flush=True)
    gpu_lib.fft_plans_import("\n".join(lines))
    try:
        got = gpu_lib.reconstruct([o], tf, dd, eta)[0].cpu().numpy()
        e_rec = rel(got, linear.reconstruct(bank, d, eta=eta))
        got = gpu_lib.forward([o], tf, ff)[0].cpu().numpy()
        e_fwd = rel(got, linear.forward(bank, f))
    finally:
        gpu_lib.fft_plans_clear()
    print(f"  rel reconstruct {e_rec:.2e} forward {e_fwd:.2e}")
    assert e_rec < 1e-4 and e_fwd < 1e-5
