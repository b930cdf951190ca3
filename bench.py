"""Throughput of the WaveOrder hot path on one MI355X.

Headline workload: polarisation-resolved label-free reconstruction, 5 channels
(swing 0.1) x 4 properties (phase, rho cos 2w, rho sin 2w, absorption) on a
64 x 1024 x 1024 grid (dz 0.25 um, dx = dy 0.1 um), lambda0 0.532 um, NA_ill
0.5, NA_det 0.75, n 1.33; 300 random spline fibres, Gaussian noise.  One step
is the whole reconstruction hot path on that volume: transfer-function
synthesis (pupils, propagators, correlation, 3D transforms; the 5 x 4 bank in
its reduced form, the label-free pair on its lateral support) followed by the
Tikhonov reconstruction (forward 3D FFT of the 5 channels, per-frequency 5 x 4
solve fused with the Z transform, inverse 3D FFT of the 4 properties).
Inputs are resident in HBM before timing starts.

Secondary workloads with the same measurements: label-free phase and
absorption, 96 x 512 x 512, 1 channel -> 2 properties; widefield fluorescence,
32 x 64 x 64, 1 -> 1.  Every workload's timed output is compared with the FP64
oracle (the whole volume where the oracle can reconstruct it in seconds,
sampled frequencies at 64 x 1024 x 1024).

Prints one JSON line.  `value` = reconstructed voxels per second of the
headline step; extra fields give the rate with a cached transfer function,
each kernel's time and algorithmic bytes, the roofline of the dominant kernel,
the parity check and the FP64 oracle timed on a bounded sample on the host.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
_OPT = dict(defocus=0.0, tilt_zenith=0.0, tilt_azimuth=0.0, edge_width=0.0, swing=0.1)
# polarisation-resolved 5 x 4, the headline workload
POL5 = dict(_OPT, model=3, nz=64, ny=1024, nx=1024, dz=0.25, dy=0.1, dx=0.1, wavelength=0.532,
            na_ill=0.5, na_det=0.75, n_medium=1.33)
# label-free phase and absorption, 1 x 2
LABELFREE = dict(_OPT, model=1, nz=96, ny=512, nx=512, dz=0.2, dy=0.1, dx=0.1, wavelength=0.532,
                 na_ill=0.5, na_det=1.2, n_medium=1.33)
# widefield fluorescence, 1 x 1
FLUOR = dict(_OPT, model=0, nz=32, ny=64, nx=64, dz=0.25, dy=0.1, dx=0.1, wavelength=0.52, na_ill=0.0,
             na_det=1.2, n_medium=1.33)
# vector (non-paraxial) label-free bank of the same 5 x 4 system as the headline:
# the five swing states through the circular analyser, properties phase,
# rho cos 2w, rho sin 2w, absorption (spherical-harmonic codes 0, 16, 8, 1)
VECTOR = dict(POL5, model=5, vec_channels=1, vec_props=(0, 16, 8, 1))
WORKLOAD = LABELFREE          # the 3D label-free sampling the extra sections reuse
ETA_REL = 1e-3
TOL_REC = 1e-4                # reconstruction parity (relative L2) vs the FP64 oracle

SECTIONS = {
    "pol5": dict(optics=POL5, name="pol5_64x1024x1024",
                 workload="polarisation-resolved label-free, 64x1024x1024, 5 channels (swing 0.1) x 4 "
                          "properties, 300 spline fibres + N(0, 1e-3^2) noise; bank in reduced form "
                          "(label-free pair on its lateral support)"),
    "labelfree": dict(optics=LABELFREE, name="labelfree3d_96x512x512",
                      workload="label-free 3D phase+absorption, 96x512x512, 1 channel x 2 properties, "
                               "200 ellipsoids + Poisson-Gaussian noise (bank kept on its lateral "
                               "support)"),
    "fluor": dict(optics=FLUOR, name="fluor3d_32x64x64",
                  workload="widefield fluorescence, 32x64x64, 1 x 1, 50 beads + N(0, 1e-3^2) noise, "
                           "eta 1e-3 (full-layout calls)"),
    "vector": dict(optics=VECTOR, name="vector_64x1024x1024",
                   workload="vector (non-paraxial) label-free bank, 64x1024x1024, the 5 swing states x "
                            "4 spherical-harmonic coefficients (phase, rho cos 2w, rho sin 2w, absorption), "
                            "300 spline fibres + N(0, 1e-3^2) noise; bank in the band layout, default "
                            "schedules"),
}


def kernel_bytes(name, Z, Y, X, sup, C=1, P=2, E=None, F=None):
    """Algorithmic HBM bytes one launch of each kernel must move in the step.

    sup: the lateral support (wo_lateral_support): the fields A and B are kept on
    field_cols columns at ly points along y, the bank and the spectra on the
    columns k < kt of every row (of the band rows once transformed along Y).
    C, P: channels and properties; E: transfer-function values read per
    frequency by the fused Z pass (C * P, or 2 for the reduced 5 x 4 bank); F: the
    vector model's field count (its synthesis works on the full grid)."""
    E = C * P if E is None else E
    fa, fb = sup["field_cols"]
    kt, nb, (ly, _) = sup["tf_cols"], sup["band_rows"], sup["tf_lengths"]
    Xh = X // 2 + 1
    cplx = 8
    full = Z * Y * X
    rows_kt = Z * Y * kt          # compact half spectrum, every row
    band = Z * nb * kt            # compact half spectrum, band rows
    tf_rows = Z * ly * kt         # compact TF before its Y transform (ly rows)
    table = {
        # reconstruction
        "k_rows_r2c": C * (4 * full + cplx * rows_kt),
        "k_cols_y_fwd": C * cplx * (rows_kt + band),
        f"k_zop<{P}>": cplx * band * (C + E + P),
        "k_cols_y_inv": P * cplx * (band + rows_kt),
        "k_rows_c2r": P * (cplx * rows_kt + 4 * full),
        # transfer-function synthesis (the label-free pair)
        "k_tf_fields_y": cplx * Z * ly * (fa + fb),
        "k_tf_rows_lf": cplx * Z * ly * (fa + fb) + 2 * cplx * tf_rows,
        "k_cols_y_tf": 2 * cplx * (tf_rows + band),
        # band rows' Z transform, plus the zeros of the rest of the bank
        "k_cols_expand": 2 * 2 * cplx * band + 2 * cplx * (Z * Y * Xh - band),
        # the same into the band layout (no zeros)
        "k_cols_z_band": 2 * 2 * cplx * band,
    }
    if F is not None:
        # vector synthesis: F field spectra written on the detection pupil's fb
        # columns and transformed along Y there (read + write), then along X into
        # full rows, read by the products, which write C P real responses; their
        # forward transform on the bank's support (kt columns, band rows), whose
        # Z pass writes the full half-spectrum bank
        half_full = Z * Y * Xh
        # the fused path works on the support's shortened transforms ly x lx
        sl = Z * ly * sup["tf_lengths"][1]
        rows_kt_s = Z * ly * kt
        table.update({
            "k_vec_spectra": F * cplx * Z * ly * fb,
            "k_cols_vec": 2 * F * cplx * Z * ly * fb,
            "k_rows_c2c": F * cplx * (Z * Y * fb + full),
            "k_vec_products": F * cplx * full + C * P * 4 * full,
            # fused X pass + responses: per row the F spectra lines of fb kept
            # columns read once, C P response rows of lx written
            "k_vec_rows_resp": Z * ly * (F * cplx * fb + C * P * 4 * sup["tf_lengths"][1]),
            "k_rows_r2c_tf": C * P * (4 * sl + cplx * rows_kt_s),
            "k_cols_y_tf": C * P * cplx * (rows_kt_s + band),
            "k_cols_expand": C * P * cplx * (band + half_full),
            "k_cols_z_band": 2 * C * P * cplx * band,
        })
    return table.get(name)


CSRC = os.path.join(ROOT, "paper_2412_09775_amd", "csrc")


def traffic_file(section):
    return os.path.join(ROOT, "profiles", f"{SECTIONS[section]['name']}_hbm_traffic.txt")


def counter_symbols(sup, Z, X, P, C, ns=None):
    """Kernel name in the library's timing report -> symbol in the counter summary
    (the column passes share one symbol across launches and are not listed); the
    TF kernels are compiled for the synthesis' transform lengths (ly, lx)."""
    ly, lx = sup["tf_lengths"]
    ct = 1 if C == 1 else (5 if C == 5 else 0)
    zop = f"wo::k_zop<{P}, {ct}, {Z}, true>" if C == 5 and P == 4 else f"wo::k_zop<{P}, {ct}, {Z}, false>"
    if ns is not None:   # the vector bank's synthesis (ns illumination states)
        return {"k_vec_products": f"wo::k_vec_products<{ns}>", "k_vec_spectra": f"wo::k_vec_spectra<{ns}>",
                "k_vec_rows_resp": f"wo::k_vec_rows_resp<{ns}, {X}>",
                "k_rows_c2c": f"wo::k_rows_c2c<{X}>", f"k_zop<{P}>": f"wo::k_zop<{P}, {ct}, {Z}, false>",
                "k_rows_r2c": f"wo::k_rows_r2c<{X}>", "k_rows_c2r": f"wo::k_rows_c2r<{X}>"}
    return {f"k_zop<{P}>": zop, "k_rows_r2c": f"wo::k_rows_r2c<{X}>",
            "k_rows_c2r": f"wo::k_rows_c2r<{X}>", "k_tf_rows_lf": f"wo::k_tf_rows_lf<{lx}>",
            "k_tf_fields_y": f"wo::k_tf_fields_y<{ly}, 2, false>",
            "k_cols_z_band": f"wo::k_cols_expand<{Z}, {min(16, 8192 // Z)}>"}


def source_sha1():
    """SHA-1 over every kernel source of the library (any change invalidates counters)."""
    import hashlib
    h = hashlib.sha1()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def measured_traffic(section, kernel, symbols):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE summary, or None
    when the kernel sources changed since the counters were taken."""
    try:
        lines = open(traffic_file(section)).read().splitlines()
    except OSError:
        return None
    rec = [ln.split()[1] for ln in lines if ln.startswith("source_sha1")]
    if not rec or rec[0] != source_sha1() or kernel not in symbols:
        return None
    want = symbols[kernel]
    best = None
    for ln in lines:
        f = ln.split("\t")
        if len(f) >= 5 and f[0] == want:
            mb = float(f[-1])
            best = mb if best is None else max(best, mb)   # the largest dispatch is the workload's
    return None if best is None else int(best * 1e6)


def _symbol(name):
    name = name[5:] if name.startswith("void ") else name
    return name.split("(")[0]


def summarise_trace(trace_dir, command, title):
    """Per (kernel, grid) call count and average duration from a rocprofv3
    --kernel-trace CSV directory, as the text committed under profiles/."""
    import csv
    import glob
    path = glob.glob(os.path.join(trace_dir, "*kernel_trace.csv"))[0]
    agg = {}
    for r in csv.DictReader(open(path)):
        k = (_symbol(r["Kernel_Name"]), int(r["Grid_Size_X"]))
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
        c, t = agg.get(k, (0, 0.0))
        agg[k] = (c + 1, t + d)
    out = [f"# Kernel durations: {title}",
           f"# command: {command}",
           f"source_sha1 {source_sha1()}",
           "kernel\tgrid\tcalls\tavg_us\ttotal_us"]
    for (k, g), (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        if k.startswith("wo::"):     # the library's kernels (not the input generation's)
            out.append(f"{k}\t{g}\t{c}\t{t / c:.1f}\t{t:.1f}")
    return "\n".join(out) + "\n"


def summarise_counters(fetch_dir, write_dir, commands, title):
    """Per-dispatch FETCH_SIZE and WRITE_SIZE (KiB) of every kernel, scaled by what the
    counters read for the 1 GiB device copy in the same run, in MB per dispatch."""
    import csv
    import glob

    def load(d, counter):
        path = glob.glob(os.path.join(d, "*counter_collection.csv"))[0]
        rows = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                rows[int(r["Dispatch_Id"])] = (_symbol(r["Kernel_Name"]), int(r["Grid_Size"]),
                                               float(r["Counter_Value"]))
        return rows

    fe, wr = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    gib = 1 << 30
    copies_f = [v for v in fe.values() if "copyBuffer" in v[0] and v[2] > 0.25 * gib / 1024]
    copies_w = [v for v in wr.values() if "copyBuffer" in v[0] and v[2] > 0.25 * gib / 1024]
    cf = max(v[2] for v in copies_f) if copies_f else 0.0
    cw = max(v[2] for v in copies_w) if copies_w else 0.0
    sf = (gib / 1024) / cf if cf else 1.0
    sw = (gib / 1024) / cw if cw else 1.0
    # dispatch ids differ between the two runs: pair the n-th dispatch of each (kernel, grid)
    from collections import defaultdict
    seq_f, seq_w = defaultdict(list), defaultdict(list)
    for i in sorted(fe):
        seq_f[fe[i][:2]].append(fe[i][2])
    for i in sorted(wr):
        seq_w[wr[i][:2]].append(wr[i][2])
    out = [f"# HBM traffic per dispatch: {title} (same workload as the kernel durations)"]
    out += [f"# command: {c}" for c in commands]
    out += [f"# calibration: 1 GiB device copy reads FETCH_SIZE={cf:.1f} KiB, "
            f"WRITE_SIZE={cw:.1f} KiB",
            f"# scale factors: fetch x{sf:.3f}, write x{sw:.3f}",
            f"source_sha1 {source_sha1()}",
            "kernel\tgrid\tFETCH_KiB\tWRITE_KiB\tscaled_MB"]
    for key in sorted(set(seq_f) & set(seq_w)):
        if not key[0].startswith("wo::"):     # the library's kernels (not the input generation's)
            continue
        f = sum(seq_f[key]) / len(seq_f[key])
        w = sum(seq_w[key]) / len(seq_w[key])
        mb = (f * sf + w * sw) * 1024 / 1e6
        out.append(f"{key[0]}\t{key[1]}\t{f:.1f}\t{w:.1f}\t{mb:.1f}")
    return "\n".join(out) + "\n"


def summarise_sq(dirs, commands, title):
    """Per-dispatch averages of the SQ counters of one or more rocprofv3 --pmc CSV
    directories for the library's kernels, with the ratios read from them:
    VALU and LDS instructions per wave, the fraction of wave-cycles issuing VALU
    work (SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES), the fraction waiting on any
    instruction (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES) and LDS bank-conflict cycles
    per LDS instruction."""
    import csv
    import glob
    from collections import defaultdict
    vals = defaultdict(lambda: defaultdict(list))
    for d in dirs:
        for path in glob.glob(os.path.join(d, "*counter_collection.csv")):
            for r in csv.DictReader(open(path)):
                k = (_symbol(r["Kernel_Name"]), int(r["Grid_Size"]))
                vals[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for v in vals.values() for c in v})
    out = [f"# SQ counters per dispatch: {title}"]
    out += [f"# command: {c}" for c in commands]
    out += ["# ratios: valu/wave = SQ_INSTS_VALU / SQ_WAVES; lds/wave = SQ_INSTS_LDS / SQ_WAVES; "
            "valu_active = SQ_ACTIVE_INST_VALU / SQ_WAVE_CYCLES; wait_any = SQ_WAIT_INST_ANY / "
            "SQ_WAVE_CYCLES; conflict/lds = SQ_LDS_BANK_CONFLICT / SQ_INSTS_LDS",
            f"source_sha1 {source_sha1()}",
            "kernel\tgrid\tdispatches\t" + "\t".join(names) +
            "\tvalu/wave\tlds/wave\tvalu_active\twait_any\tconflict/lds"]

    def ratio(a, b):
        return f"{a / b:.3f}" if a is not None and b else "-"
    for k in sorted(vals, key=lambda k: k[0]):
        if not k[0].startswith("wo::"):
            continue
        m = {c: sum(v) / len(v) for c, v in vals[k].items()}
        n = max(len(v) for v in vals[k].values())
        g = m.get
        out.append(f"{k[0]}\t{k[1]}\t{n}\t" + "\t".join(f"{m[c]:.4g}" if c in m else "-" for c in names) +
                   f"\t{ratio(g('SQ_INSTS_VALU'), g('SQ_WAVES'))}\t{ratio(g('SQ_INSTS_LDS'), g('SQ_WAVES'))}"
                   f"\t{ratio(g('SQ_ACTIVE_INST_VALU'), g('SQ_WAVE_CYCLES'))}"
                   f"\t{ratio(g('SQ_WAIT_INST_ANY'), g('SQ_WAVE_CYCLES'))}"
                   f"\t{ratio(g('SQ_LDS_BANK_CONFLICT'), g('SQ_INSTS_LDS'))}")
    return "\n".join(out) + "\n"


# ---------------------------------------------------------------- inputs

def pol5_sigma_max_sq(api, torch, o, red):
    """max over frequencies of sigma_max(H(nu))^2 for the 5 x 4 bank formed from its
    reduced form red (1, 1, 2, Z, rows, cols): per frequency the largest eigenvalue
    of the 4 x 4 Gram matrix H^H H by power iteration (elementwise torch ops)."""
    k = torch.from_numpy(api.pol5_coupling(o.swing)).to(red.device)      # (5, 4) complex64
    u, v = red[0, 0, 0].reshape(-1), red[0, 0, 1].reshape(-1)
    best = 0.0
    for s in range(0, u.numel(), 1 << 22):
        uu, vv = u[s:s + (1 << 22)], v[s:s + (1 << 22)]
        H = [[k[c, p].real * uu + k[c, p].imag * vv for p in range(4)] for c in range(5)]
        G = [[sum(H[c][p].conj() * H[c][q] for c in range(5)) for q in range(4)] for p in range(4)]
        x = [torch.ones_like(uu) for _ in range(4)]
        lam = None
        for _ in range(60):
            y = [sum(G[p][q] * x[q] for q in range(4)) for p in range(4)]
            nrm = torch.sqrt(sum((t.abs() ** 2) for t in y)) + 1e-30
            x = [t / nrm for t in y]
            lam = nrm
        best = max(best, float(lam.max()))
    return best


def bank_sigma_max_sq(torch, tf):
    """max over frequencies of sigma_max(H(nu))^2 of a full bank tf (1, C, P, Z, Y, Xh):
    per frequency the largest eigenvalue of H^H H by power iteration."""
    C, P = tf.shape[1], tf.shape[2]
    H = tf[0].reshape(C, P, -1)
    best = 0.0
    for s in range(0, H.shape[2], 1 << 21):
        h = H[:, :, s:s + (1 << 21)]
        G = [[sum(h[c, p].conj() * h[c, q] for c in range(C)) for q in range(P)] for p in range(P)]
        x = [torch.ones_like(h[0, 0]) for _ in range(P)]
        lam = None
        for _ in range(60):
            y = [sum(G[p][q] * x[q] for q in range(P)) for p in range(P)]
            nrm = torch.sqrt(sum((t.abs() ** 2) for t in y)) + 1e-30
            x = [t / nrm for t in y]
            lam = nrm
        best = max(best, float(lam.max()))
    return best


def make_inputs(api, torch, dev, key, o, sup):
    """The workload's synthetic data on the device (forward model of a seeded
    specimen through the GPU bank, plus noise) and eta.  Returns (d, eta, band)."""
    import synth
    Z, Y, X = o.nz, o.ny, o.nx
    band = key != "fluor"
    tf = api.transfer_function_band([o], device=dev) if band else api.transfer_function([o], device=dev)
    lin = ((lambda op, x: api.linear_band(op, [o], tf, x)) if band else
           (lambda op, x: api.forward([o], tf, x)))
    if key == "pol5":
        f = synth.fibres_on_device((Z, Y, X), (o.dz, o.dy, o.dx), 300, seed=3001, device=dev)[None]
        d = lin(api.OP_FORWARD, f)
        del f
        api.add_gaussian_noise(d, 1e-3, 3002)
        eta = ETA_REL * pol5_sigma_max_sq(api, torch, o, tf)
    elif key == "labelfree":
        obj = synth.ellipsoids((Z, Y, X), (o.dz, o.dy, o.dx), 200, seed=2001)
        clean = lin(api.OP_FORWARD, torch.from_numpy(obj[None]).to(dev))
        d = torch.from_numpy(synth.poisson_gaussian(clean.cpu().numpy(), seed=2002)).to(dev)
        # 1 channel: sigma_max^2 = |H_phase|^2 + |H_abs|^2
        eta = ETA_REL * float((tf.abs() ** 2).sum(dim=2).max())
    elif key == "vector":
        f = synth.fibres_on_device((Z, Y, X), (o.dz, o.dy, o.dx), 300, seed=3001, device=dev)[None]
        d = lin(api.OP_FORWARD, f)
        del f
        api.add_gaussian_noise(d, 1e-3, 3002)
        eta = ETA_REL * bank_sigma_max_sq(torch, tf)
    else:
        obj = synth.beads((Z, Y, X), 50, seed=1001)[None]
        clean = lin(api.OP_FORWARD, torch.from_numpy(obj[None]).to(dev))
        d = clean + torch.from_numpy(synth.gaussian_noise((1, 1, Z, Y, X), 1e-3, 1002).astype(np.float32)).to(dev)
        eta = 1e-3
    torch.cuda.synchronize()
    return d.contiguous(), eta, band


# ---------------------------------------------------------------- parity of the timed output

def _oracle_optics(o):
    from oracle import optics as op
    return op.Optics(model=o.model, nz=o.nz, ny=o.ny, nx=o.nx, dz=o.dz, dy=o.dy, dx=o.dx,
                     wavelength=o.wavelength, na_ill=o.na_ill, na_det=o.na_det, n_medium=o.n_medium,
                     swing=o.swing, vec_channels=o.vec_channels, vec_props=tuple(o.vec_props),
                     ill_jones=tuple(o.ill_jones))


def parity_full(o, d_host, f_gpu, eta):
    """FP64 oracle TF synthesis + reconstruction of the bench's own data, element by
    element against the timed GPU output (relative L2 over the whole volume)."""
    import scipy.fft as sfft

    from oracle import linear
    from oracle import tf as tfm
    t0 = time.perf_counter()
    with sfft.set_workers(len(os.sched_getaffinity(0))):
        bank = tfm.transfer_function(_oracle_optics(o))
        ref = linear.reconstruct(bank, d_host.astype(np.float64), None, eta)
    err = float(np.linalg.norm(f_gpu.astype(np.float64) - ref) / np.linalg.norm(ref))
    return {"kind": "whole volume", "oracle": "oracle.tf.transfer_function + oracle.linear.reconstruct (FP64)",
            "rel_l2": err, "tolerance": TOL_REC, "ok": bool(err < TOL_REC),
            "oracle_seconds": round(time.perf_counter() - t0, 1)}


def _dft_at(vol, freqs):
    """Direct DFT of vol (C, Z, Y, X) at frequency indices [(kz, ky, kx)], FP64:
    per plane, the X sum by a product with exp(-i 2 pi kx x / X), then Y, then Z."""
    C, Z, Y, X = vol.shape
    kz = np.array([f[0] for f in freqs])
    ky = np.array([f[1] for f in freqs])
    kx = np.array([f[2] for f in freqs])
    ex = np.exp(-2j * np.pi * np.outer(np.arange(X), kx) / X)          # (X, K)
    ey = np.exp(-2j * np.pi * np.outer(ky, np.arange(Y)) / Y)          # (K, Y)
    ez = np.exp(-2j * np.pi * np.outer(np.arange(Z), kz) / Z)          # (Z, K)
    out = np.zeros((C, len(freqs)), dtype=np.complex128)
    for z in range(Z):
        pl = vol[:, z].astype(np.float64)                               # (C, Y, X)
        tx = pl @ ex                                                    # (C, Y, K)
        t = np.einsum("ky,cyk->ck", ey, tx)
        out += t * ez[z][None, :]
    return out


def parity_pol5_sampled(o, d_host, f_gpu, eta, sup, n=12, seed=3003):
    """At sampled frequencies of the support: the oracle's per-frequency Tikhonov
    solve F = (H^H H + eta I)^-1 H^H D with H from the direct source sum
    (oracle.tf.pol5_3d_at, or oracle.vector.vector_3d_at for the vector bank) and D
    the direct DFT of the bench's own data, against the direct DFT of the timed GPU
    output there (relative L2 over the samples).  The whole-volume FP64 solve does
    not fit the bench's time."""
    from oracle import tf as tfm
    from oracle import vector as vec
    t0 = time.perf_counter()
    oo = _oracle_optics(o)
    bank_at = vec.vector_3d_at if o.model == 5 else tfm.pol5_3d_at
    rng = np.random.default_rng(seed)
    ky_max = (sup["band_rows"] - 1) // 2
    kt = sup["tf_cols"]
    freqs = []
    while len(freqs) < n:
        # in-band frequencies: low and moderate axial and lateral indices
        kz = int(rng.integers(-4, 5)) % o.nz
        ky = int(rng.integers(-ky_max // 2, ky_max // 2 + 1)) % o.ny
        kx = int(rng.integers(1, kt // 2))
        if (kz, ky, kx) not in freqs:
            freqs.append((kz, ky, kx))
    Dg = _dft_at(d_host, freqs)                                          # (5, K)
    Fg = _dft_at(f_gpu, freqs)                                           # (4, K)
    num = den = 0.0
    for k, (kz, ky, kx) in enumerate(freqs):
        H = bank_at(oo, kz, ky, kx)
        Hh = H.conj().T
        F = np.linalg.solve(Hh @ H + eta * np.eye(4), Hh @ Dg[:, k])
        num += float(np.sum(np.abs(Fg[:, k] - F) ** 2))
        den += float(np.sum(np.abs(F) ** 2))
    err = math.sqrt(num / den)
    return {"kind": f"{n} sampled frequencies of the support",
            "oracle": f"oracle.{'vector.vector_3d_at' if o.model == 5 else 'tf.pol5_3d_at'} (direct source "
                      "sum) + per-frequency solve; direct DFTs (FP64)",
            "rel_l2": err, "tolerance": TOL_REC, "ok": bool(err < TOL_REC),
            "oracle_seconds": round(time.perf_counter() - t0, 1)}


# ---------------------------------------------------------------- one linear workload

def linear_section(api, torch, dev, args, key, parity=True):
    """Step = TF synthesis + reconstruction of the workload, timed; per-kernel
    table, dominant-kernel roofline, cached-TF rate and the parity of the timed
    output against the oracle."""
    spec = SECTIONS[key]
    o = api.Optics(**spec["optics"])
    Z, Y, X = o.nz, o.ny, o.nx
    V = Z * Y * X
    C, P, _, _ = api.bank_shape([o])
    sup = api.lateral_support([o])
    d, eta, band = make_inputs(api, torch, dev, key, o, sup)
    print(f"[bench] {key}: inputs ready (eta {eta:.3e})", file=sys.stderr, flush=True)
    lib = api.load()
    arr = api.optics_array([o])
    stream = torch.cuda.current_stream()
    sp = api._stream(stream)
    ws_tf = torch.empty(api.workspace_size([o], api.OP_TRANSFER_FUNCTION), dtype=torch.uint8, device=dev)
    ws_rec = torch.empty(api.workspace_size([o], api.OP_RECONSTRUCT), dtype=torch.uint8, device=dev)
    fout = torch.empty((1, P, Z, Y, X), dtype=torch.float32, device=dev)
    bank = torch.empty(api.band_dims([o]) if band else api.bank_dims([o]), dtype=torch.complex64, device=dev)

    def step_tf():
        fn = lib.wo_transfer_function_band if band else lib.wo_transfer_function
        st = fn(arr, 1, api._ptr(bank), api._ptr(ws_tf), ws_tf.numel(), sp)
        assert st == 0, st

    def step_rec():
        if band:
            st = lib.wo_linear_band(api.OP_RECONSTRUCT, arr, 1, api._ptr(bank), api._ptr(d), None, eta,
                                    api._ptr(fout), api._ptr(ws_rec), ws_rec.numel(), sp)
        else:
            st = lib.wo_reconstruct(arr, 1, api._ptr(bank), api._ptr(d), None, eta, api._ptr(fout),
                                    api._ptr(ws_rec), ws_rec.numel(), sp)
        assert st == 0, st

    def full_step():
        step_tf()
        step_rec()

    def timed(fn, k):
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) * 1e3 / k

    for _ in range(args.warmup):
        full_step()
    torch.cuda.synchronize()

    # ---- FFT schedules: the library's defaults, then the tuner's picks (or a saved table)
    tuner = {}
    if args.fft_plans:
        api.fft_plans_import(open(args.fft_plans).read())
        tuner["imported"] = os.path.basename(args.fft_plans)
    elif not args.no_fft_tune and key != "vector":
        before = api.fft_plans_export()
        tuner["ms_per_step_default_schedules"] = timed(full_step, args.steps)
        a = time.perf_counter()
        tf_out = torch.empty_like(bank)
        api.fft_tune(api.OP_TRANSFER_FUNCTION, [o], out=tf_out, reps=15, ws=ws_tf, stream=stream, band=band)
        del tf_out
        step_tf()
        api.fft_tune(api.OP_RECONSTRUCT, [o], tf=bank, x=d, out=fout, eta=eta, reps=15, ws=ws_rec,
                     stream=stream, band=band)
        tuner["tune_s"] = round(time.perf_counter() - a, 3)
        for _ in range(args.warmup):
            full_step()
        # The tuner judges each call on its own; the step runs the two calls back
        # to back (other cache contents), so keep its picks only if the step is
        # faster with them by more than the run-to-run spread (1 %); otherwise
        # the timed step runs the default schedules, as the profiled runs do.
        tuner["ms_per_step_tuned_schedules"] = timed(full_step, args.steps)
        if tuner["ms_per_step_tuned_schedules"] >= 0.99 * tuner["ms_per_step_default_schedules"]:
            mine = [ln for ln in api.fft_plans_export().splitlines() if ln not in before.splitlines()]
            tuner["tuned_table_dropped"] = mine
            api.fft_plans_clear()
            if before:
                api.fft_plans_import(before)
            for _ in range(args.warmup):
                full_step()
    tuner["table"] = api.fft_plans_export().splitlines()
    print(f"[bench] {key}: fft schedules {tuner}", file=sys.stderr, flush=True)

    # ---- per-kernel pass: K steps with every library kernel bracketed by HIP events
    # (the events add gaps between launches, so this pass is not the timed one)
    api.timing_enable(True)
    for _ in range(args.steps):
        full_step()
    torch.cuda.synchronize()
    api.timing_enable(False)
    kern = api.timing_report()
    dom = max(kern, key=lambda k: kern[k][1])

    # ---- timed region: K whole steps; HIP events on the library's stream around
    # the dominant kernel only (its duration for the roofline)
    api.timing_select(dom)
    api.timing_enable(True)
    ms = timed(full_step, args.steps)
    api.timing_enable(False)
    dom_rec = api.timing_report()[dom]
    api.timing_select(None)
    f_timed = fout.cpu().numpy()[0]

    ms_rec = timed(step_rec, args.steps)      # cached transfer function

    E = 2 if key == "pol5" else None
    F = 6 + 3 * (5 if o.vec_channels == 1 else 1) if key == "vector" else None
    # the fluorescence workload (about 10 MB) stays in the caches and its kernels
    # last a few microseconds each: launch- and latency-bound, no HBM roofline
    hbm = key != "fluor"
    kernels = {}
    step_bytes = 0
    for name, (cnt, tot) in sorted(kern.items()):
        per = tot / cnt
        b = kernel_bytes(name, Z, Y, X, sup, C, P, E, F) if hbm else None
        ent = {"launches": cnt, "avg_ms": round(per, 5)}
        if b:
            ent["alg_bytes"] = b
            ent["alg_GBps"] = round(b / (per * 1e-3) / 1e9, 1)
            ent["hbm_frac"] = round(b / (per * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            step_bytes += b * cnt // args.steps
        kernels[name] = ent
    dom_ms = dom_rec[1] / dom_rec[0]
    if hbm:
        dom_b = kernel_bytes(dom, Z, Y, X, sup, C, P, E, F) or 0
        ach = dom_b / (dom_ms * 1e-3) / 1e9
        symbols = counter_symbols(sup, Z, X, P, C, (5 if o.vec_channels == 1 else 1) if key == "vector" else None)
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(key, dom, symbols), "alg_bytes": dom_b,
                "avg_ms_timed_region": round(dom_ms, 5)}
    else:
        ach = 0.0
        roof = {"kernel": dom, "bound": "latency", "avg_ms_timed_region": round(dom_ms, 5),
                "note": "cache-resident working set, kernels of a few microseconds: launch/latency-bound"}
    res = {"workload": spec["workload"], "shape_zyx": [Z, Y, X], "channels_x_properties": [C, P],
           "voxel_um": [o.dz, o.dy, o.dx], "eta": eta,
           "eta_rule": "1e-3 absolute" if key == "fluor" else "1e-3 * max_nu sigma_max(H(nu))^2",
           "ms_per_step": ms, "voxels_per_s": V / (ms * 1e-3), "steps": args.steps,
           "reconstruct_cached_tf": {"ms": ms_rec, "voxels_per_s": V / (ms_rec * 1e-3)},
           "lateral_support": {k: list(v) if isinstance(v, tuple) else v for k, v in sup.items()},
           "fft_schedules": tuner, "roofline": roof,
           # every library kernel of the step: algorithmic bytes per step over the timed
           # step duration (launch gaps and all)
           "step_hbm": ({"alg_bytes": step_bytes, "GBps": round(step_bytes / (ms * 1e-3) / 1e9, 1),
                         "frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)} if hbm else None),
           "kernels": kernels,
           # the FFT passes and the fused Tikhonov kernel against 60 % of peak HBM
           "hbm_target_60pct": ({"met": sorted(k for k, v in kernels.items()
                                               if k.startswith(("k_rows", "k_cols", "k_zop"))
                                               and v.get("hbm_frac", 0) >= 0.6),
                                 "below": sorted(k for k, v in kernels.items()
                                                 if k.startswith(("k_rows", "k_cols", "k_zop"))
                                                 and v.get("hbm_frac", 1) < 0.6)} if hbm else None)}
    print(f"[bench] {key}: {ms:.3f} ms/step, {V / (ms * 1e-3) / 1e9:.2f} G voxels/s; dominant {dom} "
          f"{dom_ms * 1e3:.1f} us" + (f", {ach:.0f} GB/s" if hbm else ""), file=sys.stderr, flush=True)
    if parity:
        d_host = d.cpu().numpy()[0]
        res["parity"] = (parity_pol5_sampled(o, d_host, f_timed, eta, sup) if key in ("pol5", "vector")
                         else parity_full(o, d_host, f_timed, eta))
        print(f"[bench] {key}: parity {res['parity']['rel_l2']:.2e} ({res['parity']['kind']})",
              file=sys.stderr, flush=True)
    del d, ws_tf, ws_rec, fout, bank
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true", help="skip the oracle checks of the timed outputs")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tune-patches", type=int, default=256)
    ap.add_argument("--tune-iters", type=int, default=100)
    ap.add_argument("--cnn-train-patches", type=int, default=51200)
    ap.add_argument("--cnn-epochs", type=int, default=8)
    ap.add_argument("--cnn-tune-iters", type=int, default=20)
    ap.add_argument("--restore-tiles", type=int, default=64)
    ap.add_argument("--fov-size", type=int, default=2048, help="field of view side (0: skip)")
    ap.add_argument("--no-multi-aperture", action="store_true")
    ap.add_argument("--no-aberration", action="store_true")
    ap.add_argument("--sections", default="pol5,labelfree,fluor,vector",
                    help="linear workloads to run, the first is the headline")
    ap.add_argument("--main-only", action="store_true",
                    help="only the headline linear workload (profiled runs: only its kernels in the trace)")
    ap.add_argument("--no-fft-tune", action="store_true", help="keep the default FFT schedules")
    ap.add_argument("--fft-plans", default="", help="import an FFT schedule table instead of tuning")
    ap.add_argument("--save-fft-plans", default="", help="write the FFT schedule table used")
    ap.add_argument("--restore-graph", type=int, default=2, choices=(0, 1, 2),
                    help="graph mode of the CNN-started restoration (multistart uses 1)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--summarise-trace", default="", help="(no GPU) write the kernel-duration "
                    "summary of a rocprofv3 --kernel-trace directory to --summary-out")
    ap.add_argument("--summarise-counters", nargs=2, default=None, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="(no GPU) write the FETCH_SIZE/WRITE_SIZE summary to --summary-out")
    ap.add_argument("--summarise-sq", nargs="+", default=None, metavar="PMC_DIR",
                    help="(no GPU) write the SQ-counter summary of rocprofv3 --pmc directories")
    ap.add_argument("--summary-command", action="append", default=[],
                    help="command line recorded in the summary header (repeatable)")
    ap.add_argument("--summary-title", default="", help="workload named in the summary header")
    ap.add_argument("--summary-out", default="")
    args = ap.parse_args()
    if args.summarise_trace or args.summarise_counters or args.summarise_sq:
        if args.summarise_trace:
            text = summarise_trace(args.summarise_trace, " ".join(args.summary_command), args.summary_title)
        elif args.summarise_counters:
            text = summarise_counters(*args.summarise_counters, args.summary_command, args.summary_title)
        else:
            text = summarise_sq(args.summarise_sq, args.summary_command, args.summary_title)
        if args.summary_out:
            open(args.summary_out, "w").write(text)
        else:
            sys.stdout.write(text)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the path is not sharded across GPUs; --gpus above 1 is not supported"}))
        sys.exit(2)

    import torch

    from paper_2412_09775_amd import api

    api.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    keys = [k for k in args.sections.split(",") if k]
    if args.main_only:
        keys = keys[:1]
        args.no_multi_aperture = args.no_aberration = args.no_autotune = True
    results = {}
    for k in keys:
        results[k] = linear_section(api, torch, dev, args, k, parity=not args.no_parity)
    head = results[keys[0]]
    if args.save_fft_plans:
        os.makedirs(os.path.dirname(os.path.abspath(args.save_fft_plans)), exist_ok=True)
        with open(args.save_fft_plans, "w") as fh:
            fh.write(api.fft_plans_export())

    out = {
        "metric": "reconstructed voxels/s (TF synthesis + Tikhonov reconstruction per step)",
        "value": head["voxels_per_s"],
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": head["workload"], "shape_zyx": head["shape_zyx"],
                   "channels_x_properties": head["channels_x_properties"], "voxel_um": head["voxel_um"],
                   "eta_rel": ETA_REL},
        "roofline": head["roofline"],
        "step_hbm": head["step_hbm"],
        "parity": head.get("parity"),
        "reconstruct_cached_tf": head["reconstruct_cached_tf"],
        "lateral_support": head["lateral_support"],
        "fft_schedules": head["fft_schedules"],
        "kernels": head["kernels"],
        "hbm_target_60pct": head["hbm_target_60pct"],
        "secondary": {SECTIONS[k]["name"]: results[k] for k in keys[1:]},
    }

    if not args.no_multi_aperture:
        out["multi_aperture"] = multi_aperture_section(api, torch, dev, args.steps)
    if not args.no_aberration:
        out["aberration"] = aberration_section(api, torch, dev, args.steps)
    if not args.no_autotune:
        net, train = None, None
        if args.cnn_train_patches > 0:
            net, train = train_cnn(api, torch, dev, args.cnn_train_patches, args.cnn_epochs)
        out["autotune"] = autotune_section(api, torch, dev, args.tune_patches, args.tune_iters, net,
                                           args.cnn_tune_iters)
        if train:
            out["autotune"]["cnn_training"] = train
        if net is not None and args.fov_size > 0:
            out["fov"] = fov_section(api, torch, dev, net, args.cnn_tune_iters, size=args.fov_size)
        if not args.no_cpu_baseline:
            out["autotune"]["cpu_baseline"] = cpu_baseline_autotune()
        if args.restore_tiles > 0:
            out["restore"] = restore_section(api, torch, dev, net, args.restore_tiles, args.cnn_tune_iters,
                                             args.tune_iters, args.restore_graph)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(keys[0])
    print(json.dumps(out))
    bad = [k for k, r in results.items() if r.get("parity") and not r["parity"]["ok"]]
    if bad:
        print(f"[bench] parity above tolerance: {bad}", file=sys.stderr, flush=True)
        sys.exit(1)


# Auto-tune workload: 256 patches of 32x128x128 (dz 0.2, dx 0.1 um), lambda0 0.532,
# NA_ill 0.5, n 1.33, soft pupil edges; per-patch truth defocus ~U(-2, 2) um,
# NA_det ~U(1.0, 1.3), illumination zenith tilt ~U(0, 30 deg).
TUNE = dict(model=2, nz=32, ny=128, nx=128, dz=0.2, dy=0.1, dx=0.1, wavelength=0.532, na_ill=0.5,
            na_det=1.15, n_medium=1.33, defocus=0.0, tilt_zenith=0.0, tilt_azimuth=0.0,
            edge_width=0.5, swing=0.1)
TUNE_RANGE = np.array([4.0, 0.3, math.radians(30.0)])
TUNE_LR = (0.02, 0.005, 0.005, 0.001)
TUNE_LO = (-2.5, 1.0, 0.0, -1.0)
TUNE_HI = (2.5, 1.3, math.radians(32.0), 1.0)
# tuned parameters: defocus and illumination zenith tilt, as in the paper's auto-tune;
# NA_det keeps its starting value (nominal, or the learned initialiser's prediction)
TUNE_MASK = 0b0101


def thin_sigma_max_sq(tf):
    """max over 2D frequencies of the largest eigenvalue of H^H H for a thin bank
    (n, Z, 2, Y, Xh): the 2x2 Gram matrix of the two property columns."""
    h0, h1 = tf[:, :, 0], tf[:, :, 1]
    a = (h0.abs() ** 2).sum(dim=1)
    b = (h1.abs() ** 2).sum(dim=1)
    m = (h0.conj() * h1).sum(dim=1).abs()
    return float(((a + b) / 2 + (((a - b) / 2) ** 2 + m ** 2).sqrt()).max())


def norm_err(th, truth):
    """Median over patches of max_j |theta_j - truth_j| / range_j, and per component."""
    e = np.abs(np.asarray(th)[:, :3] - truth) / TUNE_RANGE
    return float(np.median(e.max(axis=1))), [round(float(x), 4) for x in np.median(e, axis=0)]


def tuned_err(th, truth):
    """The same over the tuned components only (defocus, zenith tilt): the mid-band
    loss is monotone in NA, so NA is not identified by it and comes from the start."""
    e = np.abs(np.asarray(th)[:, [0, 2]] - truth[:, [0, 2]]) / TUNE_RANGE[[0, 2]]
    return round(float(np.median(e.max(axis=1))), 4)


def prior_draws(rng, n):
    return np.stack([rng.uniform(-2, 2, n), rng.uniform(1.0, 1.3, n),
                     rng.uniform(0.0, math.radians(30.0), n)], 1)


def grid_starts(n, na):
    """8 starts per patch: defocus {-1.5, -0.5, 0.5, 1.5} um x tilt {7.5, 22.5} deg."""
    grid = np.stack(np.meshgrid([-1.5, -0.5, 0.5, 1.5], [math.radians(7.5), math.radians(22.5)],
                                indexing="ij"), -1).reshape(-1, 2)
    theta0 = np.zeros((n, 8, 4))
    theta0[:, :, 0] = grid[None, :, 0]
    theta0[:, :, 1] = na
    theta0[:, :, 2] = grid[None, :, 1]
    return theta0


def autotune_section(api, torch, dev, n, iters, net, cnn_iters):
    """Patches/s of the batched GPU auto-tune (single start, 8-start multistart and
    CNN-initialised) and the median normalised parameter error |theta - truth| / range."""
    import synth
    rng = np.random.default_rng(4001)
    truth = prior_draws(rng, n)
    opts_true = [api.Optics(**dict(TUNE, defocus=t[0], na_det=t[1], tilt_zenith=t[2])) for t in truth]
    objs = np.stack([synth.thin_cells((TUNE["ny"], TUNE["nx"]), TUNE["dx"], 20, seed=5000 + i)
                     for i in range(n)])
    tf_true = api.transfer_function(opts_true, device=dev)
    clean = api.forward(opts_true, tf_true, torch.from_numpy(objs).to(dev))
    d = torch.from_numpy(synth.poisson_gaussian(clean.cpu().numpy(), seed=4002)).to(dev)
    del tf_true, clean
    nominal = api.Optics(**TUNE)
    eta = 1e-2 * thin_sigma_max_sq(api.transfer_function([nominal], device=dev))
    nu_c = (TUNE["na_det"] + TUNE["na_ill"]) / TUNE["wavelength"]
    starts = [api.Optics(**dict(TUNE, tilt_zenith=math.radians(15.0))) for _ in range(n)]

    res = {"workload": f"{n} patches 32x128x128, {iters} Adam iterations, hipGraph replay, "
                       "tuning defocus and zenith tilt",
           "tuned_parameters": "defocus and illumination zenith tilt (the paper's auto-tune optimises the "
                               "focal offset and the illumination tilt; the synthetic truth has no tilt "
                               "azimuth); NA_det keeps its start value: nominal for single start and "
                               "multistart, the CNN's prediction for the CNN start",
           "error_measure": "median_norm_err_defocus_tilt compares arms on the tuned parameters; "
                            "median_norm_err_defocus_na_tilt lists each parameter"}
    for label, M in (("single_start", 1), ("multistart_8", 8)):
        theta0 = grid_starts(n, TUNE["na_det"]) if M > 1 else None
        ws = torch.empty(api.tune_workspace_size(starts, M), dtype=torch.uint8, device=dev)
        api.autotune(starts[:1], d[:1], eta, iters=2, lr=TUNE_LR, lo=TUNE_LO, hi=TUNE_HI, multistart=M,
                     theta0=None if theta0 is None else theta0[:1], nu_c=nu_c, use_graph=True, ws=ws,
                     mask=TUNE_MASK)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, loss, _, _ = api.autotune(starts, d, eta, iters=iters, lr=TUNE_LR, lo=TUNE_LO, hi=TUNE_HI,
                                       multistart=M, theta0=theta0, nu_c=nu_c, use_graph=True, ws=ws,
                                       mask=TUNE_MASK)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        th = np.array([[o.defocus, o.na_det, o.tilt_zenith, o.tilt_azimuth] for o in out])
        med, per = norm_err(th, truth)
        res[label] = {"patches_per_s": n / dt, "seconds": round(dt, 3), "starts": M,
                      "median_norm_param_err": round(med, 4), "median_norm_err_defocus_na_tilt": per,
                      "median_norm_err_defocus_tilt": tuned_err(th, truth)}
        del ws
        print(f"[bench] autotune {label}: {n / dt:.1f} patches/s, median err {med:.3f}",
              file=sys.stderr, flush=True)

    if net is not None:
        ws = torch.empty(api.tune_workspace_size(starts, 1), dtype=torch.uint8, device=dev)
        net.predict(d[:8])
        api.autotune(starts[:1], d[:1], eta, iters=2, lr=TUNE_LR, lo=TUNE_LO, hi=TUNE_HI, nu_c=nu_c,
                     use_graph=True, ws=ws, mask=TUNE_MASK)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pred = net.predict(d)
        theta0 = np.zeros((n, 1, 4))
        theta0[:, 0, :3] = np.clip(pred, np.array(TUNE_LO[:3]), np.array(TUNE_HI[:3]))
        out, loss, _, _ = api.autotune(starts, d, eta, iters=cnn_iters, lr=TUNE_LR, lo=TUNE_LO, hi=TUNE_HI,
                                       theta0=theta0, nu_c=nu_c, use_graph=True, ws=ws, mask=TUNE_MASK)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        th = np.array([[o.defocus, o.na_det, o.tilt_zenith, o.tilt_azimuth] for o in out])
        med, per = norm_err(th, truth)
        med0, per0 = norm_err(pred, truth)
        ms = res["multistart_8"]["patches_per_s"]
        res["cnn_init"] = {"patches_per_s": n / dt, "seconds": round(dt, 3), "tune_iters": cnn_iters,
                           "median_norm_param_err": round(med, 4), "median_norm_err_defocus_na_tilt": per,
                           "median_norm_err_defocus_tilt": tuned_err(th, truth),
                           "cnn_only_median_norm_err_defocus_na_tilt": per0,
                           "speedup_vs_multistart_8": round(n / dt / ms, 2)}
        print(f"[bench] cnn init: {n / dt:.1f} patches/s, median err {med:.3f} (cnn only {med0:.3f})",
              file=sys.stderr, flush=True)
    return res


CNN_CHANNELS = (1, 32, 64, 128, 256)
BF16_PEAK_TFLOPS = 2500.0     # MI355X dense BF16 MFMA


def cnn_flops_per_sample(shape=(32, 64, 64)):
    """Convolution FLOPs of one training sample (forward, weight gradient, and the
    input gradient of every block but the first): 2 * positions * Cout * 27 * Cin
    per GEMM; stride 2, padding 1."""
    d, h, w = shape
    total = 0
    for l in range(len(CNN_CHANNELS) - 1):
        d, h, w = (d - 1) // 2 + 1, (h - 1) // 2 + 1, (w - 1) // 2 + 1
        g = 2 * d * h * w * CNN_CHANNELS[l + 1] * 27 * CNN_CHANNELS[l]
        total += g * (2 if l == 0 else 3)
    return total


def train_cnn(api, torch, dev, patches, epochs):
    """The learned initialiser trained on forward-model patches 32x64x64 (not part of
    any patches/s figure); a quarter of the patches keep only their central 16 planes
    and a quarter 24, as tiles with fewer planes present them."""
    from paper_2412_09775_amd import learned_init
    tmpl64 = api.Optics(**dict(TUNE, ny=64, nx=64, edge_width=0.25))
    t0 = time.perf_counter()
    stacks, theta = learned_init.simulate(tmpl64, patches, seed=6001, device=dev)
    learned_init.clear_outer_planes(stacks, seed=6002, keeps=(16, 24, 32, 32))
    torch.cuda.synchronize()
    t_sim = time.perf_counter() - t0
    net = learned_init.LearnedInit(dev, seed=0)
    t0 = time.perf_counter()
    hist = net.train(stacks, theta, epochs=epochs, batch=64, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del stacks
    print(f"[bench] cnn trained: {patches} patches x {epochs} epochs in {t_train:.1f}s, "
          f"loss {hist[0]:.3f} -> {hist[-1]:.3f}", file=sys.stderr, flush=True)
    flops = cnn_flops_per_sample() * patches * epochs
    achieved = flops / t_train * 1e-12
    return net, {"patches": patches, "epochs": epochs, "batch": 64, "simulate_s": round(t_sim, 2),
                 "train_s": round(t_train, 2), "loss_first_last": [round(hist[0], 4), round(hist[-1], 4)],
                 "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": BF16_PEAK_TFLOPS,
                              "unit": "TFLOP/s", "frac": round(achieved / BF16_PEAK_TFLOPS, 4),
                              "flops_per_sample": cnn_flops_per_sample(),
                              "note": "convolution FLOPs over the whole training time (AdamW, head, "
                                      "normalisation and GELU backward included in the time)"}}


RESTORE_Z = (16, 24, 32, 48, 64)
RESTORE_YX = (128, 160, 192, 240, 256, 320, 384, 480, 512)


def restore_section(api, torch, dev, net, ntiles, cnn_iters, ms_iters, graph_mode):
    """Shift-variant restoration of uneven tiles (Z in 16..64, Y, X in 128..512, each
    tile its own true optics): CNN initialisation + a short auto-tune, against plain
    8-start multistart; each arm ends with the thin reconstruction of every tile, all
    inside one wo_restore_tiles call."""
    from paper_2412_09775_amd import learned_init
    rng = np.random.default_rng(5001)
    shapes = [(int(rng.choice(RESTORE_Z)), int(rng.choice(RESTORE_YX)), int(rng.choice(RESTORE_YX)))
              for _ in range(ntiles)]
    truth = prior_draws(rng, ntiles)

    def tile_optics(shape, **kw):
        z, y, x = shape
        # soft pupil edge of the same absolute width as 0.5 px on a 128 x 128 tile
        return api.Optics(**dict(TUNE, nz=z, ny=y, nx=x, edge_width=0.5 * max(y, x) / 128.0, **kw))

    tiles, etas, nucs, nominal = [], [], [], []
    for i, (shape, t) in enumerate(zip(shapes, truth)):
        ot = tile_optics(shape, defocus=t[0], na_det=t[1], tilt_zenith=t[2])
        cells = api.synth_thin_cells(1, shape[1], shape[2], TUNE["dx"],
                                     max(1, round(20 * shape[1] * shape[2] / 128 ** 2)), 7000 + i, dev)
        d = api.forward([ot], api.transfer_function([ot], device=dev), cells)[0]
        api.add_gaussian_noise(d, 0.0317, 8000 + i)   # Poisson-Gaussian at I_bg 1000, read 2 e-
        tiles.append(d)
        on = tile_optics(shape)
        nominal.append(on)
        etas.append(1e-2 * thin_sigma_max_sq(api.transfer_function([on], device=dev)))
        nucs.append((on.na_det + on.na_ill) / on.wavelength)
    torch.cuda.synchronize()
    vox = sum(z * y * x for z, y, x in shapes)
    res = {"workload": f"{ntiles} tiles, Z in {list(RESTORE_Z)}, Y and X in {list(RESTORE_YX)} "
                       f"({vox / 1e6:.1f} M voxels, {len(set(shapes))} distinct shapes), thin model, "
                       f"tuning defocus and zenith tilt, thin reconstruction of every tile; "
                       f"tiles_per_s from a repeated call with the same buffers (graph reused), "
                       f"first_call_seconds includes the capture"}

    def run(label, M, iters, theta0, predict, graph_mode, branches):
        ws = torch.empty(api.tune_workspace_size(nominal, M), dtype=torch.uint8, device=dev)
        fo = torch.empty(sum(2 * y * x for _, y, x in shapes), dtype=torch.float32, device=dev)
        small = [tile_optics((16, 128, 128))]
        api.restore_tiles(small, [tiles[0].new_zeros((16, 128, 128))], etas[:1], iters=1, lr=TUNE_LR,
                          lo=TUNE_LO, hi=TUNE_HI, multistart=M, mask=TUNE_MASK, use_graph=graph_mode,
                          branches=branches)
        d = api.pack_stacks(tiles)
        times = []
        for _ in range(2):   # the second call reuses the graph the first one captured
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if predict:   # the library's CNN start (crop, network, denormalisation)
                pred = api.cnn_init_theta(net.params, nominal, d)
                theta0 = np.zeros((ntiles, 1, 4))
                theta0[:, 0, :3] = np.clip(pred[:, :3], np.array(TUNE_LO[:3]), np.array(TUNE_HI[:3]))
            out, loss, _, _, f = api.restore_tiles(nominal, d, etas, iters=iters, lr=TUNE_LR, lo=TUNE_LO,
                                                   hi=TUNE_HI, multistart=M, theta0=theta0, nu_c=nucs,
                                                   mask=TUNE_MASK, use_graph=graph_mode,
                                                   branches=branches, ws=ws, f_out=fo)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        dt = times[1]
        th = np.array([[o.defocus, o.na_det, o.tilt_zenith, o.tilt_azimuth] for o in out])
        med, per = norm_err(th, truth)
        r = {"tiles_per_s": ntiles / dt, "voxels_per_s": vox / dt, "seconds": round(dt, 3),
             "first_call_seconds": round(times[0], 3), "use_graph": graph_mode, "branches": branches,
             "starts": M,
             "tune_iters": iters, "median_norm_param_err": round(med, 4),
             "median_norm_err_defocus_na_tilt": per, "median_norm_err_defocus_tilt": tuned_err(th, truth)}
        if predict:
            r["cnn_only_median_norm_err_defocus_na_tilt"] = norm_err(pred, truth)[1]
        print(f"[bench] restore {label}: {ntiles / dt:.1f} tiles/s, median err {med:.3f}",
              file=sys.stderr, flush=True)
        del ws, fo
        return r

    # graph modes: the whole call as one launch (use_graph 2) suits the short CNN-started
    # tune; the 100-iteration multistart replays a one-iteration graph (use_graph 1),
    # whose capture is 100 times smaller
    res["multistart_8"] = run("multistart_8", 8, ms_iters, grid_starts(ntiles, TUNE["na_det"]), False,
                              1, 4)
    if net is not None:
        res["cnn_init"] = run("cnn_init", 1, cnn_iters, None, True, graph_mode, 8)
        res["cnn_init"]["speedup_vs_multistart_8"] = round(
            res["cnn_init"]["tiles_per_s"] / res["multistart_8"]["tiles_per_s"], 2)
    return res


def fov_section(api, torch, dev, net, cnn_iters, size=2048, nz=32, grid=6, overlap_frac=0.2):
    """Shift-variant restoration of one field of view: a grid x grid of tiles with
    about 20 % overlap (Methods, OPS data), each tile CNN-started, auto-tuned
    (defocus, tilt) and reconstructed in one call, then blended with EDT weights.
    Synthetic data: cells over the whole field; each tile imaged with its own
    parameters (defocus drifting across the field, tilt growing towards the
    periphery), and the tile images blended with the same weights."""
    from paper_2412_09775_amd import fov
    T0 = api.tile_grid(size, grid, 0)[0]
    T, starts = api.tile_grid(size, grid, int(round(overlap_frac * T0)))
    n = grid * grid
    cy = np.array([s + T / 2 for s in starts]) - size / 2
    truth = np.zeros((n, 3))
    for iy in range(grid):
        for ix in range(grid):
            r = math.hypot(cy[iy], cy[ix]) / (size / math.sqrt(2))
            truth[iy * grid + ix] = [-1.5 + 3.0 * ix / (grid - 1), 1.15 + 0.1 * (iy / (grid - 1) - 0.5),
                                     math.radians(25.0) * r]
    ew = 0.5 * T / 128.0
    tmpl = api.Optics(**dict(TUNE, nz=nz, ny=T, nx=T, edge_width=ew))
    cells = api.synth_thin_cells(1, size, size, TUNE["dx"], round(20 * size * size / 128 ** 2), 9001, dev)
    obj_tiles = torch.stack([cells[0, :, y:y + T, x:x + T] for y in starts for x in starts]).contiguous()
    opts_true = [api.Optics(**dict(TUNE, nz=nz, ny=T, nx=T, edge_width=ew, defocus=t[0], na_det=t[1],
                                   tilt_zenith=t[2])) for t in truth]
    imgs = torch.empty((n, nz, T, T), dtype=torch.float32, device=dev)
    for i in range(n):
        imgs[i] = api.forward([opts_true[i]], api.transfer_function([opts_true[i]], device=dev),
                              obj_tiles[i:i + 1])[0]
    stack = torch.stack([api.stitch_tiles(imgs[:, z:z + 1], starts, starts, size, size)[0]
                         for z in range(nz)])
    api.add_gaussian_noise(stack, 0.0317, 9002)
    del imgs, obj_tiles, cells
    eta = 1e-2 * thin_sigma_max_sq(api.transfer_function([tmpl], device=dev))
    nu_c = (TUNE["na_det"] + TUNE["na_ill"]) / TUNE["wavelength"]
    kw = dict(grid=(grid, grid), overlap=(int(round(overlap_frac * T0)),) * 2, eta=eta, net=net,
              iters=cnn_iters, mask=TUNE_MASK, lr=TUNE_LR, lo=TUNE_LO, hi=TUNE_HI, nu_c=nu_c)
    fov.restore_fov(stack, tmpl, **kw)            # capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    field, out, loss, geom = fov.restore_fov(stack, tmpl, **kw)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    th = np.array([[o.defocus, o.na_det, o.tilt_zenith, o.tilt_azimuth] for o in out])
    med, per = norm_err(th, truth)
    vox = nz * size * size
    print(f"[bench] fov {size}x{size}: {dt * 1e3:.0f} ms, median err {med:.3f}", file=sys.stderr,
          flush=True)
    return {"workload": f"field of view {nz}x{size}x{size}, {grid}x{grid} tiles of {T}x{T} "
                        f"(overlap >= {int(round(overlap_frac * T0))} px), CNN start + {cnn_iters} "
                        f"iterations per tile, EDT-weighted stitching",
            "fov_per_s": 1.0 / dt, "voxels_per_s": vox / dt, "seconds": round(dt, 3),
            "median_norm_param_err": round(med, 4), "median_norm_err_defocus_na_tilt": per,
            "median_norm_err_defocus_tilt": tuned_err(th, truth)}


def aberration_section(api, torch, dev, steps, n_patches=256, iters=20):
    """Detection aberrations (Zernike Noll 5..11 in the detection pupil, Methods
    detection-parameter branch): TF synthesis of the bench volume with every
    coefficient at 0.05 waves, and the auto-tune iteration of the 32x128x128
    patches with theta only vs theta plus the seven coefficients tuned."""
    from paper_2412_09775_amd import learned_init
    Z, Y, X = WORKLOAD["nz"], WORKLOAD["ny"], WORKLOAD["nx"]
    o = api.Optics(**dict(WORKLOAD, zernike=(0.05,) * 7))
    tf = api.transfer_function([o], device=dev)
    ws_tf = torch.empty(api.workspace_size([o], api.OP_TRANSFER_FUNCTION), dtype=torch.uint8, device=dev)
    api.transfer_function([o], out=tf, ws=ws_tf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        api.transfer_function([o], out=tf, ws=ws_tf)
    torch.cuda.synchronize()
    tf_ms = (time.perf_counter() - t0) * 1e3 / steps
    del tf, ws_tf
    tmpl = api.Optics(**TUNE)
    stacks, _ = learned_init.simulate(tmpl, n_patches, seed=31, device=dev)
    opts = [api.Optics(**TUNE) for _ in range(n_patches)]
    eta = 1e-2 * thin_sigma_max_sq(api.transfer_function([tmpl], device=dev))
    ws = torch.empty(api.tune_workspace_size(opts, 1), dtype=torch.uint8, device=dev)
    res = {"workload": f"TF synthesis {Z}x{Y}x{X} with 7 Zernike terms at 0.05 waves; auto-tune of "
                       f"{n_patches} patches 32x128x128, {iters} iterations, graph replay",
           "tf_ms": tf_ms}
    for label, mask in (("theta", 0b0101), ("theta_and_zernike", 0b0101 | (0x7F << 4))):
        kw = dict(iters=iters, mask=mask, use_graph=1, ws=ws, lr_zernike=0.01, zernike_bound=0.5)
        api.autotune(opts, stacks, eta, **dict(kw, iters=2))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.autotune(opts, stacks, eta, **kw)
        torch.cuda.synchronize()
        res[f"ms_per_iter_{label}"] = (time.perf_counter() - t0) * 1e3 / iters
    print(f"[bench] aberrations: TF {tf_ms:.2f} ms; auto-tune {res['ms_per_iter_theta']:.2f} -> "
          f"{res['ms_per_iter_theta_and_zernike']:.2f} ms/iter", file=sys.stderr, flush=True)
    return res


def multi_aperture_section(api, torch, dev, steps, shape=(48, 512, 512)):
    """9 illumination apertures (8 sectors + the full disc) fused into one phase
    estimate (Results, cardiomyocytes; Fig. 4c): TF synthesis of the 9 x 1 bank and
    the per-frequency 9 x 1 Tikhonov solve."""
    import synth
    Z, Y, X = shape
    o = api.Optics(**dict(WORKLOAD, model=api.MODEL_SECTORS9_3D, nz=Z, ny=Y, nx=X))
    tf = api.transfer_function([o], device=dev)
    obj = synth.ellipsoids((Z, Y, X), (o.dz, o.dy, o.dx), 60, seed=2101)[:1]
    clean = api.forward([o], tf, torch.from_numpy(obj[None]).to(dev))
    d = torch.from_numpy(synth.poisson_gaussian(clean.cpu().numpy(), seed=2102)).to(dev)
    h = tf[0, :, 0]
    eta = ETA_REL * float((h.abs() ** 2).sum(dim=0).max())   # P = 1: sigma_max^2 = sum_c |H_c|^2
    ws_tf = torch.empty(api.workspace_size([o], api.OP_TRANSFER_FUNCTION), dtype=torch.uint8, device=dev)
    ws_rec = torch.empty(api.workspace_size([o], api.OP_RECONSTRUCT), dtype=torch.uint8, device=dev)
    api.fft_tune(api.OP_RECONSTRUCT, [o], tf=tf, x=d, out=torch.empty((1, 1, Z, Y, X), device=dev), eta=eta,
                 ws=ws_rec)
    for _ in range(2):
        api.transfer_function([o], out=tf, ws=ws_tf)
        f = api.reconstruct([o], tf, d, eta, ws=ws_rec)
    torch.cuda.synchronize()
    api.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        api.transfer_function([o], out=tf, ws=ws_tf)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        f = api.reconstruct([o], tf, d, eta, ws=ws_rec)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    api.timing_enable(False)
    kern = api.timing_report()
    V = Z * Y * X
    zop = kern.get("k_zop<1>")
    res = {"workload": f"9 apertures x phase, {Z}x{Y}x{X}", "tf_ms": (t1 - t0) * 1e3 / steps,
           "reconstruct_ms": (t2 - t1) * 1e3 / steps, "reconstruct_voxels_per_s": V * steps / (t2 - t1)}
    if zop:
        per = zop[1] / zop[0]
        sp = api.lateral_support([o])
        b = 8 * Z * sp["band_rows"] * sp["tf_cols"] * (9 + 9 + 1)
        res["k_zop<1>"] = {"avg_ms": round(per, 5), "alg_bytes": b, "alg_GBps": round(b / (per * 1e-3) / 1e9, 1)}
    print(f"[bench] multi-aperture: TF {res['tf_ms']:.2f} ms, reconstruct {res['reconstruct_ms']:.2f} ms",
          file=sys.stderr, flush=True)
    return res


def cpu_baseline_autotune(patches=2, iters=100):
    """FP64 oracle auto-tune (analytic gradient + Adam, the full 100 iterations) of
    `patches` 32x128x128 patches, each with its own true optics, on all host cores;
    patches per second of that sample (no extrapolation)."""
    import scipy.fft as sfft

    import synth
    from oracle import autotune as at
    from oracle import linear
    from oracle import optics as op
    from oracle import tf as tfm

    cores = len(os.sched_getaffinity(0))
    o = op.Optics(model=op.LABELFREE_THIN, nz=TUNE["nz"], ny=TUNE["ny"], nx=TUNE["nx"], dz=TUNE["dz"],
                  dy=TUNE["dy"], dx=TUNE["dx"], wavelength=TUNE["wavelength"], na_ill=TUNE["na_ill"],
                  na_det=TUNE["na_det"], n_medium=TUNE["n_medium"], edge_width=TUNE["edge_width"])
    eta = 1e-2 * linear.max_singular_value_sq(tfm.labelfree_thin(o))
    start = o.replace(tilt_zenith=math.radians(15.0))
    mask = tuple((TUNE_MASK >> j) & 1 for j in range(4))
    data = []
    for i in range(patches):
        truth = o.replace(defocus=0.7 - 0.9 * i, tilt_zenith=0.2 + 0.1 * i)
        f = synth.thin_cells((o.ny, o.nx), o.dx, 20, seed=4101 + i)
        data.append(linear.forward(tfm.labelfree_thin(truth), f)
                    + synth.gaussian_noise((o.nz, o.ny, o.nx), 0.03, 4201 + i))
    t0 = time.perf_counter()
    with sfft.set_workers(cores):
        for d in data:
            at.autotune(start, d, eta, at.nominal_cutoff(o), iters, np.array(TUNE_LR), np.array(TUNE_LO),
                        np.array(TUNE_HI), mask=mask)
    dt = time.perf_counter() - t0
    return {"value": patches / dt, "unit": "patches/s", "cores": cores, "kind": "oracle",
            "sample": f"{patches} patches 32x128x128, {iters} Adam iterations each (FP64 analytic "
                      f"gradient), {dt:.1f} s"}


def cpu_baseline(key, lateral=256, budget_s=20.0):
    """The FP64 oracle (TF synthesis + reconstruction, as it stands) timed on the
    host cores on a bounded sample of the headline workload: its optics and
    voxel sizes on a lateral crop of the grid (all planes), repeated for about
    budget_s seconds; voxels per second of that sample."""
    import scipy.fft as sfft

    import synth
    from oracle import linear
    from oracle import optics as op
    from oracle import tf as tfm

    spec = dict(SECTIONS[key]["optics"])
    cores = len(os.sched_getaffinity(0))
    ny, nx = min(spec["ny"], lateral), min(spec["nx"], lateral)
    oo = op.Optics(model=spec["model"], nz=spec["nz"], ny=ny, nx=nx, dz=spec["dz"], dy=spec["dy"],
                   dx=spec["dx"], wavelength=spec["wavelength"], na_ill=spec["na_ill"], na_det=spec["na_det"],
                   n_medium=spec["n_medium"], swing=spec["swing"])
    C = tfm.bank_shape(oo)[0]
    data = synth.gaussian_noise((C, oo.nz, ny, nx), 1e-2, 77)
    reps, t_tf, t0 = 0, 0.0, time.perf_counter()
    with sfft.set_workers(cores):
        while True:
            a = time.perf_counter()
            bank = tfm.transfer_function(oo)
            t_tf += time.perf_counter() - a
            eta = 1e-3 if key == "fluor" else ETA_REL * linear.max_singular_value_sq(bank)
            linear.reconstruct(bank, data, None, eta)
            reps += 1
            del bank
            if time.perf_counter() - t0 > budget_s or reps >= 20:
                break
    t2 = time.perf_counter()
    vox = oo.nz * ny * nx * reps
    return {"value": vox / (t2 - t0), "unit": "voxels/s", "cores": cores, "kind": "oracle",
            "sample": f"{reps} x ({oo.nz}x{ny}x{nx} crop of the workload's grid, same optics and voxels: "
                      f"TF synthesis + reconstruction, FP64)",
            "seconds": round(t2 - t0, 2), "tf_seconds": round(t_tf, 2)}


if __name__ == "__main__":
    main()
