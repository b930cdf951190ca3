"""Thin Python binding of ``libwaveorder.so`` (argument marshalling only).

Every step of the hot path runs in the HIP kernels behind the C ABI declared
in ``include/waveorder.h``.  PyTorch only provides device memory (tensors)
and the current HIP stream.  There is no CPU fallback: if the library is
missing, :func:`load` raises.

Optics are passed as any object (or dict) with the fields of ``wo_optics``:
model, nz, ny, nx, dz, dy, dx, wavelength, na_ill, na_det, n_medium, defocus,
tilt_zenith, tilt_azimuth, edge_width, swing.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwaveorder.so")

MODEL_FLUOR_3D = 0
MODEL_LABELFREE_3D = 1
MODEL_LABELFREE_THIN = 2
MODEL_POL5_3D = 3
MODEL_SECTORS9_3D = 4
MODEL_VECTOR_3D = 5

OP_TRANSFER_FUNCTION = 0
OP_FORWARD = 1
OP_RECONSTRUCT = 2
OP_ADJOINT = 3

DIVERGED = -6   # WO_DIVERGED

SYMBOLS = ("wo_bank_shape", "wo_workspace_size", "wo_transfer_function", "wo_forward",
           "wo_reconstruct", "wo_adjoint", "wo_strerror", "wo_version", "wo_timing_enable",
           "wo_timing_report", "wo_tune_workspace_size", "wo_midband_loss_grad", "wo_autotune",
           "wo_restore_tiles",
           "wo_cnn_param_count", "wo_cnn_workspace_size", "wo_cnn_forward", "wo_cnn_gradient",
           "wo_cnn_train_step", "wo_conv3d_forward", "wo_conv3d_input_grad", "wo_conv3d_weight_grad",
           "wo_synth_thin_cells", "wo_add_gaussian_noise", "wo_crop_stacks", "wo_fft_tune",
           "wo_fft_plans_export", "wo_fft_plans_import", "wo_fft_plans_clear", "wo_fft_candidates",
           "wo_tile_grid", "wo_stitch_tiles", "wo_timing_select", "wo_midband_loss_grad_aberration",
           "wo_lateral_support", "wo_transfer_function_band",
           "wo_linear_band", "wo_reconstruct_noalloc", "wo_pol5_coupling",
           "wo_reconstruct_grad_workspace_size", "wo_reconstruct_grad", "wo_cnn_prior",
           "wo_cnn_init_workspace_size", "wo_cnn_init_theta")

_FIELDS = ("model", "nz", "ny", "nx", "dz", "dy", "dx", "wavelength", "na_ill", "na_det",
           "n_medium", "defocus", "tilt_zenith", "tilt_azimuth", "edge_width", "swing")


N_ZERNIKE = 7   # Noll j = 5..11


class WoOptics(ctypes.Structure):
    _fields_ = ([("model", ctypes.c_int32), ("nz", ctypes.c_int32), ("ny", ctypes.c_int32),
                 ("nx", ctypes.c_int32)] + [(f, ctypes.c_double) for f in _FIELDS[4:]]
                + [("zernike", ctypes.c_double * N_ZERNIKE)]
                + [("det_tilt", ctypes.c_double), ("det_azimuth", ctypes.c_double)]
                + [("vec_channels", ctypes.c_int32), ("vec_nprops", ctypes.c_int32),
                   ("vec_props", ctypes.c_int32 * 8), ("ill_jones", ctypes.c_double * 4)])


@dataclasses.dataclass
class Optics:
    """Python mirror of ``wo_optics``."""

    model: int
    nz: int
    ny: int
    nx: int
    dz: float
    dy: float
    dx: float
    wavelength: float
    na_ill: float
    na_det: float
    n_medium: float
    defocus: float = 0.0
    tilt_zenith: float = 0.0
    tilt_azimuth: float = 0.0
    edge_width: float = 0.0
    swing: float = 0.1
    zernike: tuple = ()   # detection aberration, waves, Noll j = 5..11 (up to 7 values)
    det_tilt: float = 0.0       # oblique detection: detection axis zenith, rad
    det_azimuth: float = 0.0    # and azimuth, rad
    # vector model (MODEL_VECTOR_3D): channel set (0 Stokes S0..S3 under ill_jones,
    # 1 the five swing states), property codes 2 b + part (up to 8), Jones vector
    vec_channels: int = 0
    vec_props: tuple = (0, 16, 8, 1)
    ill_jones: tuple = (2 ** -0.5, 1j * 2 ** -0.5)


class WoAutotuneOpts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("multistart", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("tune_mask", ctypes.c_int32),
                ("lr", ctypes.c_double * 4), ("lo", ctypes.c_double * 4), ("hi", ctypes.c_double * 4),
                ("theta0", ctypes.POINTER(ctypes.c_double)), ("nu_c", ctypes.POINTER(ctypes.c_double)),
                ("all_theta_out", ctypes.POINTER(ctypes.c_double)),
                ("all_loss_out", ctypes.POINTER(ctypes.c_double)), ("branches", ctypes.c_int32),
                ("lr_zernike", ctypes.c_double), ("zernike_bound", ctypes.c_double),
                ("status_out", ctypes.POINTER(ctypes.c_int32))]


class WoSupport(ctypes.Structure):
    _fields_ = [("field_cols", ctypes.c_int32 * 2), ("tf_cols", ctypes.c_int32),
                ("band_rows", ctypes.c_int32), ("tf_lengths", ctypes.c_int32 * 2)]


class WoError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.wo_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2412_09775_amd.build.build()")
    # torch ships its own HIP runtime: load it first so that the library binds to
    # the same one and torch's device memory and streams are valid in its calls
    # (a library loaded first would pull in the system runtime beside torch's)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
    op = ctypes.POINTER(WoOptics)
    lib.wo_bank_shape.argtypes = [op, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                  ctypes.POINTER(ctypes.c_int64)]
    lib.wo_workspace_size.argtypes = [op, i32, i32]
    lib.wo_workspace_size.restype = sz
    lib.wo_lateral_support.argtypes = [op, i32, ctypes.POINTER(WoSupport)]
    lib.wo_transfer_function.argtypes = [op, i32, vp, vp, sz, vp]
    lib.wo_forward.argtypes = [op, i32, vp, vp, vp, vp, vp, sz, vp]
    lib.wo_reconstruct.argtypes = [op, i32, vp, vp, vp, ctypes.c_double, vp, vp, sz, vp]
    lib.wo_adjoint.argtypes = [op, i32, vp, vp, vp, vp, sz, vp]
    lib.wo_transfer_function_band.argtypes = [op, i32, vp, vp, sz, vp]
    lib.wo_linear_band.argtypes = [i32, op, i32, vp, vp, vp, ctypes.c_double, vp, vp, sz, vp]
    lib.wo_reconstruct_noalloc.argtypes = [op, i32, vp, vp, vp, ctypes.c_double, vp, vp]
    lib.wo_pol5_coupling.argtypes = [ctypes.c_double, ctypes.POINTER(ctypes.c_float)]
    lib.wo_reconstruct_grad_workspace_size.argtypes = [op, i32]
    lib.wo_reconstruct_grad_workspace_size.restype = sz
    lib.wo_reconstruct_grad.argtypes = [op, i32, vp, vp, ctypes.c_double, vp,
                                        ctypes.POINTER(ctypes.c_double), vp, vp, sz, vp]
    lib.wo_strerror.argtypes = [ctypes.c_int]
    lib.wo_strerror.restype = ctypes.c_char_p
    lib.wo_version.restype = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    lib.wo_tune_workspace_size.argtypes = [op, i32, i32]
    lib.wo_tune_workspace_size.restype = sz
    lib.wo_midband_loss_grad.argtypes = [op, i32, vp, dp, dp, dp, dp, vp, sz, vp]
    lib.wo_midband_loss_grad_aberration.argtypes = [op, i32, vp, dp, dp, dp, dp, vp, sz, vp]
    lib.wo_autotune.argtypes = [op, i32, vp, dp, ctypes.POINTER(WoAutotuneOpts), dp, vp, sz, vp]
    lib.wo_restore_tiles.argtypes = [op, i32, vp, dp, ctypes.POINTER(WoAutotuneOpts), dp, vp, vp, sz,
                                     vp]
    i64, u64, f64 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.wo_cnn_param_count.restype = i64
    lib.wo_cnn_workspace_size.argtypes = [i32, i32, i32, i32]
    lib.wo_cnn_workspace_size.restype = sz
    lib.wo_cnn_forward.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, sz, vp]
    lib.wo_cnn_gradient.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp, vp, vp, vp, sz, vp]
    lib.wo_cnn_train_step.argtypes = [vp, vp, vp, i32, f64, f64, vp, vp, i32, i32, i32, i32, vp, vp, vp,
                                      sz, vp]
    lib.wo_cnn_prior.argtypes = [dp, dp]
    lib.wo_cnn_prior.restype = None
    lib.wo_cnn_init_workspace_size.argtypes = [i32]
    lib.wo_cnn_init_workspace_size.restype = sz
    lib.wo_cnn_init_theta.argtypes = [vp, op, i32, vp, dp, vp, sz, vp]
    conv = [vp, vp, i32, i32, i32, i32, i32, i32, vp]
    lib.wo_conv3d_forward.argtypes = conv + [vp]
    lib.wo_conv3d_input_grad.argtypes = conv + [vp]
    lib.wo_conv3d_weight_grad.argtypes = conv + [vp, sz, vp]
    lib.wo_synth_thin_cells.argtypes = [vp, i32, i32, i32, f64, i32, u64, vp]
    lib.wo_add_gaussian_noise.argtypes = [vp, i64, f64, u64, vp]
    i32p = ctypes.POINTER(i32)
    lib.wo_tile_grid.argtypes = [i32, i32, i32, i32p, i32p]
    lib.wo_stitch_tiles.argtypes = [vp, i32, i32, i32, i32, i32, i32p, i32p, i32, i32, vp, vp]
    szp = ctypes.POINTER(ctypes.c_size_t)
    lib.wo_fft_tune.argtypes = [i32, op, i32, vp, vp, vp, f64, i32, vp, sz, vp]
    lib.wo_fft_plans_export.argtypes = [ctypes.c_char_p, sz, szp]
    lib.wo_fft_plans_import.argtypes = [ctypes.c_char_p]
    lib.wo_fft_candidates.argtypes = [ctypes.c_char_p, ctypes.c_char_p, sz, szp]
    lib.wo_crop_stacks.argtypes = [vp, i32, i32, i32, i32, vp, i32, i32, i32, i32, i32, i32, vp, vp]
    lib.wo_timing_enable.argtypes = [ctypes.c_int]
    lib.wo_timing_report.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    lib.wo_timing_select.argtypes = [ctypes.c_char_p]
    for name in SYMBOLS:
        getattr(lib, name)
    _lib = lib
    return lib


def _get(o, name):
    return o[name] if isinstance(o, dict) else getattr(o, name)


def optics_array(optics) -> ctypes.Array:
    """ctypes array of wo_optics from one optics object or a sequence of them."""
    if not isinstance(optics, (list, tuple)):
        optics = [optics]
    arr = (WoOptics * len(optics))()
    for i, o in enumerate(optics):
        for f in _FIELDS:
            setattr(arr[i], f, int(_get(o, f)) if f in ("model", "nz", "ny", "nx") else float(_get(o, f)))
        z = getattr(o, "zernike", None)
        if z is None and isinstance(o, dict):
            z = o.get("zernike")
        z = tuple(z) if z is not None else ()
        if len(z) > N_ZERNIKE:
            raise ValueError(f"at most {N_ZERNIKE} Zernike coefficients (Noll 5..11)")
        for j in range(N_ZERNIKE):
            arr[i].zernike[j] = float(z[j]) if j < len(z) else 0.0
        for f in ("det_tilt", "det_azimuth"):
            v = o.get(f, 0.0) if isinstance(o, dict) else getattr(o, f, 0.0)
            setattr(arr[i], f, float(v))

        def opt(f, default):
            return o.get(f, default) if isinstance(o, dict) else getattr(o, f, default)

        arr[i].vec_channels = int(opt("vec_channels", 0))
        props = tuple(int(p) for p in opt("vec_props", (0, 16, 8, 1)))
        if len(props) > 8:
            raise ValueError("at most 8 vector-model properties")
        arr[i].vec_nprops = len(props)
        for k in range(8):
            arr[i].vec_props[k] = props[k] if k < len(props) else 0
        jx, jy = (complex(v) for v in opt("ill_jones", (2 ** -0.5, 1j * 2 ** -0.5)))
        for k, v in enumerate((jx.real, jx.imag, jy.real, jy.imag)):
            arr[i].ill_jones[k] = v
    return arr


def _check(status: int, where: str):
    if status != 0:
        raise WoError(status, where)


def bank_shape(optics):
    """(C, P, dims, complex elements per patch) of the model's bank."""
    lib = load()
    arr = optics_array(optics)
    C, P, dims = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    n = ctypes.c_int64()
    _check(lib.wo_bank_shape(arr, ctypes.byref(C), ctypes.byref(P), ctypes.byref(dims), ctypes.byref(n)),
           "wo_bank_shape")
    return C.value, P.value, dims.value, n.value


def lateral_support(optics):
    """Lateral support of the model for these patches (wo_lateral_support) as a dict:
    field_cols (A, B), tf_cols, band_rows, tf_lengths (y, x)."""
    lib = load()
    arr = optics_array(optics)
    out = WoSupport()
    _check(lib.wo_lateral_support(arr, len(arr), ctypes.byref(out)), "wo_lateral_support")
    return {"field_cols": tuple(out.field_cols), "tf_cols": out.tf_cols, "band_rows": out.band_rows,
            "tf_lengths": tuple(out.tf_lengths)}


def workspace_size(optics, op: int) -> int:
    lib = load()
    arr = optics_array(optics)
    return int(lib.wo_workspace_size(arr, len(arr), op))


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _workspace(optics, op, device, ws=None):
    import torch
    need = workspace_size(optics, op)
    if ws is not None and ws.numel() >= need:
        return ws, need
    return torch.empty(max(need, 1), dtype=torch.uint8, device=device), need


def bank_dims(optics):
    """Tensor shape of one call's bank: (n, C, P, [Z,] Y, X/2+1)."""
    arr = optics_array(optics)
    o = arr[0]
    C, P, dims, _ = bank_shape(optics)
    xh = o.nx // 2 + 1
    if dims == 3:
        return (len(arr), C, P, o.nz, o.ny, xh)
    return (len(arr), C, P, o.ny, xh)


def transfer_function(optics, device="cuda", out=None, ws=None, stream=None):
    """TF bank (complex64) for one or more patches; see ``wo_transfer_function``."""
    import torch
    lib = load()
    arr = optics_array(optics)
    shape = bank_dims(optics)
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=device)
    ws, need = _workspace(optics, OP_TRANSFER_FUNCTION, out.device, ws)
    _check(lib.wo_transfer_function(arr, len(arr), _ptr(out), _ptr(ws), ws.numel(), _stream(stream)),
           "wo_transfer_function")
    return out


def _linear(fn, name, optics, tf, x, out_shape, extra, ws, stream, op):
    import torch
    lib = load()
    arr = optics_array(optics)
    out = torch.empty(out_shape, dtype=torch.float32, device=x.device)
    ws, _ = _workspace(optics, op, x.device, ws)
    _check(fn(arr, len(arr), _ptr(tf), _ptr(x), *extra(out), _ptr(ws), ws.numel(), _stream(stream)), name)
    return out


def _vol(optics):
    o = optics_array(optics)[0]
    return (o.ny, o.nx) if o.model == MODEL_LABELFREE_THIN else (o.nz, o.ny, o.nx)


def forward(optics, tf, f, b=None, ws=None, stream=None):
    """d = H f + b; f: (n, P, *vol) float32 -> d: (n, C, *dvol)."""
    arr = optics_array(optics)
    C, P, dims, _ = bank_shape(optics)
    o = arr[0]
    dshape = (len(arr), C, o.ny, o.nx) if dims == 2 else (len(arr), C, o.nz, o.ny, o.nx)
    lib = load()
    return _linear(lib.wo_forward, "wo_forward", optics, tf, f.contiguous(), dshape,
                   lambda out: (_ptr(b), _ptr(out)), ws, stream, OP_FORWARD)


def reconstruct(optics, tf, d, eta, b=None, ws=None, stream=None):
    """Tikhonov reconstruction; d: (n, C, *dvol) -> f: (n, P, *vol)."""
    arr = optics_array(optics)
    C, P, dims, _ = bank_shape(optics)
    fshape = (len(arr), P) + _vol(optics)
    lib = load()
    return _linear(lib.wo_reconstruct, "wo_reconstruct", optics, tf, d.contiguous(), fshape,
                   lambda out: (_ptr(b), ctypes.c_double(eta), _ptr(out)), ws, stream, OP_RECONSTRUCT)


NOALLOC_SCRATCH_BYTES = 64 << 20   # WO_NOALLOC_SCRATCH_BYTES


def reconstruct_noalloc(optics, tf, d, eta, b=None, out=None, stream=None):
    """Tikhonov reconstruction with the library's static scratch instead of a
    workspace (``wo_reconstruct_noalloc``); `out` may be passed to avoid the one
    allocation this binding would otherwise make (the output)."""
    import torch
    lib = load()
    arr = optics_array(optics)
    C, P, dims, _ = bank_shape(optics)
    fshape = (len(arr), P) + _vol(optics)
    if out is None:
        out = torch.empty(fshape, dtype=torch.float32, device=d.device)
    _check(lib.wo_reconstruct_noalloc(arr, len(arr), _ptr(tf), _ptr(d.contiguous()), _ptr(b),
                                      ctypes.c_double(eta), _ptr(out), _stream(stream)),
           "wo_reconstruct_noalloc")
    return out


def reconstruct_grad(optics, d, eta, dL_df, b=None, want_theta=True, want_data=True, ws=None,
                     stream=None):
    """Gradient of a loss of the reconstruction (``wo_reconstruct_grad``): returns
    (dL/dtheta numpy (n, 6) over PARAMS6 or None, dL/dd tensor (n, C, *vol) or None)."""
    import numpy as np
    import torch
    lib = load()
    arr = optics_array(optics)
    n = len(arr)
    need = int(lib.wo_reconstruct_grad_workspace_size(arr, n))
    if need == 0:
        raise WoError(-2, "wo_reconstruct_grad_workspace_size")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=d.device)
    gth = np.zeros((n, 6)) if want_theta else None
    gd = torch.empty_like(d) if want_data else None
    _check(lib.wo_reconstruct_grad(arr, n, _ptr(d.contiguous()), _ptr(b), ctypes.c_double(eta),
                                   _ptr(dL_df.contiguous()),
                                   gth.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if want_theta else None,
                                   _ptr(gd), _ptr(ws), ws.numel(), _stream(stream)), "wo_reconstruct_grad")
    return gth, gd


def band_dims(optics):
    """Tensor shape of one call's bank in the band layout: (n, C, P, Z, band rows, columns);
    the polarisation model's reduced form is the label-free pair, (n, 1, 2, ...)."""
    arr = optics_array(optics)
    C, P, dims, _ = bank_shape(optics)
    if arr[0].model == MODEL_POL5_3D:
        C, P = 1, 2
    sup = lateral_support(optics)
    return (len(arr), C, P, arr[0].nz, sup["band_rows"], sup["tf_cols"])


def pol5_coupling(swing: float):
    """The FP32 coupling kappa (5, 4) complex64 the library uses for this swing."""
    import numpy as np
    out = np.zeros(40, dtype=np.float32)
    _check(load().wo_pol5_coupling(float(swing), out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
           "wo_pol5_coupling")
    return out.view(np.complex64).reshape(5, 4)


def transfer_function_band(optics, device="cuda", out=None, ws=None, stream=None):
    """TF bank on its lateral support (``wo_transfer_function_band``)."""
    import torch
    lib = load()
    arr = optics_array(optics)
    if out is None:
        out = torch.empty(band_dims(optics), dtype=torch.complex64, device=device)
    ws, _ = _workspace(optics, OP_TRANSFER_FUNCTION, out.device, ws)
    _check(lib.wo_transfer_function_band(arr, len(arr), _ptr(out), _ptr(ws), ws.numel(), _stream(stream)),
           "wo_transfer_function_band")
    return out


def linear_band(op, optics, tf_band, x, eta=0.0, b=None, ws=None, stream=None):
    """Forward, reconstruction or adjoint (op OP_FORWARD / OP_RECONSTRUCT / OP_ADJOINT)
    with a band-layout bank (``wo_linear_band``)."""
    import torch
    lib = load()
    arr = optics_array(optics)
    C, P, dims, _ = bank_shape(optics)
    nout = C if op == OP_FORWARD else P
    out = torch.empty((len(arr), nout) + _vol(optics), dtype=torch.float32, device=x.device)
    ws, _ = _workspace(optics, op, x.device, ws)
    _check(lib.wo_linear_band(op, arr, len(arr), _ptr(tf_band), _ptr(x.contiguous()), _ptr(b),
                              ctypes.c_double(eta), _ptr(out), _ptr(ws), ws.numel(), _stream(stream)),
           "wo_linear_band")
    return out


def adjoint(optics, tf, r, ws=None, stream=None):
    """g = H^H r; r: (n, C, *dvol) -> g: (n, P, *vol)."""
    arr = optics_array(optics)
    C, P, dims, _ = bank_shape(optics)
    gshape = (len(arr), P) + _vol(optics)
    lib = load()
    return _linear(lib.wo_adjoint, "wo_adjoint", optics, tf, r.contiguous(), gshape,
                   lambda out: (_ptr(out),), ws, stream, OP_ADJOINT)


def timing_enable(on: bool = True):
    """Bracket every library kernel launch with HIP events (instrumentation)."""
    load().wo_timing_enable(1 if on else 0)


def timing_select(name=None):
    """Restrict the timing events to one kernel name (None: every kernel)."""
    _check(load().wo_timing_select(name.encode() if name else None), "wo_timing_select")


def timing_report() -> dict:
    """{kernel: (launches, total_ms)} since the last report; waits for the events."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(load().wo_timing_report(buf, len(buf)), "wo_timing_report")
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


# ---------------------------------------------------------------- auto-tune (thin model)

PARAMS = ("defocus", "na_det", "tilt_zenith", "tilt_azimuth")
PARAMS6 = PARAMS + ("det_tilt", "det_azimuth")
PAPER_LR = (0.02, 0.005, 0.005, 0.001)   # um, NA (proposed), rad, rad


def _dbl(values):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(values, dtype=np.float64))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def tune_workspace_size(optics, starts: int = 1) -> int:
    arr = optics_array(optics)
    return int(load().wo_tune_workspace_size(arr, len(arr), starts))


def pack_stacks(stacks):
    """One contiguous float32 device tensor from a [n, Z, Y, X] tensor or a list of
    [Z_i, Y_i, X_i] tensors (uneven tiles), patch after patch."""
    import torch
    if isinstance(stacks, (list, tuple)):
        return torch.cat([s.contiguous().reshape(-1) for s in stacks])
    return stacks.contiguous()


def midband_loss_grad(optics, d, eta, nu_c=None, ws=None, stream=None, aberration=False):
    """Mid-band loss and dL/dtheta per patch (numpy arrays (n,), (n, 4)); `d` as in
    pack_stacks (patches may differ in shape).  aberration=True: (n, 11), theta then
    the seven Zernike coefficients (wo_midband_loss_grad_aberration)."""
    import numpy as np
    import torch
    lib = load()
    arr = optics_array(optics)
    n = len(arr)
    d = pack_stacks(d)
    need = tune_workspace_size(optics, 1)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=d.device)
    eta_a, eta_p = _dbl(np.broadcast_to(eta, (n,)))
    nu_a, nu_p = _dbl(np.zeros(n) if nu_c is None else np.broadcast_to(nu_c, (n,)))
    loss = np.zeros(n)
    grad = np.zeros((n, 4 + N_ZERNIKE if aberration else 4))
    fn = lib.wo_midband_loss_grad_aberration if aberration else lib.wo_midband_loss_grad
    _check(fn(arr, n, _ptr(d), eta_p, nu_p, loss.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
              grad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(ws), ws.numel(),
              _stream(stream)), "wo_midband_loss_grad")
    return loss, grad


def _tune_call(fn, name, optics, d, eta, iters, lr, lo, hi, mask, multistart, theta0, nu_c, use_graph,
               branches, ws, stream, extra, lr_zernike=0.0, zernike_bound=0.0, status=None):
    import copy
    import numpy as np
    import torch
    optics = list(optics) if isinstance(optics, (list, tuple)) else [optics]
    arr = optics_array(optics)
    n = len(arr)
    M = int(multistart)
    d = pack_stacks(d)
    need = tune_workspace_size(optics, M)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=d.device)
    opts = WoAutotuneOpts()
    opts.iters, opts.multistart, opts.use_graph, opts.tune_mask = int(iters), M, int(use_graph), int(mask)
    opts.branches = int(branches)
    opts.lr_zernike, opts.zernike_bound = float(lr_zernike), float(zernike_bound)
    for j in range(4):
        opts.lr[j], opts.lo[j], opts.hi[j] = float(lr[j]), float(lo[j]), float(hi[j])
    keep = []
    if theta0 is not None:
        a, p = _dbl(np.reshape(theta0, (n * M * 4,)))
        keep.append(a)
        opts.theta0 = p
    if nu_c is not None:
        a, p = _dbl(np.broadcast_to(nu_c, (n,)))
        keep.append(a)
        opts.nu_c = p
    all_theta = np.zeros((n, M, 4))
    all_loss = np.zeros((n, M))
    opts.all_theta_out = all_theta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    opts.all_loss_out = all_loss.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if status is not None:
        if status.dtype != np.int32 or status.size < n or not status.flags["C_CONTIGUOUS"]:
            raise ValueError("status must be a contiguous int32 array of n entries")
        opts.status_out = status.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    eta_a, eta_p = _dbl(np.broadcast_to(eta, (n,)))
    loss = np.zeros(n)
    _check(fn(arr, n, _ptr(d), eta_p, ctypes.byref(opts),
              loss.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), *extra, _ptr(ws), ws.numel(),
              _stream(stream)), name)
    out = []
    for i, o in enumerate(optics):
        oo = copy.copy(o)
        for f in PARAMS:
            if isinstance(oo, dict):
                oo[f] = getattr(arr[i], f)
            else:
                setattr(oo, f, getattr(arr[i], f))
        if (int(mask) >> 4) & 0x7F:
            z = tuple(float(arr[i].zernike[j]) for j in range(N_ZERNIKE))
            if isinstance(oo, dict):
                oo["zernike"] = z
            else:
                oo.zernike = z
        out.append(oo)
    return out, loss, all_theta, all_loss


def autotune(optics, d, eta, iters=100, lr=PAPER_LR, lo=(-1e300,) * 4, hi=(1e300,) * 4,
             mask=0b0111, multistart=1, theta0=None, nu_c=None, use_graph=False, branches=0, ws=None,
             stream=None, lr_zernike=0.0, zernike_bound=0.0, status=None):
    """Adam auto-tune of theta for every patch; returns (optics list, loss, all_theta, all_loss).
    `d` as in pack_stacks; use_graph 0/False, 1/True (one iteration replayed) or 2 (one launch).
    mask bits 4..10 also tune the Zernike coefficients (rate lr_zernike, box +-zernike_bound).
    status: optional int32 numpy array (n,) that receives each patch's status (0 or
    WO_DIVERGED = -6)."""
    return _tune_call(load().wo_autotune, "wo_autotune", optics, d, eta, iters, lr, lo, hi, mask,
                      multistart, theta0, nu_c, use_graph, branches, ws, stream, (),
                      lr_zernike, zernike_bound, status)


def restore_tiles(optics, d, eta, iters=20, lr=PAPER_LR, lo=(-1e300,) * 4, hi=(1e300,) * 4,
                  mask=0b0111, multistart=1, theta0=None, nu_c=None, use_graph=2, branches=0,
                  f_out=None, ws=None, stream=None, lr_zernike=0.0, zernike_bound=0.0, status=None):
    """Auto-tune then thin reconstruction of uneven tiles.  Returns (optics list, loss,
    all_theta, all_loss, f) with f a list of [2, Y_i, X_i] views into one packed buffer."""
    import torch
    optics = list(optics) if isinstance(optics, (list, tuple)) else [optics]
    sizes = [2 * int(_get(o, "ny")) * int(_get(o, "nx")) for o in optics]
    d = pack_stacks(d)
    if f_out is None:
        f_out = torch.empty(sum(sizes), dtype=torch.float32, device=d.device)
    lib = load()
    res = _tune_call(lib.wo_restore_tiles, "wo_restore_tiles", optics, d, eta, iters, lr, lo, hi, mask,
                     multistart, theta0, nu_c, use_graph, branches, ws, stream, (_ptr(f_out),),
                     lr_zernike, zernike_bound, status)
    views, off = [], 0
    for o, sz in zip(optics, sizes):
        views.append(f_out[off:off + sz].view(2, int(_get(o, "ny")), int(_get(o, "nx"))))
        off += sz
    return (*res, views)


# ---------------------------------------------------------------- autograd wrappers

def _autograd():
    import torch

    class LinearForward(torch.autograd.Function):
        """d = H f + b with the adjoint kernel as backward: grad_f = H^H grad_d."""

        @staticmethod
        def forward(ctx, f, optics, tf, b):
            ctx.optics, ctx.tf = optics, tf
            return forward(optics, tf, f, b=b)

        @staticmethod
        def backward(ctx, g):
            return adjoint(ctx.optics, ctx.tf, g.contiguous()), None, None, None

    class MidbandLoss(torch.autograd.Function):
        """Mid-band loss of each patch as a function of theta (n, 4) (float64, host);
        backward uses the hand-written transfer-function gradient."""

        @staticmethod
        def forward(ctx, theta, optics, d, eta, nu_c):
            import copy
            opts = []
            for i, o in enumerate(optics):
                oo = copy.copy(o)
                for j, f in enumerate(PARAMS):
                    setattr(oo, f, float(theta[i, j]))
                opts.append(oo)
            loss, grad = midband_loss_grad(opts, d, eta, nu_c)
            ctx.save_for_backward(torch.from_numpy(grad))
            return torch.from_numpy(loss)

        @staticmethod
        def backward(ctx, gout):
            (grad,) = ctx.saved_tensors
            return gout[:, None] * grad, None, None, None, None

    class Reconstruct(torch.autograd.Function):
        """Tikhonov reconstruction f(d, theta) of a 3D model with theta (n, 4) or
        (n, 6) (float64, host) the optics' leading PARAMS6 (defocus, na_det,
        tilt_zenith, tilt_azimuth[, det_tilt, det_azimuth]); forward:
        wo_transfer_function + wo_reconstruct at theta; backward:
        wo_reconstruct_grad (dL/dd and dL/dtheta, the bank recomputed)."""

        @staticmethod
        def forward(ctx, d, theta, optics, eta, b):
            import copy
            opts = []
            for i, o in enumerate(optics):
                oo = copy.copy(o)
                for j, f in enumerate(PARAMS6[: theta.shape[1]]):
                    setattr(oo, f, float(theta[i, j]))
                opts.append(oo)
            ctx.opts, ctx.eta, ctx.b, ctx.k = opts, eta, b, theta.shape[1]
            ctx.save_for_backward(d)
            tf = transfer_function(opts, device=d.device)
            return reconstruct(opts, tf, d, eta, b=b)

        @staticmethod
        def backward(ctx, g):
            (d,) = ctx.saved_tensors
            gth, gd = reconstruct_grad(ctx.opts, d, ctx.eta, g.contiguous(), b=ctx.b,
                                       want_theta=ctx.needs_input_grad[1],
                                       want_data=ctx.needs_input_grad[0])
            return (gd, None if gth is None else torch.from_numpy(gth[:, :ctx.k]), None, None, None)

    return LinearForward, MidbandLoss, Reconstruct


def linear_forward_fn(f, optics, tf, b=None):
    """Differentiable forward model (backward = wo_adjoint)."""
    return _autograd()[0].apply(f, optics, tf, b)


def midband_loss_fn(theta, optics, d, eta, nu_c=None):
    """Differentiable mid-band loss in theta (backward = hand-written TF gradient)."""
    return _autograd()[1].apply(theta, optics, d, eta, nu_c)


def reconstruct_fn(d, theta, optics, eta, b=None):
    """Differentiable 3D reconstruction in the data d and theta (n, 4) (backward =
    wo_reconstruct_grad)."""
    return _autograd()[2].apply(d, theta, optics, eta, b)


# ---------------------------------------------------------------- CNN and training data

def cnn_param_count() -> int:
    return int(load().wo_cnn_param_count())


def cnn_workspace(batch, shape, device):
    import torch
    n = int(load().wo_cnn_workspace_size(batch, *shape))
    return torch.empty(n, dtype=torch.uint8, device=device)


def cnn_prior():
    """(lo, hi) of the prior box the network's outputs are normalised over
    (defocus um, NA_det, tilt_zenith rad)."""
    import numpy as np
    lo, hi = (ctypes.c_double * 3)(), (ctypes.c_double * 3)()
    load().wo_cnn_prior(lo, hi)
    return np.array(lo[:]), np.array(hi[:])


def cnn_init_theta(params, optics, stacks, ws=None, stream=None):
    """Starting theta (n, 4) of the auto-tune from the network (``wo_cnn_init_theta``):
    stacks as in pack_stacks, patches of any shape."""
    import numpy as np
    import torch
    lib = load()
    arr = optics_array(optics)
    d = pack_stacks(stacks)
    if ws is None:
        ws = torch.empty(int(lib.wo_cnn_init_workspace_size(len(arr))), dtype=torch.uint8, device=d.device)
    out = np.zeros((len(arr), 4))
    _check(lib.wo_cnn_init_theta(_ptr(params), arr, len(arr), _ptr(d),
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(ws), ws.numel(),
                                 _stream(stream)), "wo_cnn_init_theta")
    return out


def cnn_forward(params, x, ws=None, stream=None):
    """y = CNN(x): params FP32 flat (device), x (batch, Z, Y, X) FP32 -> (batch, 3)."""
    import torch
    x = x.contiguous()
    B = x.shape[0]
    if ws is None:
        ws = cnn_workspace(B, x.shape[1:], x.device)
    y = torch.empty((B, 3), dtype=torch.float32, device=x.device)
    _check(load().wo_cnn_forward(_ptr(params), _ptr(x), B, *x.shape[1:], _ptr(y), _ptr(ws), ws.numel(),
                                 _stream(stream)), "wo_cnn_forward")
    return y


def cnn_gradient(params, x, target, ws=None, stream=None):
    """(y, loss, grad) of the MSE loss for a batch."""
    import torch
    x = x.contiguous()
    B = x.shape[0]
    if ws is None:
        ws = cnn_workspace(B, x.shape[1:], x.device)
    y = torch.empty((B, 3), dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    grad = torch.empty_like(params)
    _check(load().wo_cnn_gradient(_ptr(params), _ptr(x), _ptr(target.contiguous()), B, *x.shape[1:],
                                  _ptr(y), _ptr(loss), _ptr(grad), _ptr(ws), ws.numel(), _stream(stream)),
           "wo_cnn_gradient")
    return y, loss, grad


def cnn_train_step(params, m, v, t, lr, wd, x, target, ws, y, loss, stream=None):
    _check(load().wo_cnn_train_step(_ptr(params), _ptr(m), _ptr(v), int(t), float(lr), float(wd), _ptr(x),
                                    _ptr(target), x.shape[0], *x.shape[1:], _ptr(y), _ptr(loss), _ptr(ws),
                                    ws.numel(), _stream(stream)), "wo_cnn_train_step")


def conv3d_forward(x_bf16, w_bf16, cout, stream=None):
    """x (N, D, H, W, Cin) and w (Cout, 27*Cin) as int16 BF16 bit patterns -> FP32 output."""
    import torch
    N, D, H, W, Cin = x_bf16.shape
    out = torch.empty((N, (D - 1) // 2 + 1, (H - 1) // 2 + 1, (W - 1) // 2 + 1, cout),
                      dtype=torch.float32, device=x_bf16.device)
    _check(load().wo_conv3d_forward(_ptr(x_bf16), _ptr(w_bf16), N, D, H, W, Cin, cout, _ptr(out),
                                    _stream(stream)), "wo_conv3d_forward")
    return out


def conv3d_input_grad(gz_bf16, w_bf16, in_shape, stream=None):
    import torch
    N, D, H, W, Cin = in_shape
    cout = gz_bf16.shape[-1]
    out = torch.empty(in_shape, dtype=torch.float32, device=gz_bf16.device)
    _check(load().wo_conv3d_input_grad(_ptr(gz_bf16), _ptr(w_bf16), N, D, H, W, Cin, cout, _ptr(out),
                                       _stream(stream)), "wo_conv3d_input_grad")
    return out


def conv3d_weight_grad(x_bf16, gz_bf16, stream=None):
    import torch
    N, D, H, W, Cin = x_bf16.shape
    cout = gz_bf16.shape[-1]
    out = torch.empty((cout, 27 * Cin), dtype=torch.float32, device=x_bf16.device)
    ws = torch.empty(64 << 20, dtype=torch.uint8, device=x_bf16.device)
    _check(load().wo_conv3d_weight_grad(_ptr(x_bf16), _ptr(gz_bf16), N, D, H, W, Cin, cout, _ptr(out),
                                        _ptr(ws), ws.numel(), _stream(stream)), "wo_conv3d_weight_grad")
    return out


def synth_thin_cells(n, ny, nx, pixel, ncells, seed, device="cuda", stream=None):
    import torch
    out = torch.empty((n, 2, ny, nx), dtype=torch.float32, device=device)
    _check(load().wo_synth_thin_cells(_ptr(out), n, ny, nx, float(pixel), int(ncells), int(seed),
                                      _stream(stream)), "wo_synth_thin_cells")
    return out


def add_gaussian_noise(x, sigma, seed, stream=None):
    _check(load().wo_add_gaussian_noise(_ptr(x), x.numel(), float(sigma), int(seed), _stream(stream)),
           "wo_add_gaussian_noise")
    return x


def crop_stacks(x, out_shape, offsets=(0, 0, 0), keep_z=None, out=None, stream=None):
    """Windows (n, oz, oy, ox) of stacks x (n, Z, Y, X) at `offsets`, zero outside the
    input and outside the central keep_z[i] planes (see ``wo_crop_stacks``)."""
    import torch
    n, Z, Y, X = x.shape
    oz, oy, ox = out_shape
    if out is None:
        out = torch.empty((n, oz, oy, ox), dtype=torch.float32, device=x.device)
    keep = None
    if keep_z is not None:
        keep = torch.as_tensor(keep_z, dtype=torch.int32).to(x.device)
    _check(load().wo_crop_stacks(_ptr(x), n, Z, Y, X, _ptr(out), oz, oy, ox, *[int(v) for v in offsets],
                                 _ptr(keep), _stream(stream)), "wo_crop_stacks")
    return out


# ---------------------------------------------------------------- FFT schedule tuner

FFT_TUNE_BAND = 16   # WO_FFT_TUNE_BAND


def fft_tune(op, optics, tf=None, x=None, out=None, eta=0.0, reps=3, ws=None, stream=None, band=False):
    """Time every candidate schedule of the FFT passes of one call (see ``wo_fft_tune``)
    and keep the fastest; `out` and `ws` hold unspecified values afterwards.
    band=True tunes the band-layout variant of the call (tf a band-layout bank)."""
    lib = load()
    arr = optics_array(optics)
    dev = out.device
    ws, _ = _workspace(optics, op, dev, ws)
    _check(lib.wo_fft_tune(int(op) | (FFT_TUNE_BAND if band else 0), arr, len(arr), _ptr(tf), _ptr(x),
                           _ptr(out), float(eta), int(reps), _ptr(ws), ws.numel(), _stream(stream)),
           "wo_fft_tune")


def _text_call(fn, *args):
    need = ctypes.c_size_t(0)
    _check(fn(*args, None, 0, ctypes.byref(need)), fn.__name__)
    buf = ctypes.create_string_buffer(need.value)
    _check(fn(*args, buf, need.value, None), fn.__name__)
    return buf.value.decode()


def fft_plans_export() -> str:
    return _text_call(load().wo_fft_plans_export)


def fft_plans_import(text: str):
    _check(load().wo_fft_plans_import(text.encode()), "wo_fft_plans_import")


def fft_plans_clear():
    _check(load().wo_fft_plans_clear(), "wo_fft_plans_clear")


def fft_candidates(key_line: str) -> list:
    """Schedules (export-format lines) the pass "kind n m batch extra" accepts."""
    return [ln for ln in _text_call(load().wo_fft_candidates, key_line.encode()).splitlines() if ln]


# ---------------------------------------------------------------- field of view

def tile_grid(length: int, count: int, overlap: int):
    """(tile size, starts) along one axis (see ``wo_tile_grid``)."""
    T = ctypes.c_int32(0)
    starts = (ctypes.c_int32 * count)()
    _check(load().wo_tile_grid(int(length), int(count), int(overlap), ctypes.byref(T), starts),
           "wo_tile_grid")
    return T.value, list(starts)


def stitch_tiles(tiles, ys, xs, H, W, out=None, stream=None):
    """Blend tiles (n_y * n_x, P, T_y, T_x) into a (P, H, W) field (see ``wo_stitch_tiles``)."""
    import torch
    tiles = tiles.contiguous()
    n, P, ty, tx = tiles.shape
    if out is None:
        out = torch.empty((P, H, W), dtype=torch.float32, device=tiles.device)
    ya = (ctypes.c_int32 * len(ys))(*ys)
    xa = (ctypes.c_int32 * len(xs))(*xs)
    _check(load().wo_stitch_tiles(_ptr(tiles), len(ys), len(xs), P, ty, tx, ya, xa, int(H), int(W),
                                  _ptr(out), _stream(stream)), "wo_stitch_tiles")
    return out
