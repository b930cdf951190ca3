"""The C-ABI library loads and exports every symbol the header declares (CPU only).

No compute call is made here: the calls below fail argument validation,
which happens on the host before anything is enqueued on a GPU.
"""

import ctypes
import os
import re

import pytest

from paper_2412_09775_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "waveorder.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\*\s]+?\b(wo_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(api.LIB_PATH):
        pytest.fail("libwaveorder.so is not built (run __graft_entry__.build())")
    return api.load()


def test_header_declares_the_abi():
    syms = declared_symbols()
    for s in ("wo_transfer_function", "wo_forward", "wo_reconstruct", "wo_adjoint",
              "wo_workspace_size", "wo_bank_shape", "wo_strerror", "wo_version"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    for s in declared_symbols():
        assert hasattr(lib, s), s
    assert set(api.SYMBOLS) == set(declared_symbols())


def _optics(**kw):
    base = dict(model=api.MODEL_LABELFREE_3D, nz=32, ny=64, nx=64, dz=0.2, dy=0.1, dx=0.1,
                wavelength=0.532, na_ill=0.5, na_det=1.2, n_medium=1.33)
    base.update(kw)
    return api.Optics(**base)


def test_bank_shape_and_workspace(lib):
    assert api.bank_shape(_optics()) == (1, 2, 3, 2 * 32 * 64 * 33)
    assert api.bank_shape(_optics(model=api.MODEL_POL5_3D, na_det=0.75))[:3] == (5, 4, 3)
    assert api.bank_shape(_optics(model=api.MODEL_LABELFREE_THIN))[:3] == (32, 2, 2)
    assert api.bank_shape(_optics(model=api.MODEL_FLUOR_3D))[:3] == (1, 1, 3)
    ws = api.workspace_size(_optics(), api.OP_RECONSTRUCT)
    assert ws >= 2 * 32 * 64 * 33 * 8
    assert api.workspace_size([_optics()] * 3, api.OP_RECONSTRUCT) >= 3 * 2 * 32 * 64 * 33 * 8


@pytest.mark.parametrize("kw,status", [
    (dict(na_det=1.4), -1),                 # pupil beyond the shell n / lambda0
    (dict(dx=0.2, dy=0.2), -5),             # lateral aliasing
    (dict(dz=0.5), -5),                     # axial aliasing
    (dict(nx=70), -2),                      # 7 is not a supported radix
    (dict(ny=45), -2),                      # odd size
    (dict(wavelength=-1.0), -1),
    (dict(tilt_zenith=1.2), -1),            # tilted source leaves the shell
])
def test_invalid_optics_are_rejected_before_any_gpu_work(lib, kw, status):
    arr = api.optics_array(_optics(**kw))
    st = lib.wo_transfer_function(arr, 1, ctypes.c_void_p(1), ctypes.c_void_p(1), 1 << 40, None)
    assert st == status


def test_null_and_small_workspace_are_rejected(lib):
    arr = api.optics_array(_optics())
    assert lib.wo_transfer_function(arr, 1, None, None, 0, None) == -1
    assert lib.wo_transfer_function(arr, 1, ctypes.c_void_p(1), ctypes.c_void_p(1), 16, None) == -3
    assert lib.wo_reconstruct(arr, 1, ctypes.c_void_p(1), ctypes.c_void_p(1), None, -1.0,
                              ctypes.c_void_p(1), ctypes.c_void_p(1), 1 << 40, None) == -1
    assert lib.wo_reconstruct(arr, 1, ctypes.c_void_p(1), ctypes.c_void_p(1), None, 0.0,
                              ctypes.c_void_p(1), ctypes.c_void_p(1), 1 << 40, None) == -2
    # an empty batch is rejected, not treated as a no-op
    assert lib.wo_transfer_function(arr, 0, ctypes.c_void_p(1), ctypes.c_void_p(1), 1 << 40, None) == -1
    assert lib.wo_reconstruct(arr, 0, ctypes.c_void_p(1), ctypes.c_void_p(1), None, 1e-3,
                              ctypes.c_void_p(1), ctypes.c_void_p(1), 1 << 40, None) == -1
    assert lib.wo_tune_workspace_size(arr, 0, 1) == 0
    big = api.optics_array(_optics(nx=8192))        # beyond the 4096 limit
    assert lib.wo_transfer_function(big, 1, ctypes.c_void_p(1), ctypes.c_void_p(1), 1 << 40, None) == -2
    # detection aberrations: finite coefficients only
    bad = _optics(zernike=(float("nan"),))
    assert lib.wo_transfer_function(api.optics_array(bad), 1, ctypes.c_void_p(1), ctypes.c_void_p(1),
                                    1 << 40, None) == -1
    with pytest.raises(ValueError):
        api.optics_array(_optics(zernike=(0.1,) * 8))     # at most Noll 5..11
    # one Z line of both properties must fit a workgroup of the fused Z pass
    deep = api.optics_array(_optics(model=api.MODEL_POL5_3D, nz=2048))   # 5 x 2048 > 8192
    assert lib.wo_reconstruct(deep, 1, ctypes.c_void_p(1), ctypes.c_void_p(1), None, 1e-3,
                              ctypes.c_void_p(1), ctypes.c_void_p(1), 1 << 40, None) == -2
    mixed = api.optics_array([_optics(), _optics(nz=16)])
    assert lib.wo_forward(mixed, 2, ctypes.c_void_p(1), ctypes.c_void_p(1), None,
                          ctypes.c_void_p(1), ctypes.c_void_p(1), 1 << 40, None) == -1
    assert lib.wo_strerror(-5).decode().startswith("transfer-function support")


def test_fft_schedule_table_host_logic(lib):
    """Candidate enumeration, import validation and export round trip (host only)."""
    api.fft_plans_clear()
    for key, n in (("cols 96 41 48 0", 96), ("rows_r2c 80 0 2304 0", 80), ("zop 24 3936 1 2011", 24)):
        cands = api.fft_candidates(key)
        assert len(cands) >= 2 and len(set(cands)) == len(cands)
        for ln in cands:
            f = ln.split()
            assert " ".join(f[:5]) == key
            w, thr, plan = map(int, f[5:])
            assert 64 <= thr <= 1024 and thr % 64 == 0 and w >= 1
            # plan 4: the column tile loop, compiled lengths at the compiled width only
            assert 0 <= plan <= 3 or (plan == 4 and key.startswith("cols 96 ") and w == 16)
    # 80 = 8*2*5 has three distinct radix orders; 96 = 8*4*3 also; 24 = 8*3 two
    assert {int(ln.split()[-1]) for ln in api.fft_candidates("rows_r2c 80 0 2304 0")} == {0, 2, 3}
    assert {int(ln.split()[-1]) for ln in api.fft_candidates("zop 24 3936 1 2011")} == {0, 2}
    assert 4 in {int(ln.split()[-1]) for ln in api.fft_candidates("cols 96 41 48 0")}
    pick = api.fft_candidates("cols 96 41 48 0")[-1]
    api.fft_plans_import(pick)
    assert api.fft_plans_export() == pick + "\n"
    for bad in ("cols 96 41 48 0 64 64 0",       # 64 x 96 elements need 768 threads or more
                "cols 96 41 48 0 1 100 0",       # not a multiple of 64
                "zop 24 3936 1 2011 1 64 7",     # no such plan
                "zop 24 3936 1 2011 1 64 4",     # the tile loop is a column schedule
                "cols 96 41 48 0 8 192 4",       # the tile loop runs the compiled width only
                "nonsense 1 2 3"):
        with pytest.raises(api.WoError):
            api.fft_plans_import(bad)
    assert api.fft_plans_export() == pick + "\n"   # a rejected import changes nothing
    api.fft_plans_clear()
    assert api.fft_plans_export() == ""


def test_tile_grid_host_logic_matches_the_oracle(lib):
    from oracle import stitch
    for args in [(2048, 6, 410), (1000, 5, 25), (300, 1, 0), (130, 2, 0), (2048, 6, 82), (120, 2, 20)]:
        assert api.tile_grid(*args) == stitch.tile_grid(*args)
    with pytest.raises(api.WoError):
        api.tile_grid(100, 2, 200)          # tiles would not fit


def test_support_and_band_calls_validate_on_the_host(lib):
    """wo_lateral_support, wo_transfer_function_band and wo_linear_band reject bad
    arguments before any GPU work (fake device pointers are never touched)."""
    one = ctypes.c_void_p(1)
    arr = api.optics_array(_optics())
    assert lib.wo_lateral_support(arr, 1, None) == -1
    assert lib.wo_lateral_support(api.optics_array(_optics(na_det=1.4)), 1, ctypes.byref(api.WoSupport())) == -1
    # band synthesis: label-free 3D only (unless the support fills the grid)
    thin = api.optics_array(_optics(model=api.MODEL_LABELFREE_THIN))
    assert lib.wo_transfer_function_band(thin, 1, one, one, 1 << 40, None) == -2
    # the polarisation model's band layout is its reduced form (validated, then the
    # workspace check fails before any GPU work)
    pol5 = api.optics_array(_optics(model=api.MODEL_POL5_3D, na_det=0.75, ny=128, nx=128))
    assert lib.wo_transfer_function_band(pol5, 1, one, one, 16, None) == -3
    assert lib.wo_transfer_function_band(arr, 1, None, one, 1 << 40, None) == -1
    assert lib.wo_transfer_function_band(arr, 1, one, one, 16, None) == -3
    # band linear calls: forward, reconstruction or adjoint of a 3D model
    assert lib.wo_linear_band(api.OP_TRANSFER_FUNCTION, arr, 1, one, one, None, 1e-3, one, one, 1 << 40,
                              None) == -1
    assert lib.wo_linear_band(api.OP_RECONSTRUCT, thin, 1, one, one, None, 1e-3, one, one, 1 << 40,
                              None) == -2
    assert lib.wo_linear_band(api.OP_RECONSTRUCT, arr, 1, one, one, None, -1.0, one, one, 1 << 40,
                              None) == -1
    assert lib.wo_linear_band(api.OP_RECONSTRUCT, arr, 1, one, one, None, 0.0, one, one, 1 << 40,
                              None) == -2
    assert lib.wo_linear_band(api.OP_ADJOINT, arr, 1, one, one, None, 0.0, one, one, 16, None) == -3


def test_noalloc_reconstruction_validates_on_the_host(lib):
    """wo_reconstruct_noalloc rejects inputs whose scratch would exceed the static
    array, and bad arguments, before any GPU work (fake pointers never touched)."""
    one = ctypes.c_void_p(1)
    big = api.optics_array(_optics(nz=96, ny=512, nx=512))
    assert api.workspace_size(_optics(nz=96, ny=512, nx=512), api.OP_RECONSTRUCT) > api.NOALLOC_SCRATCH_BYTES
    assert lib.wo_reconstruct_noalloc(big, 1, one, one, None, 1e-3, one, None) == -3
    arr = api.optics_array(_optics())
    assert lib.wo_reconstruct_noalloc(arr, 1, None, one, None, 1e-3, one, None) == -1
    assert lib.wo_reconstruct_noalloc(arr, 1, one, one, None, -1.0, one, None) == -1
    assert lib.wo_reconstruct_noalloc(arr, 1, one, one, None, 0.0, one, None) == -2   # P = 2 needs eta > 0
    assert lib.wo_reconstruct_noalloc(arr, 0, one, one, None, 1e-3, one, None) == -1


def test_pol5_coupling_is_the_oracle_coupling_in_fp32(lib):
    """wo_pol5_coupling (host only) returns the oracle's kappa rounded to FP32: within
    one FP32 rounding (the two FP64 evaluations differ by a few FP64 ulps, which can
    move a value across an FP32 rounding boundary or leave 1e-17 where 0 is exact)."""
    import numpy as np
    from oracle import tf as tfm
    for swing in (0.0, 0.03, 0.1, 0.25):
        got = api.pol5_coupling(swing).astype(np.complex128)
        ref = tfm.pol5_coupling(swing)
        for g, r in ((got.real, ref.real), (got.imag, ref.imag)):
            assert np.all(np.abs(g - r) <= 2.0 ** -24 * np.abs(r) + 1e-15)
    assert lib.wo_pol5_coupling(float("nan"), None) == -1


def test_cnn_start_validates_on_the_host_and_shares_the_prior(lib):
    """wo_cnn_prior is learned_init's prior box; wo_cnn_init_theta rejects bad
    arguments before any GPU work (fake pointers never touched)."""
    import numpy as np
    from paper_2412_09775_amd import learned_init
    lo, hi = api.cnn_prior()
    assert np.array_equal(lo, learned_init.PRIOR_LO) and np.array_equal(hi, learned_init.PRIOR_HI)
    assert lib.wo_cnn_init_workspace_size(0) == 0
    need = lib.wo_cnn_init_workspace_size(3)
    assert need > 3 * 32 * 64 * 64 * 4
    one = ctypes.c_void_p(1)
    arr = api.optics_array([_optics()] * 3)
    out = (ctypes.c_double * 12)()
    assert lib.wo_cnn_init_theta(None, arr, 3, one, out, one, need, None) == -1
    assert lib.wo_cnn_init_theta(one, arr, 0, one, out, one, need, None) == -1
    assert lib.wo_cnn_init_theta(one, arr, 3, one, out, one, need - 1, None) == -3


def test_nine_aperture_validity_is_the_oracles_lit_criterion(lib):
    """The 9-aperture model needs light in every sector: sum S_c P^2 > 0 for c < 8
    (oracle pupils).  The library checks it on the host (scanning only the source
    disc's bounding box); wo_lateral_support reports it (WO_EINVAL when unlit)."""
    import numpy as np
    from oracle import optics as op
    cases = [dict(na_ill=0.5), dict(na_ill=0.05), dict(na_ill=0.12, tilt_zenith=0.3, tilt_azimuth=0.7),
             dict(na_ill=0.4, det_tilt=0.25, det_azimuth=-0.6, na_det=0.9), dict(na_ill=0.02, edge_width=0.5)]
    seen = set()
    for kw in cases:
        base = dict(model=op.SECTORS9_3D, nz=8, ny=64, nx=48, dz=0.2, dy=0.1, dx=0.1, wavelength=0.532,
                    na_ill=0.5, na_det=1.2, n_medium=1.33)
        base.update(kw)
        oo = op.Optics(**base)
        P = op.detection_pupil(oo)
        lit = all(np.sum(op.sector_pupil(oo, c) * P * P) > 0 for c in range(8))
        ao = api.Optics(**{k: v for k, v in base.items()})
        out = api.WoSupport()
        st = lib.wo_lateral_support(api.optics_array([ao]), 1, ctypes.byref(out))
        assert (st == 0) == lit, (kw, st, lit)
        seen.add(lit)
    assert seen == {True, False}


def test_vector_model_shape_and_validation_on_the_host(lib):
    """The vector model's bank shape follows its channel set and property list;
    malformed channel sets, property codes, Jones vectors and oblique detection
    are rejected before any GPU work, as are mixed property lists in one call and
    property counts the linear calls do not implement."""
    v = dict(model=api.MODEL_VECTOR_3D, na_det=1.2)
    assert api.bank_shape(_optics(**v))[:3] == (4, 4, 3)
    assert api.bank_shape(_optics(vec_channels=1, vec_props=(0, 1), **v))[:3] == (5, 2, 3)
    assert api.bank_shape(_optics(vec_props=tuple(range(8)), **v))[:3] == (4, 8, 3)
    one = ctypes.c_void_p(1)

    def tf_status(o):
        return lib.wo_transfer_function(api.optics_array(o), 1 if not isinstance(o, list) else len(o), one, one,
                                        1 << 40, None)

    assert tf_status(_optics(vec_channels=2, **v)) == -1
    assert tf_status(_optics(vec_props=(0, 18), **v)) == -1
    assert tf_status(_optics(vec_props=(-1,), **v)) == -1
    assert tf_status(_optics(vec_props=(), **v)) == -1
    assert tf_status(_optics(ill_jones=(float("nan"), 1.0), **v)) == -1
    assert tf_status(_optics(det_tilt=0.2, **dict(v, na_det=0.8))) == -2
    assert tf_status([_optics(**v), _optics(vec_props=(0, 16, 8, 2), **v)]) == -1
    with pytest.raises(ValueError):
        api.optics_array(_optics(vec_props=tuple(range(9)), **v))
    three = api.optics_array(_optics(vec_props=(0, 16, 8), **v))
    assert lib.wo_reconstruct(three, 1, one, one, None, 1e-3, one, one, 1 << 40, None) == -2
    assert lib.wo_forward(three, 1, one, one, None, one, one, 1 << 40, None) == -2
    ws = api.workspace_size(_optics(**v), api.OP_TRANSFER_FUNCTION)
    assert ws >= 16 * 4 * 32 * 64 * 64                      # the 16 real responses of the synthesis
