"""C-ABI contract tests that need no GPU: the library loads, exports every
entry point the header declares, its host-side trajectory helpers agree with
the oracle's own geometry, and invalid arguments are rejected with the
documented status codes before any HIP call."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pyrohip.h")


@pytest.fixture(scope="module")
def ph():
    import paper_1904_13342_amd as ph
    return ph


@pytest.fixture(scope="module")
def L(ph):
    from paper_1904_13342_amd._lib import lib
    return lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ph_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for expected in ("ph_project_par2d", "ph_project_fan2d", "ph_project_cone3d", "ph_backproject_par2d",
                     "ph_backproject_fan2d", "ph_backproject_cone3d", "ph_fdk_cone3d", "ph_fbp_par2d",
                     "ph_fbp_fan2d", "ph_weight_filter_3d"):
        assert expected in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_covers_every_symbol(ph):
    from paper_1904_13342_amd._lib import SIGNATURES
    assert set(declared_functions()) <= set(SIGNATURES)


def test_status_strings(L):
    assert L.ph_status_string(0) == b"ok"
    for s in range(-8, 0):
        assert L.ph_status_string(s) not in (b"ok", b"unknown status")
    assert b"gfx950" in L.ph_version()


def test_ray_vectors_match_angles(ph):
    spec = synth.config("fan2d_512")
    g = ph.from_spec(spec)
    rv = ph.ray_vectors_2d(g)
    beta = spec.angular_range * np.arange(spec.n_proj) / spec.n_proj
    # the range travels as FP32 (2 pi rounds by 1.7e-7 relative)
    np.testing.assert_allclose(rv[:, 0], np.cos(beta), atol=3e-7)
    np.testing.assert_allclose(rv[:, 1], np.sin(beta), atol=3e-7)


@pytest.mark.parametrize("name", ["cone3d_256_short", "cone3d_512", "cone3d_crop32"])
def test_projection_matrices_match_oracle(ph, ora, name):
    """The library's FP32 matrices equal the oracle's FP64 ones to FP32
    rounding; the oracle's are pinned to the geometry in the oracle tests."""
    spec = synth.config(name)
    P = ph.projection_matrices_3d(ph.from_spec(spec)).astype(np.float64)
    R = ora.projection_matrices(spec)
    scale = np.abs(R).max(axis=(1, 2), keepdims=True)
    assert np.max(np.abs(P - R) / scale) < 1e-6


# ------------------------------------------------------------ validation

FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first


def _call3(L, g, mats=None, vol=FAKE, proj=FAKE, batch=1, dtype=0, fn="ph_project_cone3d"):
    m = mats if mats is not None else np.zeros((g.n_proj, 3, 4), np.float32)
    return getattr(L, fn)(ctypes.byref(g), m.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), vol, proj, batch,
                          dtype, None)


def _good3(ph):
    return ph.from_spec(synth.config("cone3d_crop32"))


def test_rejects_null_and_shape(ph, L):
    g = _good3(ph)
    mats = ph.projection_matrices_3d(g)
    assert _call3(L, g, mats, vol=None) == -1
    assert _call3(L, g, mats, proj=None) == -1
    assert L.ph_project_cone3d(None, None, FAKE, FAKE, 1, 0, None) == -1
    assert _call3(L, g, mats, batch=0) == -2
    bad = _good3(ph)
    bad.vol_shape[0] = 0
    assert _call3(L, bad, mats) == -2
    bad = _good3(ph)
    bad.det_shape[1] = -3
    assert _call3(L, bad, mats) == -2


def test_rejects_dtype(ph, L):
    g = _good3(ph)
    assert _call3(L, g, ph.projection_matrices_3d(g), dtype=7) == -4


@pytest.mark.parametrize("field,value", [("sid", 0.0), ("sdd", 100.0), ("sdd", float("nan")),
                                         ("angular_range", -1.0), ("step_mm", float("inf"))])
def test_rejects_bad_geometry_scalars(ph, L, field, value):
    g = _good3(ph)
    mats = ph.projection_matrices_3d(g)
    setattr(g, field, value)
    assert _call3(L, g, mats) == -3


def test_rejects_bad_spacing(ph, L):
    g = _good3(ph)
    mats = ph.projection_matrices_3d(g)
    g.vol_spacing[1] = 0.0
    assert _call3(L, g, mats) == -3


def test_rejects_singular_or_nonfinite_matrix(ph, L):
    g = _good3(ph)
    mats = ph.projection_matrices_3d(g)
    m = mats.copy()
    m[3, :, 2] = 0.0   # singular 3x3 part
    assert _call3(L, g, m) == -3
    assert _call3(L, g, m, fn="ph_backproject_cone3d") == -3
    m = mats.copy()
    m[5, 1, 1] = np.nan
    assert _call3(L, g, m) == -3


def test_rejects_source_inside_volume(ph, L):
    spec = synth.config("cone3d_crop32").with_(vol_shape=(32, 32, 32), vol_spacing=(40.0, 40.0, 40.0))
    g = ph.from_spec(spec)   # 1280 mm wide volume around a 750 mm source circle
    assert _call3(L, g, ph.projection_matrices_3d(g)) == -3
    spec2 = synth.config("fan2d_512").with_(vol_spacing=(4.0, 4.0))
    g2 = ph.from_spec(spec2)
    rv = ph.ray_vectors_2d(g2)
    st = L.ph_project_fan2d(ctypes.byref(g2), rv.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), FAKE, FAKE, 1, 0,
                            None)
    assert st == -3


def test_rejects_bad_ray_vectors(ph, L):
    g = ph.from_spec(synth.config("par2d_64"))
    rv = ph.ray_vectors_2d(g)
    rv[7] = 0.0
    st = L.ph_project_par2d(ctypes.byref(g), rv.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), FAKE, FAKE, 1, 0,
                            None)
    assert st == -3


def test_rejects_bad_filter_length_and_workspace(ph, L):
    g = _good3(ph)
    mats = ph.projection_matrices_3d(g)
    fp = mats.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    ws_need = L.ph_fdk_workspace_bytes(ctypes.byref(g), 0, 1, 0)
    assert ws_need >= 360 * 48 * 48 * 4
    # the FP32 filtered projections whatever the filter length and storage type
    for M, dt in ((0, 0), (64, 1), (4096, 2)):
        assert L.ph_fdk_workspace_bytes(ctypes.byref(g), M, 1, dt) == ws_need
    assert L.ph_fdk_workspace_bytes(ctypes.byref(g), 0, 3, 0) == L.ph_workspace_bytes_3d(ctypes.byref(g), 3)
    for M, dt, b in ((100, 0, 1), (32, 0, 1), (8192, 0, 1), (0, 3, 1), (0, 0, 0)):
        assert L.ph_fdk_workspace_bytes(ctypes.byref(g), M, b, dt) == 0, (M, dt, b)
    # too-small workspace
    assert L.ph_fdk_cone3d(ctypes.byref(g), fp, FAKE, FAKE, None, 0, None, None, FAKE, ws_need - 1, 1, 0, None) == -5
    assert L.ph_fdk_cone3d(ctypes.byref(g), fp, FAKE, FAKE, None, 0, None, None, None, ws_need, 1, 0, None) == -5
    # filter lengths: not a power of two, shorter than the row, too long
    for M in (100, 32, 8192):
        st = L.ph_weight_filter_3d(ctypes.byref(g), FAKE, FAKE, FAKE, M, None, None, 1, 0, None)
        assert st == -2, M
    # the default Ram-Lak length must avoid wrap-around
    assert L.ph_weight_filter_3d(ctypes.byref(g), FAKE, FAKE, None, 64, None, None, 1, 0, None) == -2


def test_static_fdk_rejects_before_any_gpu_call(ph, L):
    """ph_fdk_cone3d_static (the FDK that allocates nothing) validates like
    ph_fdk_cone3d and refuses, on the host, sizes its static scratch cannot
    take: one view's filtered projections larger than the scratch, and an
    FP16 / BF16 volume that would need several shares of the views."""
    g = _good3(ph)
    mats = ph.projection_matrices_3d(g)
    fp = mats.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    scratch = 64 << 20
    assert L.ph_fdk_cone3d_static(ctypes.byref(g), fp, None, FAKE, None, 0, None, None, 1, 0, None) == -1
    assert L.ph_fdk_cone3d_static(ctypes.byref(g), fp, FAKE, FAKE, None, 0, None, None, 0, 0, None) == -2
    assert L.ph_fdk_cone3d_static(ctypes.byref(g), fp, FAKE, FAKE, None, 0, None, None, 1, 3, None) == -4
    assert L.ph_fdk_cone3d_static(ctypes.byref(g), fp, FAKE, FAKE, FAKE, 100, None, None, 1, 0, None) == -2
    # one view of a batch too large for the scratch
    per_view = 48 * 48 * 4
    big_batch = scratch // per_view + 1
    assert L.ph_fdk_cone3d_static(ctypes.byref(g), fp, FAKE, FAKE, None, 0, None, None, big_batch, 0, None) == -5
    # half-precision volumes in more than one share
    half_batch = scratch // (per_view * g.n_proj) + 1
    for dt in (1, 2):
        assert L.ph_fdk_cone3d_static(ctypes.byref(g), fp, FAKE, FAKE, None, 0, None, None, half_batch, dt,
                                      None) == -5


def test_rejects_bad_corrector_arguments(ph, L):
    g = _good3(ph)
    G = ctypes.byref(g)
    # MSE: null pointers and n = 0
    assert L.ph_mse_grad(None, FAKE, None, 10, FAKE, FAKE, None) == -1
    assert L.ph_mse_grad(FAKE, FAKE, None, 10, FAKE, None, None) == -1
    assert L.ph_mse_grad(FAKE, FAKE, None, 0, FAKE, FAKE, None) == -2
    # corrector gradient: K is required, lengths as for the filter, geometry checked
    assert L.ph_corrector_grad_3d(G, FAKE, FAKE, None, 64, None, None, FAKE, FAKE, 1, None) == -1
    assert L.ph_corrector_grad_3d(G, FAKE, FAKE, FAKE, 64, None, None, None, FAKE, 1, None) == -1
    assert L.ph_corrector_grad_3d(G, FAKE, FAKE, FAKE, 64, None, None, FAKE, FAKE, 0, None) == -2
    for M in (100, 32, 8192):
        assert L.ph_corrector_grad_3d(G, FAKE, FAKE, FAKE, M, None, None, FAKE, FAKE, 1, None) == -2
    bad = _good3(ph)
    bad.sdd = bad.sid
    assert L.ph_corrector_grad_3d(ctypes.byref(bad), FAKE, FAKE, FAKE, 64, None, None, FAKE, FAKE, 1, None) == -3
    # Adam: hyper-parameters
    ok = dict(lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, t=1)
    assert L.ph_adam_step(FAKE, FAKE, None, FAKE, 5, 1e-3, 0.9, 0.999, 1e-8, 1, None) == -1
    assert L.ph_adam_step(FAKE, FAKE, FAKE, FAKE, 0, 1e-3, 0.9, 0.999, 1e-8, 1, None) == -2
    for key, value in [("lr", 0.0), ("lr", float("nan")), ("b1", 1.0), ("b2", -0.1), ("eps", 0.0), ("t", 0)]:
        a = dict(ok, **{key: value})
        st = L.ph_adam_step(FAKE, FAKE, FAKE, FAKE, 5, a["lr"], a["b1"], a["b2"], a["eps"], a["t"], None)
        assert st == -8, key


def test_rejects_bad_tv_arguments(L):
    assert L.ph_tv_3d(None, 1, 4, 4, 1, 0, 0.1, 1.0, FAKE, None, None) == -1
    assert L.ph_tv_3d(FAKE, 0, 4, 4, 1, 0, 0.1, 1.0, FAKE, None, None) == -2
    assert L.ph_tv_3d(FAKE, 1, 4, 4, 0, 0, 0.1, 1.0, FAKE, None, None) == -2
    assert L.ph_tv_3d(FAKE, 1, 4, 4, 1, 0, 0.0, 1.0, FAKE, None, None) == -8   # isotropic needs eps > 0
    assert L.ph_tv_3d(FAKE, 1, 4, 4, 1, 1, -0.1, 1.0, FAKE, None, None) == -8
    assert L.ph_tv_3d(FAKE, 1, 4, 4, 1, 2, 0.1, 1.0, FAKE, None, None) == -8
    assert L.ph_tv_3d(FAKE, 1, 4, 4, 1, 0, 0.1, float("nan"), FAKE, None, None) == -8
    assert L.ph_tv_3d(FAKE, 1, 4, 4, 1, 0, 0.1, 1.0, None, None, None) == 0   # nothing requested: no launch
    assert L.ph_tv_3d(FAKE, 1, 4, 4, 1, 1, 0.0, 1.0, None, None, None) == 0   # anisotropic: eps = 0 is valid


def test_rejects_bad_tv_iterate_arguments(ph, L):
    from paper_1904_13342_amd._lib import TvParams
    g = ph.from_spec(synth.config("par2d_64"))
    rv = ph.ray_vectors_2d(g)
    fp = rv.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    G = ctypes.byref(g)
    ok = TvParams(1e-3, 1e-2, 1e-2, 0.9, 0.999, 1e-8)
    need = L.ph_tv_workspace_bytes_2d(G, 1)
    assert need >= 2 * 90 * 96 * 4 + 64 * 64 * 4
    args = lambda prm, ws_bytes, t0=0, n=5: (G, fp, FAKE, FAKE, FAKE, FAKE, t0, n, ctypes.byref(prm), FAKE, ws_bytes,
                                             None, 1, None)
    assert L.ph_tv_iterate_par2d(*args(ok, need - 1)) == -5
    assert L.ph_tv_iterate_par2d(*args(ok, need, n=0)) == -2
    assert L.ph_tv_iterate_par2d(*args(ok, need, t0=-1)) == -2
    for bad in (TvParams(-1.0, 1e-2, 1e-2, 0.9, 0.999, 1e-8), TvParams(1e-3, 0.0, 1e-2, 0.9, 0.999, 1e-8),
                TvParams(1e-3, 1e-2, 1e-2, 1.0, 0.999, 1e-8), TvParams(1e-3, -1e-2, 1e-2, 0.9, 0.999, 1e-8, 1),
                TvParams(1e-3, 1e-2, 1e-2, 0.9, 0.999, 1e-8, 3)):
        assert L.ph_tv_iterate_par2d(*args(bad, need)) == -8
    assert L.ph_tv_iterate_par2d(G, fp, None, FAKE, FAKE, FAKE, 0, 5, ctypes.byref(ok), FAKE, need, None, 1,
                                 None) == -1


def test_filter_response_matches_oracle(L, ora):
    for kind, ref_fn in ((0, ora.ramlak_response), (1, ora.ramp_response)):
        for M in (16, 1024):
            K = (ctypes.c_float * M)()
            assert L.ph_filter_response(kind, M, 0.625, K) == 0
            ref = ref_fn(M, 0.625)
            assert np.abs(np.array(K) - ref).max() <= 1e-7 * np.abs(ref).max()
    K = (ctypes.c_float * 16)()
    assert L.ph_filter_response(0, 16, 0.625, None) == -1
    assert L.ph_filter_response(0, 24, 0.625, K) == -2
    assert L.ph_filter_response(2, 16, 0.625, K) == -8
    assert L.ph_filter_response(1, 16, -1.0, K) == -8


def test_equiangular_response_matches_oracle(L, ora):
    for M, alpha, sid in ((16, 0.05, 300.0), (2048, 1.0 / 1200.0, 750.0)):
        K = (ctypes.c_float * M)()
        assert L.ph_filter_response_equiangular(M, alpha, sid, K) == 0
        ref = ora.equiangular_response(M, alpha, sid)
        assert np.abs(np.array(K) - ref).max() <= 1e-6 * np.abs(ref).max()
    K = (ctypes.c_float * 16)()
    assert L.ph_filter_response_equiangular(16, 0.05, 300.0, None) == -1
    assert L.ph_filter_response_equiangular(24, 0.05, 300.0, K) == -2
    assert L.ph_filter_response_equiangular(16, 0.5, 300.0, K) == -8   # alpha * M > pi
    assert L.ph_filter_response_equiangular(16, 0.05, -1.0, K) == -8


def test_curved_fan_detector_validation(ph, L):
    """fan_detector must be 0 or 1, and the arc must span less than a half
    turn about the source."""
    spec = synth.config("fan2d_512").with_(kind="fan2d_curved")
    g = ph.from_spec(spec)
    assert g.fan_detector == 1
    rv = ph.ray_vectors_2d(g)
    fp = rv.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    g.fan_detector = 2
    assert L.ph_project_fan2d(ctypes.byref(g), fp, FAKE, FAKE, 1, 0, None) == -3
    g.fan_detector = 1
    g.det_spacing = 6.0    # 725 bins * 6 mm / 1200 mm > pi rad
    assert L.ph_project_fan2d(ctypes.byref(g), fp, FAKE, FAKE, 1, 0, None) == -3
    with pytest.raises(ValueError):
        ph.geom2d((8, 8), (1.0, 1.0), 12, 1.0, 4, math.pi, 20.0, 32.0, detector="round")


def test_binding_checks_tensor_shapes(ph):
    import torch
    g = ph.from_spec(synth.config("par2d_64"))
    rv = ph.ray_vectors_2d(g)
    with pytest.raises(ValueError):
        ph.project_par2d(g, rv, torch.zeros(64, 64))          # host tensor
    with pytest.raises(ValueError):
        ph.project_par2d(g, rv[:10], torch.zeros(64, 64))     # wrong trajectory length
