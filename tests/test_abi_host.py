"""C-ABI checks that need no GPU: the library loads, exports every entry
point include/tdgl.h declares, validates arguments before touching the
device, and computes the same reduced coefficients as the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2605_28800_amd as T
import tdgl_inputs as I
from oracle import tdgl_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(T.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    T.lib()


def _declared():
    src = "".join(open(os.path.join(ROOT, "include", h)).read()
                  for h in sorted(os.listdir(os.path.join(ROOT, "include"))) if h.endswith(".h"))
    return sorted(set(re.findall(r"\b(tdgl_[A-Za-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(T.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(T.EXPORTED)


def test_abi_version():
    assert T.tdgl_abi_version() == 1


def _grid(n=(16, 16, 8), d=(1e-9, 1e-9, 1e-9), pm=0):
    return T.tdgl_grid(n[0], n[1], n[2], d[0], d[1], d[2], pm)


@pytest.mark.parametrize("n,d,pm,status", [
    ((0, 4, 4), (1e-9,) * 3, 0, T.TDGL_E_ARG),
    ((4, 4, 4), (0.0, 1e-9, 1e-9), 0, T.TDGL_E_ARG),
    ((4, 4, 4), (1e-9,) * 3, 1, T.TDGL_E_UNSUPPORTED),
    ((12, 16, 4), (1e-9,) * 3, 3, T.TDGL_E_UNSUPPORTED),     # periodic x not a power of two
    ((4, 4, 4), (1e-9,) * 3, 3, T.TDGL_E_UNSUPPORTED),       # periodic below 8
    ((600, 4, 4), (1e-9,) * 3, 0, T.TDGL_E_UNSUPPORTED),     # padded length 2048
])
def test_create_rejects(n, d, pm, status):
    with pytest.raises(T.TdglError) as e:
        T.tdgl_create(_grid(n, d, pm), T.TDGL_FP32)
    assert e.value.status == status


def test_sweep_without_field_values_is_refused():
    # an empty sweep is an argument error, found before any device work
    ctx = T.tdgl_create(_grid(), T.TDGL_FP32)
    try:
        with pytest.raises(T.TdglError) as e:
            T.tdgl_sweep_eext(ctx, np.zeros((0, 3)), 10)
        assert e.value.status == T.TDGL_E_ARG
    finally:
        T.tdgl_destroy(ctx)


def test_fp64_rows_of_at_most_512_cells():
    # FP64: the time-step kernel's two-row tile of 1024-cell rows needs more
    # than its 512 threads; FP32 takes them, and FP64 takes 512-cell rows
    # (padded to 1024 points)
    with pytest.raises(T.TdglError) as e:
        T.tdgl_create(_grid((1024, 8, 8), pm=3), T.TDGL_FP64)
    assert e.value.status == T.TDGL_E_UNSUPPORTED
    for n, pm, prec in (((1024, 8, 8), 3, T.TDGL_FP32), ((512, 4, 2), 0, T.TDGL_FP64)):
        ctx = T.tdgl_create(_grid(n, pm=pm), prec)
        try:
            assert T.tdgl_get_dims(ctx)[3] == 1024
        finally:
            T.tdgl_destroy(ctx)


@pytest.mark.parametrize("n,pm,dims", [
    ((16, 16, 8), 0, (32, 32, 16)),
    ((12, 10, 5), 0, (24, 24, 16)),          # x, y: 3 * 2^a lengths; z: powers of two
    ((96, 96, 8), 0, (192, 192, 16)),
    ((16, 12, 12), 0, (32, 24, 32)),
    ((1, 1, 1), 0, (8, 8, 8)),
    ((128, 128, 32), 3, (128, 128, 64)),
    ((256, 256, 64), 0, (512, 512, 128)),
    ((16, 8, 32), 7, (16, 8, 32)),
])
def test_padded_dims(n, pm, dims):
    ctx = T.tdgl_create(_grid(n, pm=pm), T.TDGL_FP64)
    try:
        d = T.tdgl_get_dims(ctx)
        assert d[:3] == n and d[3:6] == dims and d[6] == dims[0] // 2 + 1
        assert T.tdgl_workspace_size(ctx) > 0
    finally:
        T.tdgl_destroy(ctx)


def test_setter_validation_leaves_context_usable():
    ctx = T.tdgl_create(_grid(), T.TDGL_FP32)
    try:
        for call in (lambda: T.tdgl_set_scales(ctx, 1.0, -1.0, 5e-10, 45.0),
                     lambda: T.tdgl_set_integrator(ctx, 7, 1e-3),
                     lambda: T.tdgl_set_integrator(ctx, T.TDGL_EULER, 0.0),
                     lambda: T.tdgl_set_terms(ctx, 16),
                     lambda: T.tdgl_set_temperature(ctx, -3.0),
                     lambda: T.tdgl_set_layer_materials(ctx, [0] * 7 + [20]),
                     lambda: T.tdgl_set_z_tile(ctx, 96),
                     lambda: T.tdgl_set_store_mode(ctx, 3),
                     lambda: T.tdgl_build_tensor(ctx, 65)):
            with pytest.raises(T.TdglError) as e:
                call()
            assert e.value.status == T.TDGL_E_ARG
        with pytest.raises(T.TdglError) as e:
            T.tdgl_set_gradient(ctx, 5.1e-10, float("nan"), 2e-11, 2e-11)
        assert e.value.status == T.TDGL_E_ARG
        T.tdgl_set_gradient(ctx, 5.1e-10, -2e-11, 2e-11, 2e-11)       # full eq 4 accepted
        # the z-pass tile: a knob, resolved on the host
        assert T.tdgl_get_z_tile(ctx) in (64, 128)
        T.tdgl_set_z_tile(ctx, 256)
        assert T.tdgl_get_z_tile(ctx) == 256
        T.tdgl_set_z_tile(ctx, 0)
        assert T.tdgl_get_store_mode(ctx) == 1          # one instance: non-temporal
        T.tdgl_set_store_mode(ctx, 2)
        assert T.tdgl_get_store_mode(ctx) == 2
        T.tdgl_set_store_mode(ctx, 0)
        assert T.tdgl_get_store_mode(ctx) == 1
        with pytest.raises(T.TdglError) as e:
            T.tdgl_step(ctx, 1)                                        # no P yet
        assert e.value.status == T.TDGL_E_STATE
        with pytest.raises(T.TdglError) as e:
            T.tdgl_build_tensor(ctx, 4)                                # no scales yet
        assert e.value.status == T.TDGL_E_STATE
        assert b"scales" in T.lib().tdgl_last_error(ctx)
    finally:
        T.tdgl_destroy(ctx)


@pytest.mark.parametrize("name", ["c1", "c4_small"])
def test_reduced_coefficients_match_oracle(name):
    from oracle import tdgl_oracle as O
    cfg = I.config(name)
    cfg["T"] = 287.0
    cfg["layers"] = list(cfg["layers"])
    cfg["layers"][-1] = -1
    ctx = T.tdgl_create(_grid(cfg["n"], cfg["d"], 0), T.TDGL_FP64)
    try:
        s = cfg["scales"]
        T.tdgl_set_scales(ctx, s["P0"], s["alpha_ref"], s["G110"], s["eps_b"])
        for i, m in enumerate(cfg["materials"]):
            T.tdgl_set_material(ctx, i, m)
        T.tdgl_set_layer_materials(ctx, cfg["layers"])
        G = cfg["gradient"]
        T.tdgl_set_gradient(ctx, G["G11"], G["G12"], G["G44"], G["G44p"])
        T.tdgl_set_temperature(ctx, cfg["T"])
        coef, scal = T.tdgl_get_reduced(ctx, cfg["n"][2])
    finally:
        T.tdgl_destroy(ctx)
    prob = O.Problem(cfg, tensor=False)
    assert np.allclose(coef, prob.coef, rtol=1e-14, atol=0)
    assert scal[0] == pytest.approx(prob.kappa, rel=1e-14)
    assert np.allclose(scal[1:4], prob.h, rtol=1e-14)
    assert scal[4] == pytest.approx(prob.dV, rel=1e-14)
    assert scal[5] == pytest.approx(prob.energy_scale, rel=1e-14)
    assert scal[6] == pytest.approx(prob.field_scale, rel=1e-14)


def test_device_calls_fail_cleanly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    cfg = I.config("c1")
    ctx = T.tdgl_create(_grid(), T.TDGL_FP64)
    try:
        s = cfg["scales"]
        T.tdgl_set_scales(ctx, s["P0"], s["alpha_ref"], s["G110"], s["eps_b"])
        with pytest.raises(T.TdglError) as e:
            T.tdgl_build_tensor(ctx, 0)
        assert e.value.status == T.TDGL_E_HIP
    finally:
        T.tdgl_destroy(ctx)


def test_batch_create_limits_and_sizes():
    g = T.tdgl_grid(16, 16, 8, 1e-9, 1e-9, 1e-9, 0)
    for bad in (0, 5000):
        ctx = T._ctx_p()
        st = T.lib().tdgl_create_batch(ctypes.byref(g), bad, T.TDGL_FP32, None, ctypes.byref(ctx))
        assert st == T.TDGL_E_ARG
    g2 = T.tdgl_grid(16, 16, 64, 1e-9, 1e-9, 1e-9, 0)
    ctx = T._ctx_p()
    st = T.lib().tdgl_create_batch(ctypes.byref(g2), 2048, T.TDGL_FP32, None, ctypes.byref(ctx))
    assert st == T.TDGL_E_UNSUPPORTED              # nz * nbatch beyond one launch grid
    ctxs = [T.tdgl_create(g, T.TDGL_FP32)] + [T.tdgl_create_batch(g, n, T.TDGL_FP32)
                                              for n in (2, 4)]
    try:
        assert [T.tdgl_get_batch(c) for c in ctxs] == [1, 2, 4]
        s1, s2, s4 = [T.tdgl_workspace_size(c) for c in ctxs]
        per = s2 - s1                               # state, spectra, coefficients of one instance
        assert per > 3 * 2 * 16 * 16 * 8 * 4        # at least the two P buffers
        assert abs((s4 - s2) - 2 * per) <= 8 * 256   # the tensor and tables are shared
    finally:
        for c in ctxs:
            T.tdgl_destroy(c)


def test_batch_temperatures_reach_the_coefficients():
    cfg = I.config("c1")
    g = T.tdgl_grid(*cfg["n"], *cfg["d"], 0)
    ctx = T.tdgl_create_batch(g, 3, T.TDGL_FP64)
    try:
        s = cfg["scales"]
        T.tdgl_set_scales(ctx, s["P0"], s["alpha_ref"], s["G110"], s["eps_b"])
        T.tdgl_set_material(ctx, 0, cfg["materials"][0])
        T.tdgl_set_layer_materials(ctx, cfg["layers"])
        with pytest.raises(T.TdglError):
            T.tdgl_set_temperatures(ctx, [300.0, -1.0, 300.0])
        T.tdgl_set_temperatures(ctx, [250.0, 300.0, 350.0])
        coef, _ = T.tdgl_get_reduced(ctx, cfg["n"][2])   # instance 0
        ref = O.landau_coefficients(cfg["materials"][0], 250.0)
        assert abs(coef[0, 0] - ref["a1x"] / s["alpha_ref"]) < 1e-12 * abs(coef[0, 0])
    finally:
        T.tdgl_destroy(ctx)


def test_triangle_wave_shape():
    w = T.triangle_wave(2.0, 8)
    assert np.allclose(w, [1, 2, 1, 0, -1, -2, -1, 0])
    assert T.triangle_wave(1.0, 400).max() == 1.0 and T.triangle_wave(1.0, 400).min() == -1.0


def test_rk_tolerance_validation():
    g = T.tdgl_grid(8, 8, 8, 1e-9, 1e-9, 1e-9, 0)
    ctx = T.tdgl_create(g, T.TDGL_FP64)
    try:
        for bad in ((-1.0, 1e-6), (0.0, 0.0), (float("nan"), 1e-6), (1e-8, float("inf"))):
            with pytest.raises(T.TdglError):
                T.tdgl_set_rk_tolerances(ctx, *bad)
        T.tdgl_set_rk_tolerances(ctx, 0.0, 1e-6)
        T.tdgl_set_integrator(ctx, T.TDGL_RK45, 2e-3)
        assert T.tdgl_get_rk_state(ctx) == (0.0, 2e-3, 0)
    finally:
        T.tdgl_destroy(ctx)


def test_net_create_rejects_bad_shapes():
    from paper_2605_28800_amd.proposal import tdgl_net_cfg
    bad = [
        (64, 64, 16, 32, 8, 0),        # no batch
        (64, 64, 16, 32, 8, 5000),     # batch above 4096
        (48, 64, 16, 32, 8, 8),        # nx not a power of two
        (64, 64, 2, 32, 8, 8),         # nz below 4
        (64, 64, 16, 24, 8, 8),        # width not a power of two
        (64, 64, 16, 4, 8, 8),         # width below 8
        (64, 64, 16, 256, 8, 8),       # width above 128
        (64, 64, 16, 32, 32, 8),       # noise block larger than nz
        (64, 64, 16, 32, 3, 8),        # noise block not a power of two
    ]
    for c in bad:
        cfg = tdgl_net_cfg(*c)
        h = ctypes.c_void_p()
        st = T.lib().tdgl_net_create(ctypes.byref(cfg), None, ctypes.byref(h))
        assert st == T.TDGL_E_ARG, c
        assert not h.value
    assert T.lib().tdgl_net_create(None, None, ctypes.byref(ctypes.c_void_p())) == T.TDGL_E_ARG


def test_single_layer_entry_points_validate_before_launch():
    L = T.lib()
    dummy = ctypes.c_void_p(16)        # never dereferenced: every call below is rejected
    # cin_p not a power of two >= 16, cout_p below 16, epilogue out of range,
    # output epilogue with cout_p != 16, missing output pointer
    cases = [
        (0, dummy, 0, dummy, dummy, 1, 3, 3, 3, 24, 32, dummy, None, None, None, None),
        (0, dummy, 0, dummy, dummy, 1, 3, 3, 3, 32, 8, dummy, None, None, None, None),
        (7, dummy, 0, dummy, dummy, 1, 3, 3, 3, 32, 32, dummy, None, None, None, None),
        (2, dummy, 0, dummy, dummy, 1, 3, 3, 3, 32, 32, None, None, None, dummy, dummy),
        (3, dummy, 0, dummy, None, 1, 3, 3, 3, 32, 32, None, None, None, None, None),
        (1, dummy, 0, dummy, dummy, 1, 3, 3, 3, 32, 32, dummy, None, dummy, None, None),
        (0, dummy, 1, dummy, dummy, 1, 0, 3, 3, 32, 32, dummy, None, None, None, None),
    ]
    for c in cases:
        assert L.tdgl_nn_conv3(*c, None) == T.TDGL_E_ARG, c
    nbytes = ctypes.c_size_t()
    assert L.tdgl_nn_wgrad_workspace(1, 3, 3, 3, 24, 32, ctypes.byref(nbytes)) == T.TDGL_E_ARG
    assert L.tdgl_nn_wgrad_workspace(2, 4, 4, 3, 32, 64, ctypes.byref(nbytes)) == T.TDGL_OK
    assert nbytes.value >= 64 * 27 * 32 * 4
    # too small a workspace
    assert L.tdgl_nn_conv3_wgrad(dummy, dummy, 0, 2, 4, 4, 3, 32, 64, dummy, 16, dummy,
                                 None) == T.TDGL_E_ARG


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
