"""The relaxation criterion without a GPU: the tests' host reference of it
(which the GPU tests hold the library's on-device test to) on a stand-in
context whose energies follow known sequences -- the recorded relax step of
each instance, the floor and the step cap -- and the argument checks of
tdgl_relax, made before any device work."""
import numpy as np
import pytest

import paper_2605_28800_amd as T
from paper_2605_28800_amd import relaxation as R
from tests.relax_reference import host_relax


class FakeBatch:
    """energies(k) of each instance after k calls of step(check)."""

    def __init__(self, curves):
        self.curves = curves
        self.k = 0
        self.steps = 0

    def step(self, n):
        self.k += 1
        self.steps += n

    def energies_batch(self):
        F = np.zeros((len(self.curves), 5))
        F[:, 4] = [c(self.k) for c in self.curves]
        return F, np.zeros((len(self.curves), 3))


def test_relax_records_the_first_check_below_the_tolerance():
    floor = 1e-20
    curves = [
        lambda k: -1.0 - 0.5 ** k,           # change 0.5^k: below 1e-6 once 0.5^k < ~1e-6
        lambda k: -2.0,                       # already stationary: relaxed at the first check
        lambda k: -1.0 - 1e-3 * k,            # never relaxes
    ]
    ctx = FakeBatch(curves)
    done, steps = host_relax(ctx, floor, check=100, max_steps=5000)
    # instance 0: |F(k) - F(k-1)| = 0.5^k < 1e-6 * |F(k)| first at k = 20
    k0 = next(k for k in range(1, 100) if 0.5 ** k < 1e-6 * (1.0 + 0.5 ** k))
    assert done[0] == 100 * k0
    assert done[1] == 100
    assert done[2] == -1
    assert steps == 5000 and ctx.steps == 5000


def test_relax_stops_when_all_have_relaxed_and_uses_the_floor():
    # |F| tiny: the floor decides (paraelectric instance near F = 0)
    curves = [lambda k: 1e-12 * 0.5 ** k, lambda k: -3.0]
    ctx = FakeBatch(curves)
    done, steps = host_relax(ctx, floor=1e-3, check=50, max_steps=10000)
    assert list(done) == [50, 50]
    assert steps == 50


def test_relax_floor_scales_with_the_volume():
    import tdgl_inputs as I
    c = I.c5_recipe(8, (16, 64, 64))
    f = R.relax_floor(c)
    assert np.isclose(f, c["scales"]["alpha_ref"] * 1e-3 * 64 * 64 * 16 * 1e-27)


def test_tdgl_relax_rejects_bad_arguments_before_any_device_work():
    g = T.tdgl_grid(8, 8, 4, 1e-9, 1e-9, 1e-9, 0)
    ctx = T.tdgl_create_batch(g, 3, T.TDGL_FP32)
    try:
        for args in ((0, 100, 1e-6, 1e-3, 0), (100, -1, 1e-6, 1e-3, 0), (100, 100, 0.0, 1e-3, 0),
                     (100, 100, float("nan"), 1e-3, 0), (100, 100, 1e-6, -1.0, 0),
                     (100, 100, 1e-6, 1e-3, 2)):
            with pytest.raises(T.TdglError) as ei:
                T.tdgl_relax(ctx, 3, *args[:4], retire=args[4])
            assert ei.value.status == T.TDGL_E_ARG, args
        with pytest.raises(T.TdglError) as ei:          # no P yet
            T.tdgl_relax(ctx, 3, 100, 1000)
        assert ei.value.status == T.TDGL_E_STATE
    finally:
        T.tdgl_destroy(ctx)


def test_tdgl_relax_group_rejects_bad_arguments():
    g = T.tdgl_grid(8, 8, 4, 1e-9, 1e-9, 1e-9, 0)
    a = T.tdgl_create_batch(g, 2, T.TDGL_FP32)
    b = T.tdgl_create_batch(g, 3, T.TDGL_FP32)
    try:
        with pytest.raises(T.TdglError) as ei:              # the same context twice
            T.tdgl_relax_group([a, a], [2, 2], 100, 1000)
        assert ei.value.status == T.TDGL_E_ARG
        with pytest.raises(T.TdglError) as ei:              # bad check
            T.tdgl_relax_group([a, b], [2, 3], 0, 1000)
        assert ei.value.status == T.TDGL_E_ARG
        T.tdgl_set_integrator(b, T.TDGL_RK45, 1e-3)         # not a graphed scheme
        with pytest.raises(T.TdglError) as ei:
            T.tdgl_relax_group([a, b], [2, 3], 100, 1000)
        assert ei.value.status in (T.TDGL_E_UNSUPPORTED, T.TDGL_E_STATE)
    finally:
        T.tdgl_destroy(a)
        T.tdgl_destroy(b)
