"""Quasi-static field sweep (hysteresis driver) on the GPU against the
oracle taking the same field values and steps."""
import numpy as np
import pytest

import paper_2605_28800_amd as T
import tdgl_inputs as I
from oracle import tdgl_oracle as O
from tests.gpu_helpers import announce, gpu_context, ps_of

pytestmark = pytest.mark.gpu


def test_sweep_matches_oracle_on_the_small_bilayer():
    """32x32x8 PbTiO3/SrTiO3 bilayer, FP64, E_z along a triangle wave of
    +-4e8 V/m in 8 values of 25 steps: mean P after every value and the
    final state against the oracle."""
    cfg = I.config("c4_small")
    values = np.zeros((8, 3))
    values[:, 2] = T.triangle_wave(4e8, 8)
    P = I.initial_P(cfg, 2)
    prob = O.Problem(cfg)
    announce("field sweep c4_small fp64")
    ctx = gpu_context(cfg, "f64")
    try:
        ctx.set_P(P)
        m, F = T.tdgl_sweep_eext(ctx.ctx, values, 25)
        got = ctx.get_P()
    finally:
        ctx.close()
    Ps = ps_of(cfg)
    for i, e in enumerate(values):
        prob.eext = e / prob.field_scale
        P = O.run(P, prob, "heun", cfg["dtau"], 25)
        ref = O.energies(P, prob)
        assert np.abs(m[i, 0] - ref["meanP"] * prob.P0).max() <= 1e-12 * Ps, i
        assert abs(F[i, 0, 4] - ref["F_total"] * prob.energy_scale) <= \
            1e-10 * abs(ref["F_total"] * prob.energy_scale), i
    assert np.abs(got - P).max() / Ps <= 1e-12


@pytest.mark.timeout(300)
def test_sweep_at_the_configured_amplitude_matches_oracle():
    """The hysteresis configuration's own amplitude, +-1e8 V/m, on its
    32x32x8 downscale (FP64): a triangle wave of 40 values of 50 steps (2000
    steps, one period), mean P_z after every value against the oracle."""
    cfg = I.config("c4_small")
    n, k = 40, 50
    values = np.zeros((n, 3))
    values[:, 2] = T.triangle_wave(1e8, n)
    P = I.initial_P(cfg, 3)
    prob = O.Problem(cfg)
    announce("field sweep c4_small fp64 at +-1e8 V/m, %d x %d steps" % (n, k))
    ctx = gpu_context(cfg, "f64")
    try:
        ctx.set_P(P)
        m, F = T.tdgl_sweep_eext(ctx.ctx, values, k)
    finally:
        ctx.close()
    Ps = ps_of(cfg)
    loop = []
    for i, e in enumerate(values):
        prob.eext = e / prob.field_scale
        P = O.run(P, prob, "heun", cfg["dtau"], k)
        ref = O.energies(P, prob)["meanP"] * prob.P0
        loop.append(ref[2])
        assert np.abs(m[i, 0] - ref).max() <= 1e-12 * Ps, (i, m[i, 0], ref)
    print("P_z(E) loop: " + " ".join("%.4f" % v for v in loop))
