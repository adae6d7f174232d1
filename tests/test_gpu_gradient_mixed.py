"""The full gradient energy of eq 4 on the GPU (cross terms G12 and
G44 - G44') against the oracle: fields, energies and a trajectory."""
import numpy as np
import pytest

import paper_2605_28800_amd as T
import tdgl_inputs as I
from oracle import tdgl_oracle as O
from tests.gpu_helpers import announce, gpu_context, oracle_field, ps_of, rel_inf

pytestmark = pytest.mark.gpu

ANISO = dict(G11=5.1e-10, G12=-1.0e-10, G44=2.0e-10, G44p=0.5e-10)
CASES = {
    "open_9x7x5": dict(n=(9, 7, 5), periodic=(0, 0, 0), layers=None),
    "film_16x8x4": dict(n=(16, 8, 4), periodic=(1, 1, 0), layers=None),
    "bulk_8x8x8": dict(n=(8, 8, 8), periodic=(1, 1, 1), layers=None),
    "vacuum_8x6x5": dict(n=(8, 6, 5), periodic=(0, 0, 0), layers=[0, 0, -1, 0, 0]),
}


def _cfg(n, periodic, layers):
    cfg = I.config("c1")
    cfg.update(n=n, periodic=periodic, mimg=2, eext=(2e6, -1e6, 3e6))
    cfg["layers"] = list(layers) if layers is not None else [0] * n[2]
    cfg["gradient"] = dict(ANISO)
    cfg["d"] = (1.0e-9, 1.2e-9, 0.9e-9)
    return cfg


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cross_term_fields(case, prec):
    cfg = _cfg(**CASES[case])
    announce("gradient cross terms %s %s" % (case, prec))
    P = I.initial_P(cfg, 6, np.float32 if prec == "f32" else np.float64)
    prob = O.Problem(cfg)
    ctx = gpu_context(cfg, prec)
    try:
        ctx.set_P(P)
        tol = 1e-13 if prec == "f64" else 2e-6
        for mask in (T.TDGL_GRAD, T.TDGL_ALL):
            got = ctx.eval_field(mask).cpu().numpy()
            ref = oracle_field(P.astype(np.float64), prob, mask)
            assert rel_inf(got, ref) <= tol, (case, prec, mask)
    finally:
        ctx.close()


@pytest.mark.parametrize("case", ["open_9x7x5", "vacuum_8x6x5"])
def test_cross_term_energies(case):
    cfg = _cfg(**CASES[case])
    announce("gradient cross-term energies %s" % case)
    P = I.initial_P(cfg, 2) * 3
    prob = O.Problem(cfg)
    ctx = gpu_context(cfg, "f64")
    try:
        ctx.set_P(P)
        F, _ = ctx.energies()
    finally:
        ctx.close()
    E = O.energies(P, prob)
    ref = [E["F_land"], E["F_grad"], E["F_elec"], E["F_ext"], E["F_total"]]
    scale = max(abs(v) for v in ref) * prob.energy_scale
    for k in range(5):
        assert abs(F[k] - ref[k] * prob.energy_scale) <= 1e-12 * scale, k


def test_cross_term_trajectory_fp64():
    cfg = _cfg(**CASES["open_9x7x5"])
    cfg["scheme"] = "heun"
    announce("gradient cross-term trajectory")
    P = I.initial_P(cfg, 0)
    prob = O.Problem(cfg)
    ctx = gpu_context(cfg, "f64")
    try:
        ctx.set_P(P)
        ctx.step(100)
        got = ctx.get_P()
    finally:
        ctx.close()
    ref = O.run(P, prob, "heun", cfg["dtau"], 100)
    assert np.abs(got - ref).max() / ps_of(cfg) <= 1e-12
