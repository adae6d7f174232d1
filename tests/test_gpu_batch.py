"""Batched contexts: nbatch instances of one grid advanced by the same
launches give, instance by instance, exactly the results of separate
contexts (same kernels, same arithmetic, other indices), and each instance
follows the oracle's run at its own temperature."""
import numpy as np
import pytest

import paper_2605_28800_amd as T
import tdgl_inputs as I
from oracle import tdgl_oracle as O
from tests.gpu_helpers import PREC, announce, gpu_context, ps_of
from tests.test_gpu_parity import CASES, _cfg

pytestmark = pytest.mark.gpu


def _batch_context(cfg, prec, nb, temps, path=0):
    c = dict(cfg)
    c["T"] = list(temps)
    ctx = T.Context(c, PREC[prec], build_tensor=False, batch=nb)
    T.tdgl_set_fft_path(ctx.ctx, path)
    if c.get("terms", 15) & T.TDGL_ELEC:
        T.tdgl_build_tensor(ctx.ctx, c.get("mimg", 16))
    return ctx


def _single(cfg, prec, temp, P, steps, path=0):
    c = dict(cfg)
    c["T"] = temp
    ctx = gpu_context(c, prec, path=path)
    try:
        ctx.set_P(P)
        ctx.step(steps)
        F, m = ctx.energies()
        return ctx.get_P(PREC[prec]), np.array(F), np.array(m)
    finally:
        ctx.close()


@pytest.mark.parametrize("name,prec,path,scheme", [("c2_small", "f32", 0, None),
                                                   ("c2_small", "f32", 1, None),
                                                   ("c1", "f64", 0, None), ("c1", "f64", 1, None),
                                                   ("c2_small", "f32", 1, "ab3m2")])
def test_batch_equals_separate_runs(name, prec, path, scheme):
    cfg = I.config(name)
    if scheme:
        cfg["scheme"] = scheme
    temps = [250.0, 300.0, 350.0]
    dt = np.float32 if prec == "f32" else np.float64
    Ps = [I.initial_P(cfg, s, dt) for s in range(3)]
    steps = 40
    announce("batch of 3 %s %s path %d" % (name, prec, path))
    ctx = _batch_context(cfg, prec, 3, temps, path)
    try:
        ctx.set_P(np.stack(Ps))
        ctx.step(steps)
        Fb, mb = ctx.energies_batch()
        Pb = ctx.get_P(PREC[prec])
    finally:
        ctx.close()
    for b in range(3):
        P1, F1, m1 = _single(cfg, prec, temps[b], Ps[b], steps, path)
        assert np.array_equal(Pb[b], P1), b
        assert np.array_equal(Fb[b], F1), (b, Fb[b], F1)
        assert np.array_equal(mb[b], m1), b


def test_batch_with_vacuum_layers_and_field():
    """Two-material stack with a vacuum layer: per-instance coefficients,
    zeroed vacuum rows and the field output of each instance."""
    cfg = _cfg(**CASES["bilayer_vacuum_10x12x6"])
    temps = [280.0, 320.0]
    Ps = [I.initial_P(cfg, 7 + s) for s in range(2)]
    announce("batch with vacuum layers")
    ctx = _batch_context(cfg, "f64", 2, temps)
    try:
        ctx.set_P(np.stack(Ps))
        Eb = ctx.eval_field(T.TDGL_ALL).cpu().numpy()
        ctx.step(25)
        Pb = ctx.get_P()
    finally:
        ctx.close()
    for b in range(2):
        c = dict(cfg)
        c["T"] = temps[b]
        one = gpu_context(c, "f64")
        try:
            one.set_P(Ps[b])
            E1 = one.eval_field(T.TDGL_ALL).cpu().numpy()
            one.step(25)
            P1 = one.get_P()
        finally:
            one.close()
        assert np.array_equal(Eb[b], E1), b
        assert np.array_equal(Pb[b], P1), b
        assert np.all(Pb[b][:, 5] == 0)           # the vacuum layer stays empty


def test_autotune_restores_state_and_keeps_its_choice():
    cfg = I.config("c2_small")
    P0 = I.initial_P(cfg, 0, np.float32)
    announce("autotune c2_small")
    ctx = gpu_context(cfg, "f32")
    try:
        ctx.set_P(P0)
        ctx.step(10)
        fused, rows, ms = T.tdgl_autotune(ctx.ctx, 20)
        assert rows in (2, 4, 8, 16) and ms > 0
        assert T.tdgl_get_fft_path(ctx.ctx) == fused
        ctx.step(30)
        got = ctx.get_P(T.TDGL_FP32)
    finally:
        ctx.close()
    ref = gpu_context(cfg, "f32", path=0 if fused else 1)
    try:
        T.tdgl_set_update_rows(ref.ctx, rows)
        ref.set_P(P0)
        ref.step(40)
        want = ref.get_P(T.TDGL_FP32)
    finally:
        ref.close()
    assert np.array_equal(got, want)


@pytest.mark.parametrize("path", [0, 1])
def test_batch_against_oracle_fp64(path):
    """Three instances of the 16x16x8 box at 250, 300 and 350 K (one shared
    alpha_ref, per-instance coefficients) advanced by one batched context,
    each against the oracle's own run at its temperature: 200 Heun steps,
    |dP|/Ps <= 1e-12, energies to 1e-12 of their scale."""
    cfg = I.config("c1")
    cfg["scheme"] = "heun"
    temps = [250.0, 300.0, 350.0]
    Ps = [I.initial_P(cfg, 20 + s) for s in range(3)]
    announce("batch of 3 c1 fp64 vs oracle, path %d" % path)
    ctx = _batch_context(cfg, "f64", 3, temps, path)
    try:
        ctx.set_P(np.stack(Ps))
        ctx.step(200)
        Fb, mb = ctx.energies_batch()
        Pb = ctx.get_P(T.TDGL_FP64)
    finally:
        ctx.close()
    for b in range(3):
        c = dict(cfg)
        c["T"] = temps[b]
        prob = O.Problem(c)
        ref = O.run(Ps[b], prob, "heun", cfg["dtau"], 200)
        err = np.abs(Pb[b] - ref).max() / ps_of(c)
        assert err <= 1e-12, (b, err)
        E = O.energies(ref, prob)
        want = [E[k] * prob.energy_scale for k in ("F_land", "F_grad", "F_elec", "F_ext",
                                                  "F_total")]
        scale = max(abs(v) for v in want)
        assert np.abs(np.array(Fb[b]) - want).max() <= 1e-12 * scale, (b, Fb[b], want)
        assert np.abs(np.array(mb[b]) - E["meanP"] * prob.P0).max() <= 1e-14
