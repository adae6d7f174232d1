"""tdgl_relax: the on-device relaxation test inside captured graphs against
the tests' host loop over tdgl_energies_batch (same relax step for every
instance, same steps taken, same final state bit for bit), and retirement:
a retired instance keeps the state it relaxed in, which equals the state of
a separate context advanced exactly that many steps."""
import numpy as np
import pytest

import paper_2605_28800_amd as T
import tdgl_inputs as I
from paper_2605_28800_amd.relaxation import relax_floor
from tests.gpu_helpers import PREC, announce
from tests.relax_reference import host_relax

pytestmark = pytest.mark.gpu


def _box(n, temps, scheme="heun"):
    cfg = I.config("c1")
    cfg.update(n=n, layers=[0] * n[2], scheme=scheme, T=list(temps),
               init=dict(kind="uniform", amp=0.1))
    return cfg


def _ctx(cfg, prec, P):
    ctx = T.Context(cfg, PREC[prec], batch=len(cfg["T"]))
    ctx.set_P(P)
    return ctx


CASES = {
    # paraelectric instances relax within the cap, the 300 K one does not
    "mixed_fp32_heun": ((12, 10, 6), [420.0, 300.0, 450.0, 400.0], "f32", "heun", 100, 4000),
    # every instance relaxes: the relaxation stops at the last one
    "all_fp32_heun": ((12, 10, 6), [430.0, 450.0, 410.0], "f32", "heun", 100, 20000),
    "all_fp64_euler_odd_check": ((8, 8, 4), [440.0, 420.0], "f64", "euler", 75, 20000),
    # the multistep scheme steps through tdgl_step (no graphs, no retirement)
    "ab3m2_fp64": ((8, 8, 4), [440.0, 300.0], "f64", "ab3m2", 100, 3000),
}


@pytest.mark.parametrize("case", list(CASES))
def test_relax_on_device_equals_the_host_loop(case):
    n, temps, prec, scheme, check, cap = CASES[case]
    cfg = _box(n, temps, scheme)
    dt = np.float32 if prec == "f32" else np.float64
    P0 = np.stack([I.initial_P(cfg, 40 + b, dt) for b in range(len(temps))])
    announce("tdgl_relax vs host loop: %s" % case)
    a = _ctx(cfg, prec, P0)
    try:
        got, taken = a.relax(check, cap)
        Pa = a.get_P(PREC[prec])
    finally:
        a.close()
    b = _ctx(cfg, prec, P0)
    try:
        want, taken_h = host_relax(b, relax_floor(cfg), check, cap)
        Pb = b.get_P(PREC[prec])
    finally:
        b.close()
    print("%s: relax steps %s, steps taken %d" % (case, list(got), taken))
    np.testing.assert_array_equal(got, want)
    assert taken == taken_h
    assert np.array_equal(Pa, Pb)
    assert (got > 0).sum() >= 1
    if case.startswith("all"):
        assert (got > 0).all() and taken == got.max()


@pytest.mark.parametrize("case", ["mixed_fp32_heun", "all_fp64_euler_odd_check"])
def test_retired_instances_keep_the_state_they_relaxed_in(case):
    n, temps, prec, scheme, check, cap = CASES[case]
    cfg = _box(n, temps, scheme)
    dt = np.float32 if prec == "f32" else np.float64
    P0 = np.stack([I.initial_P(cfg, 40 + b, dt) for b in range(len(temps))])
    announce("tdgl_relax with retirement: %s" % case)
    a = _ctx(cfg, prec, P0)
    try:
        steps, taken = a.relax(check, cap, retire=True)
        Pa = a.get_P(PREC[prec])
        a.step(3)                     # the context steps every instance afterwards
        Pa3 = a.get_P(PREC[prec])
    finally:
        a.close()
    ref = _ctx(cfg, prec, P0)
    try:
        plain, _ = ref.relax(check, cap)
    finally:
        ref.close()
    np.testing.assert_array_equal(steps, plain)
    for i, temp in enumerate(temps):
        c = dict(cfg, T=temp)
        one = T.Context(c, PREC[prec])
        try:
            one.set_P(P0[i])
            one.step(steps[i] if steps[i] > 0 else taken)
            want = one.get_P(PREC[prec])
            one.step(3)
            want3 = one.get_P(PREC[prec])
        finally:
            one.close()
        assert np.array_equal(Pa[i], want), i
        assert np.array_equal(Pa3[i], want3), i


def test_group_of_three_shapes_in_one_graph_equals_separate_relaxations():
    """Three batches of different grid shapes relaxed by tdgl_relax_group (one
    graph per chunk with a branch per shape) give, instance by instance, the
    relax steps and states of tdgl_relax on each batch alone."""
    specs = [((12, 10, 6), [430.0, 300.0, 450.0]), ((8, 8, 8), [440.0, 410.0]),
             ((16, 8, 4), [420.0, 250.0, 445.0, 460.0])]
    cfgs = [_box(n, temps) for n, temps in specs]
    starts = [np.stack([I.initial_P(c, 60 + 7 * g + b, np.float32) for b in range(len(c["T"]))])
              for g, c in enumerate(cfgs)]
    announce("tdgl_relax_group of three shapes")
    import torch
    streams = [torch.cuda.Stream() for _ in cfgs]
    ctxs = [T.Context(c, T.TDGL_FP32, stream=s, batch=len(c["T"])) for c, s in zip(cfgs, streams)]
    try:
        for ctx, P in zip(ctxs, starts):
            ctx.set_P(P)
        steps, taken = T.tdgl_relax_group([c.ctx for c in ctxs], [len(c["T"]) for c in cfgs],
                                          100, 6000, retire=True)
        torch.cuda.synchronize()
        got = [ctx.get_P(T.TDGL_FP32) for ctx in ctxs]
    finally:
        for ctx in ctxs:
            ctx.close()
    most = 0
    for g, (c, P) in enumerate(zip(cfgs, starts)):
        one = _ctx(c, "f32", P)
        try:
            s1, t1 = one.relax(100, 6000, retire=True)
            want = one.get_P(T.TDGL_FP32)
        finally:
            one.close()
        np.testing.assert_array_equal(steps[g], s1)
        assert np.array_equal(got[g], want), g
        most = max(most, t1)
    assert taken == most
    assert sum((s > 0).sum() for s in steps) >= 5
