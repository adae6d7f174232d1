"""GPU runtime behaviour through the C ABI: HIP graphs vs plain launches,
bitwise determinism, split step counts, non-finite detection, state
invalidation by field/energy evaluations, time-dependent E_ext, energy
descent and caller-owned workspace."""
import numpy as np
import pytest
import torch

import paper_2605_28800_amd as T
import tdgl_inputs as I
from oracle import tdgl_oracle as O
from tests.gpu_helpers import announce, gpu_context, ps_of

pytestmark = pytest.mark.gpu


def _run(cfg, prec, steps, chunk=None, path=0, seed=0):
    ctx = gpu_context(cfg, prec, chunk=chunk, path=path)
    try:
        ctx.set_P(I.initial_P(cfg, seed, np.float32 if prec == "f32" else np.float64))
        ctx.step(steps)
        return ctx.get_P(T.TDGL_FP64 if prec == "f64" else T.TDGL_FP32)
    finally:
        ctx.close()


@pytest.mark.parametrize("scheme", ["heun", "euler", "ab3m2"])
def test_graph_chunks_equal_plain_launches(scheme):
    cfg = I.config("c2_small")
    cfg["scheme"] = scheme
    announce("graph vs plain %s" % scheme)
    a = _run(cfg, "f32", 131, chunk=0)
    b = _run(cfg, "f32", 131, chunk=64)
    c = _run(cfg, "f32", 131, chunk=7)
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_split_steps_and_rerun_bitwise():
    cfg = I.config("c2_small")
    announce("split steps bitwise")
    whole = _run(cfg, "f32", 130)
    again = _run(cfg, "f32", 130)
    ctx = gpu_context(cfg, "f32")
    try:
        ctx.set_P(I.initial_P(cfg, 0, np.float32))
        ctx.step(50)
        ctx.step(80)
        split = ctx.get_P(T.TDGL_FP32)
    finally:
        ctx.close()
    assert np.array_equal(whole, again)
    assert np.array_equal(whole, split)


def test_field_and_energy_calls_do_not_disturb_the_run():
    cfg = I.config("c2_small")
    announce("eval/energies between steps")
    ref = _run(cfg, "f32", 60)
    ctx = gpu_context(cfg, "f32")
    try:
        ctx.set_P(I.initial_P(cfg, 0, np.float32))
        ctx.step(20)
        ctx.eval_field(T.TDGL_ALL)
        ctx.energies()
        ctx.step(25)
        ctx.get_P()
        ctx.eval_field(T.TDGL_ELEC)
        ctx.step(15)
        got = ctx.get_P(T.TDGL_FP32)
    finally:
        ctx.close()
    assert np.array_equal(ref, got)


def test_nonfinite_detected_and_cleared():
    cfg = I.config("c1")
    announce("non-finite flag")
    ctx = gpu_context(cfg, "f64")
    try:
        P = I.initial_P(cfg, 0)
        bad = P.copy()
        bad[1, 3, 4, 5] = np.nan
        ctx.set_P(bad)
        ctx.step(3)
        with pytest.raises(T.TdglError) as e:
            ctx.sync()
        assert e.value.status == T.TDGL_E_NONFINITE
        ctx.set_P(P)            # a fresh state clears the flag
        ctx.step(3)
        ctx.sync()
    finally:
        ctx.close()


def test_unstable_time_step_reported():
    """dtau far above the explicit stability bound (about 2/320 here) blows
    up; the step kernel flags it and sync reports it."""
    cfg = I.config("c1")
    cfg["dtau"] = 0.05
    announce("unstable dtau")
    ctx = gpu_context(cfg, "f32")
    try:
        ctx.set_P(I.initial_P(cfg, 0, np.float32))
        ctx.step(200)
        with pytest.raises(T.TdglError) as e:
            ctx.sync()
        assert e.value.status == T.TDGL_E_NONFINITE
    finally:
        ctx.close()


def test_time_dependent_field_matches_oracle():
    cfg = I.config("c4_small")
    announce("E_ext changed between step calls")
    prob = O.Problem(cfg)
    P = I.initial_P(cfg, 1)
    ctx = gpu_context(cfg, "f64")
    try:
        ctx.set_P(P)
        for ez in (0.0, 5e7, 1e8, -5e7):
            T.tdgl_set_eext(ctx.ctx, 0.0, 0.0, ez)
            ctx.step(20)
            prob.eext = np.array([0.0, 0.0, ez]) / prob.field_scale
            P = O.run(P, prob, "heun", cfg["dtau"], 20)
        got = ctx.get_P()
    finally:
        ctx.close()
    assert np.abs(got - P).max() / ps_of(cfg) <= 1e-12


def test_energy_descends_on_gpu():
    cfg = I.config("c2_small")
    announce("energy descent")
    ctx = gpu_context(cfg, "f32")
    try:
        ctx.set_P(I.initial_P(cfg, 0, np.float32))
        F = []
        for _ in range(12):
            F.append(ctx.energies()[0][4])
            ctx.step(25)
    finally:
        ctx.close()
    assert np.all(np.diff(F) < 0), F


def test_library_and_torch_workspaces_agree():
    cfg = I.config("c2_small")
    announce("workspace ownership")
    a = _run(cfg, "f32", 40)
    ctx = T.Context(cfg, T.TDGL_FP32, torch_workspace=False)
    try:
        ctx.set_P(I.initial_P(cfg, 0, np.float32))
        ctx.step(40)
        b = ctx.get_P(T.TDGL_FP32)
    finally:
        ctx.close()
    assert np.array_equal(a, b)


def test_device_set_get_and_precision_conversion():
    cfg = I.config("c2_small")
    announce("set/get P on device")
    P = I.initial_P(cfg, 4)
    ctx = gpu_context(cfg, "f64")
    try:
        ctx.set_P(torch.from_numpy(P).cuda())
        back = ctx.get_P_device(T.TDGL_FP64).cpu().numpy()
        assert np.array_equal(back, P)
        f32 = ctx.get_P_device(T.TDGL_FP32).cpu().numpy()
        assert np.array_equal(f32, P.astype(np.float32))
        ctx.set_P(torch.from_numpy(P.astype(np.float32)).cuda())
        assert np.array_equal(ctx.get_P(), P.astype(np.float32).astype(np.float64))
    finally:
        ctx.close()


@pytest.mark.parametrize("name,path", [("c2_small", 0), ("c2_small", 1)])
def test_kernel_profile_keeps_the_state(name, path):
    """tdgl_profile_kernels times every kernel and leaves the run as it was:
    the trajectory continues bit for bit."""
    cfg = I.config(name)
    announce("kernel profile %s path %d" % (name, path))
    ref = _run(cfg, "f32", 60, path=path)
    ctx = gpu_context(cfg, "f32", path=path)
    try:
        ctx.set_P(I.initial_P(cfg, 0, np.float32))
        ctx.step(30)
        ms = T.tdgl_profile_kernels(ctx.ctx, 5)
        fused = T.tdgl_get_fft_path(ctx.ctx)
        ctx.step(30)
        got = ctx.get_P(T.TDGL_FP32)
    finally:
        ctx.close()
    used = [0, 3, 4] if fused else [0, 1, 2, 3, 4]
    assert all(ms[i] > 0 for i in used), ms
    assert all(ms[i] == 0 for i in range(5) if i not in used), ms
    assert np.array_equal(ref, got)


def test_ab3m2_split_steps_bitwise():
    """The multistep history survives split step calls and graph chunks."""
    cfg = I.config("c2_small")
    cfg["scheme"] = "ab3m2"
    announce("AB3M2 split steps")
    whole = _run(cfg, "f32", 131, chunk=16)
    ctx = gpu_context(cfg, "f32", chunk=16)
    try:
        ctx.set_P(I.initial_P(cfg, 0, np.float32))
        for n in (1, 1, 30, 16, 83):
            ctx.step(n)
        split = ctx.get_P(T.TDGL_FP32)
    finally:
        ctx.close()
    assert np.array_equal(whole, split)


def test_graph_cache_follows_term_and_gradient_changes():
    """Captured step chunks take the term mask and the cross-term kernel by
    value: turning the Landau term off, then switching on the gradient cross
    terms of eq 4 (G12 != 0, G44 != G44') between tdgl_step calls must change
    the physics of the graphed chunks as well (FP64 against the oracle)."""
    cfg = I.config("c2_small")
    cfg["n"] = (16, 16, 4)
    cfg["layers"] = [0] * 4
    announce("graph cache vs set_terms / set_gradient, FP64 16x16x4 film")
    P0 = I.initial_P(cfg, 3)
    prob = O.Problem(cfg)
    ctx = gpu_context(cfg, "f64", chunk=64)
    try:
        ctx.set_P(P0)
        ctx.step(128)
        T.tdgl_set_terms(ctx.ctx, T.TDGL_ALL & ~T.TDGL_LANDAU)
        ctx.step(128)
        T.tdgl_set_terms(ctx.ctx, T.TDGL_ALL)
        G = cfg["gradient"]
        T.tdgl_set_gradient(ctx.ctx, G["G11"], -0.3 * G["G11"], G["G44"], 0.2 * G["G44"])
        ctx.step(128)
        got = ctx.get_P(T.TDGL_FP64)
    finally:
        ctx.close()
    ref = O.run(P0, prob, "heun", cfg["dtau"], 128)
    prob.terms = T.TDGL_ALL & ~T.TDGL_LANDAU
    ref = O.run(ref, prob, "heun", cfg["dtau"], 128)
    prob.terms = T.TDGL_ALL
    prob.g12 = -0.3 * G["G11"] / prob.G110
    prob.gm = (G["G44"] - 0.2 * G["G44"]) / prob.G110
    for i in range(3):
        for d in range(3):
            prob.g[i, d] = (G["G11"] if i == d else 1.2 * G["G44"]) / prob.G110
    ref = O.run(ref, prob, "heun", cfg["dtau"], 128)
    err = np.abs(got - ref).max() / ps_of(cfg)
    print("max |dP|/Ps = %.3e" % err)
    assert err < 1e-12, err


def test_integrator_buffers_live_in_the_bound_workspace():
    """The RK45 stage buffers and the AB3M2 history come from a bound
    workspace sized after the integrator is set; a workspace sized for Heun
    refuses a later switch to RK45 with TDGL_E_STATE and stays usable."""
    cfg = I.config("c1")
    cfg["n"] = (8, 8, 4)
    cfg["layers"] = [0] * 4
    P0 = I.initial_P(cfg, 2)
    announce("integrator buffers in the bound workspace")
    sizes = {}
    for scheme in ("heun", "ab3m2", "rk45"):
        c = dict(cfg, scheme=scheme)
        ctx = gpu_context(c, "f64")
        try:
            sizes[scheme] = T.tdgl_workspace_size(ctx.ctx)
            ctx.set_P(P0)
            ctx.step(5)
            got = ctx.get_P()
        finally:
            ctx.close()
        prob = O.Problem(c)
        if scheme == "rk45":
            ref = O.run_rk45(P0, prob, c["dtau"], 5, 1e-8, 1e-6)[0]
        else:
            ref = O.run(P0, prob, scheme, c["dtau"], 5)
        assert np.abs(got - ref).max() / ps_of(c) <= 1e-12, scheme
    pbytes = 3 * 8 * 8 * 4 * 8
    assert sizes["ab3m2"] - sizes["heun"] >= 3 * pbytes
    assert sizes["rk45"] - sizes["heun"] >= 8 * pbytes
    ctx = gpu_context(dict(cfg, scheme="heun"), "f64")
    try:
        ctx.set_P(P0)
        ctx.step(2)
        T.tdgl_set_integrator(ctx.ctx, T.TDGL_RK45, 1e-3)
        with pytest.raises(T.TdglError) as ei:
            ctx.step(1)
        assert ei.value.status == T.TDGL_E_STATE
        T.tdgl_set_integrator(ctx.ctx, T.TDGL_HEUN, 1e-3)
        ctx.step(3)
        got = ctx.get_P()
    finally:
        ctx.close()
    ref = O.run(P0, O.Problem(dict(cfg, scheme="heun")), "heun", cfg["dtau"], 5)
    assert np.abs(got - ref).max() / ps_of(cfg) <= 1e-12


def test_zero_steps_leave_the_state_unchanged():
    """Empty work: step(0) right after set_P and after a run, and a sweep whose
    field values are held for 0 steps, leave P bit for bit as it was; the
    sweep's two records of the same state agree exactly."""
    cfg = I.config("c2_small")
    announce("zero steps c2_small")
    P0 = I.initial_P(cfg, 1, np.float32)
    ctx = gpu_context(cfg, "f32")
    try:
        ctx.set_P(P0)
        ctx.step(0)
        assert np.array_equal(ctx.get_P(T.TDGL_FP32), P0)
        ctx.step(7)
        P7 = ctx.get_P(T.TDGL_FP32)
        ctx.step(0)
        m, F = T.tdgl_sweep_eext(ctx.ctx, np.zeros((2, 3)), 0)
        assert np.array_equal(ctx.get_P(T.TDGL_FP32), P7)
        assert np.array_equal(m[0], m[1]) and np.array_equal(F[0], F[1])
        assert np.isfinite(F).all() and np.abs(m).max() > 0
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_tuning_knobs_do_not_change_results(prec):
    """The z-pass tile and the store mode are launch choices only: every
    combination advances the film (three passes) and a batch of three boxes
    bit for bit as the built-in choice does."""
    dt = np.float32 if prec == "f32" else np.float64
    out = T.TDGL_FP32 if prec == "f32" else T.TDGL_FP64
    film = I.config("c2_small")
    box = I.config("c1")
    box.update(n=(12, 10, 6), layers=[0] * 6, scheme="heun", T=[300.0, 350.0, 420.0])
    # a tall box: 64-point z transforms, where the tile widths change how
    # many lines a wave holds
    tall = I.config("c1")
    tall.update(n=(8, 8, 32), layers=[0] * 32, scheme="heun", T=300.0)
    for cfg, nb in ((film, 1), (box, 3), (tall, 1)):
        announce("tuning knobs %s, %d instance(s)" % (prec, nb))
        P0 = I.initial_P(cfg, 3, dt) if nb == 1 else np.stack(
            [I.initial_P(cfg, 3 + b, dt) for b in range(nb)])
        results = {}
        for zt in (0, 64, 128, 256):
            for mode in (0, 1, 2):
                ctx = T.Context(cfg, T.TDGL_FP32 if prec == "f32" else T.TDGL_FP64, batch=nb)
                try:
                    T.tdgl_set_fft_path(ctx.ctx, 1)
                    T.tdgl_set_z_tile(ctx.ctx, zt)
                    T.tdgl_set_store_mode(ctx.ctx, mode)
                    ctx.set_P(P0)
                    ctx.step(40)
                    results[(zt, mode)] = ctx.get_P(out)
                finally:
                    ctx.close()
        ref = results[(0, 0)]
        for key, P in results.items():
            assert np.array_equal(P, ref), key
