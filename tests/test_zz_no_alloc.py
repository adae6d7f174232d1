"""The allocation-free energy entry point (tdgl_energies_noalloc) against
tdgl_energies_batch on the same contexts, through the C ABI: a batch of
three 32x32x8 FP32 films first, then a smaller 12x10x5 FP64 open box (the
second call reuses the fixed device scratch of the first), and the host-side
rejection of a context whose partial sums exceed the scratch."""
import numpy as np
import pytest

import paper_2605_28800_amd as T
import tdgl_inputs as I
from tests.gpu_helpers import announce, gpu_context

pytestmark = pytest.mark.gpu


def _noalloc(ctx, nb):
    import torch
    out = torch.full((nb, 8), float("nan"), dtype=torch.float64, device="cuda")
    T.tdgl_energies_noalloc(ctx.ctx, out.data_ptr())
    ctx.stream.synchronize()
    return out.cpu().numpy()


def _check(ctx, nb):
    got = _noalloc(ctx, nb)
    F, m = T.tdgl_energies_batch(ctx.ctx)
    scale = np.abs(F).max(axis=1, keepdims=True)
    assert np.all(np.isfinite(got))
    assert np.all(np.abs(got[:, :5] - F) <= 1e-14 * scale), (got[:, :5], F)
    assert np.all(np.abs(got[:, 5:] - m) <= 1e-15), (got[:, 5:], m)
    return got


def test_noalloc_energies_two_calls_second_smaller():
    announce("noalloc energies: batch of 3 films 32x32x8 FP32, then 12x10x5 FP64")
    cfg = I.config("c2_small")
    cfg["T"] = [250.0, 300.0, 350.0]
    cfg["mimg"] = 2
    ctx = T.Context(cfg, T.TDGL_FP32, build_tensor=False, batch=3)
    try:
        T.tdgl_build_tensor(ctx.ctx, 2)
        P = np.stack([I.initial_P(cfg, s, np.float32) for s in range(3)])
        ctx.set_P(P)
        ctx.step(3)
        a = _check(ctx, 3)
        # the three instances differ (different T and seeds)
        assert len({float(v) for v in a[:, 4]}) == 3
    finally:
        ctx.close()
    cfg = I.config("c1")
    cfg.update(n=(12, 10, 5), layers=[0] * 5, mimg=0, eext=(2e6, -1e6, 3e6))
    ctx = gpu_context(cfg, "f64")
    try:
        ctx.set_P(I.initial_P(cfg, 1))
        ctx.step(2)
        b = _check(ctx, 1)
        # a second call in a row on the same context gives the same bits
        assert np.array_equal(_noalloc(ctx, 1), b)
    finally:
        ctx.close()


def test_noalloc_rejects_more_partials_than_the_scratch_holds():
    announce("noalloc energies: a batch larger than the fixed scratch is refused")
    cfg = I.config("c1")
    cfg.update(n=(8, 8, 8), layers=[0] * 8, terms=T.TDGL_LANDAU | T.TDGL_GRAD)
    nb = 4096
    ctx = T.Context(cfg, T.TDGL_FP64, build_tensor=False, batch=nb)
    try:
        T.tdgl_set_update_rows(ctx.ctx, 8)
        ctx.set_P(np.zeros((nb, 3, 8, 8, 8)))
        import torch
        out = torch.zeros((nb, 8), dtype=torch.float64, device="cuda")
        with pytest.raises(T.TdglError) as ei:
            T.tdgl_energies_noalloc(ctx.ctx, out.data_ptr())
        assert ei.value.status == -6
        assert "scratch" in str(ei.value)
        # nothing was enqueued: the output is untouched
        ctx.stream.synchronize()
        assert float(out.abs().max()) == 0.0
    finally:
        ctx.close()
