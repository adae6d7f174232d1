"""Relaxation drivers on the C ABI: batched TDGL relaxation to the energy
criterion, and the training loop of the initial-state proposal network.

Host-side control only: the steps, energies, network passes and Adam
updates run in libtdgl's kernels.  "Relaxed" means the total free energy
changed by less than 1e-6 of max(|F|, floor) over the last `check` steps,
tested every `check` steps on each instance.
"""
from __future__ import annotations

import time

import numpy as np

from . import TDGL_FP32, Context


def relax_floor(cfg):
    """Energy floor of the relaxation test near F = 0 (paraelectric runs):
    alpha_ref P0^2 * 1e-3 times the sample volume, in J."""
    s = cfg["scales"]
    n = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    dv = cfg["d"][0] * cfg["d"][1] * cfg["d"][2]
    return s["alpha_ref"] * s["P0"] ** 2 * 1e-3 * n * dv


def relax(ctx, floor, check=100, max_steps=20000):
    """Step a batch context until every instance has relaxed or max_steps.
    Returns (relax step per instance, -1 if not relaxed; steps taken)."""
    f_prev = ctx.energies_batch()[0][:, 4].copy()
    done = np.full(len(f_prev), -1)
    steps = 0
    while steps < max_steps and (done < 0).any():
        ctx.step(check)
        steps += check
        f = ctx.energies_batch()[0][:, 4]
        ok = np.abs(f - f_prev) < 1e-6 * np.maximum(np.abs(f), floor)
        done[(done < 0) & ok] = steps
        f_prev = f.copy()
    return done, steps


def relax_grouped(recipe, keys, T, start, check=100, max_steps=20000, group_max=256,
                  tune_steps=0):
    """Relax samples that share a recipe per key (e.g. film thickness) in
    batches of at most group_max.

    recipe(key) -> run recipe; keys, T: per sample; start: torch float32
    device tensor [n][3][nz][ny][nx] (C/m^2).  Returns the relaxed P (device
    tensor like start), relax steps, final energies F (J) and the seconds
    spent stepping (set-up excluded)."""
    import torch
    keys = np.asarray(keys)
    n = len(keys)
    out = torch.empty_like(start)
    steps = np.full(n, -1)
    F = np.zeros(n)
    seconds = 0.0
    for k in np.unique(keys):
        rows_all = np.flatnonzero(keys == k)
        for g0 in range(0, len(rows_all), group_max):
            rows = rows_all[g0:g0 + group_max]
            cfg = recipe(k)
            cfg["T"] = [float(T[i]) for i in rows]
            ctx = Context(cfg, TDGL_FP32, batch=len(rows))
            try:
                ridx = torch.from_numpy(rows).to(start.device)
                ctx.set_P(start.index_select(0, ridx).contiguous())
                if tune_steps:
                    from . import tdgl_autotune
                    tdgl_autotune(ctx.ctx, tune_steps)
                    ctx.set_P(start.index_select(0, ridx).contiguous())
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                done, _ = relax(ctx, relax_floor(cfg), check, max_steps)
                torch.cuda.synchronize()
                seconds += time.perf_counter() - t0
                steps[rows] = done
                F[rows] = ctx.energies_batch()[0][:, 4]
                out.index_copy_(0, ridx, ctx.get_P_device(TDGL_FP32))
            finally:
                ctx.close()
    return out, steps, F, seconds


def train(net, rows, T, thick, noise, target, steps, batch, lr, seed=0, lr_final=None):
    """Adam on minibatches drawn from `rows` (dataset row indices) with a
    seeded shuffle, `steps` steps of `batch` samples; the learning rate
    decays geometrically from lr to lr_final (default lr / 10) in 8 stages.
    Returns the per-step losses and the seconds spent (GPU-synchronised)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = np.asarray(rows, dtype=np.int32)
    order = []
    while len(order) < steps * batch:
        order.extend(rng.permutation(rows).tolist())
    idx = torch.tensor(order[:steps * batch], dtype=torch.int32, device=T.device)
    lr_final = lr / 10 if lr_final is None else lr_final
    stages = 8
    per = (steps + stages - 1) // stages
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(stages):
        a, b = s * per, min(steps, (s + 1) * per)
        if a >= b:
            break
        rate = lr * (lr_final / lr) ** (s / max(stages - 1, 1))
        losses.extend(net.train(idx[a * batch:b * batch], batch, T, thick, noise, target, rate))
    torch.cuda.synchronize()
    return np.asarray(losses), time.perf_counter() - t0


def propose(net, rows, T, thick, noise, batch):
    """Network proposals for dataset rows (device tensor [len(rows)][3][...])."""
    import torch
    out = []
    for a in range(0, len(rows), batch):
        idx = torch.tensor(np.asarray(rows[a:a + batch], dtype=np.int32), device=T.device)
        out.append(net.forward(T, thick, noise, idx=idx))
    return torch.cat(out, 0)
