"""Relaxation drivers on the C ABI: batched TDGL relaxation to the energy
criterion, and the training loop of the initial-state proposal network.

Host-side control only: the steps, energies, relaxation test, network
passes and Adam updates run in libtdgl's kernels.  "Relaxed" means the total
free energy changed by less than 1e-6 of max(|F|, floor) over the last
`check` steps, tested every `check` steps on each instance (tdgl_relax).
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


def relax(ctx, check=100, max_steps=20000, retire=False):
    """Step a batch context until every instance has relaxed or max_steps
    (tdgl_relax with rtol 1e-6 and the floor alpha_ref P0^2 1e-3 V).
    Returns (relax step per instance, -1 if not relaxed; steps taken)."""
    return ctx.relax(check, max_steps, 1e-6, 1e-3, retire)


def relax_grouped(recipe, keys, T, start, check=100, max_steps=20000, group_max=256,
                  tune_steps=100, log=None, retire=False):
    """Relax samples that share a recipe per key (e.g. film thickness) in
    batches of at most group_max.

    recipe(key) -> run recipe; keys, T: per sample; start: torch float32
    device tensor [n][3][nz][ny][nx] (C/m^2).  Each batch context is
    autotuned (FFT path and update tile, tune_steps steps per candidate)
    before its relaxation is timed.  Returns the relaxed P (device
    tensor like start), relax steps, final energies F (J), the seconds spent
    stepping (set-up excluded) and, per sample, its time to relaxed: its
    relax step count times its batch's measured time per step and instance
    (the cap for samples that did not relax).  log(message), if given, hears
    of each finished group.  retire: relaxed samples stop advancing (their
    state is the one that met the criterion)."""
    import torch
    keys = np.asarray(keys)
    n = len(keys)
    out = torch.empty_like(start)
    steps = np.full(n, -1)
    F = np.zeros(n)
    t_inst = np.zeros(n)
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
                done, taken = relax(ctx, check, max_steps, retire=retire)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                seconds += dt
                steps[rows] = done
                t_inst[rows] = np.where(done > 0, done, max_steps) * dt / (taken * len(rows))
                F[rows] = ctx.energies_batch()[0][:, 4]
                out.index_copy_(0, ridx, ctx.get_P_device(TDGL_FP32))
                if log:
                    log("relaxed group %s: %d instances, %d relaxed, %.1f s"
                        % (k, len(rows), (done > 0).sum(), seconds))
            finally:
                ctx.close()
    return out, steps, F, seconds, t_inst


def train(net, rows, T, thick, noise, target, steps, batch, lr, seed=0, lr_final=None,
          augment=True):
    """Adam on minibatches drawn from `rows` (dataset row indices) with a
    seeded shuffle, `steps` steps of `batch` samples; the learning rate
    decays geometrically from lr to lr_final (default lr / 10) in 8 stages.
    With augment, every sample is drawn under a seeded random in-plane
    symmetry op (the 8 mirrors and transposes of a square film; mirrors only
    otherwise).  Returns the per-step losses and the seconds spent
    (GPU-synchronised)."""
    import torch
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = np.asarray(rows, dtype=np.int32)
    order = []
    while len(order) < steps * batch:
        order.extend(rng.permutation(rows).tolist())
    idx = torch.tensor(order[:steps * batch], dtype=torch.int32, device=T.device)
    ops = None
    if augment:
        ops = torch.tensor(rng.integers(0, 8, size=steps * batch), dtype=torch.int32,
                           device=T.device)
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
        for c0 in range(a, b, 4096):          # tdgl_net_train takes at most 4096 steps a call
            c1 = min(b, c0 + 4096)
            losses.extend(net.train(idx[c0 * batch:c1 * batch], batch, T, thick, noise, target,
                                    rate, ops=None if ops is None else ops[c0 * batch:c1 * batch]))
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


def proposal_experiment(recipe, shape, noise_div, T, thick, noise, starts, n_train, theta0,
                        width, data_steps, eval_steps, train_steps, batch, check=100, lr=1e-3,
                        seed=0, profile=False, log=None, relaxed_only=True, augment=True):
    """The learned proposal end to end.

    Rows 0..n_train-1 of the conditions (T, thick, noise: host arrays;
    starts: device tensor of the matching random starts) are relaxed from
    their starts (cap data_steps) into the training set; a network of the
    given width, initialised with theta0, is trained on it (on the samples
    that met the criterion only, if relaxed_only and any did); the remaining
    rows are relaxed from their random starts and from the network's
    proposals (cap eval_steps).  recipe(thickness) gives the run recipe.
    Returns a dict of the measurements (relax steps -1 = not relaxed)."""
    import torch

    from .proposal import Net
    n = len(T)
    dT, dth, dn = (torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(starts.device)
                   for a in (T, thick, noise))
    tr, te = np.arange(n_train), np.arange(n_train, n)
    P_tr, s_tr, F_tr, t_data, _ = relax_grouped(recipe, thick[tr], T[tr], starts[:n_train],
                                                check, data_steps, log=log, retire=True)
    target = torch.zeros((n, 3) + tuple(shape), dtype=torch.float32, device=starts.device)
    target[:n_train] = P_tr
    net = Net(shape, width=width, noise_div=noise_div, max_batch=batch)
    try:
        net.set_params(theta0)
        rows = tr[s_tr > 0] if relaxed_only and (s_tr > 0).any() else tr
        losses, t_train = train(net, rows, dT, dth, dn, target, train_steps, batch, lr, seed=seed,
                                augment=augment)
        if log:
            log("trained %d steps in %.1f s" % (train_steps, t_train))
        prof = net.profile(batch, dT, dth, dn, target, reps=5) if profile else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prop = propose(net, te, dT, dth, dn, batch)
        torch.cuda.synchronize()
        t_net = time.perf_counter() - t0
    finally:
        net.close()
    P_pl, s_pl, F_pl, t_pl, i_pl = relax_grouped(recipe, thick[te], T[te], starts[n_train:],
                                                 check, eval_steps, log=log, retire=True)
    P_pr, s_pr, F_pr, t_pr, i_pr = relax_grouped(recipe, thick[te], T[te], prop, check,
                                                 eval_steps, log=log, retire=True)
    floor = np.array([relax_floor(recipe(k)) for k in thick[te]])
    dP = [(torch.linalg.norm(P_pr[i] - P_pl[i]) / max(torch.linalg.norm(P_pl[i]).item(), 1e-30)).item()
          for i in range(len(te))]
    return dict(train_steps_relaxed=s_tr, data_seconds=t_data, losses=losses,
                train_seconds=t_train, profile_ms=prof, network_seconds=t_net,
                plain_steps=s_pl, proposal_steps=s_pr, plain_F=F_pl, proposal_F=F_pr,
                plain_seconds=t_pl, proposal_seconds=t_pr, plain_instance_seconds=i_pl,
                proposal_instance_seconds=i_pr, energy_floor=floor,
                P_rel_diff=np.asarray(dP))
