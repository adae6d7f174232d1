"""Benchmark of the TDGL time step on one MI355X.

Workload (the metric's configuration): 128 x 128 x 32 BaTiO3 film, 1 nm cells,
periodic in x and y, open in z (z padded to 64), tetragonal 180-degree wall
with 1 % seeded noise, all four energy terms, Heun with dtau = 1e-3, FP32
field arithmetic with FP64 tensor construction.  One "step" is one full TDGL
time step (two field evaluations).  Inputs are resident in device memory
before the timed region starts.

Prints one JSON line: throughput in cell-steps/s, the roofline entry of the
dominant kernel (algorithmic bytes per launch / mean launch duration from HIP
events on the library's stream), the FP64 figure of the same workload and the
CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(dims, esz):
    """Algorithmic HBM bytes per launch of every kernel of one field
    evaluation (reads + writes the method must do in this 4-kernel design;
    Laplacian neighbours counted once, as cache hits)."""
    nx, ny, nz, mx, my, mz, hx = dims
    ncell = nx * ny * nz
    c = 2 * esz                                   # complex element
    s_phys = 3 * nz * ny * hx * c                 # x spectra, physical y rows
    s_pad = 3 * nz * my * hx * c                  # after the y pass
    tens = 6 * (mz // 2 + 1) * (my // 2 + 1) * hx * esz
    p = 3 * ncell * esz
    return {
        "y_forward": s_phys + s_pad,
        "z_tensor": 2 * s_pad + tens,
        "y_inverse": s_pad + s_phys,
        "update_predictor": s_phys + 2 * p + s_phys,
        "update_corrector": s_phys + 3 * p + s_phys,
    }


def model_bytes_per_cell_step(dims, esz):
    """Bytes per cell-step of a streaming 3-pass design with a separate x
    pass (the yardstick quoted with the target): Heun = 2 evals + 12 B."""
    nx, ny, nz, mx, my, mz, hx = dims
    n = nx * ny * nz
    h = hx * ny * nz / n
    ry = my / ny
    K = 24 * hx * (my // 2 + 1) * (mz // 2 + 1) / n
    b_eval = 36 + 96 * h + 96 * h * ry + K
    return (2 * b_eval + 12) * esz / 4


def source_hash():
    """Hash of the TDGL step's sources (the proposal network's net* files
    do not change the step's kernels)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_28800_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if not f.startswith("net"):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def run_gpu(cfg, precision, steps, warmup, profile_steps, fft_path=0, rows=0, chunk=None,
            kernel_reps=0, windows=1):
    import numpy as np
    import torch

    import paper_2605_28800_amd as T
    import tdgl_inputs as I
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t0 = time.time()
    ctx = T.Context(cfg, precision, stream=stream, build_tensor=False)
    T.tdgl_set_fft_path(ctx.ctx, fft_path)
    T.tdgl_set_update_rows(ctx.ctx, rows)
    if chunk is not None:
        T.tdgl_set_graph_chunk(ctx.ctx, chunk)
    T.tdgl_build_tensor(ctx.ctx, cfg["mimg"])
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    P0 = I.initial_P(cfg, 0, np.float32 if precision == T.TDGL_FP32 else np.float64)
    ctx.set_P(torch.from_numpy(P0).cuda())
    ctx.step(warmup)
    ctx.sync()
    torch.cuda.synchronize()
    # `windows` timed windows of `steps` steps each, back to back from the
    # evolving state; the figure is the median window
    win_ms, walls = [], []
    for _ in range(windows):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        ev0.record(stream)
        ctx.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - w0)
        ctx.sync()
        win_ms.append(ev0.elapsed_time(ev1))
    ms = float(np.median(win_ms))
    wall = float(np.median(walls))
    prof = T.tdgl_profile_step(ctx.ctx, profile_steps) if profile_steps else None
    kprof = T.tdgl_profile_kernels(ctx.ctx, kernel_reps) if kernel_reps else None
    F, meanP = ctx.energies()
    dims = ctx.dims
    fused = T.tdgl_get_fft_path(ctx.ctx)
    ctx.close()
    return dict(ms=ms, wall=wall, setup_s=setup_s, prof=prof, kprof=kprof, dims=dims, F=F,
                meanP=meanP, fused=fused, window_ms=win_ms)


def copy_calibration(mib=256, reps=3):
    """A plain device copy of known size (hipMemcpyAsync through torch's
    copy_, the runtime's copy kernel), for scaling
    the FETCH_SIZE / WRITE_SIZE counters: each launch reads and writes
    mib MiB, far more than the L2 holds."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"copy_bytes": n * 4, "launches": reps}


def stream_copy(mib=1024, reps=20):
    """Achievable HBM bandwidth of the device: a device-to-device copy of
    mib MiB (far more than the caches hold; torch's copy_ of contiguous
    tensors is hipMemcpyAsync, the runtime's copy kernel), its read plus
    written bytes over the mean of reps back-to-back copies timed with HIP
    events on torch's stream."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return {"GBps": round(2 * n * 4 / sec / 1e9, 1), "bytes_per_copy": 2 * n * 4,
            "copies": reps, "kind": "device-to-device hipMemcpyAsync, read + written bytes"}


KERNEL_KEYS = {        # rocprofv3 kernel-name fragments of the step kernels
    "y_forward": "k_rowb<float, 128, false,",
    "z_tensor": "k_zmul<float, 64,",
    "y_inverse": "k_rowb<float, 128, true,",
    "update": "k_update<float, 128, 0,",
}


def _pmc_means(path, counter):
    """Mean counter value (KiB) per dispatch, by kernel-name fragment, from a
    rocprofv3 counter_collection.csv."""
    import csv
    sums, cnts = {}, {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            name = row.get("Kernel_Name", "")
            v = float(row["Counter_Value"])
            for key, frag in list(KERNEL_KEYS.items()) + [("copy", "copy")]:
                if frag in name.replace("  ", " "):
                    sums[key] = sums.get(key, 0.0) + v
                    cnts[key] = cnts.get(key, 0) + 1
    return {k: sums[k] / cnts[k] for k in sums}, cnts


def traffic_from(fetch_kernels, write_kernels, fetch_copy, write_copy, copy_bytes, out):
    """HBM bytes per launch of each step kernel: FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch) scaled by the factor that maps the same counters of a
    plain copy of copy_bytes onto copy_bytes."""
    fk, fc = _pmc_means(fetch_kernels, "FETCH_SIZE")
    wk, wc = _pmc_means(write_kernels, "WRITE_SIZE")
    cf, _ = _pmc_means(fetch_copy, "FETCH_SIZE")
    cw, _ = _pmc_means(write_copy, "WRITE_SIZE")
    f_scale = copy_bytes / (cf["copy"] * 1024.0)
    w_scale = copy_bytes / (cw["copy"] * 1024.0)
    res = {"source_hash": source_hash(), "fetch_scale": f_scale, "write_scale": w_scale,
           "copy_bytes": copy_bytes, "bytes_per_launch": {}, "fetch_bytes": {},
           "write_bytes": {}, "dispatches": {"fetch": fc, "write": wc}}
    for k in KERNEL_KEYS:
        if k in fk and k in wk:
            fb, wb = fk[k] * 1024.0 * f_scale, wk[k] * 1024.0 * w_scale
            res["fetch_bytes"][k] = fb
            res["write_bytes"][k] = wb
            res["bytes_per_launch"][k] = fb + wb
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    return res


def run_c3(max_steps, check, tune_steps, seq_every):
    """Batched relaxation of the 64-instance workload against plain runs.

    Relaxed: |F(n) - F(n - check)| < 1e-6 max(|F(n)|, floor), tested every
    `check` steps on each instance, on the device (tdgl_relax).  Batched: one
    context per grid shape (24 / 24 / 16 instances), autotuned, all three
    relaxed by tdgl_relax_group -- one captured graph per chunk of up to 5000
    steps with a branch per shape -- with retirement: an instance stops
    advancing at the check where it relaxed.  Every instance therefore follows
    exactly its plain trajectory and stops in the same state as a plain run,
    so the two are compared at equal final energy.  Plain: every seq_every-th
    instance relaxed alone (a single-instance context, tdgl_relax) and timed;
    the plain time of the others is their relax steps times the measured
    plain time per step of their shape.  Set-up (tensor builds, uploads,
    tuning) is not timed."""
    import numpy as np
    import torch

    import paper_2605_28800_amd as T
    import tdgl_inputs as I
    groups = I.c3_groups()
    starts, ctxs, info = [], [], []
    for c in groups:
        nb = len(c["T"])
        st = torch.cuda.Stream()
        ctx = T.Context(c, T.TDGL_FP32, stream=st, batch=nb)
        P = np.stack([I.initial_P(c, sd, np.float32) for sd in c["seeds"]])
        ctx.set_P(P)
        fused, rows, ms = T.tdgl_autotune(ctx.ctx, tune_steps)
        ctx.set_P(P)
        info.append({"grid": list(c["n"]), "instances": nb, "fused_plane": fused, "rows": rows,
                     "ms_per_step_tuned": ms})
        starts.append(P)
        ctxs.append(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    relaxed, steps = T.tdgl_relax_group([ctx.ctx for ctx in ctxs], [len(c["T"]) for c in groups],
                                        check, max_steps, retire=True)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    F_batch = [ctx.energies_batch()[0][:, 4] for ctx in ctxs]
    for ctx in ctxs:
        ctx.close()
    # plain runs, one instance at a time, same start and test
    t_meas, n_meas, agree, same_F, plain_total, dF_max = 0.0, 0, 0, 0, 0.0, 0.0
    per_step = []
    for g, c in enumerate(groups):
        one = T.Context(dict(c, T=c["T"][0]), T.TDGL_FP32)
        t_g, steps_g = 0.0, 0
        try:
            for i in range(0, len(c["T"]), seq_every):
                T.tdgl_set_temperature(one.ctx, c["T"][i])
                one.set_P(starts[g][i])
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                done, taken = one.relax(check, max_steps)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t1
                t_g += dt
                steps_g += taken
                n_meas += 1
                agree += int(done[0] == relaxed[g][i])
                # equal final-energy accuracy: within 1e-6 of the plain run's F
                Fp = one.energies()[0][4]
                dF = abs(Fp - F_batch[g][i]) / max(abs(Fp), 1e-300)
                dF_max = max(dF_max, dF)
                same_F += int(dF <= 1e-6)
        finally:
            one.close()
        t_meas += t_g
        rate = t_g / max(steps_g, 1)                  # plain seconds per step of this shape
        per_step.append(rate * 1e3)
        plain_total += rate * float(np.where(relaxed[g] > 0, relaxed[g], steps).sum())
    cells = sum(c["n"][0] * c["n"][1] * c["n"][2] * len(c["T"]) for c in groups)
    nrel = int(sum((r > 0).sum() for r in relaxed))
    return {
        "workload": "64 open BaTiO3 boxes: 24 of 32x32x32, 24 of 64x64x16, 16 of 96x96x8 "
                    "(padded 64^3 / 128x128x32 / 192x192x16), T ~ U(200, 450) K, "
                    "P ~ U(-0.1, 0.1), FP32 Heun dtau=1e-3",
        "criterion": "|dF| over %d steps < 1e-6 max(|F|, alpha_ref P0^2 1e-3 V), on the device"
                     % check,
        "groups": info,
        "max_steps": max_steps,
        "batched": "tdgl_relax_group: one graph per <= 5000-step chunk with a branch per shape; "
                   "relaxed instances retired",
        "batched_steps": steps,
        "relaxed": nrel,
        "instances": int(sum(len(r) for r in relaxed)),
        "relax_steps": [r.tolist() for r in relaxed],
        "batched_s": t_batch,
        "plain_ms_per_step": per_step,
        "plain_measured_runs": n_meas,
        "plain_measured_s": t_meas,
        "plain_same_relax_step": agree,
        "plain_same_final_energy_1e-6": same_F,
        "plain_final_energy_max_rel_diff": dF_max,
        "plain_s": plain_total,
        "plain_note": "measured runs (every %d-th instance) give the per-step time of each "
                      "shape; plain_s = sum over all 64 of relax steps (the cap if not relaxed) "
                      "x that time" % seq_every,
        "speedup": plain_total / t_batch if t_batch > 0 else None,
        "cell_steps_per_s_batched_if_all_ran": cells * steps / t_batch if t_batch > 0 else None,
    }


def net_flops(width, shape):
    """Algorithmic FLOPs of one sample's forward pass (2 per multiply-add of
    the convolutions; unpadded channel counts)."""
    import tdgl_inputs as I
    nz, ny, nx = shape
    cells = [nx * ny * nz, nx * ny * nz // 8, nx * ny * nz // 64]
    level = [0, 0, 1, 1, 2, 2, 2, 1, 1, 0, 0, 0]
    return sum(2.0 * 27 * ci * co * cells[lv]
               for (ci, co), lv in zip(I.net_layer_shapes(width), level))


def equal_accuracy(s_pl, s_pr, dF, t_pl, t_pr, cap):
    """The proposal's gains over the held-out samples whose proposal-started
    run ends at an energy equal to (within 1e-6 relative) or below the plain
    run's, and both relaxed: mean relax steps and summed per-instance time to
    relaxed, plain over proposal."""
    import numpy as np
    m = (dF <= 1e-6) & (s_pl > 0) & (s_pr > 0)
    if not m.any():
        return {"samples": 0}
    return {"samples": int(m.sum()),
            "criterion": "final F(proposal) <= F(plain) (1 + 1e-6 sign), both relaxed",
            "plain_mean_steps": float(s_pl[m].mean()),
            "proposal_mean_steps": float(s_pr[m].mean()),
            "steps_ratio": float(s_pl[m].mean() / s_pr[m].mean()),
            "instance_time_ratio": float(t_pl[m].sum() / max(t_pr[m].sum(), 1e-30))}


def run_c5(n_train, n_test, data_steps, eval_steps, train_steps, batch, width, check=100,
           seed=7, augment=-1):
    """Learned initial-state proposal on 64x64x16 BaTiO3 films (thickness
    8..16 layers, T ~ U(250, 450) K): relax n_train seeded random starts
    (batched, one context per thickness) to make the training set, train the
    network on the GPU, then relax n_test held-out samples from their random
    starts and from the network's proposals, to the same criterion."""
    import numpy as np
    import torch

    import tdgl_inputs as I
    from paper_2605_28800_amd import relaxation as R
    shape, noise_div = (16, 64, 64), 8
    T, th, noise = I.net_conditions(n_train + n_test, shape, noise_div, seed=seed,
                                    T_range=(250.0, 450.0), thickness_range=(8, 16))
    starts = torch.from_numpy(I.noise_start(noise, th, shape)).cuda()
    log("c5: %d training starts (cap %d steps), %d training steps, %d held-out samples"
        % (n_train, data_steps, train_steps, n_test))
    aug = (n_train >= 512) if augment < 0 else bool(augment)
    r = R.proposal_experiment(lambda k: I.c5_recipe(int(k), shape), shape, noise_div, T, th,
                              noise, starts, n_train, I.net_params(width, seed=seed), width,
                              data_steps, eval_steps, train_steps, batch, check, seed=seed,
                              profile=True, log=lambda m: log("c5: " + m), augment=aug)
    capped = lambda s: np.where(s > 0, s, eval_steps)
    s_pl, s_pr = r["plain_steps"], r["proposal_steps"]
    dF = (r["proposal_F"] - r["plain_F"]) / np.maximum(np.abs(r["plain_F"]), r["energy_floor"])
    prof = r["profile_ms"]
    fl = net_flops(width, shape) * batch
    losses = r["losses"]
    t_pr = r["proposal_seconds"] + r["network_seconds"]
    res = {
        "workload": "64x64x16 open BaTiO3 boxes, film of 8..16 layers under vacuum, "
                    "T ~ U(250, 450) K, start: U(-0.1, 0.1) C/m^2 noise on 8^3 blocks; "
                    "FP32 Heun dtau=1e-3; network width %d (%d parameters), BF16" % (
                        width, sum(co * 27 * ci + co for ci, co in I.net_layer_shapes(width))),
        "criterion": "|dF| over %d steps < 1e-6 max(|F|, alpha_ref P0^2 1e-3 V)" % check,
        "train_samples": n_train, "train_relaxed": int((r["train_steps_relaxed"] > 0).sum()),
        "trained_on": "relaxed training states only" + (
            ", each minibatch sample under a random in-plane symmetry op" if aug else ""),
        "data_steps_cap": data_steps, "data_seconds": round(r["data_seconds"], 2),
        "train_steps": train_steps, "batch": batch, "train_seconds": round(r["train_seconds"], 2),
        "loss_first20": float(losses[:20].mean()), "loss_last20": float(losses[-20:].mean()),
        "test_samples": n_test, "eval_steps_cap": eval_steps,
        "plain": {"relaxed": int((s_pl > 0).sum()), "mean_steps": float(capped(s_pl).mean()),
                  "median_steps": float(np.median(capped(s_pl))),
                  "seconds": round(r["plain_seconds"], 3)},
        "proposal": {"relaxed": int((s_pr > 0).sum()), "mean_steps": float(capped(s_pr).mean()),
                     "median_steps": float(np.median(capped(s_pr))), "seconds": round(t_pr, 3),
                     "network_seconds": round(r["network_seconds"], 4)},
        "steps_ratio": float(capped(s_pl).mean() / capped(s_pr).mean()),
        "time_ratio": float(r["plain_seconds"] / t_pr),
        "instance_time_to_relaxed_s": {
            "plain": float(r["plain_instance_seconds"].sum()),
            "proposal": float(r["proposal_instance_seconds"].sum() + r["network_seconds"]),
            "note": "sum over held-out samples of relax steps x the batch's time per step "
                    "and instance (the cap where not relaxed), plus network inference"},
        "final_energy_rel_diff": {"median": float(np.median(dF)),
                                  "max_abs": float(np.abs(dF).max()),
                                  "lower_or_equal": int((dF <= 1e-6).sum())},
        "equal_accuracy": equal_accuracy(s_pl, s_pr, dF, r["plain_instance_seconds"],
                                         r["proposal_instance_seconds"], eval_steps),
        "P_rel_diff_median": float(np.median(r["P_rel_diff"])),
        "train_step_ms": {"forward": prof[0], "backward": prof[1], "adam": prof[2]},
        "conv_kernels_ms": {"forward": prof[3], "backward_data": prof[4], "weight_grad": prof[5]},
        "conv_tflops": {"forward": fl / (prof[3] * 1e-3) / 1e12,
                        "backward_data": fl / (prof[4] * 1e-3) / 1e12,
                        "weight_grad": fl / (prof[5] * 1e-3) / 1e12,
                        "peak_bf16_dense": 2500.0},
    }
    log("c5: steps plain %.0f vs proposal %.0f (x%.2f), time x%.2f"
        % (res["plain"]["mean_steps"], res["proposal"]["mean_steps"], res["steps_ratio"],
           res["time_ratio"]))
    return res


def run_c4(args, names=("y_forward", "z_tensor", "y_inverse", "update_predictor",
                         "update_corrector")):
    """The 256x256x64 bilayer: timed Heun steps (graph chunks unless
    --graph-chunk says otherwise) and, with --kernel-reps, each step kernel
    timed over graph replays."""
    import paper_2605_28800_amd as T
    import tdgl_inputs as I
    cfg4 = I.config("c4")
    n4 = cfg4["n"][0] * cfg4["n"][1] * cfg4["n"][2]
    log("c4 fp32 run: %d timed Heun steps" % args.c4_steps)
    r4 = run_gpu(cfg4, T.TDGL_FP32, args.c4_steps, 20, 0, chunk=args.graph_chunk,
                 kernel_reps=20 if args.kernel_reps else 0)
    v4 = n4 * args.c4_steps / (r4["ms"] / 1e3)
    b4 = model_bytes_per_cell_step(r4["dims"], 4)
    kb4 = kernel_bytes(r4["dims"], 4)
    k4 = None
    if r4["kprof"] is not None:
        k4 = {k: {"ms": round(ms, 5), "alg_bytes": kb4[k],
                  "GBps": round(kb4[k] / (ms * 1e-3) / 1e9, 1) if ms else None}
              for k, ms in zip(names, r4["kprof"])}
    c4 = {"workload": "PbTiO3/SrTiO3 bilayer 256x256x64 (48+16 layers), open, padded "
                      "512x512x128, uniform random start, all terms, Heun dtau=1e-3",
          "value": v4, "unit": "cell-steps/s", "steps": args.c4_steps,
          "ms_per_step": r4["ms"] / args.c4_steps, "bytes_per_cell_step": round(b4, 1),
          "roofline_frac_step": round(v4 * b4 / (HBM_PEAK_GBS * 1e9), 4), "kernels": k4}
    log("c4: %.4f ms/step, %.3e cell-steps/s, step roofline %.3f"
        % (c4["ms_per_step"], v4, c4["roofline_frac_step"]))
    return c4


def _one_thread():
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["MKL_NUM_THREADS"] = "1"


def _oracle_run(name, nsteps, seed=0):
    """The oracle as it stands on `nsteps` steps of the named recipe (its
    own scheme); returns (cell-steps, start, end) of the timed loop (set-up
    and one first step excluded).  The periodic film's interaction table is
    built with mimg = 0: the cost of a step does not depend on the images."""
    import numpy as np

    import tdgl_inputs as I
    from oracle import tdgl_oracle as O
    from threadpoolctl import threadpool_limits
    c = I.config(name)
    if c["periodic"][0]:
        c["mimg"] = 0
    prob = O.Problem(c)
    P = I.initial_P(c, seed).astype(np.float64)
    step = O.step_euler if c["scheme"] == "euler" else O.step_heun
    with threadpool_limits(limits=1):
        P = step(P, prob, c["dtau"])
        t0 = time.time()
        for _ in range(nsteps):
            P = step(P, prob, c["dtau"])
        t1 = time.time()
    return int(np.prod(c["n"])) * nsteps, t0, t1


def _oracle_worker(a):
    return _oracle_run(*a)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(nsteps, cores):
    """The FP64 oracle timed on the host (never tuned for this): the metric's
    film on a bounded sample, single-threaded and as `cores` concurrent
    processes on their own copies (aggregate cell-steps/s over the span of
    the timed loops), plus the small box of 1000 Euler steps and the bilayer
    downscale, single-threaded.  Runs before anything touches the GPU (the
    workers are fresh interpreters)."""
    import multiprocessing as mp
    _one_thread()
    n, t0, t1 = _oracle_run("c2", nsteps)
    one = n / (t1 - t0)
    allc = None
    if cores > 1:
        with mp.get_context("spawn").Pool(cores, initializer=_one_thread) as pool:
            res = pool.map(_oracle_worker, [("c2", nsteps, s) for s in range(cores)])
        span = max(r[2] for r in res) - min(r[1] for r in res)
        allc = sum(r[0] for r in res) / span
    n1, a1, b1 = _oracle_run("c1", 1000)
    n4, a4, b4 = _oracle_run("c4_small", 100)
    return dict(
        value=allc if allc is not None else one, unit="cell-steps/s",
        cores=cores if allc is not None else 1, kind="oracle",
        sample="%d Heun steps of the 128x128x32 film per process (numpy FP64, one thread "
               "each, %d processes on their own copies; set-up excluded)" % (nsteps, cores),
        one_thread=one, one_thread_s=round(t1 - t0, 2),
        c1_1000_euler_one_thread=n1 / (b1 - a1), c1_s=round(b1 - a1, 2),
        c4_32x32x8_100_heun_one_thread=n4 / (b4 - a4), c4_s=round(b4 - a4, 2),
        cpu_model=cpu_model(), host_cpus=os.cpu_count())


def run_c4_loop(args):
    """The bilayer under a triangle wave of E_z (the hysteresis driver): one
    tdgl_sweep_eext call per 20 field values, each held for c4_loop_steps
    Heun steps; returns the field values, the mean P_z after each and the
    wall time of the loop."""
    import numpy as np
    import torch
    import paper_2605_28800_amd as T
    import tdgl_inputs as I
    cfg4 = I.config("c4")
    log("c4 loop: %d field values x %d steps" % (args.c4_loop_values, args.c4_loop_steps))
    ctx = T.Context(cfg4, T.TDGL_FP32)
    try:
        ctx.set_P(I.initial_P(cfg4, 0, np.float32))
        vals = np.zeros((args.c4_loop_values, 3))
        vals[:, 2] = T.triangle_wave(1e8, args.c4_loop_values)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        parts = []
        for a in range(0, len(vals), 20):        # a progress line per 20 values
            parts.append(T.tdgl_sweep_eext(ctx.ctx, vals[a:a + 20], args.c4_loop_steps))
            log("c4 loop: %d / %d values, %.1f s" % (min(a + 20, len(vals)), len(vals),
                                                     time.perf_counter() - t0))
        m = np.concatenate([p[0] for p in parts])
        dt = time.perf_counter() - t0
    finally:
        ctx.close()
    log("c4 loop: %.1f s, Pz from %.4f to %.4f" % (dt, m[:, 0, 2].min(), m[:, 0, 2].max()))
    return {"Ez_V_per_m": vals[:, 2].tolist(), "Pz_mean": m[:, 0, 2].tolist(),
            "steps_per_value": args.c4_loop_steps, "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--fp64-steps", type=int, default=2000)
    ap.add_argument("--profile-steps", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=6,
                    help="Heun steps of the film per oracle process in the CPU baseline")
    ap.add_argument("--cpu-cores", type=int, default=min(16, os.cpu_count() or 1),
                    help="concurrent oracle processes of the CPU baseline")
    ap.add_argument("--windows", type=int, default=5,
                    help="timed windows of --steps steps; the headline is their median")
    ap.add_argument("--c4-steps", type=int, default=200,
                    help="FP32 Heun steps of the 256x256x64 open bilayer (0: skip)")
    ap.add_argument("--c4-loop-values", type=int, default=0,
                    help="field values of a +-1e8 V/m triangle-wave sweep of the bilayer (0: skip)")
    ap.add_argument("--c4-loop-steps", type=int, default=500)
    ap.add_argument("--c3-max-steps", type=int, default=100000,
                    help="step cap of the batched 64-instance relaxation (0: skip)")
    ap.add_argument("--c3-check", type=int, default=100)
    ap.add_argument("--c3-seq-every", type=int, default=8,
                    help="plain runs: time every k-th instance alone and scale by k")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    # learned-proposal leg; the defaults are its quarter-size version (the
    # full one: --c5-train 1024 --c5-test 64 --c5-data-steps 12000
    # --c5-train-steps 10000)
    ap.add_argument("--c5-train", type=int, default=256,
                    help="learned-proposal leg: training samples (0 = leg off)")
    ap.add_argument("--c5-test", type=int, default=32)
    ap.add_argument("--c5-data-steps", type=int, default=8000)
    ap.add_argument("--c5-eval-steps", type=int, default=20000)
    ap.add_argument("--c5-train-steps", type=int, default=2000)
    ap.add_argument("--c5-batch", type=int, default=8)
    ap.add_argument("--c5-width", type=int, default=32)
    ap.add_argument("--c5-augment", type=int, default=-1,
                    help="train under random in-plane symmetry ops: 1 on, 0 off, -1 on from "
                         "512 training samples (measured: helps with 503 relaxed states, "
                         "hurts with 90)")
    ap.add_argument("--c5-only", action="store_true", help="run only the learned-proposal leg")
    ap.add_argument("--c4-only", action="store_true", help="run only the bilayer leg")
    ap.add_argument("--fft-path", type=int, default=0, help="0 auto (fused if it fits), 1 three passes")
    ap.add_argument("--rows", type=int, default=0, help="update-kernel rows per group (0 auto)")
    ap.add_argument("--graph-chunk", type=int, default=None,
                    help="steps per captured graph (0: plain launches; default: library's)")
    ap.add_argument("--kernel-reps", type=int, default=200,
                    help="launches per kernel in the per-kernel timing graphs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain copy used to scale the traffic counters")
    ap.add_argument("--traffic-from", nargs=5, metavar=("FETCH_CSV", "WRITE_CSV",
                                                         "COPY_FETCH_CSV", "COPY_WRITE_CSV",
                                                         "COPY_BYTES"),
                    help="turn rocprofv3 counter CSVs into profiles/traffic_c2_fp32.json")
    args = ap.parse_args()
    if args.traffic_from:
        a = args.traffic_from
        res = traffic_from(a[0], a[1], a[2], a[3], int(a[4]),
                           os.path.join(ROOT, "profiles", "traffic_c2_fp32.json"))
        print(json.dumps(res["bytes_per_launch"]))
        return
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (each simulation fits one "
              "MI355X; --gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        sys.exit("--steps must be >= 1")
    if args.copy_calibration:
        print(json.dumps(copy_calibration()), flush=True)
        return

    import paper_2605_28800_amd as T
    if not os.path.exists(T.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    import tdgl_inputs as I

    if args.c4_only:
        out = {"c4_large_grid": run_c4(args) if args.c4_steps > 0 else None}
        if args.c4_loop_values > 0:
            out["c4_field_loop"] = run_c4_loop(args)
        print(json.dumps(out), flush=True)
        return
    if args.c5_only:
        print(json.dumps({"c5_learned_proposal": run_c5(
            args.c5_train, args.c5_test, args.c5_data_steps, args.c5_eval_steps,
            args.c5_train_steps, args.c5_batch, args.c5_width, augment=args.c5_augment)}),
            flush=True)
        return

    cpu = None
    if not args.no_cpu_baseline and args.cpu_steps > 0:
        # first, before anything touches the GPU: its workers are new processes
        log("cpu baseline: oracle, %d Heun steps x %d processes" % (args.cpu_steps, args.cpu_cores))
        cpu = cpu_baseline(args.cpu_steps, args.cpu_cores)
        log("cpu: %.3e cell-steps/s on %d cores, %.3e on one" % (cpu["value"], cpu["cores"],
                                                                cpu["one_thread"]))

    cfg = I.config("c2")
    ncell = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    log("fp32 run: %d warmup + %d x %d timed Heun steps" % (args.warmup, args.windows, args.steps))
    r32 = run_gpu(cfg, T.TDGL_FP32, args.steps, args.warmup, args.profile_steps,
                  args.fft_path, args.rows, args.graph_chunk, args.kernel_reps,
                  windows=max(1, args.windows))
    ms_step = r32["ms"] / args.steps
    value = ncell * args.steps / (r32["ms"] / 1e3)
    log("fp32: %.4f ms/step, %.3e cell-steps/s (wall %.3f s, setup %.2f s, fused=%d)"
        % (ms_step, value, r32["wall"], r32["setup_s"], r32["fused"]))

    if r32["prof"] is None or r32["kprof"] is None:
        print(json.dumps({"metric": "TDGL cell-steps/s", "value": value, "unit": "cell-steps/s",
                          "ms_per_step": ms_step, "note": "profiling leg skipped"}), flush=True)
        return
    # roofline of the dominant kernel: mean launch durations from graphs of
    # back-to-back launches of each kernel (HIP events on the library stream)
    kb = kernel_bytes(r32["dims"], 4)
    names = ["y_forward", "z_tensor", "y_inverse", "update_predictor", "update_corrector"]
    prof = dict(zip(names, r32["kprof"]))
    prof_ev = dict(zip(names, r32["prof"]))
    per_step = {"y_forward": 2 * prof["y_forward"], "z_tensor": 2 * prof["z_tensor"],
                "y_inverse": 2 * prof["y_inverse"],
                "update": prof["update_predictor"] + prof["update_corrector"]}
    dom = max(per_step, key=per_step.get)
    if dom == "update":
        dom_ms = 0.5 * (prof["update_predictor"] + prof["update_corrector"])
        dom_bytes = 0.5 * (kb["update_predictor"] + kb["update_corrector"])
    else:
        dom_ms = prof[dom]
        dom_bytes = kb[dom]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic_c2_fp32.json")
    if os.path.exists(tfile):
        tj = json.load(open(tfile))
        if tj.get("source_hash") == source_hash() and dom in tj.get("bytes_per_launch", {}):
            traffic = tj["bytes_per_launch"][dom]
    kernels = {k: {"ms": round(prof[k], 5), "ms_eager_events": round(prof_ev[k], 5),
                   "alg_bytes": kb[k],
                   "GBps": round(kb[k] / (prof[k] * 1e-3) / 1e9, 1) if prof[k] else None}
               for k in names}
    step_bytes = model_bytes_per_cell_step(r32["dims"], 4)
    log("kernels:", json.dumps(kernels))
    copy_bw = stream_copy()
    log("stream copy: %.1f GB/s" % copy_bw["GBps"])

    fp64 = None
    if args.fp64_steps > 0:
        log("fp64 run: %d timed steps" % args.fp64_steps)
        r64 = run_gpu(cfg, T.TDGL_FP64, args.fp64_steps, max(args.warmup // 10, 10), 0)
        v64 = ncell * args.fp64_steps / (r64["ms"] / 1e3)
        fp64 = {"value": v64, "ms_per_step": r64["ms"] / args.fp64_steps,
                "steps": args.fp64_steps,
                "roofline_frac_step": v64 * model_bytes_per_cell_step(r64["dims"], 8)
                / (HBM_PEAK_GBS * 1e9)}
        log("fp64: %.4f ms/step, %.3e cell-steps/s" % (fp64["ms_per_step"], v64))

    c4 = run_c4(args) if args.c4_steps > 0 else None
    if c4 is not None and c4.get("roofline_frac_step") is not None:
        c4["roofline_frac_step_of_stream_copy"] = round(
            c4["roofline_frac_step"] * HBM_PEAK_GBS / copy_bw["GBps"], 4)

    loop = run_c4_loop(args) if args.c4_loop_values > 0 else None

    c3 = None
    if args.c3_max_steps > 0:
        log("c3: batched relaxation of 64 instances (cap %d steps)" % args.c3_max_steps)
        c3 = run_c3(args.c3_max_steps, args.c3_check, 200, args.c3_seq_every)
        log("c3: %d/%d relaxed in %d steps, batched %.2f s, plain %.2f s (x%.1f)"
            % (c3["relaxed"], c3["instances"], c3["batched_steps"], c3["batched_s"],
               c3["plain_s"], c3["speedup"] or 0))

    c5 = None
    if args.c5_train > 0:
        c5 = run_c5(args.c5_train, args.c5_test, args.c5_data_steps, args.c5_eval_steps,
                    args.c5_train_steps, args.c5_batch, args.c5_width, augment=args.c5_augment)

    out = {
        "metric": "TDGL cell-steps/s (FP32 vs FP64) + batched time-to-relaxed vs plain, 1 GPU",
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "BaTiO3 film 128x128x32 periodic x,y open z, 180-deg wall, "
                               "all terms, FP32 Heun dtau=1e-3, mimg=16",
                   "grid": list(cfg["n"]), "padded": list(r32["dims"][3:6]),
                   "precision": "fp32 field / fp64 tensor and energies", "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": dom,
                     "alg_bytes_per_launch": dom_bytes, "mean_launch_ms": dom_ms,
                     "frac_of_stream_copy": round(achieved / copy_bw["GBps"], 4)},
        "cpu_baseline": cpu,
        "fp64": fp64,
        "c4_large_grid": c4,
        "c3_batched_relaxation": c3,
        "c4_field_sweep": loop,
        "c5_learned_proposal": c5,
        "kernels": kernels,
        "step_roofline": {"bytes_per_cell_step": round(step_bytes, 1),
                          "frac": round(value * step_bytes / (HBM_PEAK_GBS * 1e9), 4),
                          "frac_of_stream_copy": round(value * step_bytes
                                                       / (copy_bw["GBps"] * 1e9), 4),
                          "note": "whole step vs an HBM model of a 5-pass design"},
        "stream_copy": copy_bw,
        "energies_J": list(r32["F"]),
        "windows_ms": [round(w, 4) for w in r32["window_ms"]],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
