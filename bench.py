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


def survey_bytes_per_cell_step(dims, esz):
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
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_28800_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def run_gpu(cfg, precision, steps, warmup, profile_steps, fft_path=0, rows=0):
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
    T.tdgl_build_tensor(ctx.ctx, cfg["mimg"])
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    P0 = I.initial_P(cfg, 0, np.float32 if precision == T.TDGL_FP32 else np.float64)
    ctx.set_P(torch.from_numpy(P0).cuda())
    ctx.step(warmup)
    ctx.sync()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record(stream)
    ctx.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ctx.sync()
    ms = ev0.elapsed_time(ev1)
    prof = T.tdgl_profile_step(ctx.ctx, profile_steps) if profile_steps else None
    F, meanP = ctx.energies()
    dims = ctx.dims
    fused = T.tdgl_get_fft_path(ctx.ctx)
    ctx.close()
    return dict(ms=ms, wall=wall, setup_s=setup_s, prof=prof, dims=dims, F=F, meanP=meanP,
                fused=fused)


def cpu_baseline(cfg, nsteps):
    """The oracle as it stands, timed on the host on a few Heun steps of the
    same grid.  Its interaction table is built with mimg = 0 (the cost of a
    step does not depend on the number of images); set-up is not timed."""
    import numpy as np

    import tdgl_inputs as I
    from oracle import tdgl_oracle as O
    c = dict(cfg)
    c["mimg"] = 0
    prob = O.Problem(c)
    P = I.initial_P(c, 0).astype(np.float64)
    P = O.step_heun(P, prob, c["dtau"])          # first call outside the timing
    t0 = time.perf_counter()
    for _ in range(nsteps):
        P = O.step_heun(P, prob, c["dtau"])
    dt = time.perf_counter() - t0
    ncell = int(np.prod(c["n"]))
    return dict(value=ncell * nsteps / dt, unit="cell-steps/s", cores=1, kind="oracle",
                sample="%d Heun steps of the %dx%dx%d film (numpy FP64, single thread; "
                       "setup excluded), %.1f s" % (nsteps, *c["n"], dt),
                host_cpus=os.cpu_count())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--fp64-steps", type=int, default=2000)
    ap.add_argument("--profile-steps", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fft-path", type=int, default=0, help="0 auto (fused if it fits), 1 three passes")
    ap.add_argument("--rows", type=int, default=0, help="update-kernel rows per group (0 auto)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (each simulation fits one "
              "MI355X; --gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        sys.exit("--steps must be >= 1")

    import paper_2605_28800_amd as T
    if not os.path.exists(T.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    import tdgl_inputs as I

    cfg = I.config("c2")
    ncell = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    log("fp32 run: %d warmup + %d timed Heun steps" % (args.warmup, args.steps))
    r32 = run_gpu(cfg, T.TDGL_FP32, args.steps, args.warmup, args.profile_steps,
                  args.fft_path, args.rows)
    ms_step = r32["ms"] / args.steps
    value = ncell * args.steps / (r32["ms"] / 1e3)
    log("fp32: %.4f ms/step, %.3e cell-steps/s (wall %.3f s, setup %.2f s, fused=%d)"
        % (ms_step, value, r32["wall"], r32["setup_s"], r32["fused"]))

    if r32["prof"] is None:
        print(json.dumps({"metric": "TDGL cell-steps/s", "value": value, "unit": "cell-steps/s",
                          "ms_per_step": ms_step, "note": "profiling leg skipped"}), flush=True)
        return
    # roofline of the dominant kernel
    kb = kernel_bytes(r32["dims"], 4)
    names = ["y_forward", "z_tensor", "y_inverse", "update_predictor", "update_corrector"]
    prof = dict(zip(names, r32["prof"]))
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
    kernels = {k: {"ms": round(prof[k], 5), "alg_bytes": kb[k],
                   "GBps": round(kb[k] / (prof[k] * 1e-3) / 1e9, 1) if prof[k] else None}
               for k in names}
    step_bytes = survey_bytes_per_cell_step(r32["dims"], 4)
    log("kernels:", json.dumps(kernels))

    fp64 = None
    if args.fp64_steps > 0:
        log("fp64 run: %d timed steps" % args.fp64_steps)
        r64 = run_gpu(cfg, T.TDGL_FP64, args.fp64_steps, max(args.warmup // 10, 10), 0)
        v64 = ncell * args.fp64_steps / (r64["ms"] / 1e3)
        fp64 = {"value": v64, "ms_per_step": r64["ms"] / args.fp64_steps,
                "steps": args.fp64_steps,
                "roofline_frac_step": v64 * survey_bytes_per_cell_step(r64["dims"], 8)
                / (HBM_PEAK_GBS * 1e9)}
        log("fp64: %.4f ms/step, %.3e cell-steps/s" % (fp64["ms_per_step"], v64))

    cpu = None
    if not args.no_cpu_baseline and args.cpu_steps > 0:
        log("cpu baseline: oracle, %d Heun steps" % args.cpu_steps)
        cpu = cpu_baseline(cfg, args.cpu_steps)
        log("cpu: %.3e cell-steps/s" % cpu["value"])

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
        "config": {"workload": "BaTiO3 film 128x128x32, periodic x,y / open z (padded 64), "
                               "180-degree wall + 1% noise, all terms, Heun dtau=1e-3, "
                               "mimg=16",
                   "grid": list(cfg["n"]), "padded": list(r32["dims"][3:6]),
                   "precision": "fp32 field / fp64 tensor and energies", "parallelism": "1 GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": dom,
                     "alg_bytes_per_launch": dom_bytes, "mean_launch_ms": dom_ms},
        "cpu_baseline": cpu,
        "fp64": fp64,
        "kernels": kernels,
        "step_roofline": {"bytes_per_cell_step": round(step_bytes, 1),
                          "frac": round(value * step_bytes / (HBM_PEAK_GBS * 1e9), 4),
                          "note": "whole step vs an HBM model of a 5-pass design"},
        "energies_J": list(r32["F"]),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
