"""Shared helpers of the GPU parity tests: run the HIP path through the
C ABI and the oracle on the same seeded inputs."""
import sys

import numpy as np

import paper_2605_28800_amd as T
from oracle import tdgl_oracle as O

PREC = {"f32": T.TDGL_FP32, "f64": T.TDGL_FP64}


def announce(msg):
    print("[gpu case] " + msg, flush=True)
    sys.stdout.flush()


def gpu_context(cfg, prec, chunk=None, path=0):
    """Context for cfg.  path 0: fused plane pass where it fits, 1: three passes."""
    ctx = T.Context(cfg, PREC[prec] if isinstance(prec, str) else prec, build_tensor=False)
    T.tdgl_set_fft_path(ctx.ctx, path)
    if cfg.get("terms", 15) & T.TDGL_ELEC:
        T.tdgl_build_tensor(ctx.ctx, cfg.get("mimg", 16))
    if chunk is not None:
        T.tdgl_set_graph_chunk(ctx.ctx, chunk)
    return ctx


def tensor_entry(cfg, offset, mimg):
    """Oracle interaction tensor for one cell offset (with periodic images,
    no k = 0 correction), components xx yy zz xy xz yz."""
    import ctypes
    from oracle import lib as orc_lib
    n = cfg["n"]
    pm = sum(1 << k for k in range(3) if cfg["periodic"][k])
    idx = [(offset[k] % n[k]) if cfg["periodic"][k] else offset[k] + n[k] - 1 for k in range(3)]
    t, w = O.gauss_legendre_tables()
    prob_h = np.asarray(cfg["d"], float) / np.sqrt(cfg["scales"]["G110"] / cfg["scales"]["alpha_ref"])
    out = np.zeros(6)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    N = (ctypes.c_int * 3)(*n)
    I3 = (ctypes.c_int * 3)(*idx)
    orc_lib().orc_offset_entry(N, pm, int(mimg), dp(prob_h), dp(t), dp(w), I3, dp(out))
    return out


def rel_inf(a, b):
    """max |a - b| / max |b|"""
    return float(np.abs(np.asarray(a, float) - np.asarray(b, float)).max()
                 / max(np.abs(np.asarray(b, float)).max(), 1e-300))


def oracle_field(P, prob, mask):
    return O.effective_field(P, prob, terms=mask) * prob.field_scale


def ps_of(cfg):
    """Reference magnitude for |dP|/Ps: tetragonal root of the first material
    at T (reading for paraelectric runs: 0.1 C/m^2)."""
    c = O.landau_coefficients(cfg["materials"][0], cfg["T"])
    a, b, cc = c["a1x"], c["a11"], c["a111"]
    if cc != 0:
        disc = b * b - 3 * a * cc
        if disc > 0:
            x = (-b + np.sqrt(disc)) / (3 * cc)
            if x > 0:
                return float(np.sqrt(x))
    elif a < 0 and b > 0:
        return float(np.sqrt(-a / (2 * b)))
    return 0.1
