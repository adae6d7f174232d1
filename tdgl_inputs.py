"""Seeded synthetic inputs for the TDGL hot path.

This module is the only code shared by the GPU path's callers and the CPU
oracle.  It holds input *data* only: the material constants printed in the
paper's Table 1, the run recipes (grid, boundary, temperature, time step,
initial state) and the seeded generators of initial polarisation fields.  It
evaluates none of the method's arithmetic: no coefficient at a temperature,
no normalisation, no field, no time step.

Units are SI (C/m^2, V/m, K, m, J/m^3 coefficients as printed).
"""
from __future__ import annotations

import copy

import numpy as np

# --------------------------------------------------------------------------
# Table 1 (section 2).  alpha_1 has either the linear form
# alpha0*(T - T0) ("a1_form" 0) or the Barrett form
# A*(coth(Ts/T) - coth(Ts/T0)) ("a1_form" 1, SrTiO3).  alpha_11 and alpha_111
# are slope*(T - Tref) + offset.  "rs" multiplies the z part of the quadratic
# term (the strain parameter of the skyrmion study, section 4.4); 1 = none.
# --------------------------------------------------------------------------
BATIO3 = dict(
    a1_form=0, a1_slope=3.34e5, a1_T0=381.0, a1_A=0.0, a1_Ts=0.0,
    a11_slope=4.69e6, a11_Tref=393.0, a11_offset=-2.02e8,
    a12=3.23e8,
    a111_slope=-5.52e7, a111_Tref=393.0, a111_offset=2.76e9,
    a112=4.47e9, a123=4.91e9, rs=1.0,
)
BATIO3_GRADIENT = dict(G11=5.1e-10, G12=-2.0e-11, G44=2.0e-11, G44p=2.0e-11, G110=5.1e-10)

PBTIO3 = dict(
    a1_form=0, a1_slope=3.85e5, a1_T0=752.0, a1_A=0.0, a1_Ts=0.0,
    a11_slope=0.0, a11_Tref=0.0, a11_offset=-7.3e7,
    a12=7.5e8,
    a111_slope=0.0, a111_Tref=0.0, a111_offset=2.6e8,
    a112=6.1e8, a123=-3.7e9, rs=1.0,
)
PBTIO3_GRADIENT = dict(G11=1.038e-10, G12=0.0, G44=5.19e-11, G44p=5.19e-11, G110=1.73e-10)

# SrTiO3 as printed (prefactor 405 N m^2 C^-2, Ts = 54 K, reference 30 K);
# sixth-order coefficients are "-" in the table, i.e. zero.
SRTIO3 = dict(
    a1_form=1, a1_slope=0.0, a1_T0=30.0, a1_A=405.0, a1_Ts=54.0,
    a11_slope=0.0, a11_Tref=0.0, a11_offset=1.7e9,
    a12=1.37e9,
    a111_slope=0.0, a111_Tref=0.0, a111_offset=0.0,
    a112=0.0, a123=0.0, rs=1.0,
)

EPS0 = 8.8541878128e-12          # vacuum permittivity, F/m (CODATA 2018)

MATERIAL_KEYS = tuple(BATIO3.keys())


def isotropic_gradient(G: float) -> dict:
    """Gradient coefficients of an isotropic medium: G11 = G, G44 = G44' = G/2,
    G12 = 0, which turns eq 4's functional derivative into -G * Laplacian(P)."""
    return dict(G11=G, G12=0.0, G44=0.5 * G, G44p=0.5 * G)


# --------------------------------------------------------------------------
# Run recipes.  "layers": material index per z layer (-1 = vacuum).
# --------------------------------------------------------------------------
def _bto_film(nx, ny, nz, periodic, **kw):
    cfg = dict(
        n=(nx, ny, nz), d=(1e-9, 1e-9, 1e-9), periodic=periodic, mimg=16,
        materials=[copy.deepcopy(BATIO3)], layers=[0] * nz,
        gradient=isotropic_gradient(5.1e-10),
        scales=dict(P0=1.0, alpha_ref=2.7054e7, G110=5.1e-10, eps_b=45.0),
        T=300.0, eext=(0.0, 0.0, 0.0), terms=15,
    )
    cfg.update(kw)
    return cfg


def config(name: str) -> dict:
    """Return a fresh copy of a named run recipe."""
    if name == "c1":          # FP64 parity config: 16x16x8 open box
        return _bto_film(16, 16, 8, (0, 0, 0), precision="f64", scheme="euler",
                         dtau=1e-3, steps=1000, init=dict(kind="uniform", amp=0.05))
    if name == "c2":          # FP32 thin film, periodic in-plane, open z
        return _bto_film(128, 128, 32, (1, 1, 0), precision="f32", scheme="heun",
                         dtau=1e-3, steps=20000,
                         init=dict(kind="wall", Ps=0.264910, w=4.342e-9, noise=0.01,
                                   noise_xy=True))
    if name == "c2_wallcheck":  # same film, electrostatics off, noise on P_z only
        c = config("c2")
        c["terms"] = 1 | 2 | 8
        c["init"] = dict(kind="wall", Ps=0.264910, w=4.342e-9, noise=0.01, noise_xy=False)
        return c
    if name == "c2_small":    # parity-sized version of the C2 film
        return _bto_film(32, 32, 8, (1, 1, 0), precision="f32", scheme="heun",
                         dtau=1e-3, steps=1000,
                         init=dict(kind="wall", Ps=0.264910, w=4.342e-9, noise=0.01,
                                   noise_xy=True))
    if name in ("c4", "c4_small"):   # PbTiO3 / SrTiO3 bilayer, open box
        big = name == "c4"
        nx, ny, nz = (256, 256, 64) if big else (32, 32, 8)
        n_pto = 48 if big else 6
        return dict(
            n=(nx, ny, nz), d=(1e-9, 1e-9, 1e-9), periodic=(0, 0, 0), mimg=16,
            materials=[copy.deepcopy(PBTIO3), copy.deepcopy(SRTIO3)],
            layers=[0] * n_pto + [1] * (nz - n_pto),
            gradient=isotropic_gradient(1.038e-10),
            scales=dict(P0=1.0, alpha_ref=1.7402e8, G110=1.73e-10, eps_b=649.0),
            T=300.0, eext=(0.0, 0.0, 0.0), terms=15,
            precision="f32", scheme="heun", dtau=1e-3, steps=500,
            init=dict(kind="uniform", amp=0.1),
        )
    raise KeyError(name)


def c3_groups() -> list:
    """The batched workload: 64 open BaTiO3 boxes (1 nm cells, the c1 model)
    in three grid shapes -- 24 of 32x32x32, 24 of 64x64x16, 16 of 96x96x8 --
    with T ~ U(200, 450) K drawn from PCG64(2024) and P ~ U(-0.1, 0.1) C/m^2
    from per-instance seeds 100..163; FP32, Heun dtau = 1e-3.  Returns one
    recipe per grid shape with "T" a list and "seeds" the instance seeds."""
    rng = np.random.Generator(np.random.PCG64(2024))
    groups, seed = [], 100
    for n, count in (((32, 32, 32), 24), ((64, 64, 16), 24), ((96, 96, 8), 16)):
        c = _bto_film(n[0], n[1], n[2], (0, 0, 0), precision="f32", scheme="heun",
                      dtau=1e-3, steps=5000, init=dict(kind="uniform", amp=0.1))
        c["T"] = [float(t) for t in rng.uniform(200.0, 450.0, count)]
        c["seeds"] = list(range(seed, seed + count))
        seed += count
        groups.append(c)
    return groups


# --------------------------------------------------------------------------
# Seeded initial states.  numpy Generator(PCG64(seed)), C order [3][Nz][Ny][Nx];
# for single-precision runs the values are rounded to float32 first and both
# sides start from the rounded numbers.  Vacuum layers hold P = 0.
# --------------------------------------------------------------------------
def initial_P(cfg: dict, seed: int = 0, dtype=np.float64) -> np.ndarray:
    nx, ny, nz = cfg["n"]
    rng = np.random.Generator(np.random.PCG64(seed))
    init = cfg["init"]
    shape = (3, nz, ny, nx)
    if init["kind"] == "uniform":
        P = rng.uniform(-init["amp"], init["amp"], size=shape)
    elif init["kind"] == "wall":
        Ps, w = init["Ps"], init["w"]
        dx = cfg["d"][0]
        x = (np.arange(nx) + 0.5 - nx / 2) * dx
        sigma = init["noise"] * Ps
        P = np.zeros(shape)
        P[2] = Ps * np.tanh(x / w)[None, None, :]
        P[2] += rng.normal(0.0, sigma, size=(nz, ny, nx))
        if init.get("noise_xy", True):
            P[0] = rng.normal(0.0, sigma, size=(nz, ny, nx))
            P[1] = rng.normal(0.0, sigma, size=(nz, ny, nx))
    elif init["kind"] == "random_dir":
        # random orientation, magnitude uniform in (0, amp]
        v = rng.normal(size=shape)
        v /= np.linalg.norm(v, axis=0, keepdims=True)
        P = v * rng.uniform(0.0, init["amp"], size=shape[1:])[None]
    else:
        raise KeyError(init["kind"])
    lay = np.asarray(cfg["layers"])
    P[:, lay < 0] = 0.0
    P = np.ascontiguousarray(P.astype(dtype))
    return P


# --------------------------------------------------------------------------
# The learned initial-state proposal: seeded weights and sample conditions.
# Layer shapes of the encoder-decoder (width w): twelve 3x3x3 convolutions,
# (cin, cout) as listed; the parameter vector holds, per layer, W as
# [cout][27][cin] then b [cout].
# --------------------------------------------------------------------------
def net_layer_shapes(width: int) -> list:
    w = width
    return [(5, w), (w, w), (w, 2 * w), (2 * w, 2 * w), (2 * w, 4 * w), (4 * w, 4 * w),
            (4 * w, 4 * w), (4 * w, 2 * w), (2 * w, 2 * w), (2 * w, w), (w, w), (w, 3)]


def net_params(width: int, seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """Seeded weights: W ~ U(-a, a) with a = scale * sqrt(6 / (1.015625 * 27 cin))
    (He-uniform for a leaky ReLU of slope 1/8), biases ~ U(-0.05, 0.05) * scale;
    float32 values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for ci, co in net_layer_shapes(width):
        a = scale * np.sqrt(6.0 / (1.015625 * 27 * ci))
        parts.append(rng.uniform(-a, a, size=co * 27 * ci))
        parts.append(rng.uniform(-0.05 * scale, 0.05 * scale, size=co))
    return np.concatenate(parts).astype(np.float32)


def net_conditions(nsamples: int, shape, noise_div: int, seed: int,
                   T_range=(250.0, 450.0), thickness_range=None, amp: float = 0.1):
    """Sample conditions of the proposal: T ~ U(T_range) K, film thickness
    (layers) uniform in thickness_range (inclusive; default the full height),
    and low-resolution noise ~ U(-amp, amp) C/m^2 of shape
    [n][3][Z/s][Y/s][X/s].  Returns (T, thickness, noise) as float32 arrays."""
    Z, Y, X = shape
    s = noise_div
    rng = np.random.Generator(np.random.PCG64(seed))
    T = rng.uniform(T_range[0], T_range[1], size=nsamples)
    lo, hi = thickness_range if thickness_range else (Z, Z)
    th = rng.integers(lo, hi + 1, size=nsamples)
    noise = rng.uniform(-amp, amp, size=(nsamples, 3, Z // s, Y // s, X // s))
    return T.astype(np.float32), th.astype(np.float32), noise.astype(np.float32)


def noise_start(noise: np.ndarray, thickness, shape) -> np.ndarray:
    """The random start that goes with a noise field: the noise repeated to
    the cell grid, zero in the vacuum layers z >= thickness (C order
    [n][3][Z][Y][X], float32)."""
    Z, Y, X = shape
    s = Z // noise.shape[2]
    P = np.repeat(np.repeat(np.repeat(noise, s, 2), s, 3), s, 4).astype(np.float32)
    for i, t in enumerate(thickness):
        P[i, :, int(t):] = 0.0
    return np.ascontiguousarray(P)


def c5_recipe(thickness: int, shape=(16, 64, 64)) -> dict:
    """The learned-proposal workload: an open BaTiO3 box of nz x ny x nx
    1 nm cells (the c1 model) whose lowest `thickness` layers are the film
    and the rest vacuum; FP32 Heun dtau = 1e-3.  Conditions (T per sample,
    low-resolution noise) come from net_conditions; the random start that
    goes with them from noise_start."""
    nz, ny, nx = shape
    c = _bto_film(nx, ny, nz, (0, 0, 0), precision="f32", scheme="heun", dtau=1e-3,
                  steps=20000, init=dict(kind="uniform", amp=0.1))
    c["layers"] = [0] * int(thickness) + [-1] * (nz - int(thickness))
    return c
