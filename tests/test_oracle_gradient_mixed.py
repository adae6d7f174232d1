"""The full gradient energy of eq 4 (G12 and G44 - G44' cross terms) in
the oracle: the field is minus the gradient of the discrete energy, and on
a periodic grid a plane wave sees the stencil's closed-form symbol."""
import numpy as np
import pytest

import tdgl_inputs as I
from oracle import tdgl_oracle as O

ANISO = dict(G11=5.1e-10, G12=-1.0e-10, G44=2.0e-10, G44p=0.5e-10)


def _cfg(n, periodic, layers=None, terms=O.GRAD):
    cfg = I.config("c1")
    cfg.update(n=n, periodic=periodic, mimg=0, terms=terms, eext=(1e6, 0.0, -2e6))
    cfg["layers"] = list(layers) if layers is not None else [0] * n[2]
    cfg["gradient"] = dict(ANISO)
    cfg["d"] = (1.0e-9, 1.2e-9, 0.9e-9)
    return cfg


@pytest.mark.parametrize("n,periodic,layers,terms", [
    ((5, 4, 3), (0, 0, 0), None, O.GRAD),
    ((4, 4, 4), (1, 1, 0), None, O.GRAD),
    ((4, 5, 5), (0, 0, 0), [0, 0, -1, 0, 0], O.GRAD),
    ((4, 4, 3), (1, 1, 0), None, O.LANDAU | O.GRAD | O.ELEC | O.EXT)])
def test_mixed_gradient_field_is_minus_energy_gradient(n, periodic, layers, terms):
    cfg = _cfg(n, periodic, layers, terms)
    prob = O.Problem(cfg)
    P = I.initial_P(cfg, 4) * 3
    H = O.effective_field(P, prob)
    eps = 1e-6
    rng = np.random.Generator(np.random.PCG64(3))
    checked = 0
    for _ in range(40):
        c = tuple(rng.integers(0, s) for s in (3, n[2], n[1], n[0]))
        if prob.layers[c[1]] < 0:
            continue
        Pp, Pm = P.copy(), P.copy()
        Pp[c] += eps
        Pm[c] -= eps
        g = (O.energies(Pp, prob)["F_total"] - O.energies(Pm, prob)["F_total"]) / (2 * eps)
        assert -g / prob.dV == pytest.approx(H[c], rel=2e-7, abs=1e-8), c
        checked += 1
    assert checked > 20


def test_plane_wave_symbol_on_a_periodic_grid():
    """P = a cos(k.r) on a fully periodic grid: H = -M(k) P with
    M_ii = g11 s_i^2 + (g44 + g44') sum_{j != i} s_j^2 and
    M_ij = (g12 + g44 - g44') t_i t_j, s = 2 sin(k h/2)/h, t = sin(k h)/h
    (the symbols of the 3-point second difference and of the central first
    difference)."""
    n = (8, 16, 8)
    cfg = _cfg(n, (1, 1, 1))
    prob = O.Problem(cfg)
    m = np.array([1, 3, 2])
    k = 2 * np.pi * m / np.array(n) / prob.h
    x = [np.arange(n[d]) * prob.h[d] for d in range(3)]
    phase = (k[2] * x[2][:, None, None] + k[1] * x[1][None, :, None] + k[0] * x[0][None, None, :])
    a = np.array([0.3, -0.2, 0.25])
    P = a[:, None, None, None] * np.cos(phase)[None]
    H = O.gradient_field(P, prob)
    s = 2 * np.sin(k * prob.h / 2) / prob.h
    t = np.sin(k * prob.h) / prob.h
    G = cfg["gradient"]
    g11, gd = G["G11"] / prob.G110, (G["G44"] + G["G44p"]) / prob.G110
    gx = (G["G12"] + G["G44"] - G["G44p"]) / prob.G110
    M = np.empty((3, 3))
    for i in range(3):
        for j in range(3):
            M[i, j] = (g11 * s[i]**2 + gd * (np.sum(s**2) - s[i]**2)) if i == j else gx * t[i] * t[j]
    ref = -(M @ a)[:, None, None, None] * np.cos(phase)[None]
    assert np.abs(H - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(gx) > 0 and np.abs(M - np.diag(np.diag(M))).max() > 0.02 * np.abs(M).max()
