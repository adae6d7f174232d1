"""The film's own check (section 4.1, eqs 8-10): the 128x128x32 film with the
electrostatic term off and noise on P_z only, 20000 FP32 Heun steps on the
GPU, then

* the y/z-averaged profile P_z(x) against the oracle's 1-D chain (the same
  discrete model along x, periodic, FP64) relaxed over the same 20000 steps
  from the y/z-averaged start: to first order in the noise the average of
  the 3-D run is exactly that chain (the averaged Laplacian along y and z
  vanishes for periodic and natural boundaries); |dP|/Ps <= 1e-5;
* the chain against the closed-form sixth-order wall (first integral of
  eq 3 with the gradient term), whose discretisation error is O(h^2):
  0.2303 reduced cells give about 9e-3 of Ps (the oracle's convergence pin
  measures 6.7e-3 at 0.2 and the ratio 4 per halving);
* the total energy (FP64 reduction) never increases between checkpoints
  (descent of eq 1 without noise), up to the FP32 state's round-off.
"""
import numpy as np
import pytest

import tdgl_inputs as I
from oracle import tdgl_oracle as O
from tests.gpu_helpers import announce, gpu_context

pytestmark = pytest.mark.gpu

STEPS = 20000
CHECK = 1000


def _closed_form_wall(T, G, x):
    """P(x) = Ps sqrt(c) tanh(x/xi6) / sqrt(c + Ps^2 sech^2(x/xi6)) with
    c = a11/a111 + 2 Ps^2, xi6 = sqrt(G/(2 a111)) / (Ps sqrt(Ps^2 + c))."""
    m = I.BATIO3
    a1 = m["a1_slope"] * (T - m["a1_T0"])
    a11 = m["a11_slope"] * (T - m["a11_Tref"]) + m["a11_offset"]
    a111 = m["a111_slope"] * (T - m["a111_Tref"]) + m["a111_offset"]
    Ps = np.sqrt((-a11 + np.sqrt(a11 * a11 - 3 * a1 * a111)) / (3 * a111))
    c = a11 / a111 + 2 * Ps**2
    xi6 = np.sqrt(G / (2 * a111)) / (Ps * np.sqrt(Ps**2 + c))
    u = x / xi6
    return Ps, Ps * np.sqrt(c) * np.tanh(u) / np.sqrt(c + Ps**2 / np.cosh(u)**2)


def test_film_wall_check_20000_steps():
    cfg = I.config("c2_wallcheck")
    nx, ny, nz = cfg["n"]
    announce("c2 wall check: %d FP32 Heun steps, electrostatics off" % STEPS)
    P0 = I.initial_P(cfg, 0, np.float32)
    assert not P0[0].any() and not P0[1].any()
    ctx = gpu_context(cfg, "f32")
    F = []
    try:
        ctx.set_P(P0)
        F.append(ctx.energies()[0][4])
        for _ in range(STEPS // CHECK):
            ctx.step(CHECK)
            F.append(ctx.energies()[0][4])
        P = ctx.get_P()
    finally:
        ctx.close()
    assert not P[0].any() and not P[1].any()     # every term of dF/dP_x is prop. to P_x

    # energy descent at every checkpoint (slack: FP32 state round-off of F)
    F = np.array(F)
    assert F[-1] < F[0]
    assert np.all(np.diff(F) <= 1e-7 * np.abs(F[1:])), np.diff(F)

    # the oracle's 1-D chain from the averaged start
    chain = dict(cfg, n=(nx, 1, 1), layers=[0], terms=O.LANDAU | O.GRAD)
    prob = O.Problem(chain)
    Pc = np.zeros((3, 1, 1, nx))
    Pc[2, 0, 0] = P0[2].astype(np.float64).mean(axis=(0, 1))
    Pc = O.run(Pc, prob, "heun", cfg["dtau"], STEPS)
    avg = P[2].astype(np.float64).mean(axis=(0, 1))
    x = (np.arange(nx) + 0.5 - nx / 2) * cfg["d"][0]
    inner = np.abs(x) < nx * cfg["d"][0] / 4
    Ps, exact = _closed_form_wall(cfg["T"], cfg["gradient"]["G11"], x)
    err_gpu = np.abs(avg - Pc[2, 0, 0])[inner].max() / Ps
    err_cf = np.abs(Pc[2, 0, 0] - exact)[inner].max() / Ps
    print("wall check: |avg - chain|/Ps = %.3e, |chain - closed form|/Ps = %.3e"
          % (err_gpu, err_cf))
    assert err_gpu <= 1e-5, err_gpu
    assert 4e-3 <= err_cf <= 1.2e-2, err_cf
