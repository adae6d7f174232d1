"""Pins for the oracle's gradient term, integrators and energy.

* eq 10 (section 4.1): the relaxed 1-D 180-degree wall of the 2-4 model with
  the paper's parameters converges to the tanh profile at second order in h.
* the sixth-order BaTiO3 wall (closed form derived from the first integral
  G P'^2/2 = f(P) - f(Ps) of the 1-D stationary equation) converges the
  same way.
* an exact discrete eigenmode of the linear problem decays by exactly the
  Euler / Heun amplification factor (pins the Laplacian with periodic and
  open boundaries, and both integrators).
* Euler is first order, Heun second order in dtau on the nonlinear problem.
"""
import copy
import json
import os

import numpy as np
import pytest

import tdgl_inputs as I
from oracle import tdgl_oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _chain_cfg(material, gradient, scales, nx, h, T):
    return dict(n=(nx, 1, 1), d=(h, 1e-9, 1e-9), periodic=(0, 0, 0), mimg=0,
                materials=[material], layers=[0], gradient=gradient, scales=scales,
                T=T, eext=(0, 0, 0), terms=O.LANDAU | O.GRAD)


def _relax_wall(cfg, start, tau, dtau):
    """Relax a 1-D chain from start(x) (x in metres, wall centred between
    the two middle cells, so symmetry pins its position)."""
    prob = O.Problem(cfg)
    nx = cfg["n"][0]
    x = (np.arange(nx) + 0.5 - nx / 2) * prob.h[0] * prob.l0
    P = np.zeros((3, 1, 1, nx))
    P[2, 0, 0] = start(x)
    for _ in range(int(round(tau / dtau))):
        P = O.step_heun(P, prob, dtau)
    return x, P[2, 0, 0]


def test_tanh_wall_eq10_second_order():
    g = json.load(open(os.path.join(GOLD, "wall_180_params.json")))
    a1, a11, G = g["alpha1"], g["alpha11"], g["G44"] + g["G44p"]
    mat = dict(I.BATIO3)
    mat.update(a1_form=0, a1_slope=1.0, a1_T0=-a1, a11_slope=0.0, a11_offset=a11,
               a12=0.0, a111_slope=0.0, a111_offset=0.0, a112=0.0, a123=0.0)
    grad = dict(G11=0.0, G12=0.0, G44=g["G44"], G44p=g["G44p"])
    scales = dict(P0=1.0, alpha_ref=abs(a1), G110=G, eps_b=1.0)
    xi = np.sqrt(G / abs(a1))
    Ps = np.sqrt(abs(a1) / (2 * a11))
    errs = []
    for k in (4, 8, 16):
        h = xi / k
        exact_fn = lambda x: Ps * np.tanh(x / xi)
        x, Pz = _relax_wall(_chain_cfg(mat, grad, scales, 20 * k, h, 0.0), exact_fn,
                            tau=10.0, dtau=0.25 / k**2)
        exact = exact_fn(x)
        errs.append(np.abs(Pz - exact).max() / Ps)
    assert errs[-1] < 2e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def test_sixth_order_bto_wall_second_order():
    T = 300.0
    a1 = 3.34e5 * (T - 381.0)
    a11 = 4.69e6 * (T - 393.0) - 2.02e8
    a111 = -5.52e7 * (T - 393.0) + 2.76e9
    G = 5.1e-10
    Ps = np.sqrt((-a11 + np.sqrt(a11 * a11 - 3 * a1 * a111)) / (3 * a111))
    c = a11 / a111 + 2 * Ps**2
    xi6 = np.sqrt(G / (2 * a111)) / (Ps * np.sqrt(Ps**2 + c))
    scales = dict(P0=1.0, alpha_ref=abs(a1), G110=G, eps_b=45.0)
    l0 = np.sqrt(G / abs(a1))
    errs = []
    for hs in (0.2, 0.1, 0.05):
        nx = int(round(12 * xi6 / (hs * l0) / 2)) * 2
        def exact_fn(x):
            u = x / xi6
            return Ps * np.sqrt(c) * np.tanh(u) / np.sqrt(c + Ps**2 / np.cosh(u)**2)
        x, Pz = _relax_wall(_chain_cfg(copy.deepcopy(I.BATIO3), I.isotropic_gradient(G),
                                       scales, nx, hs * l0, T), exact_fn,
                            tau=10.0, dtau=0.2 * hs**2)
        exact = exact_fn(x)
        errs.append(np.abs(Pz - exact).max() / Ps)
    assert errs[-1] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def _linear_cfg(n, periodic):
    mat = dict(I.BATIO3)
    mat.update(a1_form=0, a1_slope=2.7054e7, a1_T0=0.0, a11_slope=0.0, a11_offset=0.0,
               a12=0.0, a111_slope=0.0, a111_offset=0.0, a112=0.0, a123=0.0)
    return dict(n=n, d=(1.0e-9, 1.3e-9, 0.8e-9), periodic=periodic, mimg=0,
                materials=[mat], layers=[0] * n[2], gradient=I.isotropic_gradient(5.1e-10),
                scales=dict(P0=1.0, alpha_ref=2.7054e7, G110=5.1e-10, eps_b=45.0),
                T=1.0, eext=(0, 0, 0), terms=O.LANDAU | O.GRAD)


@pytest.mark.parametrize("scheme", ["euler", "heun"])
def test_exact_discrete_mode(scheme):
    n = (8, 6, 5)
    prob = O.Problem(_linear_cfg(n, (1, 0, 0)))
    kx, ky, kz = 3, 2, 1
    nx, ny, nz = n
    xi = np.arange(nx)
    yj = np.arange(ny)
    zk = np.arange(nz)
    mode = (np.cos(np.pi * kz * (zk + 0.5) / nz)[:, None, None]
            * np.cos(np.pi * ky * (yj + 0.5) / ny)[None, :, None]
            * np.cos(2 * np.pi * kx * xi / nx)[None, None, :])
    A = np.array([0.3, -0.2, 0.1])
    P0 = A[:, None, None, None] * mode[None]
    lam = 2 * prob.coef[0, 0] + sum(
        4 * np.sin(th / 2) ** 2 / prob.h[d] ** 2
        for d, th in ((0, 2 * np.pi * kx / nx), (1, np.pi * ky / ny), (2, np.pi * kz / nz)))
    dtau, steps = 2e-3, 50
    z = -dtau * lam
    amp = (1 + z) if scheme == "euler" else (1 + z + z * z / 2)
    P = O.run(P0, prob, scheme, dtau, steps)
    assert np.allclose(P, P0 * amp**steps, rtol=0, atol=1e-14)


def test_ab3m2_third_order_on_an_exact_mode():
    """Linear Landau + gradient problem, one discrete eigenmode: dP/dtau =
    -lam P has the solution P0 exp(-lam tau); the multistep scheme's error
    against it falls 8x per halving of dtau (third order, including the
    two Heun start-up steps)."""
    n = (8, 6, 5)
    prob = O.Problem(_linear_cfg(n, (1, 0, 0)))
    nx, ny, nz = n
    mode = (np.cos(np.pi * (np.arange(nz) + 0.5) / nz)[:, None, None]
            * np.cos(np.pi * 2 * (np.arange(ny) + 0.5) / ny)[None, :, None]
            * np.cos(2 * np.pi * np.arange(nx) / nx)[None, None, :])
    P0 = np.array([0.3, -0.2, 0.1])[:, None, None, None] * mode[None]
    lam = 2 * prob.coef[0, 0] + sum(
        4 * np.sin(th / 2) ** 2 / prob.h[d] ** 2
        for d, th in ((0, 2 * np.pi / nx), (1, 2 * np.pi / ny), (2, np.pi / nz)))
    tau = 0.3
    exact = P0 * np.exp(-lam * tau)
    errs = [np.abs(O.run(P0, prob, "ab3m2", tau / m, m) - exact).max() for m in (120, 240, 480)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 3) < 0.2), (errs, rates)


@pytest.mark.parametrize("scheme,order", [("euler", 1), ("heun", 2), ("ab3m2", 3)])
def test_integrator_order(scheme, order):
    cfg = I.config("c1")
    cfg.update(n=(4, 4, 2), layers=[0, 0])
    prob = O.Problem(cfg)
    P0 = I.initial_P(cfg, 5)
    tau = 0.2
    ref = O.run(P0, prob, "heun" if order < 3 else "ab3m2", tau / 1600, 1600)
    errs = []
    for m in ((50, 100) if order < 3 else (100, 200)):
        errs.append(np.abs(O.run(P0, prob, scheme, tau / m, m) - ref).max())
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - order) < (0.15 if order < 3 else 0.2), (errs, rate)


def test_rk45_tableau_order_conditions():
    """The Dormand-Prince weights satisfy the quadrature order conditions
    (fifth order for B, fourth for BS), every row sums to its node, and the
    last stage is taken at the fifth-order solution."""
    A, B, BS, C = O.DP_A, np.array(O.DP_B), np.array(O.DP_BS), np.array(O.DP_C)
    for i in range(1, 7):
        assert abs(sum(A[i]) - C[i]) < 1e-15
    assert np.allclose(A[6] + [0.0], B, rtol=0, atol=1e-16)
    for q in range(5):
        assert abs(np.dot(B, C ** q) - 1 / (q + 1)) < 1e-14, q
    for q in range(4):
        assert abs(np.dot(BS, C ** q) - 1 / (q + 1)) < 1e-14, q
    # third-order tree sum_i b_i sum_j a_ij c_j = 1/6 (both weight sets)
    ac = np.array([0.0] + [np.dot(A[i], C[:i]) for i in range(1, 7)])
    assert abs(np.dot(B, ac) - 1 / 6) < 1e-14 and abs(np.dot(BS, ac) - 1 / 6) < 1e-14


def _mode_problem():
    n = (8, 6, 5)
    prob = O.Problem(_linear_cfg(n, (1, 0, 0)))
    nx, ny, nz = n
    mode = (np.cos(np.pi * (np.arange(nz) + 0.5) / nz)[:, None, None]
            * np.cos(np.pi * 2 * (np.arange(ny) + 0.5) / ny)[None, :, None]
            * np.cos(2 * np.pi * np.arange(nx) / nx)[None, None, :])
    P0 = np.array([0.3, -0.2, 0.1])[:, None, None, None] * mode[None]
    lam = 2 * prob.coef[0, 0] + sum(
        4 * np.sin(th / 2) ** 2 / prob.h[d] ** 2
        for d, th in ((0, 2 * np.pi / nx), (1, 2 * np.pi / ny), (2, np.pi / nz)))
    return prob, P0, lam


def test_rk45_fifth_order_on_an_exact_mode():
    """Fixed steps (tolerances so loose that every step is accepted): the
    error against P0 exp(-lam tau) falls 32x per halving of h."""
    prob, P0, lam = _mode_problem()
    tau = 0.1                                  # h lam from 0.36 down to 0.09
    errs = []
    for m in (16, 32, 64):
        P = P0
        for _ in range(m):
            P, ok, _, _ = O.step_rk45(P, prob, tau / m, 1e30, 1e30)
            assert ok
        errs.append(np.abs(P - P0 * np.exp(-lam * tau)).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 5) < 0.3), (errs, rates)


def test_rk45_error_control_follows_the_tolerance():
    """Adaptive runs to the same time: the error against the exact mode
    shrinks with rtol, stays within a small multiple of it, and the tighter
    run takes more steps."""
    prob, P0, lam = _mode_problem()
    results = []
    for rtol in (1e-5, 1e-8):
        P, tau, h, tries = P0, 0.0, 1e-3, 0
        steps = 0
        while tau < 0.4 - 1e-15:
            hh = min(h, 0.4 - tau)
            Pn, ok, h, _ = O.step_rk45(P, prob, hh, 1e-12, rtol)
            if ok:
                P, tau, steps = Pn, tau + hh, steps + 1
        err = np.abs(P - P0 * np.exp(-lam * 0.4)).max() / np.abs(P0).max()
        results.append((err, steps))
    (e1, s1), (e2, s2) = results
    assert e2 < e1 and s2 > s1
    assert e1 < 10 * 1e-5 and e2 < 10 * 1e-8, results
