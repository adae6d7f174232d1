"""Pins for the oracle's electrostatic field (eqs 5-6) and energies (eq 2).

* the FFT evaluation equals the direct double sum over cells (open, in-plane
  periodic and fully periodic grids, ragged sizes);
* exact fields: a single cube cell and a uniformly polarised cube give
  -kappa P/3; an in-plane periodic film polarised uniformly along z gives
  -kappa P_z in every cell (SI: -P/(eps0 epsB)), and 0 for in-plane P;
* the field of every term is minus the gradient of its energy (eq 1 as a
  gradient flow), and the energy decreases along an Euler trajectory.
"""
import numpy as np
import pytest

import tdgl_inputs as I
from oracle import tdgl_oracle as O


def _film(n, periodic, mimg=2, **kw):
    cfg = I.config("c1")
    cfg.update(n=n, periodic=periodic, layers=[0] * n[2], mimg=mimg)
    cfg.update(kw)
    return cfg


@pytest.mark.parametrize("n,periodic", [((4, 3, 2), (0, 0, 0)), ((5, 4, 3), (0, 0, 0)),
                                        ((7, 2, 3), (0, 0, 0)), ((8, 6, 3), (1, 1, 0)),
                                        ((4, 4, 4), (1, 1, 1))])
def test_direct_sum_equals_fft(n, periodic):
    cfg = _film(n, periodic)
    prob = O.Problem(cfg)
    P = I.initial_P(cfg, 11)
    Hd = O.elec_field_direct(P, prob)
    Hf = O.elec_field_fft(P, prob)
    assert np.abs(Hd - Hf).max() <= 1e-13 * np.abs(Hd).max()


def test_direct_sum_with_vacuum_layers():
    cfg = _film((5, 4, 4), (0, 0, 0))
    cfg["layers"] = [0, 0, -1, 0]
    prob = O.Problem(cfg)
    P = I.initial_P(cfg, 2)
    assert not np.any(P[:, 2])
    Hd = O.elec_field_direct(P, prob)
    Hf = O.elec_field_fft(P, prob)
    assert np.abs(Hd - Hf).max() <= 1e-13 * np.abs(Hd).max()


def test_single_cell_field():
    prob = O.Problem(_film((1, 1, 1), (0, 0, 0)))
    p = np.array([0.3, -0.1, 0.2])
    H = O.elec_field_fft(p[:, None, None, None], prob)[:, 0, 0, 0]
    assert np.allclose(H, -prob.kappa * p / 3, rtol=1e-14)


def test_uniform_cube_mean_field():
    prob = O.Problem(_film((6, 6, 6), (0, 0, 0)))
    p = np.array([0.3, -0.1, 0.2])
    P = np.broadcast_to(p[:, None, None, None], (3, 6, 6, 6)).copy()
    H = O.elec_field_fft(P, prob)
    assert np.allclose(H.reshape(3, -1).mean(axis=1), -prob.kappa * p / 3, rtol=1e-13)


@pytest.mark.parametrize("mimg", [0, 3])
def test_periodic_slab_depolarisation(mimg):
    n = (8, 8, 3)
    prob = O.Problem(_film(n, (1, 1, 0), mimg=mimg))
    P = np.zeros((3,) + n[::-1])
    P[2] = 0.26
    H = O.elec_field_fft(P, prob)
    assert np.allclose(H[2], -prob.kappa * 0.26, rtol=1e-13)
    assert np.abs(H[:2]).max() < 1e-13 * prob.kappa
    # SI: E = -P/(eps0 epsB)
    E_si = H[2, 0, 0, 0] * prob.field_scale
    assert E_si == pytest.approx(-0.26 / (O.EPS0 * prob.eps_b), rel=1e-13)
    P = np.zeros((3,) + n[::-1])
    P[0], P[1] = 0.2, -0.1
    H = O.elec_field_fft(P, prob)
    assert np.abs(H).max() < 1e-13 * prob.kappa


def test_periodic_images_converge():
    n = (8, 8, 3)
    P = I.initial_P(_film(n, (1, 1, 0)), 4)
    fields = [O.elec_field_fft(P, O.Problem(_film(n, (1, 1, 0), mimg=m))) for m in (2, 4, 8, 16)]
    d = [np.abs(fields[k] - fields[-1]).max() for k in range(3)]
    assert d[0] > d[1] > d[2]
    assert d[2] < 2e-4 * np.abs(fields[-1]).max()


def _total_energy(P, prob):
    return O.energies(P, prob)["F_total"]


@pytest.mark.parametrize("n,periodic,layers", [((4, 3, 3), (0, 0, 0), None),
                                               ((4, 4, 3), (1, 1, 0), None),
                                               ((4, 3, 4), (0, 0, 0), [0, 1, -1, 0])])
def test_field_is_minus_energy_gradient(n, periodic, layers):
    mats = [I.BATIO3, dict(I.BATIO3, a1_T0=400.0, a12=1e8)]
    cfg = _film(n, periodic, eext=(1e6, -2e6, 3e6), materials=mats)
    if layers is not None:
        cfg["layers"] = layers
    prob = O.Problem(cfg)
    P = I.initial_P(cfg, 9) * 4
    H = O.effective_field(P, prob)
    rng = np.random.Generator(np.random.PCG64(1))
    eps = 1e-6
    for _ in range(6):
        c = tuple(rng.integers(0, s) for s in (3, n[2], n[1], n[0]))
        if prob.layers[c[1]] < 0:
            continue
        Pp, Pm = P.copy(), P.copy()
        Pp[c] += eps
        Pm[c] -= eps
        g = (_total_energy(Pp, prob) - _total_energy(Pm, prob)) / (2 * eps)
        assert -g / prob.dV == pytest.approx(H[c], rel=2e-7, abs=1e-8)


def test_energy_descends_along_euler():
    cfg = _film((6, 5, 4), (0, 0, 0))
    prob = O.Problem(cfg)
    P = I.initial_P(cfg, 3)
    F = [_total_energy(P, prob)]
    for _ in range(60):
        P = O.step_euler(P, prob, 1e-3)
        F.append(_total_energy(P, prob))
    assert np.all(np.diff(F) < 0)
