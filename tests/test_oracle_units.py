"""Pins of the oracle's unit system (Table 2) that the parity tests at
P0 = 1 C/m^2 cannot see.

* P0 is only the unit of P: the SI trajectory, the SI fields and the
  energies in joules do not depend on it.  A wrong power of P0 in the
  reduced Landau coefficients, in E* = E/(alpha_ref P0) or in the energy
  unit alpha_ref P0^2 l0^3 breaks this (checked by planting each mistake).
* Joules: a uniform tetragonal BaTiO3 box with the Landau term only stores
  f(P_s) V, with f and P_s from Table 1 and the eq 12 root (the value at
  300 K, -2.313340e6 J/m^3, is derived from Table 1, not printed); a linear
  P_z(x) profile stores (G/2)(dP/dx)^2 per unit volume on each x edge; a
  uniformly polarised film has E = -P_z/(eps0 epsB) inside, so it stores
  P_z^2/(2 eps0 epsB) per unit volume; E_ext stores -E.P per unit volume.
"""
import numpy as np
import pytest

import tdgl_inputs as I
from oracle import tdgl_oracle as O

P0_ALT = 0.3016


def _cfg(P0, n=(8, 6, 4), periodic=(0, 0, 0), terms=15):
    cfg = I.config("c1")
    cfg.update(n=n, periodic=periodic, mimg=1, terms=terms, eext=(2e7, -1e7, 3e7))
    cfg["layers"] = [0] * n[2]
    cfg["scales"] = dict(cfg["scales"], P0=P0)
    return cfg


def _invariance_errors(n=(8, 6, 4)):
    P = I.initial_P(_cfg(1.0, n), 2)
    out = []
    res = []
    for P0 in (1.0, P0_ALT):
        prob = O.Problem(_cfg(P0, n))
        res.append((O.run_si(P, prob, "heun", 1e-3, 15), O.field_si(P, prob),
                    O.energies_si(P, prob)))
    (Pa, Ea, Fa), (Pb, Eb, Fb) = res
    out.append(np.abs(Pa - Pb).max() / np.abs(Pa).max())
    out.append(np.abs(Ea - Eb).max() / np.abs(Ea).max())
    for k in ("F_land", "F_grad", "F_elec", "F_ext"):
        out.append(abs(Fa[k] - Fb[k]) / abs(Fa[k]))
    return out


def test_si_results_do_not_depend_on_P0():
    errs = _invariance_errors()
    assert max(errs) < 1e-13, errs


@pytest.mark.parametrize("mistake", ["a111_power", "field_unit", "energy_unit"])
def test_P0_invariance_catches_planted_mistakes(monkeypatch, mistake):
    """Each plausible slip in a P0 power, planted in the oracle, fails the
    invariance above."""
    if mistake == "a111_power":
        good = O.reduce_coefficients

        def bad(c, P0, alpha_ref):
            r = good(c, P0, alpha_ref)
            r[5] = c["a111"] * P0 ** 2 / alpha_ref
            return r
        monkeypatch.setattr(O, "reduce_coefficients", bad)
    else:
        init = O.Problem.__init__

        def bad_init(self, cfg, tensor=True):
            init(self, cfg, tensor)
            if mistake == "field_unit":
                self.field_scale = self.alpha_ref * self.P0 ** 2
                self.eext = np.asarray(cfg.get("eext", (0, 0, 0)), float) / self.field_scale
            else:
                self.energy_scale = self.alpha_ref * self.P0 * self.l0 ** 3
        monkeypatch.setattr(O.Problem, "__init__", bad_init)
    assert max(_invariance_errors()) > 1e-3


def _tetragonal_root(T):
    m = I.BATIO3
    a = m["a1_slope"] * (T - m["a1_T0"])
    b = m["a11_slope"] * (T - m["a11_Tref"]) + m["a11_offset"]
    c = m["a111_slope"] * (T - m["a111_Tref"]) + m["a111_offset"]
    x = (-b + np.sqrt(b * b - 3 * a * c)) / (3 * c)        # x = P^2 (eq 12)
    return np.sqrt(x), a * x + b * x * x + c * x ** 3


@pytest.mark.parametrize("P0", [1.0, P0_ALT])
def test_landau_joules_of_a_uniform_tetragonal_box(P0):
    Ps, f = _tetragonal_root(300.0)
    assert abs(Ps - 0.264910) < 5e-7
    assert abs(f / -2.313340e6 - 1) < 5e-7               # Appendix value from Table 1
    n = (4, 3, 2)
    cfg = _cfg(P0, n, terms=O.LANDAU)
    prob = O.Problem(cfg)
    P = np.zeros((3, n[2], n[1], n[0]))
    P[2] = Ps
    V = np.prod(n) * 1e-27
    F = O.energies_si(P, prob)
    assert abs(F["F_land"] / (f * V) - 1) < 1e-12
    assert abs(F["meanP"][2] / Ps - 1) < 1e-14


@pytest.mark.parametrize("P0", [1.0, P0_ALT])
def test_gradient_joules_of_a_linear_profile(P0):
    n = (6, 3, 2)
    cfg = _cfg(P0, n, terms=O.GRAD)
    prob = O.Problem(cfg)
    G = cfg["gradient"]["G44"] + cfg["gradient"]["G44p"]    # P_z varying along x
    slope = 2.0e7                                            # C/m^2 per m
    h = cfg["d"][0]
    P = np.zeros((3, n[2], n[1], n[0]))
    P[2] = slope * (np.arange(n[0]) * h)[None, None, :]
    edges = (n[0] - 1) * n[1] * n[2]
    want = 0.5 * G * slope ** 2 * edges * h ** 3
    F = O.energies_si(P, prob)
    assert abs(F["F_grad"] / want - 1) < 1e-12


@pytest.mark.parametrize("P0", [1.0, P0_ALT])
def test_electrostatic_and_external_joules_of_a_uniform_film(P0):
    n = (8, 8, 3)
    cfg = _cfg(P0, n, periodic=(1, 1, 0), terms=O.ELEC | O.EXT)
    prob = O.Problem(cfg)
    Pz = 0.2
    P = np.zeros((3, n[2], n[1], n[0]))
    P[2] = Pz
    V = np.prod(n) * 1e-27
    eps = I.EPS0 * cfg["scales"]["eps_b"]
    F = O.energies_si(P, prob)
    assert abs(F["F_elec"] / (Pz * Pz / (2 * eps) * V) - 1) < 1e-12
    assert abs(F["F_ext"] / (-cfg["eext"][2] * Pz * V) - 1) < 1e-12
    E = O.field_si(P, prob, terms=O.ELEC)
    assert np.abs(E[2] / (-Pz / eps) - 1).max() < 1e-12
