"""Pins for the oracle's dipolar tensor (eq 6 for cell-wise uniform P).

Each check ties the C oracle to something it does not compute itself: the
defining differential identities of Newell's f and g, exact values of the
self term, Laplace's equation, the point-dipole limit, an independent closed
form (Aharoni's prism factor), and agreement of two unrelated evaluations
(long-double closed form vs Gauss-Legendre quadrature).
"""
import numpy as np
import pytest

from oracle import lib as tensor_lib
from oracle import tdgl_oracle as O


def _mixed_fd(fn, p, orders, h=2e-2):
    """Central finite difference of fn at p with the given derivative orders
    (each 0, 1 or 2), Richardson-extrapolated to O(h^4)."""
    def once(hh):
        w1 = {-1: -0.5, 0: 0.0, 1: 0.5}
        w2 = {-1: 1.0, 0: -2.0, 1: 1.0}
        stencils = [({0: 1.0} if o == 0 else (w1 if o == 1 else w2)) for o in orders]
        s = 0.0
        for a, wa in stencils[0].items():
            for b, wb in stencils[1].items():
                for c, wc in stencils[2].items():
                    if wa * wb * wc == 0.0:
                        continue
                    s += wa * wb * wc * fn(p[0] + a * hh, p[1] + b * hh, p[2] + c * hh)
        return s / hh ** sum(orders)
    return (4 * once(h / 2) - once(h)) / 3


@pytest.mark.parametrize("p", [(0.7, 1.3, 0.9), (2.1, 0.4, 1.7), (1.2, 2.5, 3.1)])
def test_newell_f_g_identities(p):
    L = tensor_lib()
    r = np.sqrt(sum(v * v for v in p))
    d_f = _mixed_fd(L.orc_newell_f, p, (0, 2, 2))
    d_g = _mixed_fd(L.orc_newell_g, p, (1, 1, 2))
    assert abs(d_f * r - 1.0) < 1e-5
    assert abs(d_g * r - 1.0) < 1e-5


def test_self_term_cube_is_one_third():
    N = O.newell_tensor((0, 0, 0), (1, 1, 1))
    assert np.allclose(N[:3], 1 / 3, rtol=0, atol=2e-16)
    assert np.all(np.abs(N[3:]) < 1e-18)


@pytest.mark.parametrize("d", [(1, 2, 3), (1, 1, 0.5), (2.0, 0.7, 1.3)])
def test_self_term_trace_is_one(d):
    N = O.newell_tensor((0, 0, 0), d)
    assert abs(N[:3].sum() - 1.0) < 1e-15


@pytest.mark.parametrize("o", [(1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 1, 0), (3, 2, 1),
                               (7, 0, 2), (12, 9, 4), (40, 3, 1)])
def test_trace_vanishes_off_origin(o):
    N = O.cell_tensor(o, (1, 1, 1))
    assert abs(N[:3].sum()) < 1e-15 * max(1.0, np.abs(N).max() * 1e3)


@pytest.mark.parametrize("R", [(2, 0, 0), (2, 1, 1), (2, 2, 2), (3, 2, 1), (3, 0, 1)])
def test_closed_form_matches_quadrature(R):
    """Two unrelated evaluations of the same double integral."""
    a = O.newell_tensor(R, (1, 1, 1))
    b = O.quad_tensor(R, (1, 1, 1), 20)
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(a))


def test_closed_form_matches_quadrature_noncubic():
    d = (1.0, 1.5, 0.8)
    for o in [(2, 1, 0), (2, 0, 3)]:
        R = tuple(o[k] * d[k] for k in range(3))
        a = O.newell_tensor(R, d)
        b = O.quad_tensor(R, d, 22)
        assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_quadrature_order_rule_converged():
    """The adaptive order gives the same value as a much higher order."""
    for o in [(2, 0, 0), (2, 1, 1), (4, 0, 1), (6, 5, 3), (20, 3, 7), (130, 0, 2)]:
        a = O.cell_tensor(o, (1, 1, 1))
        b = O.quad_tensor(o, (1, 1, 1), 23)
        assert np.max(np.abs(a - b)) <= 2e-15 * np.max(np.abs(a)), o


def test_parity_and_symmetry():
    for o in [(3, 2, 1), (1, 1, 0), (5, 0, 2)]:
        N = O.cell_tensor(o, (1, 1, 1))
        for sx, sy, sz in [(-1, 1, 1), (1, -1, 1), (1, 1, -1), (-1, -1, -1)]:
            M = O.cell_tensor((sx * o[0], sy * o[1], sz * o[2]), (1, 1, 1))
            exp = N * np.array([1, 1, 1, sx * sy, sx * sz, sy * sz])
            assert np.allclose(M, exp, rtol=1e-15, atol=1e-19)
        # exchanging x and y exchanges xx<->yy and xz<->yz
        P = O.cell_tensor((o[1], o[0], o[2]), (1, 1, 1))
        assert np.allclose(P, N[[1, 0, 2, 3, 5, 4]], rtol=1e-14, atol=1e-19)


def test_far_field_tends_to_point_dipole():
    for o in [(40, 17, 9), (90, 0, 30)]:
        R = np.array(o, float)
        r = np.linalg.norm(R)
        dip = np.array([r * r - 3 * R[0] ** 2, r * r - 3 * R[1] ** 2, r * r - 3 * R[2] ** 2,
                        -3 * R[0] * R[1], -3 * R[0] * R[2], -3 * R[1] * R[2]]) / (4 * np.pi * r ** 5)
        N = O.cell_tensor(o, (1, 1, 1))
        # cubes: the (d/r)^2 correction vanishes (harmonic kernel), next is (d/r)^4
        assert np.max(np.abs(N - dip)) <= 5.0 / r ** 4 * np.max(np.abs(dip))


def _aharoni_nzz(a, b, c):
    """Demagnetising factor along z of a 2a x 2b x 2c prism (Aharoni 1998)."""
    r = np.sqrt(a * a + b * b + c * c)
    ab, bc, ac = np.sqrt(a * a + b * b), np.sqrt(b * b + c * c), np.sqrt(a * a + c * c)
    s = ((b * b - c * c) / (2 * b * c) * np.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * np.log((r - b) / (r + b))
         + b / (2 * c) * np.log((ab + a) / (ab - a)) + a / (2 * c) * np.log((ab + b) / (ab - b))
         + c / (2 * a) * np.log((bc - b) / (bc + b)) + c / (2 * b) * np.log((ac - a) / (ac + a))
         + 2 * np.arctan(a * b / (c * r)) + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r
         + c / (a * b) * (ac + bc) - (ab ** 3 + bc ** 3 + ac ** 3) / (3 * a * b * c))
    return s / np.pi


@pytest.mark.parametrize("n", [(4, 3, 2), (5, 5, 5), (9, 4, 3)])
def test_box_sum_rule(n):
    """Sum of N over all cell pairs of a box / cells = the box's own average
    tensor (near and far entries together)."""
    nx, ny, nz = n
    tab = O.offset_table(n, (0, 0, 0), 0, (1.0, 1.0, 1.0))
    cnt = [np.array([s - abs(i - (s - 1)) for i in range(2 * s - 1)], float) for s in n]
    w = cnt[2][:, None, None] * cnt[1][None, :, None] * cnt[0][None, None, :]
    S = np.array([(tab[q] * w).sum() for q in range(6)]) / (nx * ny * nz)
    box = O.newell_tensor((0, 0, 0), (nx, ny, nz))
    assert np.max(np.abs(S - box)) < 1e-14
    assert abs(box[2] - _aharoni_nzz(nx / 2, ny / 2, nz / 2)) < 1e-13
    if nx == ny == nz:
        assert np.allclose(S[:3], 1 / 3, atol=1e-14)
