"""Pins for the oracle's 40-digit dipolar tensor (oracle/tensor_mp.py) and
its stored tables, which the GPU tensor is compared with.

The 40-digit closed form is tied to facts it does not compute itself: the
defining differential identities of Newell's f and g (checked by mpmath's
numerical differentiation), the exact self term of a cube, the traces fixed
by Laplace's equation, the parity rules, the point-dipole limit and
Aharoni's independent closed form for a prism.  The stored tables are
re-derived at sampled entries (so a stale file fails), and the oracle's fast
C quadrature is held to them on every stored grid.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import tdgl_oracle as O
from oracle import tensor_mp as TM
from oracle import tensor_tables as TT
from tests.test_oracle_tensor import _aharoni_nzz


@pytest.mark.parametrize("p", [(0.7, 1.3, 0.9), (2.1, 0.4, 1.7)])
def test_newell_identities_in_high_precision(p):
    with mp.workdps(30):
        x, y, z = (mp.mpf(v) for v in p)
        r = mp.sqrt(x * x + y * y + z * z)
        df = mp.diff(lambda a, b, c: TM.newell_f(a, b, c), (x, y, z), (0, 2, 2))
        dg = mp.diff(lambda a, b, c: TM.newell_g(a, b, c), (x, y, z), (1, 1, 2))
        assert abs(df * r - 1) < mp.mpf(10) ** -15
        assert abs(dg * r - 1) < mp.mpf(10) ** -15


def test_self_terms():
    cube = TM.Lattice((1.0, 1.0, 1.0)).tensor((0, 0, 0))
    box = TM.Lattice((1.0, 2.0, 3.0)).tensor((0, 0, 0))
    with mp.workdps(TM.DPS):
        for q in range(3):
            assert abs(cube[q] - mp.mpf(1) / 3) < mp.mpf(10) ** -35
        for q in range(3, 6):
            assert abs(cube[q]) < mp.mpf(10) ** -35
        assert abs(box[0] + box[1] + box[2] - 1) < mp.mpf(10) ** -35


@pytest.mark.parametrize("o", [(1, 0, 0), (1, 1, 1), (3, 2, 1), (12, 9, 4), (150, 3, 1)])
def test_trace_vanishes_and_parity(o):
    lat = TM.Lattice((0.9, 1.1, 0.7))
    N = lat.tensor(o)
    with mp.workdps(TM.DPS):
        scale = max(abs(v) for v in N)
        assert abs(N[0] + N[1] + N[2]) < mp.mpf(10) ** -24 * scale
        for s in [(-1, 1, 1), (1, -1, 1), (1, 1, -1)]:
            M = lat.tensor((s[0] * o[0], s[1] * o[1], s[2] * o[2]))
            sign = [1, 1, 1, s[0] * s[1], s[0] * s[2], s[1] * s[2]]
            for q in range(6):
                assert abs(M[q] - sign[q] * N[q]) < mp.mpf(10) ** -24 * scale


def test_far_field_point_dipole():
    """Cubes: the (d/r)^2 correction vanishes, the next term is (d/r)^4."""
    lat = TM.Lattice((1.0, 1.0, 1.0))
    for o in [(40, 17, 9), (300, 0, 100)]:
        R = np.array(o, float)
        r = np.linalg.norm(R)
        dip = np.array([r * r - 3 * R[0] ** 2, r * r - 3 * R[1] ** 2, r * r - 3 * R[2] ** 2,
                        -3 * R[0] * R[1], -3 * R[0] * R[2], -3 * R[1] * R[2]]) / (4 * np.pi * r ** 5)
        N = np.array([float(v) for v in lat.tensor(o)])
        assert np.max(np.abs(N - dip)) <= 5.0 / r ** 4 * np.max(np.abs(dip))


@pytest.mark.parametrize("n", [(4, 3, 2), (3, 3, 3)])
def test_box_sum_equals_aharoni(n):
    """Sum of N over all cell pairs of a box / cells = the box's own average
    tensor; its zz entry is Aharoni's prism factor."""
    lat = TM.Lattice((1.0, 1.0, 1.0))
    S = [mp.mpf(0)] * 6
    for oz in range(-(n[2] - 1), n[2]):
        for oy in range(-(n[1] - 1), n[1]):
            for ox in range(-(n[0] - 1), n[0]):
                w = (n[0] - abs(ox)) * (n[1] - abs(oy)) * (n[2] - abs(oz))
                t = lat.tensor((ox, oy, oz))
                for q in range(6):
                    S[q] += w * t[q]
    ncell = n[0] * n[1] * n[2]
    S = [float(v / ncell) for v in S]
    assert abs(S[2] - _aharoni_nzz(n[0] / 2, n[1] / 2, n[2] / 2)) < 1e-13
    assert abs(S[0] - _aharoni_nzz(n[1] / 2, n[2] / 2, n[0] / 2)) < 1e-13
    assert max(abs(v) for v in S[3:]) < 1e-15


def test_stored_tables_match_the_module():
    """Sampled octant entries of every stored table, recomputed."""
    keys = TT.stored_keys()
    assert len(keys) >= 6
    rng = np.random.Generator(np.random.PCG64(5))
    for key in keys:
        n, per, mimg, h = key
        oct_tab = TT._load_all()[key]
        lat = TM.Lattice(h)
        for _ in range(3):
            a = [int(rng.integers(0, oct_tab.shape[3 - k])) for k in range(3)]
            acc = [mp.mpf(0)] * 6
            with mp.workdps(TM.DPS):
                im = [TM.image_offsets(a[k] if per[k] else a[k] + n[k] - 1, n[k], per[k], mimg)
                      for k in range(3)]
                for ox, wx in im[0]:
                    for oy, wy in im[1]:
                        for oz, wz in im[2]:
                            t = lat.tensor((ox, oy, oz))
                            for q in range(6):
                                acc[q] += wx * wy * wz * t[q]
            want = np.array([float(v) for v in acc])
            got = oct_tab[:, a[2], a[1], a[0]]
            assert np.array_equal(got, want), (key, a)


def test_quadrature_tables_agree_with_the_closed_form():
    """The C quadrature (used where no 40-digit table is stored, e.g. large
    image windows) against the 40-digit tables, component by component."""
    for key in TT.stored_keys():
        n, per, mimg, h = key
        mp_tab = TT.lookup(n, per, mimg, h)
        q_tab = O.offset_table(n, per, mimg, h, k0_correction=False)
        for q in range(6):
            err = np.abs(mp_tab[q] - q_tab[q]).max() / np.abs(q_tab[q]).max()
            assert err < 1e-15, (key, q, err)


def test_oracle_problem_uses_the_closed_form_where_stored():
    import tdgl_inputs as I
    prob = O.Problem(I.config("c1"))
    assert prob.tensor_source == "newell_mp"
    prob2 = O.Problem(I.config("c2_small"))       # 16 images: quadrature
    assert prob2.tensor_source == "quadrature"
