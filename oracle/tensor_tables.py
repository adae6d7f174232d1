"""Stored 40-digit tensor tables — TEST INFRASTRUCTURE ONLY.

The tables under tests/golden/tensor_mp/ hold the octant of the
cell-averaged dipolar tensor (Newell closed form in 40-digit arithmetic,
oracle/tensor_mp.py) for the grids the parity tests use.  They are written
by tests/golden/make_tensor_mp_tables.py, which calls nothing but oracle/.
This module unfolds an octant to the full offset table of the oracle's
layout ([6][Kz][Ky][Kx]; K = 2n - 1 for open, n for periodic dimensions).
"""
from __future__ import annotations

import glob
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "tests", "golden", "tensor_mp")

# sign of each component under a mirror of one axis: xx yy zz even; xy odd
# in x and y; xz odd in x and z; yz odd in y and z
_ODD = [(), (), (), (0, 1), (0, 2), (1, 2)]


def unfold(oct_tab, n, periodic):
    """Full table from the octant oct_tab[6][Az][Ay][Ax]."""
    idx, sgn = [], []
    for k in range(3):
        if periodic[k]:
            i = np.arange(n[k])
            a = np.minimum(i, n[k] - i)
            s = np.where(i <= n[k] // 2, 1.0, -1.0)
        else:
            o = np.arange(2 * n[k] - 1) - (n[k] - 1)
            a = np.abs(o)
            s = np.where(o >= 0, 1.0, -1.0)
        idx.append(a)
        sgn.append(s)
    full = oct_tab[:, idx[2][:, None, None], idx[1][None, :, None], idx[0][None, None, :]].copy()
    for q in range(6):
        for k in _ODD[q]:
            shape = [1, 1, 1]
            shape[2 - k] = -1
            full[q] *= sgn[k].reshape(shape)
    return full


def key_of(n, periodic, mimg, h):
    m = int(mimg) if any(periodic) else 0
    return (tuple(int(v) for v in n), tuple(int(bool(p)) for p in periodic), m,
            tuple(float(v) for v in h))


_CACHE = None


def _load_all():
    global _CACHE
    if _CACHE is None:
        _CACHE = {}
        for f in sorted(glob.glob(os.path.join(GOLDEN, "*.npz"))):
            with np.load(f, allow_pickle=False) as d:
                k = key_of(d["n"], d["periodic"], int(d["mimg"]), d["h"])
                _CACHE[k] = np.array(d["octant"])
    return _CACHE


def lookup(n, periodic, mimg, h):
    """Full table for the geometry if a stored one matches exactly, else None."""
    oct_tab = _load_all().get(key_of(n, periodic, mimg, h))
    if oct_tab is None:
        return None
    return unfold(oct_tab, n, periodic)


def stored_keys():
    return list(_load_all())
