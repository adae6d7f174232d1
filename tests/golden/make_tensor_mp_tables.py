"""Write the 40-digit tensor tables of tests/golden/tensor_mp/.

Calls nothing but oracle/ (oracle.tensor_mp, the Newell closed form in
mpmath) and the seeded-input module for the grid recipes.  Each file holds
the octant of the cell-averaged dipolar tensor of one parity-test geometry
(cells n, periodic flags, image count mimg, reduced cell size h).  Run from
the repository root:  python tests/golden/make_tensor_mp_tables.py
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import tdgl_inputs as I  # noqa: E402
from oracle import tensor_mp  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "tensor_mp")


def geometries():
    """(name, n, periodic, mimg, h) of the stored tables."""
    c1 = I.config("c1")
    s = c1["scales"]
    h_bto = tuple(float(v) for v in np.asarray(c1["d"], float) / np.sqrt(s["G110"] / s["alpha_ref"]))
    c4 = I.config("c4_small")
    s4 = c4["scales"]
    h_pto = tuple(float(v) for v in np.asarray(c4["d"], float) / np.sqrt(s4["G110"] / s4["alpha_ref"]))
    return [
        ("open_16x16x8", (16, 16, 8), (0, 0, 0), 0, h_bto),
        ("open_12x10x5", (12, 10, 5), (0, 0, 0), 0, h_bto),
        ("open_7x9x3", (7, 9, 3), (0, 0, 0), 0, h_bto),
        ("open_10x12x6", (10, 12, 6), (0, 0, 0), 0, h_bto),
        ("open_8x6x4", (8, 6, 4), (0, 0, 0), 0, h_bto),
        ("film_16x16x4_m2", (16, 16, 4), (1, 1, 0), 2, h_bto),
        ("bulk_8x16x8_m2", (8, 16, 8), (1, 1, 1), 2, h_bto),
        ("open_32x32x8_pto", (32, 32, 8), (0, 0, 0), 0, h_pto),
    ]


def make(geo):
    name, n, periodic, mimg, h = geo
    tab = np.asarray(tensor_mp.octant_table(n, periodic, mimg, h), dtype=np.float64)
    np.savez_compressed(os.path.join(OUT, name + ".npz"), octant=tab, n=np.asarray(n),
                        periodic=np.asarray(periodic), mimg=np.asarray(mimg), h=np.asarray(h),
                        dps=np.asarray(tensor_mp.DPS))
    return name, tab.shape


if __name__ == "__main__":
    os.makedirs(OUT, exist_ok=True)
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        for name, shape in pool.imap_unordered(make, geometries()):
            print("wrote", name, shape, flush=True)
