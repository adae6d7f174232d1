"""Dipolar interaction tensor in 40-digit arithmetic (mpmath) — TEST
INFRASTRUCTURE ONLY.

Part of the CPU oracle: the parity tests, the smoke check and the
benchmark's CPU baseline may use it; the product library never does.

What it computes (paper section 2, eq 6, with P uniform inside every
finite-difference cell as section 3 prescribes): for cell-wise uniform P the
bound charges of eq 6 sit on the cell faces, and the field averaged over a
target cell is

    E_i(target) = -(1/(eps0 epsB)) sum_src N_ij(r_t - r_s) P_j(src),

with N the cell-averaged demagnetising tensor of two boxes.  This module
evaluates N by the closed form of Newell, Williams and Dunlop (J. Geophys.
Res. 98, 9551, 1993) at every offset, in 40 significant digits, so the
27-term difference that cancels as the offset grows keeps ~30 digits even
hundreds of cells away.  It is the plain definition of the tensor written
out; it uses no quadrature and no far-field approximation, and it shares
nothing with the library's construction (which integrates the kernel
numerically away from touching cells).

    Newell f: d^2/dy^2 d^2/dz^2 f(x, y, z) = 1/r, even in every argument,
    Newell g: d/dx d/dy d^2/dz^2 g(x, y, z) = 1/r, odd in x and y, even in z;
    N_xx(X) = (1/(4 pi V)) sum_{e in {-1,0,1}^3} c(e) f(X + e*h),
    N_xy(X) = (1/(4 pi V)) sum_e c(e) g(X + e*h),
    c(e) = prod_k (2 if e_k = 0 else -1), V = hx hy hz,
and the other components by permuting the arguments (f is symmetric in its
last two arguments, g in its first two).

Periodic dimensions follow the same reading as the rest of the oracle:
lattice images o + m n_k with |o + m n_k| <= (mimg + 1/2) n_k per periodic
dimension, weight 1/2 on the window boundary.
"""
from __future__ import annotations

import mpmath as mp

DPS = 40


def newell_f(x, y, z):
    """Newell's f at (x, y, z) (mpf arguments >= 0 are expected; f is even)."""
    x, y, z = abs(x), abs(y), abs(z)
    x2, y2, z2 = x * x, y * y, z * z
    R = mp.sqrt(x2 + y2 + z2)
    if R == 0:
        return mp.mpf(0)
    r = (2 * x2 - y2 - z2) * R / 6
    if y != 0 and z2 != x2:
        r += y * (z2 - x2) / 2 * mp.asinh(y / mp.sqrt(x2 + z2))
    if z != 0 and y2 != x2:
        r += z * (y2 - x2) / 2 * mp.asinh(z / mp.sqrt(x2 + y2))
    if x != 0 and y != 0 and z != 0:
        r -= x * y * z * mp.atan(y * z / (x * R))
    return r


def newell_g(x, y, z):
    """Newell's g at (x, y, z): odd in x and in y, even in z."""
    sgn = 1
    if x < 0:
        sgn, x = -sgn, -x
    if y < 0:
        sgn, y = -sgn, -y
    z = abs(z)
    x2, y2, z2 = x * x, y * y, z * z
    R = mp.sqrt(x2 + y2 + z2)
    if R == 0:
        return mp.mpf(0)
    r = -x * y * R / 3
    if z != 0 and x2 + y2 != 0:
        r += x * y * z * mp.asinh(z / mp.sqrt(x2 + y2))
    if x != 0 and y2 + z2 != 0:
        r += y * (3 * z2 - y2) / 6 * mp.asinh(x / mp.sqrt(y2 + z2))
    if y != 0 and x2 + z2 != 0:
        r += x * (3 * z2 - x2) / 6 * mp.asinh(y / mp.sqrt(x2 + z2))
    if z != 0:
        r -= z2 * z / 6 * mp.atan(x * y / (z * R))
    if y != 0:
        r -= z * y2 / 2 * mp.atan(x * z / (y * R))
    if x != 0:
        r -= z * x2 / 2 * mp.atan(y * z / (x * R))
    return sgn * r


class Lattice:
    """Newell functions on the lattice of non-negative cell multiples
    (a hx, b hy, c hz), computed once each and reused by every offset's
    27-point combination.  Six functions (component order xx yy zz xy xz yz):
    f(X,Y,Z), f(Y,X,Z), f(Z,Y,X), g(X,Y,Z), g(X,Z,Y), g(Y,Z,X)."""

    def __init__(self, h):
        with mp.workdps(DPS):
            self.h = tuple(mp.mpf(repr(float(v))) for v in h)
        self.cache = {}

    def values(self, a, b, c):
        key = (a, b, c)
        v = self.cache.get(key)
        if v is None:
            with mp.workdps(DPS):
                X, Y, Z = a * self.h[0], b * self.h[1], c * self.h[2]
                v = (newell_f(X, Y, Z), newell_f(Y, X, Z), newell_f(Z, Y, X),
                     newell_g(X, Y, Z), newell_g(X, Z, Y), newell_g(Y, Z, X))
            self.cache[key] = v
        return v

    def tensor(self, o):
        """N(o) for an integer cell offset o = (ox, oy, oz); six mpf values."""
        with mp.workdps(DPS):
            acc = [mp.mpf(0)] * 6
            for ex in (-1, 0, 1):
                px = o[0] + ex
                for ey in (-1, 0, 1):
                    py = o[1] + ey
                    for ez in (-1, 0, 1):
                        pz = o[2] + ez
                        w = (2 if ex == 0 else -1) * (2 if ey == 0 else -1) * (2 if ez == 0 else -1)
                        v = self.values(abs(px), abs(py), abs(pz))
                        sx = (px > 0) - (px < 0)
                        sy = (py > 0) - (py < 0)
                        sz = (pz > 0) - (pz < 0)
                        acc[0] += w * v[0]
                        acc[1] += w * v[1]
                        acc[2] += w * v[2]
                        acc[3] += w * sx * sy * v[3]
                        acc[4] += w * sx * sz * v[4]
                        acc[5] += w * sy * sz * v[5]
            V = self.h[0] * self.h[1] * self.h[2]
            s = 1 / (4 * mp.pi * V)
            return [a * s for a in acc]


def image_offsets(idx, n, periodic, mimg):
    """(offset, weight) pairs of one table index along one dimension: the
    offset itself for an open dimension (index i <-> offset i - (n - 1)),
    the lattice images of the class i mod n in the window |o| <= (mimg+1/2) n
    for a periodic one (weight 1/2 on the boundary)."""
    if not periodic:
        return [(idx - (n - 1), 1)]
    out = []
    lim2 = (2 * mimg + 1) * n           # compare 2|o| with (2 mimg + 1) n exactly
    for m in range(-mimg - 1, mimg + 2):
        o = idx + m * n
        if 2 * abs(o) < lim2:
            out.append((o, 1))
        elif 2 * abs(o) == lim2:
            out.append((o, mp.mpf(1) / 2))
    return out


def offset_table(n, periodic, mimg, h):
    """The interaction tensor for every table index of a grid, as nested
    lists [6][Kz][Ky][Kx] of Python floats (layout of the oracle's offset
    table: K = 2n - 1 for open, n for periodic dimensions), without the
    k_parallel = 0 correction."""
    lat = Lattice(h)
    K = [n[k] if periodic[k] else 2 * n[k] - 1 for k in range(3)]
    out = [[[[0.0] * K[0] for _ in range(K[1])] for _ in range(K[2])] for _ in range(6)]
    imgs = [[image_offsets(i, n[k], periodic[k], mimg) for i in range(K[k])] for k in range(3)]
    with mp.workdps(DPS):
        for iz in range(K[2]):
            for iy in range(K[1]):
                for ix in range(K[0]):
                    acc = [mp.mpf(0)] * 6
                    for ox, wx in imgs[0][ix]:
                        for oy, wy in imgs[1][iy]:
                            for oz, wz in imgs[2][iz]:
                                t = lat.tensor((ox, oy, oz))
                                w = wx * wy * wz
                                for q in range(6):
                                    acc[q] += w * t[q]
                    for q in range(6):
                        out[q][iz][iy][ix] = float(acc[q])
    return out


# --------------------------------------------------------------------------
# Octant storage of a table.  The tensor is even under o -> -o in every
# dimension for xx, yy, zz and odd in the two coordinates it names for
# xy, xz, yz; the image window is symmetric, so a table is fixed by its
# entries at non-negative offsets (open dimension: |o| = 0..n-1; periodic
# dimension: classes 0..n/2).
# --------------------------------------------------------------------------
def octant_table(n, periodic, mimg, h):
    """[6][Az][Ay][Ax] floats at non-negative offsets (A = n for open,
    n//2 + 1 for periodic dimensions), without the k_parallel = 0 correction."""
    lat = Lattice(h)
    A = [n[k] // 2 + 1 if periodic[k] else n[k] for k in range(3)]

    def imgs(a, k):
        # table index of offset +a: open i = a + n - 1, periodic class a
        return image_offsets(a if periodic[k] else a + n[k] - 1, n[k], periodic[k], mimg)

    im = [[imgs(a, k) for a in range(A[k])] for k in range(3)]
    out = [[[[0.0] * A[0] for _ in range(A[1])] for _ in range(A[2])] for _ in range(6)]
    with mp.workdps(DPS):
        for az in range(A[2]):
            for ay in range(A[1]):
                for ax in range(A[0]):
                    acc = [mp.mpf(0)] * 6
                    for ox, wx in im[0][ax]:
                        for oy, wy in im[1][ay]:
                            for oz, wz in im[2][az]:
                                t = lat.tensor((ox, oy, oz))
                                w = wx * wy * wz
                                for q in range(6):
                                    acc[q] += w * t[q]
                    for q in range(6):
                        out[q][az][ay][ax] = float(acc[q])
    return out
