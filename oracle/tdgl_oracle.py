"""TDGL oracle: plain FP64 numpy — TEST INFRASTRUCTURE ONLY.

Every function follows a passage of the paper (sections 2-3) and is written
for checking by eye, not for speed.  Readings where the paper is silent are
marked "reading"; they match the readings the GPU path documents.

Reduced units (Table 2) with a fixed reference stiffness alpha_ref > 0
(reading: one value per run, so reduced time means the same at every T):
    P* = P/P0, tau = alpha_ref L t, r* = r sqrt(alpha_ref/G110),
    alpha1* = alpha1/alpha_ref, alpha11* = alpha11 P0^2/alpha_ref,
    alpha111* = alpha111 P0^4/alpha_ref, G* = G/G110, E* = E/(alpha_ref P0),
    energy density f* = f/(alpha_ref P0^2).
Electrostatic coupling (eq 6 with E* above): kappa = 1/(eps0 epsB alpha_ref).

Array layout: P[c, z, y, x] (component first, x fastest).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import lib as _tensor_lib

EPS0 = 8.8541878128e-12
LANDAU, GRAD, ELEC, EXT = 1, 2, 4, 8


# --------------------------------------------------------------------------
# Table 1: coefficients at temperature T (SI)
# --------------------------------------------------------------------------
def landau_coefficients(mat: dict, T: float) -> dict:
    """alpha coefficients of eq 3 at temperature T, forms of Table 1."""
    if mat["a1_form"] == 0:
        a1 = mat["a1_slope"] * (T - mat["a1_T0"])
    else:  # Barrett form used for SrTiO3
        a1 = mat["a1_A"] * (1.0 / np.tanh(mat["a1_Ts"] / T)
                            - 1.0 / np.tanh(mat["a1_Ts"] / mat["a1_T0"]))
    return dict(
        a1x=a1, a1y=a1, a1z=mat.get("rs", 1.0) * a1,
        a11=mat["a11_slope"] * (T - mat["a11_Tref"]) + mat["a11_offset"],
        a12=mat["a12"],
        a111=mat["a111_slope"] * (T - mat["a111_Tref"]) + mat["a111_offset"],
        a112=mat["a112"], a123=mat["a123"],
    )


def reduce_coefficients(c: dict, P0: float, alpha_ref: float) -> np.ndarray:
    """Table 2 normalisation of the Landau coefficients.
    Returns [a1x, a1y, a1z, a11, a12, a111, a112, a123] (dimensionless)."""
    return np.array([
        c["a1x"] / alpha_ref, c["a1y"] / alpha_ref, c["a1z"] / alpha_ref,
        c["a11"] * P0**2 / alpha_ref, c["a12"] * P0**2 / alpha_ref,
        c["a111"] * P0**4 / alpha_ref, c["a112"] * P0**4 / alpha_ref,
        c["a123"] * P0**4 / alpha_ref,
    ])


# --------------------------------------------------------------------------
# Problem set-up
# --------------------------------------------------------------------------
class Problem:
    """All reduced quantities of one run (grid, materials, scales, terms)."""

    def __init__(self, cfg: dict, tensor: bool = True):
        self.n = tuple(int(v) for v in cfg["n"])
        nx, ny, nz = self.n
        s = cfg["scales"]
        self.P0, self.alpha_ref, self.G110, self.eps_b = (
            s["P0"], s["alpha_ref"], s["G110"], s["eps_b"])
        self.l0 = np.sqrt(self.G110 / self.alpha_ref)          # length unit (m)
        self.h = np.array(cfg["d"], dtype=float) / self.l0      # reduced cell sizes
        self.dV = float(np.prod(self.h))
        self.periodic = tuple(bool(p) for p in cfg["periodic"])
        self.mimg = int(cfg.get("mimg", 16))
        self.kappa = 1.0 / (EPS0 * self.eps_b * self.alpha_ref)
        self.terms = int(cfg.get("terms", 15))
        self.energy_scale = self.alpha_ref * self.P0**2 * self.l0**3   # J per reduced unit
        self.field_scale = self.alpha_ref * self.P0                    # V/m per reduced unit
        self.eext = np.asarray(cfg.get("eext", (0.0, 0.0, 0.0)), float) / self.field_scale
        self.layers = np.asarray(cfg["layers"], dtype=int)
        assert self.layers.shape == (nz,)
        self.materials = cfg["materials"]
        self.set_temperature(cfg["T"])
        # gradient (eq 4): g[i, d] multiplies the squared derivative of P_i
        # along d (G11 along the component, G44 + G44' across); g12 and gm
        # (= G44 - G44') multiply the cross products P_i,i P_j,j and P_i,j P_j,i
        G = cfg["gradient"]
        self.g = np.empty((3, 3))
        for i in range(3):
            for d in range(3):
                self.g[i, d] = (G["G11"] if i == d else G["G44"] + G["G44p"]) / self.G110
        self.g12 = G["G12"] / self.G110
        self.gm = (G["G44"] - G["G44p"]) / self.G110
        self.tab = None
        self.tensor_source = None
        if tensor and (self.terms & ELEC):
            self.tab, self.tensor_source = tensor_table(self.n, self.periodic, self.mimg, self.h,
                                                        cfg.get("tensor_source", "auto"))

    def set_temperature(self, T: float):
        self._nb_cache = {}
        self.T = T
        nz = self.n[2]
        self.coef = np.zeros((nz, 8))
        self.material = self.layers >= 0
        for z in range(nz):
            m = self.layers[z]
            if m >= 0:
                self.coef[z] = reduce_coefficients(
                    landau_coefficients(self.materials[m], T), self.P0, self.alpha_ref)

    def to_reduced_P(self, P_si):
        return np.asarray(P_si, dtype=np.float64) / self.P0

    def mask(self, P):
        """Vacuum layers carry P = 0 (section 2: P = 0 outside the sample)."""
        P = P.copy()
        P[:, ~self.material] = 0.0
        return P


# --------------------------------------------------------------------------
# Landau field: minus the derivative of eq 3 (per layer coefficients)
# --------------------------------------------------------------------------
def landau_energy_density(P, coef):
    """f_L* of eq 3 at every cell.  coef: [nz, 8] broadcast along z."""
    a1x, a1y, a1z, a11, a12, a111, a112, a123 = [coef[:, k][:, None, None] for k in range(8)]
    # powers of the squares, written as products (numpy's general power
    # routine is many times slower than a multiplication)
    x, y, z = P[0] * P[0], P[1] * P[1], P[2] * P[2]          # Px^2, Py^2, Pz^2
    return (a1x * x + a1y * y + a1z * z
            + a11 * (x * x + y * y + z * z)
            + a12 * (x * y + y * z + z * x)
            + a111 * (x * x * x + y * y * y + z * z * z)
            + a112 * (x * x * (y + z) + y * y * (x + z) + z * z * (x + y))
            + a123 * x * y * z)


def landau_field(P, coef):
    """H_L = -d f_L / dP, term by term from eq 3."""
    a1 = [coef[:, k][:, None, None] for k in range(3)]
    a11, a12, a111, a112, a123 = [coef[:, k][:, None, None] for k in range(3, 8)]
    H = np.empty_like(P)
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        Pi = P[i]
        si, sj, sk = P[i] * P[i], P[j] * P[j], P[k] * P[k]   # squares, as products
        dfdPi = Pi * (2 * a1[i]
                      + 4 * a11 * si
                      + 2 * a12 * (sj + sk)
                      + 6 * a111 * si * si
                      + a112 * (4 * si * (sj + sk) + 2 * (sj * sj + sk * sk))
                      + 2 * a123 * sj * sk)
        H[i] = -dfdPi
    return H


# --------------------------------------------------------------------------
# Gradient field: eq 4 (diagonal part), 7-point finite differences.
# Reading: neighbours outside an open surface or in vacuum are dropped
# (natural/Neumann boundary), periodic dimensions wrap.
# --------------------------------------------------------------------------
def _neighbour_valid(prob: Problem, axis_arr: int, shift: int):
    """Boolean array [nz, ny, nx]: the neighbour at +shift along the array
    axis (0=z, 1=y, 2=x) exists and is material."""
    cache = prob.__dict__.setdefault("_nb_cache", {})
    if (axis_arr, shift) not in cache:
        cache[(axis_arr, shift)] = _neighbour_valid_uncached(prob, axis_arr, shift)
    return cache[(axis_arr, shift)]


def _neighbour_valid_uncached(prob: Problem, axis_arr: int, shift: int):
    nx, ny, nz = prob.n
    shape = (nz, ny, nx)
    dim = 2 - axis_arr                      # physical dimension index (x=0)
    size = shape[axis_arr]
    idx = np.arange(size)
    nb = idx + shift
    if prob.periodic[dim]:
        ok1 = np.ones(size, bool)
    else:
        ok1 = (nb >= 0) & (nb < size)
    sh = [1, 1, 1]
    sh[axis_arr] = size
    valid = np.broadcast_to(ok1.reshape(sh), shape).copy()
    mat = np.broadcast_to(prob.material[:, None, None], shape)
    nb_mat = np.roll(mat, -shift, axis=axis_arr)
    return valid & mat & nb_mat


def _cdiff(Q, prob: Problem, dim: int):
    """Central difference of the cell field Q ([nz][ny][nx]) along physical
    dimension dim, (Q(c+d) - Q(c-d)) / (2 h_d), where a missing neighbour
    (open surface, vacuum) is replaced by Q(c)."""
    axis_arr = 2 - dim
    up = np.where(_neighbour_valid(prob, axis_arr, +1), np.roll(Q, -1, axis=axis_arr), Q)
    dn = np.where(_neighbour_valid(prob, axis_arr, -1), np.roll(Q, 1, axis=axis_arr), Q)
    return (up - dn) / (2.0 * prob.h[dim])


def _cdiff_adj(F, prob: Problem, dim: int):
    """Adjoint of _cdiff: (A^T F)(c) = sum_c' F(c') d(_cdiff Q)(c')/dQ(c)."""
    axis_arr = 2 - dim
    vup = _neighbour_valid(prob, axis_arr, +1)
    vdn = _neighbour_valid(prob, axis_arr, -1)
    out = np.where(vdn, np.roll(F, 1, axis=axis_arr), 0.0)      # c' = c - d sees c as its +d
    out -= np.where(vup, np.roll(F, -1, axis=axis_arr), 0.0)    # c' = c + d sees c as its -d
    out += F * ((~vup).astype(float) - (~vdn).astype(float))    # c' = c where c replaced a neighbour
    return out / (2.0 * prob.h[dim])


# the cross terms of eq 4, one per unordered component pair (i, j):
#   G12: P_i,i P_j,j  and  G44 - G44': P_i,j P_j,i
_CROSS_PAIRS = ((0, 1), (1, 2), (2, 0))


def gradient_field(P, prob: Problem):
    """H_G = -(1/dV) dF_G/dP for the discrete eq 4: the diagonal part
    sum_d g[i,d] sum_{existing nb along d} (P_nb - P_c)/h_d^2 plus, when
    G12 or G44 - G44' is non-zero, the derivative of the cross terms
    (central differences with missing neighbours replaced by the cell)."""
    H = np.zeros_like(P)
    for axis_arr in range(3):
        dim = 2 - axis_arr
        for shift in (-1, 1):
            valid = _neighbour_valid(prob, axis_arr, shift)
            Pnb = np.roll(P, -shift, axis=axis_arr + 1)
            for i in range(3):
                H[i] += np.where(valid, prob.g[i, dim] * (Pnb[i] - P[i]) / prob.h[dim]**2, 0.0)
    if prob.g12 != 0.0 or prob.gm != 0.0:
        D = {(i, d): _cdiff(P[i], prob, d) for i in range(3) for d in range(3)}
        for i, j in _CROSS_PAIRS:
            # G12 P_i,i P_j,j
            H[i] -= prob.g12 * _cdiff_adj(D[(j, j)], prob, i)
            H[j] -= prob.g12 * _cdiff_adj(D[(i, i)], prob, j)
            # (G44 - G44') P_i,j P_j,i
            H[i] -= prob.gm * _cdiff_adj(D[(j, i)], prob, j)
            H[j] -= prob.gm * _cdiff_adj(D[(i, j)], prob, i)
        H[:, ~prob.material] = 0.0
    return H


def gradient_energy(P, prob: Problem):
    """F_G* = dV* [sum over edges (a,b) along d of (g[i,d]/2)|P_a,i - P_b,i|^2/h_d^2
    + sum over material cells of the cross terms of eq 4]."""
    F = 0.0
    for axis_arr in range(3):
        dim = 2 - axis_arr
        valid = _neighbour_valid(prob, axis_arr, +1)     # each edge once
        Pnb = np.roll(P, -1, axis=axis_arr + 1)
        for i in range(3):
            e = np.where(valid, 0.5 * prob.g[i, dim] * (Pnb[i] - P[i])**2 / prob.h[dim]**2, 0.0)
            F += e.sum()
    if prob.g12 != 0.0 or prob.gm != 0.0:
        D = {(i, d): _cdiff(P[i], prob, d) for i in range(3) for d in range(3)}
        mat = np.broadcast_to(prob.material[:, None, None], P.shape[1:])
        for i, j in _CROSS_PAIRS:
            cross = prob.g12 * D[(i, i)] * D[(j, j)] + prob.gm * D[(i, j)] * D[(j, i)]
            F += np.where(mat, cross, 0.0).sum()
    return prob.dV * F


# --------------------------------------------------------------------------
# Electrostatic field (eqs 5-6): H_E = -kappa * sum_c' N(r_c - r_c') P_c'
# --------------------------------------------------------------------------
_GL = None


def gauss_legendre_tables():
    """Gauss-Legendre nodes/weights on [0,1] for n = 0..23 nodes, as the C
    code's [24][24] tables (row n holds n nodes)."""
    global _GL
    if _GL is None:
        t = np.zeros((24, 24))
        w = np.zeros((24, 24))
        for n in range(1, 24):
            x, wt = np.polynomial.legendre.leggauss(n)
            t[n, :n] = 0.5 * (x + 1.0)
            w[n, :n] = 0.5 * wt
        _GL = (np.ascontiguousarray(t), np.ascontiguousarray(w))
    return _GL


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def cell_tensor(o, h):
    """N(o) for an integer cell offset o (6 comps xx,yy,zz,xy,xz,yz), no images."""
    t, w = gauss_legendre_tables()
    out = np.zeros(6)
    oo = np.asarray(o, float)
    hh = np.asarray(h, float)
    _tensor_lib().orc_cell_tensor(_dp(oo), _dp(hh), _dp(t), _dp(w), _dp(out))
    return out


def newell_tensor(R, h):
    """Closed-form N at physical offset R (long double Newell formulas)."""
    out = np.zeros(6)
    RR = np.asarray(R, float)
    hh = np.asarray(h, float)
    _tensor_lib().orc_newell(_dp(RR), _dp(hh), _dp(out))
    return out


def quad_tensor(R, h, n):
    """Tent-weighted Gauss-Legendre N at physical offset R with n nodes per half."""
    t, w = gauss_legendre_tables()
    out = np.zeros(6)
    RR = np.asarray(R, float)
    hh = np.asarray(h, float)
    _tensor_lib().orc_quad(_dp(RR), _dp(hh), int(n), _dp(t[n]), _dp(w[n]), _dp(out))
    return out


def offset_table(n, periodic, mimg, h, k0_correction=True):
    """N for every cell offset of the grid by the C quadrature (see
    tensor_oracle.c for indexing), then the k_parallel = 0 correction."""
    pm = sum((1 << k) for k in range(3) if periodic[k])
    if pm not in (0, 3, 7):
        raise NotImplementedError("periodic mask %d" % pm)
    if mimg > 64:
        raise ValueError("mimg <= 64")
    t, w = gauss_legendre_tables()
    N = (ctypes.c_int * 3)(*[int(v) for v in n])
    K = [n[k] if periodic[k] else 2 * n[k] - 1 for k in range(3)]
    out = np.zeros((6, K[2], K[1], K[0]))
    hh = np.asarray(h, float)
    _tensor_lib().orc_offset_table(N, pm, int(mimg), _dp(hh), _dp(t), _dp(w), _dp(out))
    return k0_correct(out, n, periodic) if k0_correction else out


def k0_correct(tab, n, periodic):
    """Reading for periodic dimensions (the paper treats open samples only):
    lattice images in a symmetric window; afterwards, per z-offset and
    component, a constant is added so the in-plane sum takes its exact
    infinite-lattice value: zz -> 1 at dz = 0 (an infinite uniformly polarised
    sheet has E = -P_z/(eps0 epsB) inside and 0 outside), all others -> 0.
    Fully periodic grids use the short-circuit value 0 for every sum."""
    pm = sum((1 << k) for k in range(3) if periodic[k])
    out = np.array(tab, dtype=np.float64)
    K = out.shape[1:][::-1]
    if pm == 3:
        nz = n[2]
        for q in range(6):
            for iz in range(K[2]):
                dz = iz - (nz - 1)
                target = 1.0 if (q == 2 and dz == 0) else 0.0
                S = out[q, iz].sum()
                out[q, iz] += (target - S) / (n[0] * n[1])
    elif pm == 7:
        for q in range(6):
            out[q] -= out[q].sum() / (n[0] * n[1] * n[2])
    return out


def tensor_table(n, periodic, mimg, h, source="auto"):
    """The oracle's interaction-tensor table with the k_parallel = 0
    correction, and where it came from.

    "newell_mp": the Newell closed form in 40-digit arithmetic
    (oracle/tensor_mp.py), stored for the parity-test grids under
    tests/golden/tensor_mp/ by a script that calls only the oracle;
    "quadrature": the C evaluation (tensor_oracle.c), pinned against the
    40-digit tables.  "auto" takes the stored table when one matches the
    geometry exactly and the quadrature otherwise (large image windows)."""
    from . import tensor_tables
    if source in ("auto", "newell_mp"):
        tab = tensor_tables.lookup(n, periodic, mimg, h)
        if tab is not None:
            return k0_correct(tab, n, periodic), "newell_mp"
        if source == "newell_mp":
            raise KeyError("no stored 40-digit table for n=%s periodic=%s mimg=%d"
                           % (tuple(n), tuple(periodic), mimg))
    return offset_table(n, periodic, mimg, h), "quadrature"


_PAIRS = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 0): 3,
          (0, 2): 4, (2, 0): 4, (1, 2): 5, (2, 1): 5}


def elec_field_direct(P, prob: Problem):
    """Plain definition: double loop over target and source cells."""
    nx, ny, nz = prob.n
    tab = prob.tab
    H = np.zeros_like(P)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")

    def index(delta, dim, size):
        return delta % size if prob.periodic[dim] else delta + (size - 1)

    for sz in range(nz):
        for sy in range(ny):
            for sx in range(nx):
                p = P[:, sz, sy, sx]
                if not np.any(p):
                    continue
                iz = index(z - sz, 2, nz)
                iy = index(y - sy, 1, ny)
                ix = index(x - sx, 0, nx)
                for i in range(3):
                    for j in range(3):
                        H[i] += -prob.kappa * tab[_PAIRS[(i, j)], iz, iy, ix] * p[j]
    return H


def padded_sizes(prob: Problem):
    """Reading: open dimensions zero-padded to 2N, periodic ones not padded."""
    return tuple(prob.n[k] if prob.periodic[k] else 2 * prob.n[k] for k in range(3))


def kernel_spectrum(prob: Problem):
    """Spectrum of the interaction table placed on the padded grid in
    wrap-around order (offset -o at index M - o; the entry at index N of an
    open dimension stays 0)."""
    nx, ny, nz = prob.n
    Mx, My, Mz = padded_sizes(prob)
    kern = np.zeros((6, Mz, My, Mx))
    # wrap-around placement of offsets
    def positions(dim, size, M):
        if prob.periodic[dim]:
            return np.arange(size), np.arange(size)
        idx = np.arange(2 * size - 1)
        return idx, (idx - (size - 1)) % M
    iz, pz = positions(2, nz, Mz)
    iy, py = positions(1, ny, My)
    ix, px = positions(0, nx, Mx)
    kern[:, pz[:, None, None], py[None, :, None], px[None, None, :]] = \
        prob.tab[:, iz[:, None, None], iy[None, :, None], ix[None, None, :]]
    Nk = np.fft.rfftn(kern, axes=(1, 2, 3))
    prob._nk_cache = (prob.tab, Nk)
    return Nk


def elec_field_fft(P, prob: Problem):
    """Same sum as elec_field_direct, as a circular convolution on the padded
    grid (section 3: FFT evaluation of the electrostatic field)."""
    nx, ny, nz = prob.n
    Mx, My, Mz = padded_sizes(prob)
    cached = prob.__dict__.get("_nk_cache")
    # the kernel spectrum depends on the table only: transformed once per table
    Nk = cached[1] if cached is not None and cached[0] is prob.tab else kernel_spectrum(prob)
    Pp = np.zeros((3, Mz, My, Mx))
    Pp[:, :nz, :ny, :nx] = P
    Pk = np.fft.rfftn(Pp, axes=(1, 2, 3))
    Hk = np.zeros_like(Pk)
    for i in range(3):
        for j in range(3):
            Hk[i] += Nk[_PAIRS[(i, j)]] * Pk[j]
    H = np.fft.irfftn(Hk, s=(Mz, My, Mx), axes=(1, 2, 3))[:, :nz, :ny, :nx]
    return -prob.kappa * H


# --------------------------------------------------------------------------
# Effective field (eq 1 with eq 2) and integrators
# --------------------------------------------------------------------------
def effective_field(P, prob: Problem, terms=None, elec_mode="fft", parts=False):
    """E_eff* = H_L + H_G + H_E + E_ext*, terms switched by the mask (section 3)."""
    terms = prob.terms if terms is None else terms
    out = {}
    H = np.zeros_like(P)
    if terms & LANDAU:
        out["landau"] = landau_field(P, prob.coef)
        H += out["landau"]
    if terms & GRAD:
        out["grad"] = gradient_field(P, prob)
        H += out["grad"]
    if terms & ELEC:
        out["elec"] = (elec_field_direct if elec_mode == "direct" else elec_field_fft)(P, prob)
        H += out["elec"]
    if terms & EXT:
        out["ext"] = np.broadcast_to(prob.eext[:, None, None, None], P.shape).copy()
        H += out["ext"]
    H[:, ~prob.material] = 0.0
    return (H, out) if parts else H


def step_euler(P, prob: Problem, dtau):
    """Explicit Euler for eq 1 (L = 1 in reduced time)."""
    return prob.mask(P + dtau * effective_field(P, prob))


def step_heun(P, prob: Problem, dtau):
    """Heun's predictor-corrector (section 3): predictor with the field at P,
    corrector averaging the old state and predictor plus half a step of the
    field at the predictor."""
    Pt = prob.mask(P + dtau * effective_field(P, prob))
    return prob.mask(0.5 * (P + Pt) + 0.5 * dtau * effective_field(Pt, prob))


def step_ab3m2(P, prob: Problem, dtau, hist):
    """One step of the multistep scheme section 3 names AB3M2, read as a
    predictor-corrector pair: the three-step Adams-Bashforth predictor
    P* = P_n + dtau (23 E_n - 16 E_{n-1} + 5 E_{n-2}) / 12 and the two-step
    Adams-Moulton corrector P_{n+1} = P_n + dtau (5 E(P*) + 8 E_n - E_{n-1}) / 12,
    both third order.  hist holds the fields of earlier steps at their
    corrected states, newest last; while it holds fewer than two, the step
    is a Heun step.  E_n is appended; returns the new state."""
    En = effective_field(P, prob)
    if len(hist) < 2:
        Pt = prob.mask(P + dtau * En)
        Pn = prob.mask(0.5 * (P + Pt) + 0.5 * dtau * effective_field(Pt, prob))
    else:
        E1, E2 = hist[-1], hist[-2]
        Ps = prob.mask(P + dtau * (23.0 * En - 16.0 * E1 + 5.0 * E2) / 12.0)
        Pn = prob.mask(P + dtau * (5.0 * effective_field(Ps, prob) + 8.0 * En - E1) / 12.0)
    hist.append(En)
    del hist[:-2]
    return Pn


# Dormand-Prince 5(4) tableau (Dormand & Prince 1980), the RK45 of
# section 3: nodes C, stage weights A (row i for stage i + 1), the fifth-order
# weights B (used to advance) and the fourth-order weights BS.
DP_C = [0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0, 1.0]
DP_A = [[],
        [1 / 5],
        [3 / 40, 9 / 40],
        [44 / 45, -56 / 15, 32 / 9],
        [19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729],
        [9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656],
        [35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84]]
DP_B = [35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84, 0.0]
DP_BS = [5179 / 57600, 0.0, 7571 / 16695, 393 / 640, -92097 / 339200, 187 / 2100, 1 / 40]


def step_rk45(P, prob: Problem, h, atol, rtol):
    """One attempt of the adaptive RK45 step (section 3): the seven stages
    of the tableau, the fifth-order solution P5 and the error estimate
    err = max over cells and components of |h sum_j (B_j - BS_j) k_j| /
    (atol + rtol max(|P|, |P5|)).  Accepted if err <= 1.  The next step
    size is h min(5, max(0.2, 0.9 err^(-1/5))) when accepted and
    h max(0.2, 0.9 err^(-1/5)) when rejected.  Returns (P5 or P, accepted,
    h_next, err)."""
    k = []
    X = P
    for i in range(7):
        if i > 0:
            X = prob.mask(P + h * sum(a * kj for a, kj in zip(DP_A[i], k)))
        k.append(effective_field(X, prob))
    P5 = X                                   # stage 7 is evaluated at the new state
    e = h * sum((b - bs) * kj for b, bs, kj in zip(DP_B, DP_BS, k))
    sc = atol + rtol * np.maximum(np.abs(P), np.abs(P5))
    err = float(np.max(np.abs(e) / sc)) if e.size else 0.0
    fac = 0.9 * err ** -0.2 if err > 0 else 5.0
    if err <= 1.0:
        return P5, True, h * min(5.0, max(0.2, fac)), err
    return P, False, h * max(0.2, fac), err


def run_rk45(P, prob: Problem, h, nsteps: int, atol, rtol):
    """nsteps accepted RK45 steps from step size h; returns (P, tau, h,
    rejected attempts)."""
    tau, rejected, done = 0.0, 0, 0
    while done < nsteps:
        Pn, ok, hn, _ = step_rk45(P, prob, h, atol, rtol)
        if ok:
            tau += h
            done += 1
            P = Pn
        else:
            rejected += 1
        h = hn
    return P, tau, h, rejected


def run(P, prob: Problem, scheme: str, dtau: float, nsteps: int, hist=None):
    """nsteps steps of "euler", "heun" or "ab3m2" (hist: the multistep
    history to continue from; a fresh run starts with an empty one)."""
    if scheme == "ab3m2":
        hist = [] if hist is None else hist
        for _ in range(nsteps):
            P = step_ab3m2(P, prob, dtau, hist)
        return P
    step = step_euler if scheme == "euler" else step_heun
    for _ in range(nsteps):
        P = step(P, prob, dtau)
    return P


# --------------------------------------------------------------------------
# Energies (eqs 2, 3, 4, 5, 7) in reduced units; multiply by
# prob.energy_scale for joules.
# --------------------------------------------------------------------------
def energies(P, prob: Problem, terms=None):
    """Returns dict F_land, F_grad, F_elec, F_ext, F_total, meanP (reduced)."""
    terms = prob.terms if terms is None else terms
    F = dict(F_land=0.0, F_grad=0.0, F_elec=0.0, F_ext=0.0)
    mat = prob.material
    if terms & LANDAU:
        F["F_land"] = prob.dV * landau_energy_density(P, prob.coef)[mat].sum()
    if terms & GRAD:
        F["F_grad"] = gradient_energy(P, prob)
    if terms & ELEC:
        HE = elec_field_fft(P, prob)
        F["F_elec"] = -0.5 * prob.dV * (P * HE).sum(axis=0)[mat].sum()
    if terms & EXT:
        F["F_ext"] = -prob.dV * np.einsum("c,c...->...", prob.eext, P)[mat].sum()
    F["F_total"] = F["F_land"] + F["F_grad"] + F["F_elec"] + F["F_ext"]
    ncell = mat.sum() * prob.n[0] * prob.n[1]
    F["meanP"] = P[:, mat].reshape(3, -1).sum(axis=1) / max(ncell, 1)
    return F


# --------------------------------------------------------------------------
# SI entry points (Table 2 in reverse): P in C/m^2, fields in V/m, energies
# in J.  The reduced functions above work in units of P0, alpha_ref and l0.
# --------------------------------------------------------------------------
def run_si(P_si, prob: Problem, scheme: str, dtau: float, nsteps: int):
    """run() on an SI state; returns the SI state."""
    return prob.P0 * run(prob.to_reduced_P(P_si), prob, scheme, dtau, nsteps)


def field_si(P_si, prob: Problem, terms=None):
    """E_eff of an SI state in V/m."""
    return effective_field(prob.to_reduced_P(P_si), prob, terms) * prob.field_scale


def energies_si(P_si, prob: Problem, terms=None):
    """energies() of an SI state: F terms in J, meanP in C/m^2."""
    F = energies(prob.to_reduced_P(P_si), prob, terms)
    out = {k: v * prob.energy_scale for k, v in F.items() if k != "meanP"}
    out["meanP"] = F["meanP"] * prob.P0
    return out
