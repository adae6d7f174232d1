"""MI355X TDGL time step: Python binding of libtdgl (include/tdgl.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of libtdgl.so.  PyTorch is used for device memory (the context workspace and
device-side P / field buffers) and for the HIP stream the work is enqueued
on.  Importing this package fails loudly if the library has not been built
(``python -m paper_2605_28800_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdgl.so")

TDGL_OK, TDGL_E_ARG, TDGL_E_NOMEM, TDGL_E_HIP = 0, -1, -2, -3
TDGL_E_NONFINITE, TDGL_E_STATE, TDGL_E_UNSUPPORTED = -4, -5, -6
TDGL_FP32, TDGL_FP64 = 0, 1
TDGL_EULER, TDGL_HEUN, TDGL_AB3M2, TDGL_RK45 = 0, 1, 2, 3
TDGL_LANDAU, TDGL_GRAD, TDGL_ELEC, TDGL_EXT, TDGL_ALL = 1, 2, 4, 8, 15
TDGL_MAX_MATERIALS = 16

_STATUS = {0: "TDGL_OK", -1: "TDGL_E_ARG", -2: "TDGL_E_NOMEM", -3: "TDGL_E_HIP",
           -4: "TDGL_E_NONFINITE", -5: "TDGL_E_STATE", -6: "TDGL_E_UNSUPPORTED"}

c_int, c_uint, c_double, c_void_p, c_size_t = (ctypes.c_int, ctypes.c_uint, ctypes.c_double,
                                                ctypes.c_void_p, ctypes.c_size_t)
c_longlong = ctypes.c_longlong


class tdgl_grid(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("nz", c_int),
                ("dx", c_double), ("dy", c_double), ("dz", c_double),
                ("periodic_mask", c_uint)]


class tdgl_material(ctypes.Structure):
    _fields_ = [("a1_form", c_int), ("a1_slope", c_double), ("a1_T0", c_double),
                ("a1_A", c_double), ("a1_Ts", c_double),
                ("a11_slope", c_double), ("a11_Tref", c_double), ("a11_offset", c_double),
                ("a12", c_double),
                ("a111_slope", c_double), ("a111_Tref", c_double), ("a111_offset", c_double),
                ("a112", c_double), ("a123", c_double), ("rs", c_double)]


class TdglError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


_ctx_p = c_void_p
_SIGS = {
    "tdgl_abi_version": ([], c_int),
    "tdgl_create": ([ctypes.POINTER(tdgl_grid), c_int, c_void_p, ctypes.POINTER(_ctx_p)], c_int),
    "tdgl_create_batch": ([ctypes.POINTER(tdgl_grid), c_int, c_int, c_void_p,
                           ctypes.POINTER(_ctx_p)], c_int),
    "tdgl_get_batch": ([_ctx_p, ctypes.POINTER(c_int)], c_int),
    "tdgl_destroy": ([_ctx_p], None),
    "tdgl_last_error": ([_ctx_p], ctypes.c_char_p),
    "tdgl_get_dims": ([_ctx_p, ctypes.POINTER(c_int)], c_int),
    "tdgl_workspace_size": ([_ctx_p, ctypes.POINTER(c_size_t)], c_int),
    "tdgl_bind_workspace": ([_ctx_p, c_void_p, c_size_t], c_int),
    "tdgl_relax": ([_ctx_p, c_longlong, c_longlong, c_double, c_double, c_int,
                    ctypes.POINTER(c_longlong), ctypes.POINTER(c_longlong)], c_int),
    "tdgl_relax_group": ([ctypes.POINTER(_ctx_p), c_int, c_longlong, c_longlong, c_double,
                          c_double, c_int, ctypes.POINTER(c_longlong),
                          ctypes.POINTER(c_longlong)], c_int),
    "tdgl_energies_noalloc": ([_ctx_p, c_void_p], c_int),
    "tdgl_set_scales": ([_ctx_p, c_double, c_double, c_double, c_double], c_int),
    "tdgl_set_material": ([_ctx_p, c_int, ctypes.POINTER(tdgl_material)], c_int),
    "tdgl_set_layer_materials": ([_ctx_p, ctypes.POINTER(ctypes.c_byte)], c_int),
    "tdgl_set_gradient": ([_ctx_p, c_double, c_double, c_double, c_double], c_int),
    "tdgl_build_tensor": ([_ctx_p, c_int], c_int),
    "tdgl_get_tensor_spectrum": ([_ctx_p, ctypes.POINTER(c_double), c_size_t], c_int),
    "tdgl_set_temperature": ([_ctx_p, c_double], c_int),
    "tdgl_set_temperatures": ([_ctx_p, ctypes.POINTER(c_double)], c_int),
    "tdgl_set_eext": ([_ctx_p, c_double, c_double, c_double], c_int),
    "tdgl_set_terms": ([_ctx_p, c_uint], c_int),
    "tdgl_set_integrator": ([_ctx_p, c_int, c_double], c_int),
    "tdgl_set_graph_chunk": ([_ctx_p, c_int], c_int),
    "tdgl_set_rk_tolerances": ([_ctx_p, c_double, c_double], c_int),
    "tdgl_get_rk_state": ([_ctx_p, ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                           ctypes.POINTER(ctypes.c_longlong)], c_int),
    "tdgl_set_P": ([_ctx_p, c_void_p, c_int, c_int], c_int),
    "tdgl_get_P": ([_ctx_p, c_void_p, c_int, c_int], c_int),
    "tdgl_step": ([_ctx_p, ctypes.c_longlong], c_int),
    "tdgl_eval_field": ([_ctx_p, c_uint, c_void_p], c_int),
    "tdgl_energies": ([_ctx_p, ctypes.POINTER(c_double), ctypes.POINTER(c_double)], c_int),
    "tdgl_energies_batch": ([_ctx_p, ctypes.POINTER(c_double), ctypes.POINTER(c_double)], c_int),
    "tdgl_get_reduced": ([_ctx_p, ctypes.POINTER(c_double), ctypes.POINTER(c_double)], c_int),
    "tdgl_profile_step": ([_ctx_p, c_int, ctypes.POINTER(c_double)], c_int),
    "tdgl_profile_kernels": ([_ctx_p, c_int, ctypes.POINTER(c_double)], c_int),
    "tdgl_autotune": ([_ctx_p, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_double)], c_int),
    "tdgl_set_z_tile": ([_ctx_p, c_int], c_int),
    "tdgl_set_store_mode": ([_ctx_p, c_int], c_int),
    "tdgl_get_store_mode": ([_ctx_p, ctypes.POINTER(c_int)], c_int),
    "tdgl_get_z_tile": ([_ctx_p, ctypes.POINTER(c_int)], c_int),
    "tdgl_sweep_eext": ([_ctx_p, ctypes.POINTER(c_double), c_int, ctypes.c_longlong,
                         ctypes.POINTER(c_double), ctypes.POINTER(c_double)], c_int),
    "tdgl_set_fft_path": ([_ctx_p, c_int], c_int),
    "tdgl_get_fft_path": ([_ctx_p, ctypes.POINTER(c_int)], c_int),
    "tdgl_set_update_rows": ([_ctx_p, c_int], c_int),
    "tdgl_sync": ([_ctx_p], c_int),
    # initial-state proposal network (include/tdgl_net.h)
    "tdgl_net_create": ([ctypes.c_void_p, c_void_p, ctypes.POINTER(c_void_p)], c_int),
    "tdgl_net_destroy": ([c_void_p], None),
    "tdgl_net_last_error": ([c_void_p], ctypes.c_char_p),
    "tdgl_net_num_params": ([c_void_p, ctypes.POINTER(ctypes.c_longlong)], c_int),
    "tdgl_net_set_params": ([c_void_p, c_void_p, ctypes.c_longlong], c_int),
    "tdgl_net_get_params": ([c_void_p, c_void_p, ctypes.c_longlong], c_int),
    "tdgl_net_forward": ([c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
                         c_int),
    "tdgl_net_loss_grad": ([c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                            c_void_p, ctypes.POINTER(c_double), c_void_p], c_int),
    "tdgl_net_adam": ([c_void_p, c_double, c_double, c_double, c_double], c_int),
    "tdgl_net_train": ([c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                        c_void_p, c_double, c_double, c_double, c_double, c_void_p], c_int),
    "tdgl_net_profile": ([c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                          ctypes.POINTER(c_double)], c_int),
    "tdgl_nn_conv3": ([c_int, c_void_p, c_int, c_void_p, c_void_p, c_int, c_int, c_int, c_int,
                       c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
                      c_int),
    "tdgl_nn_wgrad_workspace": ([c_int, c_int, c_int, c_int, c_int, c_int,
                                 ctypes.POINTER(c_size_t)], c_int),
    "tdgl_nn_conv3_wgrad": ([c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_int, c_int, c_int,
                             c_void_p, c_size_t, c_void_p, c_void_p], c_int),
}
EXPORTED = tuple(_SIGS)

_lib = None


def lib():
    """The loaded libtdgl.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError("libtdgl.so not built: run python -m paper_2605_28800_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(ctx, st):
    if st != TDGL_OK:
        msg = lib().tdgl_last_error(ctx) if ctx else b""
        raise TdglError(st, (msg or b"").decode())


# ---------------------------------------------------------------- thin layer
def tdgl_abi_version():
    return lib().tdgl_abi_version()


def tdgl_create(grid: tdgl_grid, precision: int, hip_stream=None):
    ctx = _ctx_p()
    st = lib().tdgl_create(ctypes.byref(grid), precision, hip_stream, ctypes.byref(ctx))
    if st != TDGL_OK:
        raise TdglError(st, "tdgl_create")
    return ctx


def tdgl_create_batch(grid: tdgl_grid, nbatch: int, precision: int, hip_stream=None):
    ctx = _ctx_p()
    st = lib().tdgl_create_batch(ctypes.byref(grid), nbatch, precision, hip_stream,
                                 ctypes.byref(ctx))
    if st != TDGL_OK:
        raise TdglError(st, "tdgl_create_batch")
    return ctx


def tdgl_get_batch(ctx):
    n = c_int()
    _check(ctx, lib().tdgl_get_batch(ctx, ctypes.byref(n)))
    return n.value


def tdgl_destroy(ctx):
    lib().tdgl_destroy(ctx)


def tdgl_get_dims(ctx):
    out = (c_int * 7)()
    _check(ctx, lib().tdgl_get_dims(ctx, out))
    return tuple(out)


def tdgl_workspace_size(ctx):
    b = c_size_t()
    _check(ctx, lib().tdgl_workspace_size(ctx, ctypes.byref(b)))
    return b.value


def tdgl_bind_workspace(ctx, dev_ptr: int, nbytes: int):
    _check(ctx, lib().tdgl_bind_workspace(ctx, dev_ptr, nbytes))


def tdgl_set_scales(ctx, P0, alpha_ref, G110, eps_b):
    _check(ctx, lib().tdgl_set_scales(ctx, P0, alpha_ref, G110, eps_b))


def make_material(d: dict) -> tdgl_material:
    return tdgl_material(**{k: d[k] for k, _ in tdgl_material._fields_})


def tdgl_set_material(ctx, mid: int, mat: dict):
    m = make_material(mat)
    _check(ctx, lib().tdgl_set_material(ctx, mid, ctypes.byref(m)))


def tdgl_set_layer_materials(ctx, ids):
    arr = (ctypes.c_byte * len(ids))(*[int(v) for v in ids])
    _check(ctx, lib().tdgl_set_layer_materials(ctx, arr))


def tdgl_set_gradient(ctx, G11, G12, G44, G44p):
    _check(ctx, lib().tdgl_set_gradient(ctx, G11, G12, G44, G44p))


def tdgl_build_tensor(ctx, mimg: int):
    _check(ctx, lib().tdgl_build_tensor(ctx, mimg))


def tdgl_get_tensor_spectrum(ctx):
    """Octant spectrum as [6][mz/2+1][my/2+1][hx] (the device stores it kx-major)."""
    nx, ny, nz, mx, my, mz, hx = tdgl_get_dims(ctx)
    out = np.zeros((hx, 6, mz // 2 + 1, my // 2 + 1))
    _check(ctx, lib().tdgl_get_tensor_spectrum(
        ctx, out.ctypes.data_as(ctypes.POINTER(c_double)), out.size))
    return np.ascontiguousarray(out.transpose(1, 2, 3, 0))


def tdgl_set_fft_path(ctx, path: int):
    _check(ctx, lib().tdgl_set_fft_path(ctx, path))


def tdgl_set_update_rows(ctx, rows: int):
    _check(ctx, lib().tdgl_set_update_rows(ctx, rows))


def tdgl_set_z_tile(ctx, row_bytes: int):
    _check(ctx, lib().tdgl_set_z_tile(ctx, row_bytes))


def tdgl_get_z_tile(ctx):
    v = c_int()
    _check(ctx, lib().tdgl_get_z_tile(ctx, ctypes.byref(v)))
    return v.value


def tdgl_set_store_mode(ctx, mode: int):
    _check(ctx, lib().tdgl_set_store_mode(ctx, mode))


def tdgl_get_store_mode(ctx):
    v = c_int()
    _check(ctx, lib().tdgl_get_store_mode(ctx, ctypes.byref(v)))
    return v.value


def tdgl_get_fft_path(ctx):
    f = c_int()
    _check(ctx, lib().tdgl_get_fft_path(ctx, ctypes.byref(f)))
    return f.value


def tdgl_set_temperature(ctx, T):
    _check(ctx, lib().tdgl_set_temperature(ctx, T))


def tdgl_set_temperatures(ctx, T):
    arr = (c_double * len(T))(*[float(v) for v in T])
    _check(ctx, lib().tdgl_set_temperatures(ctx, arr))


def tdgl_set_eext(ctx, ex, ey, ez):
    _check(ctx, lib().tdgl_set_eext(ctx, ex, ey, ez))


def tdgl_set_terms(ctx, mask):
    _check(ctx, lib().tdgl_set_terms(ctx, mask))


def tdgl_set_integrator(ctx, scheme, dtau):
    _check(ctx, lib().tdgl_set_integrator(ctx, scheme, dtau))


def tdgl_set_graph_chunk(ctx, steps):
    _check(ctx, lib().tdgl_set_graph_chunk(ctx, steps))


def tdgl_set_P(ctx, src_ptr: int, src_on_device: int, src_precision: int):
    _check(ctx, lib().tdgl_set_P(ctx, src_ptr, src_on_device, src_precision))


def tdgl_get_P(ctx, dst_ptr: int, dst_on_device: int, dst_precision: int):
    _check(ctx, lib().tdgl_get_P(ctx, dst_ptr, dst_on_device, dst_precision))


def tdgl_step(ctx, nsteps: int):
    _check(ctx, lib().tdgl_step(ctx, nsteps))


def tdgl_eval_field(ctx, mask: int, dst_ptr: int):
    _check(ctx, lib().tdgl_eval_field(ctx, mask, dst_ptr))


def tdgl_energies(ctx):
    F = (c_double * 5)()
    m = (c_double * 3)()
    _check(ctx, lib().tdgl_energies(ctx, F, m))
    return tuple(F), tuple(m)


def tdgl_energies_noalloc(ctx, out_dev_ptr: int):
    """Enqueue the energies of every instance into device memory
    out_dev_ptr ([nbatch][8] float64: F_Land, F_Grad, F_Elec, F_Ext, F in J,
    mean P in C/m^2) without allocating; asynchronous."""
    _check(ctx, lib().tdgl_energies_noalloc(ctx, out_dev_ptr))


def tdgl_energies_batch(ctx):
    nb = tdgl_get_batch(ctx)
    F = np.zeros((nb, 5))
    m = np.zeros((nb, 3))
    _check(ctx, lib().tdgl_energies_batch(ctx, F.ctypes.data_as(ctypes.POINTER(c_double)),
                                          m.ctypes.data_as(ctypes.POINTER(c_double))))
    return F, m


def tdgl_get_reduced(ctx, nz: int):
    coef = np.zeros((nz, 8))
    scal = np.zeros(8)
    _check(ctx, lib().tdgl_get_reduced(ctx, coef.ctypes.data_as(ctypes.POINTER(c_double)),
                                       scal.ctypes.data_as(ctypes.POINTER(c_double))))
    return coef, scal


def tdgl_profile_step(ctx, nsteps: int):
    ms = (c_double * 5)()
    _check(ctx, lib().tdgl_profile_step(ctx, nsteps, ms))
    return tuple(ms)


def tdgl_profile_kernels(ctx, nrep: int):
    ms = (c_double * 5)()
    _check(ctx, lib().tdgl_profile_kernels(ctx, nrep, ms))
    return tuple(ms)


def tdgl_relax(ctx, nbatch: int, check: int, max_steps: int, rtol: float = 1e-6,
               floor_factor: float = 1e-3, retire: bool = False):
    """Relax every instance (tdgl_relax); returns (relax step per instance,
    -1 if not relaxed; steps taken)."""
    steps = (c_longlong * nbatch)()
    taken = c_longlong(0)
    _check(ctx, lib().tdgl_relax(ctx, check, max_steps, rtol, floor_factor, int(retire),
                                 steps, ctypes.byref(taken)))
    return np.array(steps[:], dtype=np.int64), int(taken.value)


def tdgl_relax_group(ctxs, nbatches, check: int, max_steps: int, rtol: float = 1e-6,
                     floor_factor: float = 1e-3, retire: bool = False):
    """Relax several contexts in one graph per chunk (tdgl_relax_group);
    returns (list of per-instance relax steps per context; steps taken)."""
    n = len(ctxs)
    arr = (_ctx_p * n)(*ctxs)
    total = int(sum(nbatches))
    steps = (c_longlong * total)()
    taken = c_longlong(0)
    st = lib().tdgl_relax_group(arr, n, check, max_steps, rtol, floor_factor, int(retire), steps,
                                ctypes.byref(taken))
    if st != TDGL_OK:
        msgs = [(lib().tdgl_last_error(c) or b"").decode() for c in ctxs]
        raise TdglError(st, "tdgl_relax_group: " + " | ".join(m for m in msgs if m))
    out, off = [], 0
    for nb in nbatches:
        out.append(np.array(steps[off:off + nb], dtype=np.int64))
        off += nb
    return out, int(taken.value)


def tdgl_sweep_eext(ctx, e, steps_per_value: int):
    """e: (n, 3) applied fields in V/m.  Returns meanP (n, nbatch, 3) and
    F (n, nbatch, 5)."""
    e = np.ascontiguousarray(e, dtype=np.float64).reshape(-1, 3)
    nb = tdgl_get_batch(ctx)
    m = np.zeros((len(e), nb, 3))
    F = np.zeros((len(e), nb, 5))
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(c_double))
    _check(ctx, lib().tdgl_sweep_eext(ctx, dp(e), len(e), steps_per_value, dp(m), dp(F)))
    return m, F


def triangle_wave(amp: float, n: int) -> np.ndarray:
    """n values of a triangle wave 0 -> +amp -> -amp -> 0 (one period, the
    first value one step above 0)."""
    ph = np.arange(1, n + 1) / n
    return amp * np.where(ph < 0.25, 4 * ph, np.where(ph < 0.75, 2 - 4 * ph, 4 * ph - 4))


def tdgl_autotune(ctx, nsteps: int):
    """Returns (fused, rows, ms_per_step) of the configuration it kept."""
    ch = (c_int * 2)()
    ms = c_double()
    _check(ctx, lib().tdgl_autotune(ctx, nsteps, ch, ctypes.byref(ms)))
    return ch[0], ch[1], ms.value


def tdgl_set_rk_tolerances(ctx, atol: float, rtol: float):
    _check(ctx, lib().tdgl_set_rk_tolerances(ctx, atol, rtol))


def tdgl_get_rk_state(ctx):
    """(reduced time, current step, rejected attempts) of the RK45 run."""
    tau, h, rej = c_double(), c_double(), ctypes.c_longlong()
    _check(ctx, lib().tdgl_get_rk_state(ctx, ctypes.byref(tau), ctypes.byref(h),
                                        ctypes.byref(rej)))
    return tau.value, h.value, rej.value


def tdgl_sync(ctx):
    _check(ctx, lib().tdgl_sync(ctx))


# --------------------------------------------------------- convenience class
class Context:
    """One simulation, or a batch of `batch` simulations of the same grid, on
    the current torch CUDA (HIP) device and stream.

    cfg: a run recipe dict (grid "n", cell size "d", "periodic", "materials",
    "layers", "gradient", "scales", "T", "eext", "terms", "scheme", "dtau",
    "mimg").  For a batch, "T" may be a list of per-instance temperatures
    and P carries a leading instance dimension.  The workspace is a torch
    uint8 tensor bound to the context.
    """

    def __init__(self, cfg: dict, precision: int = TDGL_FP32, stream=None, build_tensor=True,
                 torch_workspace=True, batch: int = 0):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.precision = precision
        nx, ny, nz = cfg["n"]
        pm = sum(1 << k for k in range(3) if cfg["periodic"][k])
        g = tdgl_grid(nx, ny, nz, cfg["d"][0], cfg["d"][1], cfg["d"][2], pm)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.batch = batch
        if batch:
            self.ctx = tdgl_create_batch(g, batch, precision, c_void_p(self.stream.cuda_stream))
        else:
            self.ctx = tdgl_create(g, precision, c_void_p(self.stream.cuda_stream))
        self.dims = tdgl_get_dims(self.ctx)
        self.workspace = None
        s = cfg["scales"]
        tdgl_set_scales(self.ctx, s["P0"], s["alpha_ref"], s["G110"], s["eps_b"])
        for i, m in enumerate(cfg["materials"]):
            tdgl_set_material(self.ctx, i, m)
        tdgl_set_layer_materials(self.ctx, cfg["layers"])
        G = cfg["gradient"]
        tdgl_set_gradient(self.ctx, G["G11"], G["G12"], G["G44"], G["G44p"])
        if np.ndim(cfg["T"]) == 0:
            tdgl_set_temperature(self.ctx, cfg["T"])
        else:
            tdgl_set_temperatures(self.ctx, cfg["T"])
        tdgl_set_eext(self.ctx, *cfg.get("eext", (0.0, 0.0, 0.0)))
        tdgl_set_terms(self.ctx, cfg.get("terms", TDGL_ALL))
        schemes = {"euler": TDGL_EULER, "heun": TDGL_HEUN, "ab3m2": TDGL_AB3M2,
                   "rk45": TDGL_RK45}
        tdgl_set_integrator(self.ctx, schemes[cfg.get("scheme", "heun")], cfg.get("dtau", 1e-3))
        if torch_workspace:       # sized for the integrator just set
            nbytes = tdgl_workspace_size(self.ctx)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            ptr = self.workspace.data_ptr()
            ptr = (ptr + 255) // 256 * 256
            tdgl_bind_workspace(self.ctx, ptr, nbytes)
        if build_tensor and (cfg.get("terms", TDGL_ALL) & TDGL_ELEC):
            tdgl_build_tensor(self.ctx, cfg.get("mimg", 16))

    @property
    def shape(self):
        nx, ny, nz = self.cfg["n"]
        return (self.batch, 3, nz, ny, nx) if self.batch else (3, nz, ny, nx)

    def _tdtype(self, prec):
        return self.torch.float32 if prec == TDGL_FP32 else self.torch.float64

    def set_P(self, P):
        """P: numpy array (host) or torch tensor (device or host), C/m^2."""
        torch = self.torch
        if isinstance(P, torch.Tensor):
            P = P.contiguous()
            prec = TDGL_FP32 if P.dtype == torch.float32 else TDGL_FP64
            if P.dtype not in (torch.float32, torch.float64):
                raise TypeError("P must be float32 or float64")
            tdgl_set_P(self.ctx, P.data_ptr(), 1 if P.is_cuda else 0, prec)
            self._keep = P
        else:
            P = np.ascontiguousarray(P)
            if P.dtype not in (np.float32, np.float64):
                raise TypeError("P must be float32 or float64")
            prec = TDGL_FP32 if P.dtype == np.float32 else TDGL_FP64
            tdgl_set_P(self.ctx, P.ctypes.data, 0, prec)

    def get_P(self, precision=TDGL_FP64) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.float32 if precision == TDGL_FP32 else np.float64)
        tdgl_get_P(self.ctx, out.ctypes.data, 0, precision)
        return out

    def get_P_device(self, precision=None):
        precision = self.precision if precision is None else precision
        out = self.torch.empty(self.shape, dtype=self._tdtype(precision), device="cuda")
        tdgl_get_P(self.ctx, out.data_ptr(), 1, precision)
        return out

    def step(self, n: int):
        tdgl_step(self.ctx, n)

    def eval_field(self, mask: int = TDGL_ALL):
        out = self.torch.empty(self.shape, dtype=self._tdtype(self.precision), device="cuda")
        tdgl_eval_field(self.ctx, mask, out.data_ptr())
        return out

    def energies(self):
        return tdgl_energies(self.ctx)

    def energies_batch(self):
        """Per instance: F[nb][5] (J), meanP[nb][3] (C/m^2)."""
        return tdgl_energies_batch(self.ctx)

    def relax(self, check=100, max_steps=20000, rtol=1e-6, floor_factor=1e-3, retire=False):
        """tdgl_relax: (relax step per instance, -1 if not relaxed; steps taken)."""
        return tdgl_relax(self.ctx, max(self.batch, 1), check, max_steps, rtol, floor_factor,
                          retire)

    def sync(self):
        tdgl_sync(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            tdgl_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
