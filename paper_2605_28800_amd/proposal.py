"""Initial-state proposal network: thin binding of include/tdgl_net.h.

Argument marshalling only; forward, backward, loss and Adam run in the HIP
kernels of libtdgl.so.  Device arrays are torch tensors (float32 / int32 /
raw BF16 as int16, contiguous, on the current HIP device); the network works
on the stream given at construction (default: torch's current stream).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import TdglError, TDGL_OK, lib

c_int, c_double, c_void_p, c_size_t = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t

# epilogues of tdgl_nn_conv3
EPI_ACT, EPI_ACT_SKIP, EPI_P, EPI_RAW, EPI_RAW_D, EPI_RAW_AND_D = range(6)


class tdgl_net_cfg(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("nz", c_int), ("width", c_int),
                ("noise_div", c_int), ("max_batch", c_int)]


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


class Net:
    """A proposal network for samples of shape (nz, ny, nx)."""

    def __init__(self, shape, width=32, noise_div=8, max_batch=16, stream=None):
        import torch
        self.torch = torch
        nz, ny, nx = shape
        self.shape = (nz, ny, nx)
        self.width, self.noise_div, self.max_batch = width, noise_div, max_batch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        cfg = tdgl_net_cfg(nx, ny, nz, width, noise_div, max_batch)
        h = c_void_p()
        st = lib().tdgl_net_create(ctypes.byref(cfg), c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(h))
        if st != TDGL_OK:
            raise TdglError(st, "tdgl_net_create")
        self.h = h
        n = ctypes.c_longlong()
        self._check(lib().tdgl_net_num_params(self.h, ctypes.byref(n)))
        self.num_params = n.value

    def _check(self, st):
        if st != TDGL_OK:
            msg = lib().tdgl_net_last_error(self.h) or b""
            raise TdglError(st, msg.decode())

    def close(self):
        if getattr(self, "h", None):
            lib().tdgl_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == self.num_params
        self._check(lib().tdgl_net_set_params(self.h, a.ctypes.data_as(c_void_p), a.size))

    def get_params(self):
        a = np.empty(self.num_params, dtype=np.float32)
        self._check(lib().tdgl_net_get_params(self.h, a.ctypes.data_as(c_void_p), a.size))
        return a

    def forward(self, T, thick, noise, idx=None, nb=None):
        """P [nb][3][nz][ny][nx] (torch float32 on the device)."""
        nb = nb if nb is not None else (len(idx) if idx is not None else T.shape[0])
        P = self.torch.empty((nb, 3) + self.shape, dtype=self.torch.float32, device=T.device)
        self._check(lib().tdgl_net_forward(self.h, nb, _ptr(idx), _ptr(T), _ptr(thick),
                                           _ptr(noise), _ptr(P)))
        return P

    def loss_grad(self, T, thick, noise, target, idx=None, nb=None, want_grad=True, ops=None):
        """ops: int32 device tensor of per-sample in-plane symmetry ops, or None."""
        nb = nb if nb is not None else (len(idx) if idx is not None else T.shape[0])
        loss = c_double()
        g = np.empty(self.num_params, dtype=np.float32) if want_grad else None
        self._check(lib().tdgl_net_loss_grad(
            self.h, nb, _ptr(idx), _ptr(ops), _ptr(T), _ptr(thick), _ptr(noise), _ptr(target),
            ctypes.byref(loss), g.ctypes.data_as(c_void_p) if want_grad else None))
        return loss.value, g

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self._check(lib().tdgl_net_adam(self.h, lr, b1, b2, eps))

    def train(self, idx, nb, T, thick, noise, target, lr, b1=0.9, b2=0.999, eps=1e-8, ops=None):
        """len(idx) / nb steps; idx: int32 device tensor of dataset rows; ops:
        int32 device tensor of the samples' symmetry ops (same length) or None."""
        nsteps = idx.numel() // nb
        losses = np.empty(nsteps, dtype=np.float64)
        self._check(lib().tdgl_net_train(self.h, nsteps, nb, _ptr(idx), _ptr(ops), _ptr(T),
                                         _ptr(thick), _ptr(noise), _ptr(target), lr, b1, b2, eps,
                                         losses.ctypes.data_as(c_void_p)))
        return losses

    def profile(self, nb, T, thick, noise, target, reps=5):
        ms = (c_double * 6)()
        self._check(lib().tdgl_net_profile(self.h, nb, _ptr(T), _ptr(thick), _ptr(noise),
                                           _ptr(target), reps, ms))
        return list(ms)


def nn_conv3(epi, inp, w, bias, nb, lx, ly, lz, cin_p, cout_p, out=None, out2=None, aux=None,
             P=None, thick=None, in_up2=0, stream=None):
    """One convolution through tdgl_nn_conv3 (BF16 tensors as torch int16)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    st = lib().tdgl_nn_conv3(epi, _ptr(inp), int(in_up2), _ptr(w), _ptr(bias), nb, lx, ly, lz,
                             cin_p, cout_p, _ptr(out), _ptr(out2), _ptr(aux), _ptr(P),
                             _ptr(thick), c_void_p(s.cuda_stream))
    if st != TDGL_OK:
        raise TdglError(st, "tdgl_nn_conv3")


def nn_conv3_wgrad(g, inp, nb, lx, ly, lz, cin_p, cout_p, in_up2=0, stream=None):
    """Weight and bias gradient (torch float32 [cout_p * 27 * cin_p + cout_p])."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    nbytes = c_size_t()
    st = lib().tdgl_nn_wgrad_workspace(nb, lx, ly, lz, cin_p, cout_p, ctypes.byref(nbytes))
    if st != TDGL_OK:
        raise TdglError(st, "tdgl_nn_wgrad_workspace")
    ws = torch.empty(nbytes.value // 4 + 1, dtype=torch.float32, device=g.device)
    grad = torch.empty(cout_p * 27 * cin_p + cout_p, dtype=torch.float32, device=g.device)
    st = lib().tdgl_nn_conv3_wgrad(_ptr(g), _ptr(inp), int(in_up2), nb, lx, ly, lz, cin_p, cout_p,
                                   _ptr(ws), nbytes.value, _ptr(grad), c_void_p(s.cuda_stream))
    if st != TDGL_OK:
        raise TdglError(st, "tdgl_nn_conv3_wgrad")
    return grad
