"""CPU oracle for the TDGL time step — TEST INFRASTRUCTURE ONLY.

Plain, slow FP64 implementation of what one time step of the paper's method
computes (sections 2-3: eqs 1-7, Tables 1-2).  It is imported only by the
tests, the smoke check and the benchmark's CPU-baseline leg; the product
library never calls it, and the two share no code.  The only module both sides
use is ``tdgl_inputs`` (seeded input data, no arithmetic of the method).

Layout: ``tdgl_oracle`` (numpy: coefficients, normalisation, Landau and
gradient fields, electrostatic field by direct sum or FFT, integrators,
energies) and ``tensor_oracle.c`` (plain C: the dipolar tensor of two box
cells, built as ``_tensor_oracle.so`` with gcc).
"""
import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_tensor_oracle.so")
_SRC = os.path.join(_HERE, "tensor_oracle.c")


def gcc_command(src=_SRC, out=_SO):
    return ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
            "-o", out, src, "-lm"]


def build(force=False):
    """Compile tensor_oracle.c (gcc, OpenMP) if it is missing or stale."""
    if (not force and os.path.exists(_SO)
            and os.path.getmtime(_SO) >= os.path.getmtime(_SRC)):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(gcc_command(out=tmp))
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_newell.argtypes = [dp, dp, dp]
        L.orc_quad.argtypes = [dp, dp, ctypes.c_int, dp, dp, dp]
        L.orc_quad_order.argtypes = [ctypes.c_double]
        L.orc_quad_order.restype = ctypes.c_int
        L.orc_cell_tensor.argtypes = [dp, dp, dp, dp, dp]
        L.orc_offset_table.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_uint,
                                       ctypes.c_int, dp, dp, dp, dp]
        L.orc_offset_entry.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_uint,
                                       ctypes.c_int, dp, dp, dp,
                                       ctypes.POINTER(ctypes.c_int), dp]
        L.orc_newell_f.argtypes = [ctypes.c_double] * 3
        L.orc_newell_f.restype = ctypes.c_double
        L.orc_newell_g.argtypes = [ctypes.c_double] * 3
        L.orc_newell_g.restype = ctypes.c_double
        _lib = L
    return _lib
