"""Thin ctypes binding of ``libfraclap.so`` (C ABI in ``include/fraclap.h``).

Argument marshalling only: every step of assembly, matvec and solve runs in
the HIP library.  PyTorch supplies device memory and the stream.  The
library must have been built (``paper_1708_03912_amd/csrc/build.py``); a
missing library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfraclap.so")

FL_OK, FL_EINVAL, FL_EMESH, FL_ENOMEM, FL_EDEVICE = 0, -1, -2, -3, -4
FL_ESTATE, FL_ENONFINITE, FL_EBREAKDOWN, FL_ENOCONV = -5, -6, -7, 1
FL_DOF_PAPER, FL_DOF_INTERIOR = 0, 1
FL_FP64, FL_MIXED = 0, 1
FL_MAX_CLASSES = 8

ERROR_NAMES = {0: "FL_OK", -1: "FL_EINVAL", -2: "FL_EMESH", -3: "FL_ENOMEM", -4: "FL_EDEVICE",
               -5: "FL_ESTATE", -6: "FL_ENONFINITE", -7: "FL_EBREAKDOWN", 1: "FL_ENOCONV"}

# every symbol include/fraclap.h declares
EXPORTS = ["fl_default_opts", "fl_create", "fl_destroy", "fl_last_error", "fl_set_mesh",
           "fl_assemble", "fl_matrix_ld", "fl_matrix_ptr", "fl_dofs", "fl_export_matrix",
           "fl_load_vector_one", "fl_matvec", "fl_solve", "fl_energy_error2", "fl_stats"]


class FlOpts(C.Structure):
    _fields_ = [("dof_mode", C.c_int), ("with_boundary", C.c_int), ("k_touch", C.c_int),
                ("k_touch_bnd", C.c_int), ("n_classes", C.c_int),
                ("theta", C.c_double * FL_MAX_CLASSES),
                ("k_far", C.c_int * (FL_MAX_CLASSES + 1)),
                ("k_far_bnd", C.c_int * (FL_MAX_CLASSES + 1)), ("precision", C.c_int)]


class FlStats(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_cells", C.c_int64), ("n_verts", C.c_int64),
                ("n_bfacets", C.c_int64), ("pairs_identical", C.c_int64),
                ("pairs_edge", C.c_int64), ("pairs_vertex", C.c_int64),
                ("pairs_far", C.c_int64 * (FL_MAX_CLASSES + 1)),
                ("pairs_bnd_touch", C.c_int64), ("pairs_bnd_far", C.c_int64),
                ("kernel_evals", C.c_int64), ("t_plan_ms", C.c_double),
                ("t_assemble_ms", C.c_double), ("t_far_ms", C.c_double), ("t_self_ms", C.c_double),
                ("t_touch_ms", C.c_double), ("t_scatter_ms", C.c_double), ("t_solve_ms", C.c_double),
                ("last_iters", C.c_int32), ("last_relres", C.c_double), ("last_outer", C.c_int32)]


class FraclapError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libfraclap.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FraclapError(FL_EDEVICE, f"{LIB_PATH} not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, dp = C.c_void_p, C.c_int64, C.c_double
        L.fl_default_opts.argtypes = [C.POINTER(FlOpts)]
        L.fl_create.argtypes = [C.POINTER(vp), C.c_int, vp]
        L.fl_destroy.argtypes = [vp]
        L.fl_destroy.restype = None
        L.fl_last_error.argtypes = [vp]
        L.fl_last_error.restype = C.c_char_p
        L.fl_set_mesh.argtypes = [vp, C.c_int, i64, vp, i64, vp, i64, vp]
        L.fl_assemble.argtypes = [vp, dp, C.POINTER(FlOpts), C.POINTER(i64)]
        L.fl_matrix_ld.argtypes = [vp]
        L.fl_matrix_ld.restype = i64
        L.fl_matrix_ptr.argtypes = [vp]
        L.fl_matrix_ptr.restype = vp
        L.fl_dofs.argtypes = [vp, vp]
        L.fl_export_matrix.argtypes = [vp, vp, i64, C.c_int]
        L.fl_load_vector_one.argtypes = [vp, vp]
        L.fl_matvec.argtypes = [vp, vp, vp]
        L.fl_solve.argtypes = [vp, vp, vp, dp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(dp)]
        L.fl_energy_error2.argtypes = [vp, dp, vp, vp, C.POINTER(dp)]
        L.fl_stats.argtypes = [vp, C.POINTER(FlStats)]
        _lib = L
    return _lib


def default_opts() -> FlOpts:
    o = FlOpts()
    lib().fl_default_opts(C.byref(o))
    return o


def make_opts(k_touch=None, k_touch_bnd=None, theta=None, k_far=None, k_far_bnd=None,
              dof_mode=None, with_boundary=None, precision=None) -> FlOpts:
    o = default_opts()
    if precision is not None:
        o.precision = {"fp64": FL_FP64, "mixed": FL_MIXED}.get(precision, precision)
    if dof_mode is not None:
        o.dof_mode = {"paper": FL_DOF_PAPER, "interior": FL_DOF_INTERIOR}.get(dof_mode, dof_mode)
    if with_boundary is not None:
        o.with_boundary = int(with_boundary)
    if k_touch is not None:
        o.k_touch = k_touch
    if k_touch_bnd is not None:
        o.k_touch_bnd = k_touch_bnd
    if theta is not None:
        o.n_classes = len(theta)
        for i, t in enumerate(theta):
            o.theta[i] = t
    if k_far is not None:
        for i, k in enumerate(k_far):
            o.k_far[i] = k
    if k_far_bnd is not None:
        for i, k in enumerate(k_far_bnd):
            o.k_far_bnd[i] = k
    return o


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Handle:
    """One library handle on ``device`` bound to torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._torch = torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.device = device
        h = C.c_void_p()
        rc = lib().fl_create(C.byref(h), device, C.c_void_p(stream.cuda_stream))
        if rc != FL_OK:
            raise FraclapError(rc, "fl_create failed")
        self.h = h
        self.n = 0

    def close(self):
        if getattr(self, "h", None):
            lib().fl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=(FL_OK,)):
        if rc not in allow:
            raise FraclapError(rc, lib().fl_last_error(self.h).decode())
        return rc

    def set_mesh(self, mesh):
        dim = int(mesh["dim"])
        v = np.ascontiguousarray(mesh["verts"], dtype=np.float64)
        c = np.ascontiguousarray(mesh["cells"], dtype=np.int32)
        b = np.ascontiguousarray(mesh["bfacets"], dtype=np.int32)
        self._check(lib().fl_set_mesh(self.h, dim, v.size // dim, v.ctypes.data_as(C.c_void_p),
                                      c.shape[0], c.ctypes.data_as(C.c_void_p), b.shape[0],
                                      b.ctypes.data_as(C.c_void_p)))

    def assemble(self, s: float, opts: FlOpts | None = None) -> int:
        n = C.c_int64()
        self._check(lib().fl_assemble(self.h, s, None if opts is None else C.byref(opts), C.byref(n)))
        self.n = n.value
        return self.n

    @property
    def ld(self) -> int:
        return lib().fl_matrix_ld(self.h)

    def dofs(self) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.int32)
        self._check(lib().fl_dofs(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def export_matrix(self) -> np.ndarray:
        out = np.zeros((self.n, self.n), dtype=np.float64)
        self._check(lib().fl_export_matrix(self.h, out.ctypes.data_as(C.c_void_p), self.n, 0))
        return out

    def export_matrix_device(self, dst):
        self._check(lib().fl_export_matrix(self.h, _ptr(dst), dst.stride(0), 1))

    def matrix_view(self):
        """torch view (n x n, row stride ld) of the handle-owned matrix."""
        torch = self._torch
        ptr = lib().fl_matrix_ptr(self.h)
        if not ptr:
            raise FraclapError(FL_ESTATE, "no matrix")
        return _device_view(torch, ptr, self.n, self.ld, self.device)

    def load_vector_one(self, b):
        self._check(lib().fl_load_vector_one(self.h, _ptr(b)))

    def matvec(self, x, y):
        self._check(lib().fl_matvec(self.h, _ptr(x), _ptr(y)))

    def solve(self, b, u, rtol=1e-12, maxit=100000):
        it = C.c_int32()
        rel = C.c_double()
        rc = self._check(lib().fl_solve(self.h, _ptr(b), _ptr(u), rtol, maxit, C.byref(it), C.byref(rel)),
                         allow=(FL_OK, FL_ENOCONV))
        return it.value, rel.value, rc

    def energy_error2(self, fu, b, uh) -> float:
        e2 = C.c_double()
        self._check(lib().fl_energy_error2(self.h, fu, _ptr(b), _ptr(uh), C.byref(e2)))
        return e2.value

    def stats(self) -> FlStats:
        st = FlStats()
        self._check(lib().fl_stats(self.h, C.byref(st)))
        return st


def _device_view(torch, ptr, n, ld, device):
    """Wrap a library-owned device pointer as a strided torch tensor without
    copying (DLPack-free: via a typed-storage-less from_blob equivalent)."""
    class _Cai:
        __cuda_array_interface__ = {
            "shape": (n, n), "typestr": "<f8", "data": (ptr, False),
            "strides": (ld * 8, 8), "version": 2}
    return torch.as_tensor(_Cai(), device=f"cuda:{device}")
