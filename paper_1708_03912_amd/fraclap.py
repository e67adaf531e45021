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
FL_F64, FL_F32, FL_BF16, FL_BF16X2 = 0, 1, 2, 3
FL_RHS_ONE, FL_RHS_FOURIER16, FL_RHS_P1_NODAL = 0, 1, 2
FL_MAX_BATCH = 16
FL_MAX_CLASSES = 8
DTYPES = {"f64": FL_F64, "f32": FL_F32, "bf16": FL_BF16, "bf16x2": FL_BF16X2}

ERROR_NAMES = {0: "FL_OK", -1: "FL_EINVAL", -2: "FL_EMESH", -3: "FL_ENOMEM", -4: "FL_EDEVICE",
               -5: "FL_ESTATE", -6: "FL_ENONFINITE", -7: "FL_EBREAKDOWN", 1: "FL_ENOCONV"}

# every symbol include/fraclap.h declares
EXPORTS = ["fl_default_opts", "fl_create", "fl_destroy", "fl_last_error", "fl_set_mesh",
           "fl_assemble", "fl_matrix_ld", "fl_matrix_ptr", "fl_dofs", "fl_export_matrix",
           "fl_load_vector_one", "fl_matvec", "fl_solve", "fl_energy_error2", "fl_stats",
           "fl_import_matrix", "fl_load_vector", "fl_assemble_batch", "fl_export_batch_matrix",
           "fl_matmul", "fl_solve_batch", "fl_autotune", "fl_default_train_opts", "fl_pair_integrals",
           "fl_surrogate_dataset", "fl_surrogate_init", "fl_surrogate_fit_scaling",
           "fl_surrogate_set_params", "fl_surrogate_get_params", "fl_surrogate_grad", "fl_surrogate_train",
           "fl_surrogate_predict", "fl_surrogate_certify", "fl_mass_matvec", "fl_mg_setup", "fl_solve_mg",
           "fl_eval_points", "fl_strong_form", "fl_indicators", "fl_cluster_build", "fl_cluster_matvec",
           "fl_solve_cluster", "fl_cluster_info", "fl_set_symmetry",
           "fl_strong_form_cluster", "fl_solve_cluster_mg", "fl_matvec_noalloc", "fl_cluster_assemble"]
SUR_NIN, SUR_NOUT, SUR_NPARAM, SUR_NRB, SUR_NSB, SUR_BLOB = 9, 21, 8352, 6, 4, 8454


class FlOpts(C.Structure):
    _fields_ = [("dof_mode", C.c_int), ("with_boundary", C.c_int), ("k_touch", C.c_int),
                ("k_touch_bnd", C.c_int), ("n_classes", C.c_int),
                ("theta", C.c_double * FL_MAX_CLASSES),
                ("k_far", C.c_int * (FL_MAX_CLASSES + 1)),
                ("k_far_bnd", C.c_int * (FL_MAX_CLASSES + 1)), ("precision", C.c_int),
                ("surrogate", C.c_int), ("sur_tol", C.c_double), ("mass_shift", C.c_double),
                ("deterministic", C.c_int)]


class FlStats(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_cells", C.c_int64), ("n_verts", C.c_int64),
                ("n_bfacets", C.c_int64), ("pairs_identical", C.c_int64),
                ("pairs_edge", C.c_int64), ("pairs_vertex", C.c_int64),
                ("pairs_far", C.c_int64 * (FL_MAX_CLASSES + 1)),
                ("pairs_bnd_touch", C.c_int64), ("pairs_bnd_far", C.c_int64),
                ("kernel_evals", C.c_int64), ("t_plan_ms", C.c_double),
                ("t_assemble_ms", C.c_double), ("t_far_ms", C.c_double), ("t_self_ms", C.c_double),
                ("t_touch_ms", C.c_double), ("t_scatter_ms", C.c_double), ("t_solve_ms", C.c_double),
                ("last_iters", C.c_int32), ("last_relres", C.c_double), ("last_outer", C.c_int32),
                ("pairs_surrogate", C.c_int64), ("pairs_fallback", C.c_int64),
                ("t_cg_kernels_ms", C.c_double), ("cg_launched", C.c_int64)]


class FlTrainOpts(C.Structure):
    _fields_ = [("steps", C.c_int), ("batch", C.c_int), ("lr", C.c_double), ("lr_min", C.c_double),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double), ("seed", C.c_uint64)]


class FlTuneEntry(C.Structure):
    _fields_ = [("wm", C.c_int), ("waves", C.c_int), ("bk", C.c_int), ("planes", C.c_int),
                ("ms", C.c_double), ("tflops", C.c_double), ("gbps", C.c_double)]


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
        L.fl_matvec_noalloc.argtypes = [vp, vp, vp]
        L.fl_mass_matvec.argtypes = [vp, vp, vp]
        L.fl_mg_setup.argtypes = [vp, C.c_int, vp, vp]
        L.fl_eval_points.argtypes = [vp, C.c_int32, vp, vp]
        L.fl_cluster_build.argtypes = [vp, C.c_int32, dp, C.c_int32]
        L.fl_cluster_assemble.argtypes = [vp, dp, C.POINTER(FlOpts), C.c_int32, dp, C.c_int32, C.POINTER(i64)]
        L.fl_set_symmetry.argtypes = [vp, C.c_int32, i64, vp, vp, vp]
        L.fl_cluster_matvec.argtypes = [vp, vp, vp]
        L.fl_solve_cluster.argtypes = [vp, vp, vp, dp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(dp)]
        L.fl_cluster_info.argtypes = [vp, vp]
        L.fl_strong_form.argtypes = [vp, dp, vp, C.c_int32, C.c_int32, C.c_int32, vp]
        L.fl_strong_form_cluster.argtypes = [vp, dp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, dp,
                                             C.c_int32, vp]
        L.fl_indicators.argtypes = [vp, dp, vp, vp, C.c_int32, vp, vp]
        L.fl_solve_mg.argtypes = [vp, vp, vp, dp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(dp)]
        L.fl_solve_cluster_mg.argtypes = [vp, vp, vp, dp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(dp)]
        L.fl_solve.argtypes = [vp, vp, vp, dp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(dp)]
        L.fl_energy_error2.argtypes = [vp, dp, vp, vp, C.POINTER(dp)]
        L.fl_stats.argtypes = [vp, C.POINTER(FlStats)]
        L.fl_import_matrix.argtypes = [vp, vp, i64, C.c_int]
        L.fl_load_vector.argtypes = [vp, C.c_int, vp, i64, vp]
        L.fl_assemble_batch.argtypes = [vp, vp, C.c_int, C.POINTER(FlOpts), C.POINTER(i64)]
        L.fl_export_batch_matrix.argtypes = [vp, C.c_int, vp, i64, C.c_int]
        L.fl_matmul.argtypes = [vp, C.c_int, C.c_int, vp, i64, vp, i64, i64]
        L.fl_solve_batch.argtypes = [vp, vp, i64, i64, vp, i64, i64, i64, dp, C.c_int32, C.c_int, vp, vp]
        L.fl_autotune.argtypes = [vp, C.c_int, C.POINTER(FlTuneEntry), C.c_int, C.POINTER(C.c_int),
                                  C.POINTER(C.c_int)]
        L.fl_default_train_opts.argtypes = [C.POINTER(FlTrainOpts)]
        L.fl_pair_integrals.argtypes = [vp, i64, vp, vp, vp, C.c_int, vp]
        L.fl_surrogate_dataset.argtypes = [vp, i64, vp, vp, vp, C.c_int, vp, vp]
        L.fl_surrogate_init.argtypes = [vp, C.c_uint64]
        L.fl_surrogate_fit_scaling.argtypes = [vp, vp, vp, i64]
        L.fl_surrogate_set_params.argtypes = [vp, vp]
        L.fl_surrogate_get_params.argtypes = [vp, vp]
        L.fl_surrogate_grad.argtypes = [vp, vp, vp, i64, vp, C.POINTER(dp)]
        L.fl_surrogate_train.argtypes = [vp, vp, vp, i64, C.POINTER(FlTrainOpts), vp]
        L.fl_surrogate_predict.argtypes = [vp, vp, i64, vp]
        L.fl_surrogate_certify.argtypes = [vp, vp, vp, i64, vp]
        _lib = L
    return _lib


def default_opts() -> FlOpts:
    o = FlOpts()
    lib().fl_default_opts(C.byref(o))
    return o


def default_train_opts(**kw) -> FlTrainOpts:
    o = FlTrainOpts()
    lib().fl_default_train_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def make_opts(k_touch=None, k_touch_bnd=None, theta=None, k_far=None, k_far_bnd=None,
              dof_mode=None, with_boundary=None, precision=None, surrogate=None, sur_tol=None,
              mass_shift=None, deterministic=None) -> FlOpts:
    o = default_opts()
    if deterministic is not None:
        o.deterministic = int(bool(deterministic))
    if mass_shift is not None:
        o.mass_shift = float(mass_shift)
    if surrogate is not None:
        o.surrogate = int(surrogate)
    if sur_tol is not None:
        o.sur_tol = float(sur_tol)
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

    def matvec_noalloc(self, x, y):
        self._check(lib().fl_matvec_noalloc(self.h, _ptr(x), _ptr(y)))

    def mass_matvec(self, x, y):
        self._check(lib().fl_mass_matvec(self.h, _ptr(x), _ptr(y)))

    def mg_setup(self, nv, parents):
        """nv: vertex counts of the nested levels (coarsest first, the last
        = this mesh); parents: the (nv[l] x 2) parent arrays of levels 1.."""
        import numpy as np
        nv = np.ascontiguousarray(nv, dtype=np.int64)
        par = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.int32).reshape(-1)
                                                   for p in parents]), dtype=np.int32)
        self._check(lib().fl_mg_setup(self.h, len(nv), nv.ctypes.data_as(C.c_void_p),
                                      par.ctypes.data_as(C.c_void_p)))

    def solve_mg(self, b, u, rtol=1e-12, maxit=1000):
        it = C.c_int32()
        rel = C.c_double()
        rc = self._check(lib().fl_solve_mg(self.h, _ptr(b), _ptr(u), rtol, maxit, C.byref(it), C.byref(rel)),
                         allow=(FL_OK, FL_ENOCONV))
        return it.value, rel.value, rc

    def eval_points(self, k_eval, x, w):
        """Evaluation points (nc x Q x d) and weights (nc x Q) into device x, w."""
        self._check(lib().fl_eval_points(self.h, k_eval, _ptr(x), _ptr(w)))

    def strong_form(self, s, u, Lu, k_eval=2, q_far=2, q_near=12):
        """(-Delta)^s u_h at the evaluation points into device Lu (nc x Q)."""
        self._check(lib().fl_strong_form(self.h, s, _ptr(u), k_eval, q_far, q_near, _ptr(Lu)))

    def strong_form_cluster(self, s, u, Lu, k_eval=2, q_far=2, q_near=12, m=6, eta=2.0, leaf=16):
        """fl_strong_form with the all-pairs part by the cluster method."""
        self._check(lib().fl_strong_form_cluster(self.h, s, _ptr(u), k_eval, q_far, q_near, m, eta, leaf, _ptr(Lu)))

    def indicators(self, s, Lu, eta_cell, eta_node=None, f=None, k_eval=2):
        """eta_K^2 into eta_cell (nc), their vertex sums into eta_node (nv)."""
        self._check(lib().fl_indicators(self.h, s, _ptr(Lu), None if f is None else _ptr(f), k_eval,
                                        _ptr(eta_cell), None if eta_node is None else _ptr(eta_node)))

    def set_symmetry(self, order, ncells_sector, vfold, pre=None, rot=None):
        """Symmetry reduction: sector cells first in the mesh, vfold the
        representative of every vertex, optionally every cell's preimage and
        rotation index; order 1 with 0 cells switches it off."""
        import numpy as np
        vf = np.ascontiguousarray(vfold, dtype=np.int32)
        pr = None if pre is None else np.ascontiguousarray(pre, dtype=np.int32)
        ro = None if rot is None else np.ascontiguousarray(rot, dtype=np.int32)
        self._check(lib().fl_set_symmetry(self.h, order, ncells_sector, vf.ctypes.data_as(C.c_void_p),
                                          None if pr is None else pr.ctypes.data_as(C.c_void_p),
                                          None if ro is None else ro.ctypes.data_as(C.c_void_p)))

    def cluster_build(self, m=6, eta=2.0, leaf=32):
        """Cluster approximation of the assembled matrix (order m, admissibility eta)."""
        self._check(lib().fl_cluster_build(self.h, m, eta, leaf))

    def cluster_assemble(self, s: float, opts: FlOpts | None = None, m=6, eta=2.0, leaf=32) -> int:
        """Cluster approximation assembled from the mesh, without the dense
        matrix (near field from the pair kernels); returns n."""
        n = C.c_int64()
        self._check(lib().fl_cluster_assemble(self.h, s, None if opts is None else C.byref(opts), m, eta, leaf,
                                              C.byref(n)))
        self.n = n.value
        return self.n

    def cluster_matvec(self, x, y):
        self._check(lib().fl_cluster_matvec(self.h, _ptr(x), _ptr(y)))

    def solve_cluster(self, b, u, rtol=1e-12, maxit=100000):
        it = C.c_int32()
        rel = C.c_double()
        rc = self._check(lib().fl_solve_cluster(self.h, _ptr(b), _ptr(u), rtol, maxit, C.byref(it), C.byref(rel)),
                         allow=(FL_OK, FL_ENOCONV))
        return it.value, rel.value, rc

    def solve_cluster_mg(self, b, u, rtol=1e-12, maxit=1000):
        """CG on the cluster approximation, preconditioned by one V-cycle whose
        finest level smooths with the cluster product."""
        it = C.c_int32()
        rel = C.c_double()
        rc = self._check(lib().fl_solve_cluster_mg(self.h, _ptr(b), _ptr(u), rtol, maxit, C.byref(it),
                                                   C.byref(rel)), allow=(FL_OK, FL_ENOCONV))
        return it.value, rel.value, rc

    def cluster_info(self) -> dict:
        import numpy as np
        out = np.zeros(7, dtype=np.int64)
        self._check(lib().fl_cluster_info(self.h, out.ctypes.data_as(C.c_void_p)))
        keys = ("clusters", "leaves", "far_pairs", "near_pairs", "near_entries", "bytes", "depth")
        return {k: int(v) for k, v in zip(keys, out)}

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

    def import_matrix(self, A):
        """A: host numpy (n x n) or device torch tensor (n x n, row stride)."""
        if isinstance(A, np.ndarray):
            a = np.ascontiguousarray(A, dtype=np.float64)
            self._check(lib().fl_import_matrix(self.h, a.ctypes.data_as(C.c_void_p), a.shape[1], 0))
        else:
            self._check(lib().fl_import_matrix(self.h, _ptr(A), A.stride(0), 1))

    # ---- many right-hand sides / several s ----
    def load_vector(self, kind, b, coeffs=None):
        """b: device tensor (nrhs, n) float64 (= column-major n x nrhs).
        kind: "one" | "fourier16" (coeffs (nrhs, 16)) | "nodal" (coeffs (nrhs, nv))."""
        k = {"one": FL_RHS_ONE, "fourier16": FL_RHS_FOURIER16, "nodal": FL_RHS_P1_NODAL}.get(kind, kind)
        nrhs = b.shape[0] if b.dim() == 2 else 1
        cp = None
        if coeffs is not None:
            c = np.ascontiguousarray(coeffs, dtype=np.float64)
            cp = c.ctypes.data_as(C.c_void_p)
        self._check(lib().fl_load_vector(self.h, k, cp, nrhs, _ptr(b)))

    def assemble_batch(self, svals, opts: FlOpts | None = None) -> int:
        sv = np.ascontiguousarray(svals, dtype=np.float64)
        n = C.c_int64()
        self._check(lib().fl_assemble_batch(self.h, sv.ctypes.data_as(C.c_void_p), sv.size,
                                            None if opts is None else C.byref(opts), C.byref(n)))
        self.n = n.value
        self.ns = sv.size
        return self.n

    def export_batch_matrix(self, j) -> np.ndarray:
        out = np.zeros((self.n, self.n), dtype=np.float64)
        self._check(lib().fl_export_batch_matrix(self.h, j, out.ctypes.data_as(C.c_void_p), self.n, 0))
        return out

    def matmul(self, X, Y, dtype="f64", s_index=-1):
        """X, Y: device tensors (ns, nrhs, n) for s_index = -1, else (nrhs, n)
        (each row a column of the column-major operand)."""
        dt = DTYPES.get(dtype, dtype)
        nrhs = X.shape[-2]
        self._check(lib().fl_matmul(self.h, s_index, dt, _ptr(X), X.stride(-2), _ptr(Y), Y.stride(-2), nrhs))

    def solve_batch(self, Bt, U, rtol=1e-12, maxit=20000, inner="f64"):
        """Bt: device (ns, nrhs, n) or (nrhs, n) shared by every s; U: (ns, nrhs, n).
        Returns (iters (ns, nrhs), relres (ns, nrhs), rc)."""
        ns, nrhs = U.shape[0], U.shape[1]
        sb = Bt.stride(0) if Bt.dim() == 3 else 0
        it = np.zeros(ns * nrhs, dtype=np.int32)
        rel = np.zeros(ns * nrhs, dtype=np.float64)
        rc = self._check(lib().fl_solve_batch(self.h, _ptr(Bt), Bt.stride(-2), sb, _ptr(U), U.stride(-2),
                                              U.stride(0), nrhs, rtol, maxit, DTYPES.get(inner, inner),
                                              it.ctypes.data_as(C.c_void_p), rel.ctypes.data_as(C.c_void_p)),
                         allow=(FL_OK, FL_ENOCONV))
        return it.reshape(ns, nrhs), rel.reshape(ns, nrhs), rc

    def autotune(self, dtype="f64"):
        out = (FlTuneEntry * 64)()
        cnt, best = C.c_int(), C.c_int()
        self._check(lib().fl_autotune(self.h, DTYPES.get(dtype, dtype), out, 64, C.byref(cnt), C.byref(best)))
        rows = [dict(wm=e.wm, waves=e.waves, bk=e.bk, planes=e.planes, ms=e.ms, tflops=e.tflops, gbps=e.gbps)
                for e in out[:cnt.value]]
        return rows, best.value

    # ---- learned pair-integral surrogate ----
    def pair_integrals(self, X, Y, s, k, out):
        """X, Y: device (m, 6) float64; s: device (m,); out: device (m, 21)."""
        self._check(lib().fl_pair_integrals(self.h, X.shape[0], _ptr(X), _ptr(Y), _ptr(s), k, _ptr(out)))

    def surrogate_dataset(self, X, Y, s, feats, targets, k_exact=8):
        self._check(lib().fl_surrogate_dataset(self.h, X.shape[0], _ptr(X), _ptr(Y), _ptr(s), k_exact,
                                               _ptr(feats), _ptr(targets)))

    def surrogate_init(self, seed=1):
        self._check(lib().fl_surrogate_init(self.h, seed))

    def surrogate_fit_scaling(self, feats, targets):
        self._check(lib().fl_surrogate_fit_scaling(self.h, _ptr(feats), _ptr(targets), feats.shape[0]))

    def surrogate_set_params(self, blob):
        b = np.ascontiguousarray(blob, dtype=np.float64)
        if b.size != SUR_BLOB:
            raise ValueError("blob must hold %d doubles" % SUR_BLOB)
        self._check(lib().fl_surrogate_set_params(self.h, b.ctypes.data_as(C.c_void_p)))

    def surrogate_get_params(self) -> np.ndarray:
        b = np.zeros(SUR_BLOB)
        self._check(lib().fl_surrogate_get_params(self.h, b.ctypes.data_as(C.c_void_p)))
        return b

    def surrogate_grad(self, feats, targets):
        g = np.zeros(SUR_NPARAM, dtype=np.float32)
        L = C.c_double()
        self._check(lib().fl_surrogate_grad(self.h, _ptr(feats), _ptr(targets), feats.shape[0],
                                            g.ctypes.data_as(C.c_void_p), C.byref(L)))
        return L.value, g

    def surrogate_train(self, feats, targets, opts: FlTrainOpts | None = None):
        o = opts if opts is not None else default_train_opts()
        hist = np.zeros(max(o.steps, 1))
        self._check(lib().fl_surrogate_train(self.h, _ptr(feats), _ptr(targets), feats.shape[0], C.byref(o),
                                             hist.ctypes.data_as(C.c_void_p)))
        return hist[:o.steps]

    def surrogate_predict(self, feats, out):
        self._check(lib().fl_surrogate_predict(self.h, _ptr(feats), feats.shape[0], _ptr(out)))

    def surrogate_certify(self, feats, targets) -> np.ndarray:
        b = np.zeros(SUR_NRB * SUR_NSB)
        self._check(lib().fl_surrogate_certify(self.h, _ptr(feats), _ptr(targets), feats.shape[0],
                                               b.ctypes.data_as(C.c_void_p)))
        return b.reshape(SUR_NRB, SUR_NSB)


def _device_view(torch, ptr, n, ld, device):
    """Wrap a library-owned device pointer as a strided torch tensor without
    copying (DLPack-free: via a typed-storage-less from_blob equivalent)."""
    class _Cai:
        __cuda_array_interface__ = {
            "shape": (n, n), "typestr": "<f8", "data": (ptr, False),
            "strides": (ld * 8, 8), "version": 2}
    return torch.as_tensor(_Cai(), device=f"cuda:{device}")
