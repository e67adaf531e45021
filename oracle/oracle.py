"""Plain FP64 CPU oracle for the dense fractional-Laplacian stiffness matrix.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It shares
no code with the HIP path: quadrature nodes come from numpy / scipy library
routines, the pair integrals live in ``fl_oracle.c`` (compiled with gcc),
and the DOF map, normals, solves and closed forms below are written from
the paper.

References are to Ainsworth & Glusa, arXiv:1708.03912:
  * Sec. 2   -- operator, C(d,s), variational form with the boundary term
               (inward normal).
  * Sec. 3   -- P1 space, DOF rule (all nodes if s < 1/2, interior nodes
               otherwise), stiffness matrix A^s.
  * Sec. 5   -- element-pair decomposition, Gauss-type quadrature with
               regularised touching pairs, Jacobi-preconditioned CG.
  * Sec. 5   -- implicit steps of the fractional heat equation,
               (M + dt A^s) u = b with the P1 mass matrix M.
  * Sec. 7   -- closed-form solutions on the unit ball, energy-error
               identity ||u-u_h||^2 = (f,u) - (f,u_h).
  * App. B   -- per-pair quadrature orders decreasing with dist/h.

Parity status: every function here is pinned by ``tests/test_oracle_pins.py``
(closed forms, the exact 1D Toeplitz matrix, self-similarity of the
singular integrals under subdivision, boundary-term closed forms, limits
s -> 0 and s -> 1, invariances, convergence rates).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg
import scipy.special

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fl_oracle.c")
_LIB = os.path.join(_HERE, "libfl_oracle.so")
MAXK = 32


_LIB_SAN = os.path.join(_HERE, "libfl_oracle_san.so")
_CFLAGS = ["-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-D_DEFAULT_SOURCE",
           "-shared", "-fPIC"]


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile the C oracle with gcc (FP64, no fast-math, no contraction).
    ``sanitize``: a separate AddressSanitizer + UndefinedBehaviorSanitizer
    build (libfl_oracle_san.so, loaded when FL_ORACLE_SANITIZED=1; the
    process must preload libasan)."""
    out = _LIB_SAN if sanitize else _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        opt = (["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                "-fno-sanitize-recover=undefined"] if sanitize else ["-O3"])
        subprocess.check_call(["gcc"] + opt + _CFLAGS + [_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        san = os.environ.get("FL_ORACLE_SANITIZED") == "1"
        path = build(sanitize=san)
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.orc_cdn.restype = C.c_double
        L.orc_cdn.argtypes = [C.c_int, C.c_double]
        L.orc_pcg.restype = C.c_int
        _lib = L
    return _lib


# ----------------------------------------------------------------- rules --

class _Rules(C.Structure):
    _fields_ = [("gl_x", C.POINTER(C.c_double)), ("gl_w", C.POINTER(C.c_double)),
                ("gj_x", C.POINTER(C.c_double)), ("gj_w", C.POINTER(C.c_double)),
                ("r0_x", C.c_double * 2), ("r0_w", C.c_double * 2),
                ("r1_x", C.c_double * 2), ("r1_w", C.c_double * 2)]


def gauss_legendre01(k: int):
    """k-point Gauss-Legendre rule on [0,1] (numpy.polynomial.legendre)."""
    x, w = np.polynomial.legendre.leggauss(k)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_jacobi01(k: int, a: float, b: float):
    """k-point rule for int_0^1 (1-u)^a u^b f(u) du (scipy roots_jacobi)."""
    x, w = scipy.special.roots_jacobi(k, a, b)
    return 0.5 * (x + 1.0), w * 0.5 ** (a + b + 1.0)


_rule_cache: dict = {}


def rules(s: float):
    key = float(s)
    if key in _rule_cache:
        return _rule_cache[key]
    n = MAXK * (MAXK + 1) // 2
    glx, glw, gjx, gjw = (np.zeros(n) for _ in range(4))
    for k in range(1, MAXK + 1):
        o = k * (k - 1) // 2
        glx[o:o + k], glw[o:o + k] = gauss_legendre01(k)
        gjx[o:o + k], gjw[o:o + k] = gauss_jacobi01(k, 1.0, 0.0)
    R = _Rules()
    dp = C.POINTER(C.c_double)
    R.gl_x, R.gl_w = glx.ctypes.data_as(dp), glw.ctypes.data_as(dp)
    R.gj_x, R.gj_w = gjx.ctypes.data_as(dp), gjw.ctypes.data_as(dp)
    if s < 0.5:
        x0, w0 = gauss_jacobi01(2, 0.0, -2.0 * s)
    else:
        x0, w0 = np.full(2, np.nan), np.full(2, np.nan)
    x1, w1 = gauss_jacobi01(2, 0.0, 1.0 - 2.0 * s)
    for i in range(2):
        R.r0_x[i], R.r0_w[i] = x0[i], w0[i]
        R.r1_x[i], R.r1_w[i] = x1[i], w1[i]
    _rule_cache[key] = (R, (glx, glw, gjx, gjw))  # keep arrays alive
    return _rule_cache[key]


def _rp(s):
    return C.byref(rules(s)[0])


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# -------------------------------------------------------- pair integrals --
# Raw integrals (no C(d,s) factor); see fl_oracle.c for the derivations.

def far_pair(s, k, X, Y):
    X = np.ascontiguousarray(X, dtype=np.float64).ravel()
    Y = np.ascontiguousarray(Y, dtype=np.float64).ravel()
    dim = 1 if X.size == 2 else 2
    m = dim + 1
    SK, ST, O = np.zeros(m * m), np.zeros(m * m), np.zeros(m * m)
    f = lib().orc_far1 if dim == 1 else lib().orc_far2
    f(_rp(s), C.c_double(s), C.c_int(k), _dp(X), _dp(Y), _dp(SK), _dp(ST), _dp(O))
    return SK.reshape(m, m), ST.reshape(m, m), O.reshape(m, m)


def far_pair_full(s, k, X, Y):
    """Separated pair as a (2m x 2m) matrix over the union basis
    (K's vertices then Kt's)."""
    SK, ST, O = far_pair(s, k, X, Y)
    return np.block([[SK, O], [O.T, ST]])


def ident(s, k, X):
    X = np.ascontiguousarray(X, dtype=np.float64).ravel()
    if X.size == 2:
        I = np.zeros(4)
        lib().orc_ident1(C.c_double(s), _dp(X), _dp(I))
        return I.reshape(2, 2)
    I = np.zeros(9)
    lib().orc_ident2(_rp(s), C.c_double(s), C.c_int(k), _dp(X), _dp(I))
    return I.reshape(3, 3)


def vert1(s, k, xl, xq, xr):
    I = np.zeros(9)
    lib().orc_vert1(_rp(s), C.c_double(s), C.c_int(k), C.c_double(xl), C.c_double(xq),
                    C.c_double(xr), _dp(I))
    return I.reshape(3, 3)


def edge2(s, k, q0, q1, a, b):
    pts = [np.ascontiguousarray(p, dtype=np.float64) for p in (q0, q1, a, b)]
    I = np.zeros(16)
    lib().orc_edge2(_rp(s), C.c_double(s), C.c_int(k), *[_dp(p) for p in pts], _dp(I))
    return I.reshape(4, 4)


def vert2(s, k, q, b1, b2, c1, c2):
    pts = [np.ascontiguousarray(p, dtype=np.float64) for p in (q, b1, b2, c1, c2)]
    I = np.zeros(25)
    lib().orc_vert2(_rp(s), C.c_double(s), C.c_int(k), *[_dp(p) for p in pts], _dp(I))
    return I.reshape(5, 5)


def bnd_far2(s, k, X, p0, p1, n):
    X = np.ascontiguousarray(X, dtype=np.float64).ravel()
    pts = [np.ascontiguousarray(p, dtype=np.float64) for p in (p0, p1, n)]
    I = np.zeros(9)
    lib().orc_bndfar2(_rp(s), C.c_double(s), C.c_int(k), _dp(X), *[_dp(p) for p in pts], _dp(I))
    return I.reshape(3, 3)


def bnd_edge2(s, k, p0, p1, a, n):
    pts = [np.ascontiguousarray(p, dtype=np.float64) for p in (p0, p1, a, n)]
    I = np.zeros(9)
    lib().orc_bndedge2(_rp(s), C.c_double(s), C.c_int(k), *[_dp(p) for p in pts], _dp(I))
    return I.reshape(3, 3)


def bnd_vert2(s, k, q, b1, b2, p, n):
    pts = [np.ascontiguousarray(v, dtype=np.float64) for v in (q, b1, b2, p, n)]
    I = np.zeros(9)
    lib().orc_bndvert2(_rp(s), C.c_double(s), C.c_int(k), *[_dp(v) for v in pts], _dp(I))
    return I.reshape(3, 3)


def bnd1(s, k, X, ye, touching):
    X = np.ascontiguousarray(X, dtype=np.float64).ravel()
    I = np.zeros(4)
    lib().orc_bnd1(_rp(s), C.c_double(s), C.c_int(k), _dp(X), C.c_double(ye), C.c_int(touching),
                   _dp(I))
    return I.reshape(2, 2)


# --------------------------------------------------------- problem data --

def cdn(d: int, s: float) -> float:
    """C(d,s) = 2^{2s} s Gamma(s+d/2) / (pi^{d/2} Gamma(1-s))  (Sec. 2)."""
    return 2.0 ** (2 * s) * s * math.gamma(s + d / 2) / (math.pi ** (d / 2) * math.gamma(1 - s))


@dataclass
class Orders:
    """Quadrature orders (App. B).  Separated pairs are binned by the ratio
    r = |c_K - c_Kt| / max(h_K, h_Kt) (centroid distance over the larger
    longest edge) against the increasing thresholds ``theta``; class m gets
    ``k_far[m]`` (element pairs) / ``k_far_bnd[m]`` (element-facet pairs)."""
    k_touch: int = 8
    k_touch_bnd: int = 8
    theta: list = field(default_factory=lambda: [1.5, 3.0, 6.0])
    k_far: list = field(default_factory=lambda: [5, 4, 3, 2])
    k_far_bnd: list = field(default_factory=lambda: [5, 4, 3, 2])

    def check(self):
        assert len(self.k_far) == len(self.theta) + 1 == len(self.k_far_bnd)
        assert all(1 <= k <= MAXK for k in self.k_far + self.k_far_bnd + [self.k_touch, self.k_touch_bnd])
        assert all(a < b for a, b in zip(self.theta, self.theta[1:]))


class _Opts(C.Structure):
    _fields_ = [("s", C.c_double), ("k_touch", C.c_int), ("k_touch_bnd", C.c_int),
                ("ncls", C.c_int), ("theta", C.POINTER(C.c_double)),
                ("k_far", C.POINTER(C.c_int)), ("k_far_bnd", C.POINTER(C.c_int)),
                ("with_boundary", C.c_int), ("which", C.c_int), ("far_skip_below", C.c_int),
                ("cell_w", C.POINTER(C.c_double)), ("cell_pre", C.POINTER(C.c_int)),
                ("cell_rot", C.POINTER(C.c_int)), ("sym_order", C.c_int),
                ("cell_leaf", C.POINTER(C.c_int)), ("nleaf", C.c_int), ("leaf_near", C.POINTER(C.c_ubyte))]


def boundary_normals(dim, verts, cells, bfacets):
    """Inward unit normal of each boundary facet: it points from the facet
    into the (unique) cell that owns it (Sec. 2: n_y is the inward normal)."""
    verts = np.asarray(verts, dtype=np.float64).reshape(-1, dim)
    cells = np.asarray(cells).reshape(-1, dim + 1)
    bf = np.asarray(bfacets).reshape(-1, dim)
    owner = {}
    for K, c in enumerate(cells):
        for a in range(dim + 1):
            face = tuple(sorted(int(c[b]) for b in range(dim + 1) if b != a))
            owner.setdefault(face, []).append((K, int(c[a])))
    out = np.zeros((len(bf), dim))
    for e, f in enumerate(bf):
        own = owner[tuple(sorted(int(v) for v in f))]
        assert len(own) == 1, "boundary facet must lie on exactly one cell"
        opp = verts[own[0][1]]
        if dim == 1:
            out[e, 0] = 1.0 if opp[0] > verts[f[0], 0] else -1.0
        else:
            p0, p1 = verts[f[0]], verts[f[1]]
            t = p1 - p0
            nn = np.array([-t[1], t[0]]) / np.hypot(t[0], t[1])
            if np.dot(opp - p0, nn) < 0:
                nn = -nn
            out[e] = nn
    return out


def dof_nodes(nv, bfacets, s, mode="paper"):
    """Sec. 3: I_h = all nodes if s < 1/2, interior nodes if s >= 1/2
    (mode 'paper'); mode 'interior' always drops boundary nodes."""
    on_b = np.zeros(nv, dtype=bool)
    on_b[np.asarray(bfacets).ravel()] = True
    if mode == "paper" and s < 0.5:
        return np.arange(nv)
    return np.nonzero(~on_b)[0]


def assemble_full(mesh, s, orders: Orders, rows=None, which=7, with_boundary=True, threads=None,
                  far_skip_below=0, compact=False, cell_w=None, cell_pre=None, cell_rot=None, sym_order=0,
                  cell_leaf=None, leaf_near=None):
    """Full-node matrix (nv x nv) of a(phi_i, phi_j) by the element-pair
    decomposition of Sec. 5.  ``rows``: optional vertex indices; only those
    rows are accumulated (others stay zero); with ``compact`` the result is
    just those rows (len(rows) x nv, in the order given).
    ``far_skip_below``: separated pairs of a lower order class are left out
    (still counted).  ``cell_w``: optional weight per cell, a pair counting
    with the mean of its two cells' weights (the symmetry reduction of
    Sec. 7: 1 on the sector, 0 on its images); with ``cell_pre`` /
    ``cell_rot`` (preimage sector cell and rotation index of every cell) and
    ``sym_order`` only one of each equal couple of cross pairs counts, with
    weight 1 (see pair_weight in fl_oracle.c).  ``cell_leaf`` (a label per
    cell, 0..L-1) with ``leaf_near`` (L x L, 0/1): a separated pair adds its
    diagonal-block parts only where leaf_near[label K, label Kt] is 1 (the
    near-field self terms of the cluster method); its off-diagonal block
    always.  Returns (A, class_counts)."""
    orders.check()
    dim = mesh["dim"]
    verts = np.ascontiguousarray(mesh["verts"], dtype=np.float64).reshape(-1)
    cells = np.ascontiguousarray(mesh["cells"], dtype=np.int32).reshape(-1)
    bf = np.ascontiguousarray(mesh["bfacets"], dtype=np.int32).reshape(-1)
    nv = verts.size // dim
    nc = cells.size // (dim + 1)
    nb = bf.size // dim
    normals = np.ascontiguousarray(boundary_normals(dim, verts, cells, bf), dtype=np.float64).reshape(-1)
    mask = None
    if rows is not None:
        rows = np.asarray(rows, dtype=np.int64)
        mask = np.full(nv, -1, dtype=np.int32)
        mask[rows] = np.arange(len(rows)) if compact else rows
    A = np.zeros((len(rows) if (compact and rows is not None) else nv, nv))
    th = np.ascontiguousarray(orders.theta, dtype=np.float64)
    kf = np.ascontiguousarray(orders.k_far, dtype=np.int32)
    kb = np.ascontiguousarray(orders.k_far_bnd, dtype=np.int32)
    cw = None if cell_w is None else np.ascontiguousarray(cell_w, dtype=np.float64)
    cpre = None if cell_pre is None else np.ascontiguousarray(cell_pre, dtype=np.int32)
    crot = None if cell_rot is None else np.ascontiguousarray(cell_rot, dtype=np.int32)
    cl = None if cell_leaf is None else np.ascontiguousarray(cell_leaf, dtype=np.int32)
    ln = None if leaf_near is None else np.ascontiguousarray(leaf_near, dtype=np.uint8)
    if cl is not None:
        assert ln is not None and ln.ndim == 2 and ln.shape[0] == ln.shape[1] and len(cl) == nc
        assert cl.min() >= 0 and cl.max() < ln.shape[0]
    o = _Opts(s, orders.k_touch, orders.k_touch_bnd, len(orders.theta), _dp(th),
              kf.ctypes.data_as(C.POINTER(C.c_int)), kb.ctypes.data_as(C.POINTER(C.c_int)),
              1 if with_boundary else 0, which, int(far_skip_below),
              None if cw is None else _dp(cw),
              None if cpre is None else cpre.ctypes.data_as(C.POINTER(C.c_int)),
              None if crot is None else crot.ctypes.data_as(C.POINTER(C.c_int)), int(sym_order),
              None if cl is None else cl.ctypes.data_as(C.POINTER(C.c_int)), 0 if ln is None else ln.shape[0],
              None if ln is None else ln.ctypes.data_as(C.POINTER(C.c_ubyte)))
    cnt = np.zeros(16, dtype=np.int64)
    if threads is not None:
        os.environ["OMP_NUM_THREADS"] = str(threads)
    lib().orc_assemble(_rp(s), C.byref(o), C.c_int(dim), C.c_int64(nv), _dp(verts), C.c_int64(nc),
                       cells.ctypes.data_as(C.c_void_p), C.c_int64(nb), bf.ctypes.data_as(C.c_void_p),
                       _dp(normals), None if mask is None else mask.ctypes.data_as(C.c_void_p),
                       _dp(A), cnt.ctypes.data_as(C.c_void_p))
    return A, cnt[:len(orders.theta) + 1]


def assemble(mesh, s, orders: Orders, mode="paper", **kw):
    """Stiffness matrix A^s on the DOF set (canonical increasing vertex
    order) and the DOF node list."""
    nv = np.asarray(mesh["verts"]).size // mesh["dim"]
    dofs = dof_nodes(nv, mesh["bfacets"], s, mode)
    A, cnt = assemble_full(mesh, s, orders, **kw)
    return A[np.ix_(dofs, dofs)].copy(), dofs, cnt


def load_vector_one(mesh, dofs):
    """b_i = int phi_i for f = 1: sum over cells containing i of |K|/(d+1)."""
    dim = mesh["dim"]
    verts = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1, dim)
    cells = np.asarray(mesh["cells"]).reshape(-1, dim + 1)
    if dim == 1:
        meas = np.abs(verts[cells[:, 1], 0] - verts[cells[:, 0], 0])
    else:
        a, b, c = verts[cells[:, 0]], verts[cells[:, 1]], verts[cells[:, 2]]
        meas = 0.5 * np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1]))
    full = np.zeros(verts.shape[0])
    for j in range(dim + 1):
        np.add.at(full, cells[:, j], meas / (dim + 1))
    return full[dofs]


def mass_matrix(mesh, dofs):
    """P1 mass matrix M_ij = int phi_i phi_j on the DOF set (Sec. 5: the
    fractional heat equation's implicit step solves (M + dt A^s) u = b).
    On each cell the integral of lambda_a lambda_b is |K| (1 + delta_ab) /
    ((d+1)(d+2))."""
    dim = mesh["dim"]
    verts = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1, dim)
    cells = np.asarray(mesh["cells"]).reshape(-1, dim + 1)
    if dim == 1:
        meas = np.abs(verts[cells[:, 1], 0] - verts[cells[:, 0], 0])
    else:
        a, b, c = verts[cells[:, 0]], verts[cells[:, 1]], verts[cells[:, 2]]
        meas = 0.5 * np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1]))
    nv = verts.shape[0]
    full = np.zeros((nv, nv))
    den = (dim + 1) * (dim + 2)
    for i in range(dim + 1):
        for j in range(dim + 1):
            np.add.at(full, (cells[:, i], cells[:, j]), meas * (2.0 if i == j else 1.0) / den)
    return full[np.ix_(dofs, dofs)].copy()


def load_vector_fn(mesh, dofs, f, k=4):
    """b_i = int f phi_i with the order-k collapsed triangle rule (2D) /
    k-point Gauss-Legendre (1D) on every cell."""
    dim = mesh["dim"]
    verts = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1, dim)
    cells = np.asarray(mesh["cells"]).reshape(-1, dim + 1)
    full = np.zeros(verts.shape[0])
    if dim == 1:
        t, w = gauss_legendre01(k)
        x0, x1 = verts[cells[:, 0], 0], verts[cells[:, 1], 0]
        h = np.abs(x1 - x0)
        for ti, wi in zip(t, w):
            x = x0 + ti * (x1 - x0)
            fv = f(x[:, None]) * h * wi
            np.add.at(full, cells[:, 0], fv * (1 - ti))
            np.add.at(full, cells[:, 1], fv * ti)
        return full[dofs]
    ux, uw = gauss_jacobi01(k, 1.0, 0.0)
    vx, vw = gauss_legendre01(k)
    a, b, c = verts[cells[:, 0]], verts[cells[:, 1]], verts[cells[:, 2]]
    area = 0.5 * np.abs((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1]))
    for i in range(k):
        for j in range(k):
            l1, l2 = ux[i], (1 - ux[i]) * vx[j]
            wt = 2 * uw[i] * vw[j]
            x = (1 - l1 - l2) * a + l1 * b + l2 * c
            fv = f(x) * area * wt
            np.add.at(full, cells[:, 0], fv * (1 - l1 - l2))
            np.add.at(full, cells[:, 1], fv * l1)
            np.add.at(full, cells[:, 2], fv * l2)
    return full[dofs]


# ----------------------------------------------------------------- solve --

def solve_cholesky(A, b):
    c = scipy.linalg.cho_factor(A)
    return scipy.linalg.cho_solve(c, b)


def pcg(A, b, rtol=1e-12, maxit=100000):
    """Jacobi-PCG (Sec. 5), x0 = 0, stop at ||r|| <= rtol ||b||."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    rel = C.c_double(0)
    it = lib().orc_pcg(C.c_int64(b.size), _dp(A), _dp(b), _dp(x), C.c_double(rtol), C.c_int(maxit),
                       C.byref(rel))
    return x, it, rel.value


def matvec(A, x):
    A = np.ascontiguousarray(A, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(A.shape[0])
    lib().orc_matvec(C.c_int64(x.size), _dp(A), _dp(x), _dp(y))
    return y


# ---------------------------------------------------------- closed forms --

def ball_constant(d, s):
    """u = c (1-|x|^2)_+^s solves (-Delta)^s u = 1 on the unit ball,
    c = 2^{-2s} Gamma(d/2) / (Gamma(d/2+s) Gamma(1+s)) (Sec. 7 with n = l = 0;
    for d = 2 this is the Sec. 3 example divided by 2^{2s} Gamma(1+s)^2)."""
    return 2.0 ** (-2 * s) * math.gamma(d / 2) / (math.gamma(d / 2 + s) * math.gamma(1 + s))


def ball_fu(d, s):
    """(f,u) for f = 1 on the unit ball: c |S^{d-1}| int_0^1 (1-r^2)^s r^{d-1} dr."""
    c = ball_constant(d, s)
    if d == 1:
        return c * scipy.special.beta(0.5, s + 1.0)
    return c * math.pi / (s + 1.0)


def energy_error(fu, b, uh, A):
    """e^2 = (f,u) - 2 b.u_h + u_h.A u_h; equals (f,u) - (f,u_h) at the
    Galerkin solution (Sec. 7 identity) and stays valid for any u_h."""
    e2 = fu - 2.0 * float(b @ uh) + float(uh @ (A @ uh))
    return math.sqrt(max(e2, 0.0)), e2
