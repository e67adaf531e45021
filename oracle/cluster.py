"""Cluster (H-matrix) approximation of the stiffness matrix, plain numpy
(test infrastructure only, like the rest of ``oracle/``).

Sec. 6 of arXiv:1708.03912: a hierarchical cluster tree over the DOFs,
cluster boxes (cubes containing the supports of their basis functions),
admissible pairs eta dist(s, t) >= max(diam s, diam t), whose block of A is
-C int int k phi_i phi_j (disjoint supports) and is replaced by the tensor
Chebyshev interpolation of k of order m on the two boxes:

  A[s, t] ~ -C V_s K_st V_t^T,  K_st[a, b] = k(xi_a^s, xi_b^t),
  V_s[i, a] = int phi_i L_a^s,

with nested bases V_parent = sum over sons of V_son T_son,
T_son[b, a] = L_a^parent(xi_b^son) (the shift coefficients).  The other
leaf pairs form the near field, kept exactly (here: taken from a dense
matrix).  The product runs upward (x_hat = V^T x), through the kernel
blocks, and downward.

Readings (the paper defers the details to the boundary-element
literature): leaves hold at most `leaf` DOFs (the paper's leaves are single
DOFs); a cluster is split at the median of its DOF coordinates along the
longest side of their bounding box; its box is the cube with the side of
the largest extent of the supports' bounding box, centred on it; the basis
coefficients use the m+1 point rule of each cell (exact for these
polynomials); Chebyshev points of the first kind.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import oracle as O


def cheb_nodes(m):
    """Chebyshev points of the first kind on [0, 1], increasing."""
    k = np.arange(m)
    return np.sort(0.5 - 0.5 * np.cos((2 * k + 1) * math.pi / (2 * m)))


def lagrange(nodes, x):
    """Lagrange polynomials of the nodes at the points x: (len(x), m)."""
    x = np.asarray(x, dtype=np.float64)
    m = len(nodes)
    L = np.ones((len(x), m))
    for a in range(m):
        for b in range(m):
            if b != a:
                L[:, a] *= (x - nodes[b]) / (nodes[a] - nodes[b])
    return L


@dataclass
class Cluster:
    lo: int                    # DOF range [lo, hi) in tree order
    hi: int
    box_lo: np.ndarray         # cube corner
    side: float
    level: int
    parent: int = -1
    sons: list = field(default_factory=list)


@dataclass
class Tree:
    perm: np.ndarray           # tree order -> DOF index
    clusters: list
    dim: int

    def leaves(self):
        return [c for c, cl in enumerate(self.clusters) if not cl.sons]


def _supports(mesh, dofs):
    """Bounding box of the support (union of the cells) of every DOF."""
    d = mesh["dim"]
    V = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1, d)
    C = np.asarray(mesh["cells"], dtype=np.int64)
    nv = len(V)
    lo = np.full((nv, d), np.inf)
    hi = np.full((nv, d), -np.inf)
    P = V[C]                                       # (T, d+1, d)
    clo, chi = P.min(1), P.max(1)
    for a in range(C.shape[1]):
        np.minimum.at(lo, C[:, a], clo)
        np.maximum.at(hi, C[:, a], chi)
    dofs = np.asarray(dofs)
    return V[dofs], lo[dofs], hi[dofs]


def build_tree(mesh, dofs, leaf=32):
    """Cluster tree by recursive median bisection of the DOF coordinates."""
    d = mesh["dim"]
    X, slo, shi = _supports(mesh, dofs)
    perm = np.arange(len(dofs))
    clusters = []

    def make(idx, lo, level, parent):
        blo = slo[idx].min(0)
        bhi = shi[idx].max(0)
        side = float((bhi - blo).max())
        cen = 0.5 * (blo + bhi)
        c = Cluster(lo, lo + len(idx), cen - 0.5 * side, side, level, parent)
        cid = len(clusters)
        clusters.append(c)
        perm[lo:lo + len(idx)] = idx
        if len(idx) > leaf:
            ext = X[idx].max(0) - X[idx].min(0)
            ax = int(np.argmax(ext))
            order = idx[np.argsort(X[idx, ax], kind="stable")]
            h = len(order) // 2
            for part, off in ((order[:h], 0), (order[h:], h)):
                sid = make(part, lo + off, level + 1, cid)
                c.sons.append(sid)
        return cid

    make(np.arange(len(dofs)), 0, 0, -1)
    return Tree(perm.copy(), clusters, d)


def box_dist(a: Cluster, b: Cluster):
    gap = np.maximum(0.0, np.maximum(b.box_lo - (a.box_lo + a.side), a.box_lo - (b.box_lo + b.side)))
    return float(np.sqrt((gap ** 2).sum()))


def diam(c: Cluster, dim):
    return c.side * math.sqrt(dim)


def admissible(a: Cluster, b: Cluster, eta, dim):
    return eta * box_dist(a, b) >= max(diam(a, dim), diam(b, dim))


def block_tree(tree: Tree, eta):
    """(far, near): admissible cluster pairs, and the leaf pairs that are
    not admissible (recursion from (root, root), splitting the non-leaf
    side(s))."""
    far, near = [], []
    cl = tree.clusters

    def rec(s, t):
        if admissible(cl[s], cl[t], eta, tree.dim):
            far.append((s, t))
            return
        ls, lt = not cl[s].sons, not cl[t].sons
        if ls and lt:
            near.append((s, t))
        elif ls:
            for tt in cl[t].sons:
                rec(s, tt)
        elif lt:
            for ss in cl[s].sons:
                rec(ss, t)
        else:
            for ss in cl[s].sons:
                for tt in cl[t].sons:
                    rec(ss, tt)

    rec(0, 0)
    return far, near


def cheb_points(c: Cluster, m, dim):
    """Tensor Chebyshev points of the box, (m^dim, dim), first coordinate
    slowest."""
    t = cheb_nodes(m)
    g = [c.box_lo[j] + c.side * t for j in range(dim)]
    if dim == 1:
        return g[0][:, None]
    return np.stack(np.meshgrid(g[0], g[1], indexing="ij"), -1).reshape(-1, 2)


def lagrange_box(c: Cluster, m, dim, x):
    """Tensor Lagrange basis of the box at the points x (p, dim): (p, m^dim)."""
    t = cheb_nodes(m)
    x = np.asarray(x, dtype=np.float64).reshape(-1, dim)
    L0 = lagrange(t, (x[:, 0] - c.box_lo[0]) / c.side)
    if dim == 1:
        return L0
    L1 = lagrange(t, (x[:, 1] - c.box_lo[1]) / c.side)
    return (L0[:, :, None] * L1[:, None, :]).reshape(len(x), -1)


def _cell_rule(mesh, k):
    """Points, barycentric coordinates and weights (times |K|) of the k-point
    rule on every cell (collapsed Gauss in 2D, Gauss-Legendre in 1D)."""
    d = mesh["dim"]
    V = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1, d)
    C = np.asarray(mesh["cells"], dtype=np.int64)
    if d == 1:
        t, w = O.gauss_legendre01(k)
        lam = np.stack([1 - t, t], 1)
        meas = np.abs(V[C[:, 1], 0] - V[C[:, 0], 0])
    else:
        ux, uw = O.gauss_jacobi01(k, 1.0, 0.0)
        vx, vw = O.gauss_legendre01(k)
        lam, w = [], []
        for i in range(k):
            for j in range(k):
                l1, l2 = ux[i], (1 - ux[i]) * vx[j]
                lam.append((1 - l1 - l2, l1, l2))
                w.append(2 * uw[i] * vw[j])
        lam, w = np.array(lam), np.array(w)
        P = V[C]
        meas = 0.5 * np.abs((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1])
                            - (P[:, 2, 0] - P[:, 0, 0]) * (P[:, 1, 1] - P[:, 0, 1]))
    X = np.einsum("qa,tad->tqd", lam, V[C])
    return X, lam, meas[:, None] * w[None, :]


def basis_coeffs(mesh, dofs, tree: Tree, c: int, m):
    """V_c[i, a] = int phi_i L_a^c over the support of phi_i, for the DOFs of
    cluster c (tree order), by the (m+1)-point rule on every cell."""
    d = mesh["dim"]
    C = np.asarray(mesh["cells"], dtype=np.int64)
    X, lam, W = _cell_rule(mesh, m + 1)
    cl = tree.clusters[c]
    nodes = np.asarray(dofs)[tree.perm[cl.lo:cl.hi]]
    out = np.zeros((len(nodes), m ** d))
    for r, v in enumerate(nodes):
        Ks, As = np.nonzero(C == v)
        for K, a in zip(Ks, As):
            L = lagrange_box(cl, m, d, X[K])
            out[r] += (W[K] * lam[:, a]) @ L
    return out


def transfer(tree: Tree, c: int, m):
    """T_c[b, a] = L_a^parent(xi_b^c)."""
    cl = tree.clusters[c]
    par = tree.clusters[cl.parent]
    return lagrange_box(par, m, tree.dim, cheb_points(cl, m, tree.dim))


def kernel_block(tree: Tree, s: int, t: int, m, sval):
    d = tree.dim
    Xs = cheb_points(tree.clusters[s], m, d)
    Xt = cheb_points(tree.clusters[t], m, d)
    r2 = ((Xs[:, None, :] - Xt[None, :, :]) ** 2).sum(-1)
    return r2 ** (-(d + 2 * sval) / 2)


@dataclass
class HMatrix:
    tree: Tree
    far: list
    near: list
    m: int
    s: float
    C: float
    Vleaf: dict                # leaf -> V (|leaf| x m^d)
    T: dict                    # cluster (non-root) -> transfer
    K: dict                    # (s, t) admissible -> kernel block
    Anear: dict                # (s, t) near -> dense block (tree order)


def build(mesh, dofs, A, s, m=6, eta=2.0, leaf=32):
    """The H-matrix of the dense matrix A (DOF order): near blocks copied
    from A, far blocks by interpolation."""
    tree = build_tree(mesh, dofs, leaf)
    far, near = block_tree(tree, eta)
    Vleaf = {c: basis_coeffs(mesh, dofs, tree, c, m) for c in tree.leaves()}
    T = {c: transfer(tree, c, m) for c in range(1, len(tree.clusters))}
    K = {(a, b): kernel_block(tree, a, b, m, s) for a, b in far}
    P = tree.perm
    cl = tree.clusters
    An = {(a, b): A[np.ix_(P[cl[a].lo:cl[a].hi], P[cl[b].lo:cl[b].hi])] for a, b in near}
    return HMatrix(tree, far, near, m, s, O.cdn(mesh["dim"], s), Vleaf, T, K, An)


def matvec(H: HMatrix, x):
    """y = A_near x - C sum_far V_s K_st V_t^T x, upward / far / downward."""
    tree, cl = H.tree, H.tree.clusters
    P = tree.perm
    xp = np.asarray(x, dtype=np.float64)[P]
    nc = len(cl)
    xh = [None] * nc
    order = sorted(range(nc), key=lambda c: -cl[c].level)   # leaves and deep levels first
    for c in order:
        if not cl[c].sons:
            xh[c] = H.Vleaf[c].T @ xp[cl[c].lo:cl[c].hi]
        else:
            xh[c] = sum(H.T[sn].T @ xh[sn] for sn in cl[c].sons)
    yh = [np.zeros(H.m ** tree.dim) for _ in range(nc)]
    for a, b in H.far:
        yh[a] = yh[a] + H.K[(a, b)] @ xh[b]
    yp = np.zeros(len(xp))
    for c in sorted(range(nc), key=lambda c: cl[c].level):  # root first
        for sn in cl[c].sons:
            yh[sn] = yh[sn] + H.T[sn] @ yh[c]
        if not cl[c].sons:
            yp[cl[c].lo:cl[c].hi] += -H.C * (H.Vleaf[c] @ yh[c])
    for a, b in H.near:
        yp[cl[a].lo:cl[a].hi] += H.Anear[(a, b)] @ xp[cl[b].lo:cl[b].hi]
    y = np.empty_like(yp)
    y[P] = yp
    return y


def dense(H: HMatrix, n):
    """The approximated matrix itself (DOF order), for checks."""
    Y = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        Y[:, j] = matvec(H, e)
    return Y
