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
matrix by ``build``, or assembled from the mesh by ``build_direct``).
The product runs upward (x_hat = V^T x), through the kernel blocks, and
downward.

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


def cell_anchors(mesh, dofs, perm):
    """Anchor DOF (index into ``dofs``) of every cell: among the cell's
    vertices that carry a DOF, the one first in tree order (``perm``: tree
    position -> DOF index).  A cell with no DOF vertex takes the anchor of
    its neighbour across a facet (2D: a common edge, 1D: a common vertex)
    of smallest cell index that has one; such passes repeat until no cell
    changes.  -1 where none is found (no DOF in the cell's component)."""
    d = mesh["dim"]
    C = np.asarray(mesh["cells"], dtype=np.int64)
    nv = np.asarray(mesh["verts"]).size // d
    T = len(C)
    node2dof = np.full(nv, -1, dtype=np.int64)
    node2dof[np.asarray(dofs)] = np.arange(len(dofs))
    pos = np.empty(len(dofs), dtype=np.int64)
    pos[np.asarray(perm)] = np.arange(len(dofs))
    anchor = np.full(T, -1, dtype=np.int64)
    for K in range(T):
        ds = [node2dof[v] for v in C[K] if node2dof[v] >= 0]
        if ds:
            anchor[K] = min(ds, key=lambda i: pos[i])
    if (anchor >= 0).all():
        return anchor
    nbr = [[] for _ in range(T)]
    owners = {}
    for K in range(T):
        for a in range(d + 1):
            face = tuple(sorted(int(C[K, b]) for b in range(d + 1) if b != a))
            owners.setdefault(face, []).append(K)
    for ks in owners.values():
        for K in ks:
            nbr[K].extend(k for k in ks if k != K)
    changed = True
    while changed:
        changed = False
        for K in range(T):
            if anchor[K] >= 0:
                continue
            cand = sorted(k for k in nbr[K] if anchor[k] >= 0)
            if cand:
                anchor[K] = anchor[cand[0]]
                changed = True
    return anchor


def build_tree(mesh, dofs, leaf=32):
    """Cluster tree by recursive median bisection of the DOF coordinates;
    then every cluster's box: the cube with the side of the largest extent
    of the supports' bounding box, centred on it.  A cell without a DOF
    vertex widens the support box of its anchor DOF (cell_anchors), so that
    every cell lies in the box of its anchor's clusters."""
    d = mesh["dim"]
    X, slo, shi = _supports(mesh, dofs)
    perm = np.arange(len(dofs))
    clusters = []

    def make(idx, lo, level, parent):
        c = Cluster(lo, lo + len(idx), np.zeros(d), 0.0, level, parent)
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

    if len(dofs):
        make(np.arange(len(dofs)), 0, 0, -1)
    anchor = cell_anchors(mesh, dofs, perm)
    V = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1, d)
    C = np.asarray(mesh["cells"], dtype=np.int64)
    nv = len(V)
    on_dof = np.zeros(nv, dtype=bool)
    on_dof[np.asarray(dofs, dtype=np.int64)] = True
    for K in np.nonzero(~on_dof[C].any(1) & (anchor >= 0))[0]:
        P = V[C[K]]
        i = anchor[K]
        slo[i] = np.minimum(slo[i], P.min(0))
        shi[i] = np.maximum(shi[i], P.max(0))
    for c in clusters:
        idx = perm[c.lo:c.hi]
        blo = slo[idx].min(0)
        bhi = shi[idx].max(0)
        c.side = float((bhi - blo).max())
        c.box_lo = 0.5 * (blo + bhi) - 0.5 * c.side
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


def leaf_labels(tree: Tree, near):
    """Leaf index of every leaf cluster (increasing cluster id), the leaf
    cluster of every tree position, and the near table (nleaf x nleaf, 0/1)
    of the leaf pairs that are not admissible."""
    leaves = tree.leaves()
    li = {c: i for i, c in enumerate(leaves)}
    rleaf = np.empty(len(tree.perm), dtype=np.int64)
    for c in leaves:
        rleaf[tree.clusters[c].lo:tree.clusters[c].hi] = c
    tab = np.zeros((len(leaves), len(leaves)), dtype=np.uint8)
    for a, b in near:
        tab[li[a], li[b]] = 1
    return leaves, li, rleaf, tab


def self_far(mesh, tree: Tree, far, T_shift, m, sval, cell_leafc):
    """Far part of the cells' diagonal blocks.  For x in a cell K, the sum
    over the separated cells Kt whose anchor leaf is not near K's of
    int_Kt k(x, y) dy is the far field of the density 1 on those cells:
    with the interpolation of k on every admissible pair of boxes it is
    sum_a L_a(x) P_a, where the leaf coefficients of the density,
    int_Kt L_b^leaf over the cells anchored in the leaf ((m+1)-point rule),
    run upward through the shift coefficients, through the kernel blocks and
    downward (the matrix-vector product's passes).  Returns (T, d+1, d+1):
    int_K l_a l_b(x) sum_a L_a(x) P_a dx by the same rule (exact for these
    polynomials)."""
    d = tree.dim
    cl = tree.clusters
    M = m ** d
    X, lam, W = _cell_rule(mesh, m + 1)
    nc = len(cl)
    xh = [np.zeros(M) for _ in range(nc)]
    for K in range(len(cell_leafc)):
        c = cell_leafc[K]
        if c >= 0:
            xh[c] = xh[c] + W[K] @ lagrange_box(cl[c], m, d, X[K])
    for c in sorted(range(nc), key=lambda c: -cl[c].level):
        if cl[c].sons:
            xh[c] = sum(T_shift[sn].T @ xh[sn] for sn in cl[c].sons)
    yh = [np.zeros(M) for _ in range(nc)]
    for a, b in far:
        yh[a] = yh[a] + kernel_block(tree, a, b, m, sval) @ xh[b]
    for c in sorted(range(nc), key=lambda c: cl[c].level):
        for sn in cl[c].sons:
            yh[sn] = yh[sn] + T_shift[sn] @ yh[c]
    S = np.zeros((len(cell_leafc), d + 1, d + 1))
    for K in range(len(cell_leafc)):
        c = cell_leafc[K]
        if c < 0:
            continue
        g = lagrange_box(cl[c], m, d, X[K]) @ yh[c]          # (q,)
        S[K] = np.einsum("q,qa,qb->ab", W[K] * g, lam, lam)
    return S


def build_direct(mesh, dofs, s, orders, m=6, eta=2.0, leaf=32, with_boundary=True):
    """The cluster approximation assembled from the mesh, without the dense
    matrix (Sec. 6: the near field from the pair contributions of Sec. 5).
    Near blocks: every off-diagonal pair block and touching-pair
    contribution in full; the diagonal-block (self) parts of a separated
    pair only when the anchor leaves of its two cells are a near pair
    (masked assembly, oracle.assemble_full with cell labels), the rest of
    every cell's self part from the far field (self_far).  Far blocks as in
    build.  Returns the HMatrix."""
    tree = build_tree(mesh, dofs, leaf)
    far, near = block_tree(tree, eta)
    d = mesh["dim"]
    C = np.asarray(mesh["cells"], dtype=np.int64)
    nv = np.asarray(mesh["verts"]).size // d
    n = len(dofs)
    leaves, li, rleaf, tab = leaf_labels(tree, near)
    Vleaf = {c: basis_coeffs(mesh, dofs, tree, c, m) for c in leaves}
    Tsh = {c: transfer(tree, c, m) for c in range(1, len(tree.clusters))}
    Kb = {(a, b): kernel_block(tree, a, b, m, s) for a, b in far}
    if n == 0:
        return HMatrix(tree, far, near, m, s, O.cdn(d, s), Vleaf, Tsh, Kb, {})
    anchor = cell_anchors(mesh, dofs, tree.perm)
    pos = np.empty(n, dtype=np.int64)
    pos[tree.perm] = np.arange(n)
    cell_leafc = np.where(anchor >= 0, rleaf[pos[np.maximum(anchor, 0)]], -1)
    lab = np.array([li[c] if c >= 0 else 0 for c in cell_leafc], dtype=np.int32)
    Afull, _ = O.assemble_full(mesh, s, orders, with_boundary=with_boundary, cell_leaf=lab, leaf_near=tab)
    node2dof = np.full(nv, -1, dtype=np.int64)
    node2dof[np.asarray(dofs)] = np.arange(n)
    A = Afull[np.ix_(dofs, dofs)].copy()
    Cds = O.cdn(d, s)
    S = self_far(mesh, tree, far, Tsh, m, s, cell_leafc)
    for K in range(len(C)):
        for a in range(d + 1):
            i = node2dof[C[K, a]]
            if i < 0:
                continue
            for b in range(d + 1):
                j = node2dof[C[K, b]]
                if j >= 0:
                    A[i, j] += Cds * S[K, a, b]
    P = tree.perm
    cl = tree.clusters
    An = {(a, b): A[np.ix_(P[cl[a].lo:cl[a].hi], P[cl[b].lo:cl[b].hi])] for a, b in near}
    return HMatrix(tree, far, near, m, s, Cds, Vleaf, Tsh, Kb, An)


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
