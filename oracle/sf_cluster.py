"""Cluster evaluation of the strong form's all-pairs part, plain numpy
(test infrastructure only, like the rest of ``oracle/``).

Sec. 6 (the strong form by the cluster method): the strong form at the
indicator points is a sum over all edges weighted by the same kernel, so
its far part can use the same low-rank blocks as the matrix.  Written
here for the library's splitting of eq. 8 (d = 2): the edges' Gauss points
y_j carry the jumps of the normal derivative,

  c_j = w_j (grad u|K1 - grad u|K2) . N_K1 / (2s (d+2s-2)),

and the all-pairs part is P(x) = sum_j c_j |x - y_j|^{-2s}.  A cluster
tree over the cells (each cell owns its evaluation points and the Gauss
points of the edges it is the first cell of), admissible pairs of boxes
eta dist >= max diam, and for them the tensor Chebyshev interpolation of
the kernel on both boxes with nested moments (upward) and local
expansions (downward); the other leaf pairs are summed directly.  The
strong form then differs from the oracle's literal one by C (P_tree -
P_direct).

Readings: leaves of at most `leaf` cells; median split of the cell
centroids along their longest extent (stable order); the box is the cube
of the largest extent of the cells' vertex bounding box, centred on it.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import cluster as CL
from . import oracle as O
from . import strong_form as SF


@dataclass
class CellCluster:
    lo: int                     # cell range [lo, hi) in tree order
    hi: int
    box_lo: np.ndarray
    side: float
    level: int
    parent: int = -1
    sons: list = field(default_factory=list)


def cell_tree(mesh, leaf=16):
    V = np.asarray(mesh["verts"], dtype=np.float64)
    C = np.asarray(mesh["cells"], dtype=np.int64)
    P = V[C]
    cen = P.mean(1)
    blo, bhi = P.min(1), P.max(1)
    perm = np.arange(len(C))
    clusters = []

    def make(idx, lo, level, parent):
        lo_ = blo[idx].min(0)
        hi_ = bhi[idx].max(0)
        side = float((hi_ - lo_).max())
        c = CellCluster(lo, lo + len(idx), 0.5 * (lo_ + hi_) - 0.5 * side, side, level, parent)
        cid = len(clusters)
        clusters.append(c)
        perm[lo:lo + len(idx)] = idx
        if len(idx) > leaf:
            ext = cen[idx].max(0) - cen[idx].min(0)
            ax = int(np.argmax(ext))
            order = idx[np.argsort(cen[idx, ax], kind="stable")]
            h = len(order) // 2
            c.sons.append(make(order[:h], lo, level + 1, cid))
            c.sons.append(make(order[h:], lo + h, level + 1, cid))
        return cid

    make(np.arange(len(C)), 0, 0, -1)
    return perm.copy(), clusters


def _adm(a, b, eta):
    return CL.admissible(a, b, eta, 2)


def block_tree(clusters, eta):
    far, near = [], []

    def rec(s, t):
        if _adm(clusters[s], clusters[t], eta):
            far.append((s, t))
            return
        ls, lt = not clusters[s].sons, not clusters[t].sons
        if ls and lt:
            near.append((s, t))
        elif ls:
            for tt in clusters[t].sons:
                rec(s, tt)
        elif lt:
            for ss in clusters[s].sons:
                rec(ss, t)
        else:
            for ss in clusters[s].sons:
                for tt in clusters[t].sons:
                    rec(ss, tt)

    rec(0, 0)
    return far, near


def jump_sources(mesh, dofs, u, s, q):
    """Gauss points of every edge (q per edge, in the orientation of its
    first cell = the cell of lowest index), their coefficients and owning
    cell.  Returns (Y (ns, 2), c (ns,), owner (ns,))."""
    V = np.asarray(mesh["verts"], dtype=np.float64)
    C = np.asarray(mesh["cells"], dtype=np.int64)
    nod = np.zeros(len(V))
    nod[np.asarray(dofs)] = u
    P = V[C]
    U = nod[C]
    Ex = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]], axis=1)
    du = np.stack([U[:, 1] - U[:, 0], U[:, 2] - U[:, 0]], axis=1)
    G = np.linalg.solve(Ex, du[..., None])[..., 0]
    det = (P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1]) - (P[:, 2, 0] - P[:, 0, 0]) * (P[:, 1, 1] - P[:, 0, 1])
    owner = {}
    for K in range(len(C)):
        for e in range(3):
            key = tuple(sorted((int(C[K, e]), int(C[K, (e + 1) % 3]))))
            owner.setdefault(key, []).append((K, e))
    t, w = O.gauss_legendre01(q)
    cg = 1.0 / (2 * s * (2 * s))
    Y, c, own = [], [], []
    for key, lst in owner.items():
        K1, e = min(lst)
        A_, B_ = P[K1, e], P[K1, (e + 1) % 3]
        dx, dy = B_ - A_
        N = np.sign(det[K1]) * np.array([dy, -dx])
        J = G[K1] @ N
        for K2, _ in lst:
            if K2 != K1:
                J -= G[K2] @ N
        for tj, wj in zip(t, w):
            Y.append(A_ + tj * (B_ - A_))
            c.append(wj * J * cg)
            own.append(K1)
    return np.array(Y), np.array(c), np.array(own)


def potential_direct(X, Y, c, s):
    r2 = ((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
    return (r2 ** (-s)) @ c


def treecode(mesh, Xc, Y, c, own, s, m=6, eta=2.0, leaf=16):
    """Xc: (T, Q, 2) evaluation points per cell; Y, c, own: sources.  Returns
    the potential at every point, (T, Q), and (far, near, clusters)."""
    perm, cl = cell_tree(mesh, leaf)
    far, near = block_tree(cl, eta)
    T, Q = Xc.shape[:2]
    pos = np.empty(len(perm), dtype=np.int64)
    pos[perm] = np.arange(len(perm))
    # sources grouped by the tree position of their owner
    src_pos = pos[own]
    nc = len(cl)
    M = m * m

    def lagr(c_, pts):
        return CL.lagrange_box(c_, m, 2, pts)

    def in_cluster(ci):
        return (src_pos >= cl[ci].lo) & (src_pos < cl[ci].hi)

    mom = [None] * nc
    for ci in sorted(range(nc), key=lambda k: -cl[k].level):
        if not cl[ci].sons:
            sel = in_cluster(ci)
            mom[ci] = lagr(cl[ci], Y[sel]).T @ c[sel]
        else:
            mom[ci] = sum(CL.transfer(_as_tree(cl), sn, m).T @ mom[sn] for sn in cl[ci].sons)
    loc = [np.zeros(M) for _ in range(nc)]
    for a, b in far:
        Xa = CL.cheb_points(cl[a], m, 2)
        Xb = CL.cheb_points(cl[b], m, 2)
        r2 = ((Xa[:, None, :] - Xb[None, :, :]) ** 2).sum(-1)
        loc[a] = loc[a] + (r2 ** (-s)) @ mom[b]
    out = np.zeros((T, Q))
    for ci in sorted(range(nc), key=lambda k: cl[k].level):
        for sn in cl[ci].sons:
            loc[sn] = loc[sn] + CL.transfer(_as_tree(cl), sn, m) @ loc[ci]
        if not cl[ci].sons:
            cells = perm[cl[ci].lo:cl[ci].hi]
            Xt = Xc[cells].reshape(-1, 2)
            out[cells] += (lagr(cl[ci], Xt) @ loc[ci]).reshape(len(cells), Q)
    for a, b in near:
        cells = perm[cl[a].lo:cl[a].hi]
        Xt = Xc[cells].reshape(-1, 2)
        sel = in_cluster(b)
        out[cells] += potential_direct(Xt, Y[sel], c[sel], s).reshape(len(cells), Q)
    return out, far, near, cl


class _TreeView:
    def __init__(self, cl):
        self.clusters = cl
        self.dim = 2


def _as_tree(cl):
    return _TreeView(cl)


def strong_form_cluster(mesh, dofs, u, s, k_eval=2, q_far=2, q_near=12, m=6, eta=2.0, leaf=16):
    """The oracle's strong form with its all-pairs part evaluated by the
    cluster tree instead of directly: Lu + C (P_tree - P_direct)."""
    Lu = SF.strong_form(mesh, dofs, u, s, k_eval=k_eval, q_far=q_far, q_near=q_near)
    Xc, _, _ = SF.eval_points(mesh, k_eval)
    Y, c, own = jump_sources(mesh, dofs, u, s, q_far)
    Pt, far, near, cl = treecode(mesh, Xc, Y, c, own, s, m=m, eta=eta, leaf=leaf)
    Pd = potential_direct(Xc.reshape(-1, 2), Y, c, s).reshape(Pt.shape)
    return Lu + O.cdn(2, s) * (Pt - Pd), (far, near, cl)
