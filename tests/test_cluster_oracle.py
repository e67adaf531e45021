"""Pins of the oracle's cluster (H-matrix) approximation (Sec. 6): the
Chebyshev interpolation, the tree and block partition, the exactness of
the shift coefficients, and convergence to the dense matrix in m."""
import numpy as np
import pytest

from oracle import cluster as H
from oracle import oracle as O
from paper_1708_03912_amd import meshgen as M


def test_lagrange_basis():
    for m in (1, 2, 5, 8):
        t = H.cheb_nodes(m)
        assert np.all(np.diff(t) > 0) and t[0] > 0 and t[-1] < 1
        assert np.allclose(H.lagrange(t, t), np.eye(m), atol=1e-14)
        # interpolation reproduces polynomials of degree < m
        x = np.linspace(-0.3, 1.2, 17)
        for p in range(m):
            assert np.allclose(H.lagrange(t, x) @ t ** p, x ** p, atol=1e-11)
    # Chebyshev points of the first kind: roots of T_m on [0, 1]
    t = H.cheb_nodes(6)
    assert np.allclose(np.cos(6 * np.arccos(2 * t - 1)), 0.0, atol=1e-13)


@pytest.fixture(scope="module")
def disk():
    s = 0.75
    mesh = M.disk_for_cells(1200, seed=2)
    A, dofs, _ = O.assemble(mesh, s, O.Orders())
    return mesh, dofs, A, s


def test_tree_and_blocks_partition(disk):
    mesh, dofs, A, s = disk
    n = len(dofs)
    tree = H.build_tree(mesh, dofs, leaf=16)
    assert sorted(tree.perm.tolist()) == list(range(n))
    cl = tree.clusters
    X, slo, shi = H._supports(mesh, dofs)
    for c in cl:
        idx = tree.perm[c.lo:c.hi]
        assert np.all(slo[idx] >= c.box_lo - 1e-15) and np.all(shi[idx] <= c.box_lo + c.side + 1e-15)
        if c.sons:
            assert cl[c.sons[0]].lo == c.lo and cl[c.sons[-1]].hi == c.hi
            assert cl[c.sons[0]].hi == cl[c.sons[1]].lo
        else:
            assert c.hi - c.lo <= 16
    far, near = H.block_tree(tree, 2.0)
    cover = np.zeros((n, n), dtype=int)
    for a, b in far + near:
        cover[np.ix_(tree.perm[cl[a].lo:cl[a].hi], tree.perm[cl[b].lo:cl[b].hi])] += 1
    assert np.all(cover == 1)
    C = np.asarray(mesh["cells"])
    node = np.asarray(dofs)
    for a, b in far:
        assert H.admissible(cl[a], cl[b], 2.0, 2)
        # disjoint supports: no cell touches a vertex of both clusters
        va = set(node[tree.perm[cl[a].lo:cl[a].hi]].tolist())
        vb = set(node[tree.perm[cl[b].lo:cl[b].hi]].tolist())
        touch_a = np.isin(C, list(va)).any(1)
        touch_b = np.isin(C, list(vb)).any(1)
        assert not np.any(touch_a & touch_b)
    for a, b in near:
        assert not H.admissible(cl[a], cl[b], 2.0, 2)
        assert not cl[a].sons and not cl[b].sons


def test_shift_coefficients_are_exact(disk):
    """V_parent = sum_sons V_son T_son (the parent's Lagrange polynomials
    are of the son's interpolation degree), and the m+1 point rule is
    exact for the basis coefficients."""
    mesh, dofs, A, s = disk
    tree = H.build_tree(mesh, dofs, leaf=16)
    m = 5
    internal = [c for c, cl in enumerate(tree.clusters) if cl.sons]
    for c in (internal[1], internal[len(internal) // 2], internal[-1]):
        cl = tree.clusters[c]
        Vp = H.basis_coeffs(mesh, dofs, tree, c, m)
        stack = np.concatenate([H.basis_coeffs(mesh, dofs, tree, sn, m) @ H.transfer(tree, sn, m)
                                for sn in cl.sons])
        assert np.abs(Vp - stack).max() <= 1e-13 * np.abs(Vp).max()
    leaf = tree.leaves()[3]
    V1 = H.basis_coeffs(mesh, dofs, tree, leaf, m)
    X, lam, W = H._cell_rule(mesh, m + 3)
    cl = tree.clusters[leaf]
    C = np.asarray(mesh["cells"])
    ref = np.zeros_like(V1)
    for r, v in enumerate(np.asarray(dofs)[tree.perm[cl.lo:cl.hi]]):
        for K, a in zip(*np.nonzero(C == v)):
            ref[r] += (W[K] * lam[:, a]) @ H.lagrange_box(cl, m, 2, X[K])
    assert np.abs(V1 - ref).max() <= 1e-14 * np.abs(ref).max()


def test_converges_to_the_dense_matrix(disk):
    """Interpolation error falls geometrically in m (admissible blocks of
    eta = 1 and 2); at m = 6 the product is within 1e-7 of the dense one;
    the approximated matrix is symmetric."""
    mesh, dofs, A, s = disk
    n = len(dofs)
    x = np.random.default_rng(0).standard_normal(n)
    y = A @ x
    for eta, tol6 in ((1.0, 2e-8), (2.0, 5e-7)):
        err = []
        for m in (2, 4, 6):
            Hm = H.build(mesh, dofs, A, s, m=m, eta=eta, leaf=16)
            assert len(Hm.far) > 0
            err.append(np.linalg.norm(H.matvec(Hm, x) - y) / np.linalg.norm(y))
        assert err[0] > 10 * err[1] > 100 * err[2], err
        assert err[2] <= tol6, err
    Hs = H.build(mesh, dofs, A, s, m=3, eta=2.0, leaf=16)
    D = H.dense(Hs, n)
    assert np.abs(D - D.T).max() <= 1e-13 * np.abs(D).max()
    # the far field really is a low-rank replacement: entries differ
    assert np.abs(D - A).max() > 0


def test_1d_interval():
    s = 0.25
    mesh = M.interval(256)
    A, dofs, _ = O.assemble(mesh, s, O.Orders())
    x = np.random.default_rng(1).standard_normal(len(dofs))
    errs = []
    for m in (2, 4, 6):
        Hm = H.build(mesh, dofs, A, s, m=m, eta=1.0, leaf=8)
        errs.append(np.linalg.norm(H.matvec(Hm, x) - A @ x) / np.linalg.norm(A @ x))
    assert errs[0] > 10 * errs[1] > 100 * errs[2], errs


# ------------------------------------------------ direct near-field assembly

HI = O.Orders(k_touch=6, k_touch_bnd=6, theta=[1.5, 3.0, 6.0], k_far=[6, 6, 6, 6], k_far_bnd=[4, 3, 2, 2])
LO = O.Orders(k_touch=5, k_touch_bnd=5, theta=[1.5, 3.0, 6.0], k_far=[4, 3, 2, 2], k_far_bnd=[4, 3, 2, 2])


def _grid_square(k):
    """Unit square, (k+1)^2 vertices; every square cell split by its
    diagonal, the four corner squares by the diagonal that leaves a corner
    triangle with all three vertices on the boundary (a cell without DOF in
    the interior-DOF mode)."""
    xs = np.linspace(0.0, 1.0, k + 1)
    V = np.array([(x, y) for y in xs for x in xs])
    vid = lambda i, j: j * (k + 1) + i  # noqa: E731
    cells = []
    for j in range(k):
        for i in range(k):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            corner_lo = (i, j) in ((0, 0), (k - 1, k - 1))
            if corner_lo or (i + j) % 2 == 0 and (i, j) not in ((k - 1, 0), (0, k - 1)):
                cells += [(a, b, d), (b, c, d)] if (i, j) == (0, 0) else [(a, b, c), (a, c, d)]
            else:
                cells += [(a, b, c), (a, c, d)] if (i, j) in ((k - 1, 0),) else [(a, b, d), (b, c, d)]
    cells = np.array(cells)
    bf = []
    for t in range(k):
        bf += [(vid(t, 0), vid(t + 1, 0)), (vid(k, t), vid(k, t + 1)),
               (vid(t + 1, k), vid(t, k)), (vid(0, t + 1), vid(0, t))]
    return {"dim": 2, "verts": V, "cells": cells, "bfacets": np.array(bf)}


def test_direct_all_near_equals_dense():
    """With no admissible pair (eta -> 0) every leaf pair is near, no self
    part is masked and the far field is empty: the directly assembled
    cluster matrix is the dense matrix (2D disk, 1D interval, both s)."""
    for mesh, leaf in ((M.disk_for_cells(500, seed=4), 8), (M.interval(96), 4)):
        for s in (0.25, 0.75):
            A, dofs, _ = O.assemble(mesh, s, LO, mode="interior")
            Hd = H.build_direct(mesh, dofs, s, LO, m=3, eta=1e-12, leaf=leaf)
            assert not Hd.far
            D = H.dense(Hd, len(dofs))
            assert np.abs(D - A).max() <= 1e-13 * np.abs(A).max()


def test_masked_assembly_brute_force():
    """The masked assembly (cell labels, near table) equals the full one
    minus C times the diagonal-block parts SK, ST of every separated pair
    whose labels the table marks far, each pair integrated here one by one
    with the order of its distance class."""
    mesh = M.disk_for_cells(90, seed=6)
    s = 0.4
    V = np.asarray(mesh["verts"], dtype=np.float64)
    C = np.asarray(mesh["cells"])
    T = len(C)
    rng = np.random.default_rng(3)
    L = 4
    lab = rng.integers(0, L, T).astype(np.int32)
    tab = rng.integers(0, 2, (L, L)).astype(np.uint8)
    tab = np.maximum(tab, tab.T)
    Afull, _ = O.assemble_full(mesh, s, LO)
    Amask, _ = O.assemble_full(mesh, s, LO, cell_leaf=lab, leaf_near=tab)
    P = V[C]
    cen = (P[:, 0] + P[:, 1] + P[:, 2]) / 3.0
    h2 = np.max([((P[:, (a + 1) % 3] - P[:, a]) ** 2).sum(1) for a in range(3)], axis=0)
    ref = Afull.copy()
    Cds = O.cdn(2, s)
    dropped = 0
    for K in range(T):
        for Kt in range(K + 1, T):
            if set(C[K]) & set(C[Kt]) or tab[lab[K], lab[Kt]]:
                continue
            d2 = ((cen[K] - cen[Kt]) ** 2).sum()
            hm = max(h2[K], h2[Kt])
            cls = sum(1 for th in LO.theta if d2 >= th * th * hm)
            SK, ST, _ = O.far_pair(s, LO.k_far[cls], P[K], P[Kt])
            ref[np.ix_(C[K], C[K])] -= Cds * SK
            ref[np.ix_(C[Kt], C[Kt])] -= Cds * ST
            dropped += 1
    assert dropped > 100
    assert np.abs(Amask - ref).max() <= 1e-13 * np.abs(Afull).max()
    # off-diagonal blocks untouched: entries of vertices sharing no cell
    # agree (up to the order of the OpenMP sums)
    share = np.zeros_like(Afull, dtype=bool)
    for c in C:
        share[np.ix_(c, c)] = True
    assert np.abs(Amask[~share] - Afull[~share]).max() <= 1e-15 * np.abs(Afull).max()


@pytest.mark.parametrize("s", [0.25, 0.75])
def test_direct_converges_geometrically(s):
    """Against a dense matrix whose separated pairs all use order 6 (so that
    its own quadrature error is below the interpolation error), the directly
    assembled cluster matrix converges geometrically in m, both in the
    far blocks and in the far part of the diagonal blocks."""
    mesh = M.disk_for_cells(600, seed=3)
    A, dofs, _ = O.assemble(mesh, s, HI, mode="interior")
    err = []
    for m in (4, 6, 8):
        Hd = H.build_direct(mesh, dofs, s, HI, m=m, eta=2.0, leaf=8)
        assert len(Hd.far) > 0
        D = H.dense(Hd, len(dofs))
        err.append(np.abs(D - A).max() / np.abs(A).max())
        assert np.abs(D - D.T).max() <= 1e-13 * np.abs(D).max()
    assert err[0] > 10 * err[1] > 100 * err[2], err
    assert err[2] <= 1e-7, err


def test_direct_cells_without_dof():
    """Corner cells with all vertices on the boundary (no DOF in the
    interior mode) take the anchor of a neighbour across an edge; the
    anchor's clusters' boxes contain them; with every pair near the direct
    matrix is the dense one, and it converges in m."""
    mesh = _grid_square(8)
    C = np.asarray(mesh["cells"])
    s = 0.6
    A, dofs, _ = O.assemble(mesh, s, HI, mode="interior")
    on_dof = np.zeros(len(mesh["verts"]), dtype=bool)
    on_dof[dofs] = True
    dofless = np.nonzero(~on_dof[C].any(1))[0]
    assert len(dofless) >= 2
    tree = H.build_tree(mesh, dofs, leaf=4)
    anchor = H.cell_anchors(mesh, dofs, tree.perm)
    assert (anchor >= 0).all()
    V = np.asarray(mesh["verts"])
    pos = np.empty(len(dofs), dtype=int)
    pos[tree.perm] = np.arange(len(dofs))
    for K in dofless:
        nb = [k for k in range(len(C)) if k != K and len(set(C[k]) & set(C[K])) == 2]
        assert anchor[K] in [anchor[k] for k in nb]
        for c in tree.clusters:
            if c.lo <= pos[anchor[K]] < c.hi:
                assert np.all(V[C[K]] >= c.box_lo - 1e-15) and np.all(V[C[K]] <= c.box_lo + c.side + 1e-15)
    Hn = H.build_direct(mesh, dofs, s, HI, m=3, eta=1e-12, leaf=4)
    assert np.abs(H.dense(Hn, len(dofs)) - A).max() <= 1e-13 * np.abs(A).max()
    err = []
    for m in (3, 5, 7):
        Hd = H.build_direct(mesh, dofs, s, HI, m=m, eta=1.5, leaf=4)
        assert len(Hd.far) > 0
        err.append(np.abs(H.dense(Hd, len(dofs)) - A).max() / np.abs(A).max())
    assert err[0] > 5 * err[1] > 25 * err[2], err
