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
