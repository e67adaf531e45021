"""Pins of the symmetry reduction (Sec. 7): the reduced system P^T A P / K
reproduces the symmetric full solution exactly, and its load vector is the
sector's own."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import symmetry as SY
from paper_1708_03912_amd import meshgen as M


@pytest.mark.parametrize("K", [2, 4, 8])
def test_mesh_is_symmetric(K):
    mesh, vfold, Tw, pre, rot = M.disk_symmetric(0.2, K, seed=3)
    V = np.asarray(mesh["verts"])
    C = np.asarray(mesh["cells"])
    al = 2 * math.pi / K
    R = np.array([[math.cos(al), -math.sin(al)], [math.sin(al), math.cos(al)]])
    key = {(round(x * 1e9), round(y * 1e9)): i for i, (x, y) in enumerate(V)}
    img = np.array([key[(round(p[0] * 1e9), round(p[1] * 1e9))] for p in V @ R.T])
    assert np.all(vfold[img] == vfold) and np.all(vfold[vfold] == vfold)
    cells = {tuple(sorted(c)) for c in C.tolist()}
    assert {tuple(sorted(img[c])) for c in C.tolist()} == cells
    a = V[C]
    area = 0.5 * np.abs((a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1])
                        - (a[:, 2, 0] - a[:, 0, 0]) * (a[:, 1, 1] - a[:, 0, 1]))
    assert abs(K * area[:Tw].sum() - area.sum()) <= 1e-12
    # representatives are vertices of the sector
    assert set(np.unique(vfold).tolist()) <= set(np.unique(C[:Tw]).tolist())


@pytest.mark.parametrize("K,s", [(2, 0.3), (4, 0.75), (8, 0.5)])
def test_reduced_solution_is_the_full_one(K, s):
    mesh, vfold, Tw, pre, rot = M.disk_symmetric(0.25, K, seed=4)
    A, dofs, _ = O.assemble(mesh, s, O.Orders())
    b = O.load_vector_one(mesh, dofs)
    u = O.solve_cholesky(A, b)
    Ar, br, red = SY.reduce(A, b, dofs, vfold, K)
    assert np.abs(Ar - Ar.T).max() <= 1e-14 * np.abs(Ar).max()
    assert np.linalg.eigvalsh(Ar).min() > 0
    ur = O.solve_cholesky(Ar, br)
    pos = np.searchsorted(dofs, red)
    assert np.all(np.asarray(dofs)[pos] == red)
    # the full solution is symmetric up to the rotation asymmetry of the
    # quadrature (a rotated pair may take another distance class)
    assert np.abs(ur - u[pos]).max() <= 1e-8 * np.abs(u).max()
    # energies: K u_r.A_r u_r = u.A u
    assert abs(K * ur @ Ar @ ur - u @ A @ u) <= 1e-8 * (u @ A @ u)
    # the reduced load vector is the sector's: sum over the omega cells
    # around each representative of |K|/3 (f = 1)
    V = np.asarray(mesh["verts"])
    C = np.asarray(mesh["cells"])
    rep_col = {v: i for i, v in enumerate(red)}
    bw = np.zeros(len(red))
    for c in C[:Tw]:
        P = V[c]
        ar = 0.5 * abs((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1]))
        for v in c:
            r = vfold[v]
            if r in rep_col:
                bw[rep_col[r]] += ar / 3.0
    assert np.abs(bw - br).max() <= 1e-14 * np.abs(br).max()


def test_no_symmetry_is_identity():
    mesh = M.disk_for_cells(150, seed=2)
    A, dofs, _ = O.assemble(mesh, 0.4, O.Orders())
    b = O.load_vector_one(mesh, dofs)
    Ar, br, red = SY.reduce(A, b, dofs, np.arange(len(mesh["verts"])), 1)
    assert np.array_equal(Ar, A) and np.array_equal(br, b)


@pytest.mark.parametrize("K,s", [(2, 0.3), (4, 0.75)])
def test_weighted_pair_sum_is_the_fold(K, s):
    """The sector-against-images pair sum (what the effective kernel
    computes) equals P^T A P / K up to the quadrature rules' rotation
    asymmetry, and costs about 1/K of the full pair count."""
    mesh, vfold, Tw, pre, rot = M.disk_symmetric(0.25, K, seed=5)
    A, dofs, cnt_full = O.assemble(mesh, s, O.Orders())
    b = O.load_vector_one(mesh, dofs)
    Ar, br, red = SY.reduce(A, b, dofs, vfold, K)
    Aw, redw, cnt = SY.assemble_reduced(mesh, s, O.Orders(), vfold, Tw)
    assert np.array_equal(red, redw)
    assert np.abs(Aw - Ar).max() <= 1e-7 * np.abs(Ar).max()
    bw = SY.load_vector_reduced(mesh, vfold, Tw, red)
    assert np.abs(bw - br).max() <= 1e-14 * np.abs(br).max()
    uw = O.solve_cholesky(Aw, bw)
    u = O.solve_cholesky(A, b)
    pos = np.searchsorted(dofs, red)
    assert np.abs(uw - u[pos]).max() <= 1e-7 * np.abs(u).max()
    T = len(mesh["cells"])
    assert cnt.sum() < (1.5 / K + 0.1) * cnt_full.sum()


@pytest.mark.parametrize("K,s", [(2, 0.3), (4, 0.75), (8, 0.5)])
def test_one_of_each_cross_couple(K, s):
    """Counting one member of each couple (S, B^i T) ~ (T, B^-i S) with
    weight 1 gives the same reduced matrix as counting both with 1/2 (up to
    the rotation asymmetry of the rules), with about 1/K of the full pairs."""
    mesh, vfold, Tw, pre, rot = M.disk_symmetric(0.25, K, seed=5)
    Ah, red, cnt_h = SY.assemble_reduced(mesh, s, O.Orders(), vfold, Tw)
    Aq, red2, cnt_q = SY.assemble_reduced(mesh, s, O.Orders(), vfold, Tw, pre=pre, rot=rot, K=K)
    assert np.array_equal(red, red2)
    assert np.abs(Aq - Ah).max() <= 1e-7 * np.abs(Ah).max()
    assert np.abs(Aq - Aq.T).max() <= 1e-14 * np.abs(Aq).max()
    A, dofs, cnt_full = O.assemble(mesh, s, O.Orders())
    assert cnt_q.sum() <= (1.0 / K + 0.05) * cnt_full.sum() + 1


# one order for every separated pair: no distance-class threshold, so a
# rotated copy of a pair takes the same rule as the pair itself
_ONE_CLASS = O.Orders(k_touch=5, k_touch_bnd=5, theta=[], k_far=[3], k_far_bnd=[3])


@pytest.mark.parametrize("K,s", [(2, 0.3), (4, 0.75)])
def test_weighted_pair_sum_is_the_fold_exactly(K, s):
    """With a single separated-pair order the weighted pair sum is the
    definition P^T A P / K up to rounding, both when each couple of equal
    cross pairs counts twice with weight 1/2 and when one member counts with
    weight 1.  (For K = 2, 4 the images keep the vertex-id order of every
    touching pair, so the touching rules are the same on every copy.)"""
    mesh, vfold, Tw, pre, rot = M.disk_symmetric(0.25, K, seed=5)
    A, dofs, _ = O.assemble(mesh, s, _ONE_CLASS)
    b = O.load_vector_one(mesh, dofs)
    Ar, br, red = SY.reduce(A, b, dofs, vfold, K)
    Ah, red_h, _ = SY.assemble_reduced(mesh, s, _ONE_CLASS, vfold, Tw)
    Aq, red_q, _ = SY.assemble_reduced(mesh, s, _ONE_CLASS, vfold, Tw, pre=pre, rot=rot, K=K)
    assert np.array_equal(red, red_h) and np.array_equal(red, red_q)
    scale = np.abs(Ar).max()
    assert np.abs(Ah - Ar).max() <= 1e-12 * scale
    assert np.abs(Aq - Ar).max() <= 1e-12 * scale
    assert np.linalg.norm(Aq - Ar) <= 1e-12 * np.linalg.norm(Ar)


def test_weighted_pair_sum_gap_is_the_touching_rules():
    """K = 8: rotated copies of a touching pair are labelled in another
    vertex-id order, so their regularised rules differ by the rules' own
    error; the gap to P^T A P / K falls with the touching order."""
    K, s = 8, 0.5
    mesh, vfold, Tw, pre, rot = M.disk_symmetric(0.25, K, seed=5)
    gaps = []
    for kt in (5, 10):
        ords = O.Orders(k_touch=kt, k_touch_bnd=kt, theta=[], k_far=[3], k_far_bnd=[3])
        A, dofs, _ = O.assemble(mesh, s, ords)
        b = O.load_vector_one(mesh, dofs)
        Ar, _, _ = SY.reduce(A, b, dofs, vfold, K)
        Aq, _, _ = SY.assemble_reduced(mesh, s, ords, vfold, Tw, pre=pre, rot=rot, K=K)
        gaps.append(np.abs(Aq - Ar).max() / np.abs(Ar).max())
    assert gaps[1] <= 1e-9 and gaps[1] <= 1e-2 * gaps[0]
