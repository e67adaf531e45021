"""Host logic of the adaptive loop: maximum marking and conforming
refinement (newest-vertex bisection in d = 2, halving in d = 1)."""
from collections import Counter

import numpy as np
import pytest

from paper_1708_03912_amd import meshgen as M
from paper_1708_03912_amd.adaptive import mark_max


def _area(mesh):
    V = np.asarray(mesh["verts"])
    C = np.asarray(mesh["cells"])
    a, b, c = V[C[:, 0]], V[C[:, 1]], V[C[:, 2]]
    return 0.5 * ((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1]))


def _min_angle(mesh):
    V = np.asarray(mesh["verts"])
    C = np.asarray(mesh["cells"])
    ang = []
    for i in range(3):
        p, q, r = V[C[:, i]], V[C[:, (i + 1) % 3]], V[C[:, (i + 2) % 3]]
        u, v = q - p, r - p
        ang.append(np.arccos(np.clip((u * v).sum(1) / np.linalg.norm(u, axis=1) / np.linalg.norm(v, axis=1), -1, 1)))
    return np.min(ang)


def _conforming(mesh):
    """Every edge lies on one or two cells, the one-cell edges are exactly
    the boundary facets, and no vertex lies inside another cell's edge."""
    C = np.asarray(mesh["cells"])
    cnt = Counter(tuple(sorted((int(c[i]), int(c[(i + 1) % 3])))) for c in C for i in range(3))
    assert max(cnt.values()) <= 2
    bnd = {e for e, k in cnt.items() if k == 1}
    assert bnd == {tuple(sorted(map(int, f))) for f in mesh["bfacets"]}
    V = np.asarray(mesh["verts"])
    used = np.unique(C)
    assert len(used) == len(V)
    # a hanging node would be the midpoint of some edge
    mids = {tuple(np.round(0.5 * (V[a] + V[b]), 12)) for a, b in cnt}
    verts = {tuple(np.round(v, 12)) for v in V}
    for a, b in cnt:
        m = tuple(np.round(0.5 * (V[a] + V[b]), 12))
        assert m not in verts, "hanging node"
    return True


def test_nvb_refinement_is_conforming_and_nested():
    m = M.nvb_label(M.disk_for_cells(300, seed=2))
    area0 = _area(m).sum()
    ang0 = _min_angle(m)
    assert np.all(_area(m) > 0)
    rng = np.random.default_rng(0)
    for _ in range(6):
        T = len(m["cells"])
        marked = rng.choice(T, max(1, T // 10), replace=False)
        big = _area(m)[marked].max()
        m2 = M.refine_marked(m, marked)
        assert len(m2["cells"]) >= T + len(marked)
        assert np.all(_area(m2) > 0)
        assert abs(_area(m2).sum() - area0) <= 1e-12 * area0
        assert _conforming(m2)
        # nested: every old vertex survives
        old = {tuple(v) for v in np.asarray(m["verts"])}
        assert old <= {tuple(v) for v in np.asarray(m2["verts"])}
        m = m2
    # newest-vertex bisection keeps the shapes in finitely many classes
    assert _min_angle(m) >= 0.5 * ang0


def test_refine_1d_halves_marked_cells():
    m = M.interval(8)
    m2 = M.refine_marked(m, [0, 3, 7])
    x = np.asarray(m2["verts"]).ravel()
    assert len(x) == 12 and np.all(np.diff(x) > 0)
    C = np.asarray(m2["cells"])
    assert np.all(C[:, 1] == C[:, 0] + 1)
    h = np.diff(x)
    assert np.allclose(sorted(h), sorted([0.125] * 6 + [0.25] * 5))
    assert m2["bfacets"].tolist() == [[0], [11]]


def test_nvb_label_keeps_orientation():
    m = M.disk_for_cells(200, seed=4)
    m2 = M.nvb_label(m)
    assert np.all(np.sign(_area(m2)) == np.sign(_area(m)))
    V = np.asarray(m2["verts"])
    C = np.asarray(m2["cells"])
    L = [((V[C[:, (i + 1) % 3]] - V[C[:, (i + 2) % 3]]) ** 2).sum(1) for i in range(3)]
    assert np.all(L[0] >= L[1]) and np.all(L[0] >= L[2])


def test_mark_max():
    cells = np.array([[0, 1], [1, 2], [2, 3], [3, 4]])
    eta2 = np.array([1.0, 0.1, 0.0, 0.63, 0.65])     # eta-hat = sqrt
    got = mark_max(eta2, cells, 0.8)
    # sqrt(0.63) = 0.794 < 0.8, sqrt(0.65) = 0.806 >= 0.8
    assert got.tolist() == [0, 3]


def test_boundary_projection_disk():
    m = M.nvb_label(M.disk_for_cells(150, seed=2))
    V0 = np.asarray(m["verts"])
    C = np.asarray(m["cells"])
    r = np.hypot(*V0[C].mean(1).T)
    m2 = m
    for _ in range(3):  # a boundary cell's refinement edge need not be on the boundary
        V1 = np.asarray(m2["verts"])
        r = np.hypot(*V1[np.asarray(m2["cells"])].mean(1).T)
        m2 = M.refine_marked(m2, np.nonzero(r > 0.8)[0], project=M.project_disk)
    V = np.asarray(m2["verts"])
    b = np.unique(np.asarray(m2["bfacets"]))
    assert np.allclose(np.hypot(V[b, 0], V[b, 1]), 1.0, atol=1e-14)
    assert len(b) > len(np.unique(np.asarray(m["bfacets"])))
    assert np.all(_area(m2) > 0) and _conforming(m2)
