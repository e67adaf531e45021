"""The bound the repeatable assembly scales its fixed-point words by: for
the hat function of vertex v, (phi(x) - phi(y))^2 <= min(L_v^2 |x-y|^2, 1)
on {x in supp} or {y in supp} gives
  a(phi_v, phi_v) <= C |supp_v| |S^{d-1}| L_v^{2s} (1/(2-2s) + 1/(2s)),
and |a(phi_i, phi_j)| <= sqrt(a_ii a_jj).  Checked here, without the
library's safety factor 2, against the oracle's matrices (all nodes, with
the boundary term) in 1D and 2D, on quasi-uniform and graded meshes."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1708_03912_amd import meshgen as M


def hat_bound(mesh, s):
    d = mesh["dim"]
    V = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1, d)
    C = np.asarray(mesh["cells"])
    supp = np.zeros(len(V))
    L = np.zeros(len(V))
    for c in C:
        if d == 1:
            h = abs(V[c[1], 0] - V[c[0], 0])
            for a in range(2):
                supp[c[a]] += h
                L[c[a]] = max(L[c[a]], 1.0 / h)
        else:
            P = V[c]
            area = 0.5 * abs((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1]))
            for a in range(3):
                e = np.linalg.norm(P[(a + 2) % 3] - P[(a + 1) % 3])
                supp[c[a]] += area
                L[c[a]] = max(L[c[a]], e / (2 * area))   # 1 / height over the opposite edge
    sphere = 2.0 if d == 1 else 2.0 * math.pi
    return O.cdn(d, s) * supp * sphere * L ** (2 * s) * (1 / (2 - 2 * s) + 1 / (2 * s))


@pytest.mark.parametrize("case", ["interval", "graded_interval", "disk", "lshape"])
@pytest.mark.parametrize("s", [0.1, 0.45, 0.9])
def test_hat_function_bound(case, s):
    mesh = {"interval": lambda: M.interval(128), "graded_interval": lambda: M.interval_graded(96, 2.0),
            "disk": lambda: M.disk_for_cells(500, seed=3),
            "lshape": lambda: M.lshape(h_max=0.5, ratio=16.0)}[case]()
    orders = O.Orders(k_touch=6, k_touch_bnd=6, theta=[1.5, 3.0, 6.0], k_far=[4, 3, 2, 2], k_far_bnd=[4, 3, 2, 2])
    nv = np.asarray(mesh["verts"]).size // mesh["dim"]
    dofs = O.dof_nodes(nv, mesh["bfacets"], s, "interior")   # the boundary term is finite on these rows
    A, _ = O.assemble_full(mesh, s, orders)
    A = A[np.ix_(dofs, dofs)]
    B = hat_bound(mesh, s)[dofs]
    diag = np.diag(A)
    assert np.all(diag > 0)
    ratio = diag / B
    assert ratio.max() < 1.0, ratio.max()
    # off-diagonal entries by the geometric mean of the diagonal bounds
    assert np.all(np.abs(A) <= np.sqrt(np.outer(B, B)) * (1 + 1e-12))
    # the bound is not loose by more than the fixed-point margin needs
    assert ratio.max() > 1e-3
