"""Pins of the oracle's P1 mass matrix and of the implicit heat step
(Sec. 5: (M + dt A^s) u = b) against facts other than its own formula."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import oracle as O  # noqa: E402
from paper_1708_03912_amd import meshgen as M  # noqa: E402


def _quadrature_mass(mesh, dofs):
    """int phi_i phi_j by the edge-midpoint rule on each triangle (weights
    |K|/3, exact for quadratics), assembled point by point."""
    V = np.asarray(mesh["verts"], dtype=np.float64).reshape(-1, 2)
    Cc = np.asarray(mesh["cells"])
    full = np.zeros((len(V), len(V)))
    for K in Cc:
        P = V[K]
        area = 0.5 * abs((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[2, 0] - P[0, 0]) * (P[1, 1] - P[0, 1]))
        T = np.array([[1.0, P[0, 0], P[0, 1]], [1.0, P[1, 0], P[1, 1]], [1.0, P[2, 0], P[2, 1]]])
        coef = np.linalg.inv(T)  # column a: coefficients of the hat function of vertex a
        for m0, m1 in ((0, 1), (1, 2), (2, 0)):
            x = 0.5 * (P[m0] + P[m1])
            phi = np.array([1.0, x[0], x[1]]) @ coef
            full[np.ix_(K, K)] += area / 3.0 * np.outer(phi, phi)
    return full[np.ix_(dofs, dofs)]


@pytest.mark.parametrize("s", [0.3, 0.7])
def test_mass_matrix_against_quadrature(s):
    mesh = M.disk_for_cells(300, seed=4)
    nv = len(mesh["verts"])
    dofs = O.dof_nodes(nv, mesh["bfacets"], s)
    Mo = O.mass_matrix(mesh, dofs)
    Mq = _quadrature_mass(mesh, dofs)
    assert np.abs(Mo - Mq).max() <= 1e-15 * 50 * np.abs(Mq).max()


def test_mass_row_sums_are_the_load_vector():
    """With every node a DOF (s < 1/2), sum_j M_ij = int phi_i = b_i for
    f = 1, and 1^T M 1 is the area of the polygon."""
    mesh = M.disk_for_cells(500, seed=6)
    nv = len(mesh["verts"])
    dofs = O.dof_nodes(nv, mesh["bfacets"], 0.25)
    assert len(dofs) == nv
    Mo = O.mass_matrix(mesh, dofs)
    b = O.load_vector_one(mesh, dofs)
    assert np.abs(Mo.sum(1) - b).max() <= 1e-15 * 10 * b.max()
    # the hull is the regular polygon on the N_b equispaced circle points
    nb = len(mesh["bfacets"])
    assert abs(Mo.sum() - 0.5 * nb * math.sin(2 * math.pi / nb)) <= 1e-12


def test_mass_matrix_1d_uniform():
    """Textbook: on a uniform grid of width h the interior rows of M are
    h/6 (1, 4, 1)."""
    mesh = M.interval(16)
    h = 2.0 / 16
    dofs = O.dof_nodes(17, mesh["bfacets"], 0.75)
    Mo = O.mass_matrix(mesh, dofs)
    ref = h / 6.0 * (4 * np.eye(15) + np.eye(15, k=1) + np.eye(15, k=-1))
    assert np.abs(Mo - ref).max() <= 1e-16 * 10


def test_heat_step_fixed_point_and_conditioning():
    """The Poisson solution is the fixed point of the implicit step, and with
    dt = h^(2s) the Jacobi-scaled (M + dt A^s) stays well conditioned under
    refinement while A^s does not (Sec. 5 lemma on the condition number)."""
    s = 0.75
    kappa = {}
    for T in (300, 1200):
        mesh = M.disk_for_cells(T, seed=3)
        A, dofs, _ = O.assemble(mesh, s, O.Orders())
        Mm = O.mass_matrix(mesh, dofs)
        b = O.load_vector_one(mesh, dofs)
        V = np.asarray(mesh["verts"]).reshape(-1, 2)
        P = V[np.asarray(mesh["cells"])]
        h = np.sqrt(((P[:, [1, 2, 0]] - P) ** 2).sum(-1)).max()
        dt = h ** (2 * s)
        u = O.solve_cholesky(A, b)
        u1 = O.solve_cholesky(Mm + dt * A, Mm @ u + dt * b)
        assert np.abs(u1 - u).max() <= 1e-10 * np.abs(u).max()
        for name, K in (("poisson", A), ("heat", Mm + dt * A)):
            d = np.sqrt(np.diag(K))
            ev = np.linalg.eigvalsh(K / d[:, None] / d[None, :])
            kappa[(name, T)] = ev[-1] / ev[0]
    assert kappa[("heat", 1200)] / kappa[("heat", 300)] <= 1.6
    assert kappa[("poisson", 1200)] / kappa[("poisson", 300)] >= 2.0
