"""Pins of the oracle's multigrid (prolongation, Galerkin operators,
V-cycle, MG-preconditioned CG) against facts other than its own code."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import multigrid as G  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_1708_03912_amd import meshgen as M  # noqa: E402


def _levels(mesh0, L, s, mode="paper"):
    meshes, parents = M.hierarchy(mesh0, L)
    dofs = [O.dof_nodes(len(m["verts"]), m["bfacets"], s, mode) for m in meshes]
    nv = [len(m["verts"]) for m in meshes]
    return meshes, parents, dofs, nv


def test_prolongation_reproduces_linear_functions():
    meshes, parents, dofs, nv = _levels(M.disk_for_cells(200, seed=1), 3, 0.25)
    for l in (1, 2):
        P = G.prolongation(parents[l - 1], dofs[l - 1], dofs[l], nv[l - 1])
        Vc = meshes[l - 1]["verts"][dofs[l - 1]]
        Vf = meshes[l]["verts"][dofs[l]]
        f = lambda V: 0.3 - 1.7 * V[:, 0] + 2.1 * V[:, 1]
        assert np.abs(P @ f(Vc) - f(Vf)).max() <= 1e-14


@pytest.mark.parametrize("s,mode", [(0.25, "paper"), (0.75, "paper"), (0.4, "interior")])
def test_galerkin_mass_matrix_is_the_coarse_mass_matrix(s, mode):
    """The coarse P1 space is a subspace of the fine one, so P^T M_f P is the
    coarse mass matrix exactly (both integrated in closed form)."""
    meshes, parents, dofs, nv = _levels(M.disk_for_cells(150, seed=2), 3, s, mode)
    Mf = O.mass_matrix(meshes[2], dofs[2])
    Ms, Ps = G.hierarchy_operators(Mf, parents, dofs, nv)
    for l in (0, 1):
        ref = O.mass_matrix(meshes[l], dofs[l])
        assert np.abs(Ms[l] - ref).max() <= 1e-14 * 10


def test_galerkin_stiffness_close_to_coarse_assembly():
    """P^T A_f P against the coarse-mesh assembly: equal up to quadrature
    error (a wrong prolongation weight would be an O(1) difference)."""
    s = 0.6
    meshes, parents, dofs, nv = _levels(M.disk_for_cells(120, seed=3), 2, s)
    o = O.Orders(k_touch=8, k_touch_bnd=8, k_far=[6, 5, 4, 4], k_far_bnd=[6, 5, 4, 4])
    Af, _, _ = O.assemble(meshes[1], s, o)
    Ac, _, _ = O.assemble(meshes[0], s, o)
    As, _ = G.hierarchy_operators(Af, parents, dofs, nv)
    assert np.abs(As[0] - Ac).max() <= 2e-3 * np.abs(Ac).max()


def test_vcycle_solver_and_mg_pcg():
    """The V-cycle as a stationary solver contracts the error at a rate
    bounded away from 1 on 2 and 3 levels; MG-PCG reaches the Cholesky
    solution, and its iteration count stays flat from 2 to 3 levels while
    Jacobi-PCG's grows (Sec. 5)."""
    s = 0.75
    rates, its_mg, its_j = [], [], []
    base = M.disk_for_cells(150, seed=4)
    for L in (2, 3):
        meshes, parents, dofs, nv = _levels(base, L, s)
        A, _, _ = O.assemble(meshes[-1], s, O.Orders())
        b = O.load_vector_one(meshes[-1], dofs[-1])
        As, Ps = G.hierarchy_operators(A, parents, dofs, nv)
        u = O.solve_cholesky(A, b)
        x = np.zeros_like(b)
        e0 = np.sqrt((u - x) @ A @ (u - x))
        for _ in range(6):
            x = x + G.vcycle(As, Ps, b - A @ x)
        e6 = np.sqrt((u - x) @ A @ (u - x))
        rates.append((e6 / e0) ** (1 / 6))
        xm, it = G.mg_pcg(As, Ps, b, rtol=1e-12)
        assert np.sqrt((xm - u) @ A @ (xm - u)) <= 1e-10 * np.sqrt(u @ A @ u)
        its_mg.append(it)
        its_j.append(O.pcg(A, b, rtol=1e-12)[1])
    assert max(rates) < 0.35, rates
    assert its_mg[1] <= its_mg[0] + 2, its_mg
    assert its_j[1] >= its_j[0] + 5, its_j
    assert its_mg[1] < its_j[1] / 2
