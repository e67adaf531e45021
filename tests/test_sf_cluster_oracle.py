"""Pins of the cluster evaluation of the strong form (Sec. 6): the jump
sources, the treecode against the direct sum, and the strong form it
gives against the literal one."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import sf_cluster as SC
from oracle import strong_form as SF
from paper_1708_03912_amd import meshgen as M


@pytest.fixture(scope="module")
def disk():
    s = 0.75
    mesh = M.disk_for_cells(900, seed=2)
    V = np.asarray(mesh["verts"])
    dofs = O.dof_nodes(len(V), mesh["bfacets"], s)
    u = np.clip(1 - (V[dofs] ** 2).sum(1), 0, None) ** 0.5 + 0.05 * np.sin(7 * V[dofs, 0])
    return mesh, dofs, u, s


def test_jump_sources():
    """The outward normals of a cell sum to zero, so the jump coefficients
    sum to zero for any P1 function; a globally linear function has no
    jump on interior edges (sign of the second cell's term)."""
    s = 0.3
    mesh = M.disk_for_cells(300, seed=4)
    V = np.asarray(mesh["verts"])
    dofs = O.dof_nodes(len(V), mesh["bfacets"], s)
    u = np.random.default_rng(0).standard_normal(len(dofs))
    Y, c, own = SC.jump_sources(mesh, dofs, u, s, 2)
    assert abs(c.sum()) <= 1e-12 * np.abs(c).sum()
    lin = 0.3 + 1.7 * V[dofs, 0] - 0.4 * V[dofs, 1]
    Y, c, own = SC.jump_sources(mesh, dofs, lin, s, 2)
    C = np.asarray(mesh["cells"])
    bnd = {tuple(sorted(e)) for e in np.asarray(mesh["bfacets"]).tolist()}
    # sources come edge by edge, two per edge: interior edges carry nothing
    nz = np.abs(c) > 1e-12
    assert 0 < nz.sum() <= 2 * len(bnd)


def test_treecode_is_the_direct_sum_without_far_pairs(disk):
    mesh, dofs, u, s = disk
    Xc, _, _ = SF.eval_points(mesh, 2)
    Y, c, own = SC.jump_sources(mesh, dofs, u, s, 2)
    P, far, near, cl = SC.treecode(mesh, Xc, Y, c, own, s, m=3, eta=1e-9, leaf=16)
    assert len(far) == 0
    Pd = SC.potential_direct(Xc.reshape(-1, 2), Y, c, s).reshape(P.shape)
    assert np.abs(P - Pd).max() <= 1e-13 * np.abs(Pd).max()


def test_treecode_converges_in_m(disk):
    mesh, dofs, u, s = disk
    Xc, _, _ = SF.eval_points(mesh, 2)
    Y, c, own = SC.jump_sources(mesh, dofs, u, s, 2)
    Pd = SC.potential_direct(Xc.reshape(-1, 2), Y, c, s).reshape(-1, 4)
    err = []
    for m in (2, 4, 6):
        P, far, near, cl = SC.treecode(mesh, Xc, Y, c, own, s, m=m, eta=2.0, leaf=16)
        assert len(far) > 0
        err.append(np.abs(P - Pd).max() / np.abs(Pd).max())
    assert err[0] > 10 * err[1] > 100 * err[2], err
    assert err[2] < 1e-5


def test_strong_form_cluster_approaches_the_literal_one(disk):
    mesh, dofs, u, s = disk
    L0 = SF.strong_form(mesh, dofs, u, s)
    gaps = []
    for m in (3, 6):
        L1, _ = SC.strong_form_cluster(mesh, dofs, u, s, m=m, eta=2.0, leaf=16)
        gaps.append(np.abs(L1 - L0).max() / np.abs(L0).max())
    assert gaps[1] < gaps[0] / 10 and gaps[1] < 1e-5, gaps
