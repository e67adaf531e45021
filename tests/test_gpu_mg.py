"""Geometric multigrid on the GPU (Sec. 5) against the oracle's: the same
cycle on the same nested hierarchy reaches the oracle's solution with the
oracle's iteration count (+-1), and the count stays flat under refinement
while Jacobi-PCG's grows."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import multigrid as G  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_1708_03912_amd import fraclap as F, meshgen as M  # noqa: E402

from test_gpu_parity import oracle_orders  # noqa: E402


def _gpu_mg(meshes, parents, s, opts):
    h = F.Handle(0)
    h.set_mesh(meshes[-1])
    n = h.assemble(s, opts)
    h.mg_setup([len(m["verts"]) for m in meshes], parents)
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    h.load_vector_one(b)
    u = torch.zeros_like(b)
    it, rel, rc = h.solve_mg(b, u, rtol=1e-12, maxit=200)
    return h, it, rel, rc, u.cpu().numpy()


@pytest.mark.parametrize("s,mode", [(0.3, "paper"), (0.75, "paper"), (0.5, "interior")])
def test_mg_pcg_parity(s, mode):
    meshes, parents = M.hierarchy(M.disk_for_cells(150, seed=4), 3)
    o = F.make_opts(dof_mode=mode)
    h, it, rel, rc, u = _gpu_mg(meshes, parents, s, o)
    assert rc == F.FL_OK and rel <= 1e-12
    dofs = [O.dof_nodes(len(m["verts"]), m["bfacets"], s, mode) for m in meshes]
    A, _, _ = O.assemble(meshes[-1], s, oracle_orders(o), mode=mode)
    b = O.load_vector_one(meshes[-1], dofs[-1])
    As, Ps = G.hierarchy_operators(A, parents, dofs, [len(m["verts"]) for m in meshes])
    uo = O.solve_cholesky(A, b)
    _, ito = G.mg_pcg(As, Ps, b, rtol=1e-12)
    e = u - uo
    assert np.sqrt(e @ A @ e) <= 1e-10 * np.sqrt(uo @ A @ uo)
    assert abs(it - ito) <= 1, (it, ito)
    h.close()


def test_mg_iterations_flat_under_refinement():
    s = 0.75
    base = M.disk_for_cells(150, seed=4)
    its_mg, its_j = [], []
    for L in (2, 3, 4):
        meshes, parents = M.hierarchy(base, L)
        h, it, rel, rc, _ = _gpu_mg(meshes, parents, s, F.default_opts())
        assert rc == F.FL_OK
        b = torch.empty(h.n, dtype=torch.float64, device="cuda")
        h.load_vector_one(b)
        u = torch.zeros_like(b)
        itj, _, rcj = h.solve(b, u, rtol=1e-12)
        its_mg.append(it)
        its_j.append(itj)
        h.close()
    assert its_mg[-1] <= its_mg[0] + 3, its_mg
    assert its_j[-1] >= 2.5 * its_j[0], its_j
    assert its_mg[-1] * 5 < its_j[-1]


def test_mg_errors():
    meshes, parents = M.hierarchy(M.disk_for_cells(150, seed=4), 2)
    nv = [len(m["verts"]) for m in meshes]
    h = F.Handle(0)
    h.set_mesh(meshes[-1])
    with pytest.raises(F.FraclapError) as e:
        h.mg_setup(nv, parents)
    assert e.value.code == F.FL_ESTATE
    n = h.assemble(0.4)
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    u = torch.zeros_like(b)
    with pytest.raises(F.FraclapError) as e:
        h.solve_mg(b, u)
    assert e.value.code == F.FL_ESTATE
    bad = parents[0].copy()
    inh = np.nonzero(bad[:, 0] == bad[:, 1])[0]
    bad[inh[0]] = bad[inh[1]]  # one coarse vertex copied twice, another never
    with pytest.raises(F.FraclapError) as e:
        h.mg_setup(nv, [bad])
    assert e.value.code == F.FL_EMESH
    with pytest.raises(F.FraclapError) as e:
        h.mg_setup([nv[0], nv[1] + 1], parents)
    assert e.value.code == F.FL_EINVAL
    h.mg_setup(nv, parents)
    it, rel, rc = h.solve_mg(b, u, rtol=1e-10)
    assert rc == F.FL_OK
    h.assemble(0.6)  # a new matrix discards the hierarchy
    with pytest.raises(F.FraclapError) as e:
        h.solve_mg(b[: h.n].contiguous(), u[: h.n].contiguous())
    assert e.value.code == F.FL_ESTATE
    h.close()
