"""Cluster (H-matrix) approximation on the GPU (Sec. 6) against the
oracle's: the same tree and block partition, the same product to 1e-10;
convergence to the dense product in m; CG on the approximation."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import cluster as H  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_1708_03912_amd import fraclap as F, meshgen as M  # noqa: E402

from test_gpu_parity import oracle_orders  # noqa: E402


def _handle(mesh, s):
    h = F.Handle(0)
    h.set_mesh(mesh)
    n = h.assemble(s, F.default_opts())
    return h, n


@pytest.mark.parametrize("case", ["disk", "interval", "lshape"])
def test_cluster_parity(case):
    if case == "disk":
        mesh, s, m, eta, leaf = M.disk_for_cells(1200, seed=2), 0.75, 5, 2.0, 16
    elif case == "interval":
        mesh, s, m, eta, leaf = M.interval(256), 0.25, 6, 1.0, 8
    else:
        mesh, s, m, eta, leaf = M.lshape(h_max=0.8, ratio=16.0), 0.5, 4, 1.5, 24
    h, n = _handle(mesh, s)
    h.cluster_build(m=m, eta=eta, leaf=leaf)
    info = h.cluster_info()
    A, dofs, _ = O.assemble(mesh, s, oracle_orders(F.default_opts()))
    Ho = H.build(mesh, dofs, A, s, m=m, eta=eta, leaf=leaf)
    assert info["clusters"] == len(Ho.tree.clusters)
    assert info["leaves"] == len(Ho.tree.leaves())
    assert info["far_pairs"] == len(Ho.far) and info["far_pairs"] > 0
    assert info["near_pairs"] == len(Ho.near)
    rng = np.random.default_rng(3)
    for _ in range(2):
        x = rng.standard_normal(n)
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        h.cluster_matvec(torch.tensor(x, device="cuda"), y)
        yo = H.matvec(Ho, x)
        err = np.abs(y.cpu().numpy() - yo).max()
        assert err <= 1e-10 * np.abs(yo).max(), err / np.abs(yo).max()
    h.close()


def test_cluster_converges_to_dense_and_solves():
    """c2-sized disk (~8k triangles): the approximation error falls
    geometrically in m; CG on the approximation reaches the dense solution
    to the approximation's accuracy."""
    s = 0.75
    mesh = M.disk_for_cells(8000, seed=2)
    h, n = _handle(mesh, s)
    x = torch.tensor(np.random.default_rng(5).standard_normal(n), device="cuda")
    yd = torch.empty_like(x)
    h.matvec(x, yd)
    errs = []
    for m in (2, 4, 6):
        h.cluster_build(m=m, eta=2.0, leaf=32)
        yh = torch.empty_like(x)
        h.cluster_matvec(x, yh)
        errs.append(float(torch.linalg.norm(yh - yd) / torch.linalg.norm(yd)))
    assert errs[0] > 5 * errs[1] > 25 * errs[2], errs
    assert errs[2] < 1e-6, errs
    info = h.cluster_info()
    assert info["near_entries"] < 0.5 * n * n
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    h.load_vector_one(b)
    u = torch.zeros_like(b)
    ud = torch.zeros_like(b)
    it, rel, rc = h.solve_cluster(b, u, rtol=1e-10)
    assert rc == F.FL_OK and rel <= 1e-10
    itd, _, _ = h.solve(b, ud, rtol=1e-10)
    assert abs(it - itd) <= max(3, itd // 10)
    e = u - ud
    Ae = torch.empty_like(e)
    h.matvec(e, Ae)
    Au = torch.empty_like(e)
    h.matvec(ud, Au)
    assert float(torch.dot(e, Ae)) ** 0.5 <= 1e-5 * float(torch.dot(ud, Au)) ** 0.5
    h.close()


def test_cluster_errors():
    mesh = M.disk_for_cells(300, seed=1)
    h = F.Handle(0)
    h.set_mesh(mesh)
    x = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FraclapError) as e:
        h.cluster_build()
    assert e.value.code == F.FL_ESTATE
    n = h.assemble(0.4, F.default_opts())
    for kw in ({"m": 0}, {"m": 16}, {"eta": 0.0}, {"leaf": 0}):
        with pytest.raises(F.FraclapError) as e:
            h.cluster_build(**kw)
        assert e.value.code == F.FL_EINVAL
    h.cluster_build(m=3)
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    h.cluster_matvec(x, y)
    h.assemble(0.4, F.default_opts())   # a new matrix drops the approximation
    with pytest.raises(F.FraclapError) as e:
        h.cluster_matvec(x, y)
    assert e.value.code == F.FL_ESTATE
    h.close()


def test_cluster_degenerate():
    """One leaf (no admissible pair): the product is the dense one; no DOFs
    at all (one triangle, s >= 1/2): build, product and solve are no-ops."""
    mesh = M.disk_for_cells(60, seed=3)
    h, n = _handle(mesh, 0.3)
    h.cluster_build(m=4, eta=2.0, leaf=1024)
    info = h.cluster_info()
    assert info["clusters"] == 1 and info["far_pairs"] == 0 and info["near_entries"] == n * n
    x = torch.tensor(np.random.default_rng(2).standard_normal(n), device="cuda")
    y, yd = torch.empty_like(x), torch.empty_like(x)
    h.cluster_matvec(x, y)
    h.matvec(x, yd)
    assert float((y - yd).abs().max()) <= 1e-13 * float(yd.abs().max())
    h.close()
    h, n = _handle(M.tiny("one"), 0.75)
    assert n == 0
    h.cluster_build()
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    h.cluster_matvec(e, e.clone())
    it, rel, rc = h.solve_cluster(e, e.clone())
    assert it == 0 and rc == F.FL_OK
    h.close()


def _mg_cluster_handle(meshes, parents, s, m=4, leaf=16):
    h = F.Handle(0)
    h.set_mesh(meshes[-1])
    n = h.assemble(s, F.default_opts())
    h.mg_setup([len(x["verts"]) for x in meshes], parents)
    h.cluster_build(m=m, eta=2.0, leaf=leaf)
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    h.load_vector_one(b)
    return h, n, b


def test_cluster_mg_parity():
    """Multigrid-preconditioned CG on the cluster approximation against the
    oracle's mg_pcg on the same hierarchy with the finest operator replaced
    by the oracle's cluster matrix: the oracle's iteration count (+-1) and
    the solution of A_H u = b."""
    from oracle import multigrid as G
    s = 0.75
    meshes, parents = M.hierarchy(M.disk_for_cells(150, seed=4), 3)
    mesh = meshes[-1]
    h, n, b = _mg_cluster_handle(meshes, parents, s)
    assert h.cluster_info()["far_pairs"] > 0
    u = torch.zeros_like(b)
    it, rel, rc = h.solve_cluster_mg(b, u, rtol=1e-12, maxit=200)
    assert rc == F.FL_OK and rel <= 1e-12
    dofs = [O.dof_nodes(len(x["verts"]), x["bfacets"], s) for x in meshes]
    A, _, _ = O.assemble(mesh, s, oracle_orders(F.default_opts()))
    Hd = H.dense(H.build(mesh, dofs[-1], A, s, m=4, eta=2.0, leaf=16), n)
    # the diagonal blocks are copied from A, so the smoother's diagonal is A's
    assert np.array_equal(np.diag(Hd), np.diag(A))
    As, Ps = G.hierarchy_operators(A, parents, dofs, [len(x["verts"]) for x in meshes])
    As[-1] = Hd
    bo = O.load_vector_one(mesh, dofs[-1])
    assert np.abs(b.cpu().numpy() - bo).max() <= 1e-13 * np.abs(bo).max()
    _, ito = G.mg_pcg(As, Ps, bo, rtol=1e-12)
    uo = np.linalg.solve(Hd, bo)
    e = u.cpu().numpy() - uo
    assert np.sqrt(e @ Hd @ e) <= 1e-10 * np.sqrt(uo @ Hd @ uo)
    assert abs(it - ito) <= 1, (it, ito)
    h.close()


def test_cluster_mg_flat_under_refinement():
    """The iteration count of the cluster operator's MG-PCG stays flat over
    2..4 levels and within 2 of the dense operator's."""
    s = 0.75
    base = M.disk_for_cells(150, seed=4)
    its = []
    for L in (2, 3, 4):
        meshes, parents = M.hierarchy(base, L)
        h, n, b = _mg_cluster_handle(meshes, parents, s, m=5, leaf=24)
        u = torch.zeros_like(b)
        it, rel, rc = h.solve_cluster_mg(b, u, rtol=1e-10)
        assert rc == F.FL_OK and rel <= 1e-10
        ud = torch.zeros_like(b)
        itd, _, rcd = h.solve_mg(b, ud, rtol=1e-10)
        assert rcd == F.FL_OK and abs(it - itd) <= 2, (it, itd)
        # the dense residual of the cluster solution: b - A u_H =
        # (b - A_H u_H) + (A_H - A) u_H, the first at most 1e-10 |b|
        yd, yh = torch.empty_like(b), torch.empty_like(b)
        h.matvec(u, yd)
        h.cluster_matvec(u, yh)
        lhs = float(torch.linalg.norm(b - yd))
        rhs = float(torch.linalg.norm(yh - yd)) + 1e-10 * float(torch.linalg.norm(b))
        assert lhs <= 1.001 * rhs, (lhs, rhs)
        its.append(it)
        h.close()
    assert its[-1] <= its[0] + 3, its


def test_cluster_mg_errors():
    s = 0.75
    meshes, parents = M.hierarchy(M.disk_for_cells(150, seed=4), 2)
    h = F.Handle(0)
    h.set_mesh(meshes[-1])
    n = h.assemble(s, F.default_opts())
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    u = torch.zeros_like(b)
    h.cluster_build(m=4, eta=2.0, leaf=16)
    with pytest.raises(F.FraclapError) as e:
        h.solve_cluster_mg(b, u)                      # no hierarchy
    assert e.value.code == F.FL_ESTATE
    h.assemble(s, F.default_opts())                   # discards both
    h.mg_setup([len(x["verts"]) for x in meshes], parents)
    with pytest.raises(F.FraclapError) as e:
        h.solve_cluster_mg(b, u)                      # no cluster approximation
    assert e.value.code == F.FL_ESTATE
    h.cluster_build(m=4, eta=2.0, leaf=16)
    with pytest.raises(F.FraclapError) as e:
        h.solve_cluster_mg(b, u, rtol=-1.0)
    assert e.value.code == F.FL_EINVAL
    it, rel, rc = h.solve_cluster_mg(b, u, rtol=1e-10)
    assert rc == F.FL_OK and it > 0
    h.close()
