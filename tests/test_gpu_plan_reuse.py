"""Reuse of the s-independent plan (element order, DOF map, touching-pair
lists, tiles) by the next fl_assemble / fl_assemble_batch on the same mesh:
the kept plan gives the matrix a fresh handle gives (bit for bit in the
repeatable mode), and every change of its inputs -- DOF set, distance
classes, mesh, symmetry, a cluster assembly in between -- plans again
(t_plan_ms > 0 reports a new plan, 0 a reused one)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1708_03912_amd import fraclap as F, meshgen as M  # noqa: E402


def _bits(A):
    return np.ascontiguousarray(A).view(np.int64)


def _fresh(mesh, s, opts, sym=None):
    h = F.Handle(0)
    h.set_mesh(mesh)
    if sym is not None:
        h.set_symmetry(*sym)
    h.assemble(s, opts)
    A = h.export_matrix()
    h.close()
    return A


def test_plan_reused_across_s():
    mesh = M.disk_for_cells(3000, seed=3)
    od = F.make_opts(deterministic=1, dof_mode="interior")  # one DOF set for every s
    h = F.Handle(0)
    h.set_mesh(mesh)
    h.assemble(0.25, od)
    assert h.stats().t_plan_ms > 0.0
    A25 = h.export_matrix()
    h.assemble(0.75, od)
    assert h.stats().t_plan_ms == 0.0
    A75 = h.export_matrix()
    assert np.array_equal(_bits(A75), _bits(_fresh(mesh, 0.75, od)))
    # and back: still the kept plan
    h.assemble(0.25, od)
    assert h.stats().t_plan_ms == 0.0
    assert np.array_equal(_bits(h.export_matrix()), _bits(A25))
    # other orders on the same classes keep the plan as well
    od2 = F.make_opts(deterministic=1, dof_mode="interior", k_touch=5)
    h.assemble(0.5, od2)
    assert h.stats().t_plan_ms == 0.0
    assert np.array_equal(_bits(h.export_matrix()), _bits(_fresh(mesh, 0.5, od2)))
    h.close()


def test_plan_inputs_replan():
    mesh = M.disk_for_cells(2500, seed=5)
    h = F.Handle(0)
    h.set_mesh(mesh)
    od = F.make_opts(deterministic=1, dof_mode="interior")
    h.assemble(0.6, od)
    assert h.stats().t_plan_ms > 0.0
    # other distance classes: new tiles
    oc = F.make_opts(deterministic=1, dof_mode="interior", theta=(2.0, 4.0), k_far=(4, 3, 2))
    h.assemble(0.6, oc)
    assert h.stats().t_plan_ms > 0.0
    assert np.array_equal(_bits(h.export_matrix()), _bits(_fresh(mesh, 0.6, oc)))
    # the paper's DOF rule: all nodes below s = 1/2, interior ones above
    op = F.make_opts(deterministic=1, dof_mode="paper")
    n1 = h.assemble(0.3, op)
    assert h.stats().t_plan_ms > 0.0
    n2 = h.assemble(0.7, op)
    assert h.stats().t_plan_ms > 0.0 and n1 > n2
    assert np.array_equal(_bits(h.export_matrix()), _bits(_fresh(mesh, 0.7, op)))
    # a new mesh
    mesh2 = M.disk_for_cells(2000, seed=6)
    h.set_mesh(mesh2)
    h.assemble(0.6, od)
    assert h.stats().t_plan_ms > 0.0
    assert np.array_equal(_bits(h.export_matrix()), _bits(_fresh(mesh2, 0.6, od)))
    h.close()


def test_plan_after_symmetry_and_cluster():
    K, s = 4, 0.75
    mesh, vfold, Tw, pre, rot = M.disk_symmetric(0.2, K, seed=6)
    od = F.make_opts(deterministic=1)
    h = F.Handle(0)
    h.set_mesh(mesh)
    h.assemble(s, od)
    h.set_symmetry(K, Tw, vfold, pre, rot)
    h.assemble(s, od)
    assert h.stats().t_plan_ms > 0.0
    assert np.array_equal(_bits(h.export_matrix()), _bits(_fresh(mesh, s, od, sym=(K, Tw, vfold, pre, rot))))
    # a cluster assembly plans its own tiles into the plan buffer
    mesh3 = M.disk_for_cells(3000, seed=7)
    h.set_mesh(mesh3)
    h.assemble(s, od)
    h.cluster_assemble(s, F.make_opts(), m=4)
    h.assemble(s, od)
    assert h.stats().t_plan_ms > 0.0
    assert np.array_equal(_bits(h.export_matrix()), _bits(_fresh(mesh3, s, od)))
    h.close()


def test_plan_reused_by_batch():
    mesh = M.disk_for_cells(1400, seed=2)
    oi = F.make_opts(dof_mode="interior")
    h = F.Handle(0)
    h.set_mesh(mesh)
    h.assemble(0.4, oi)
    h.assemble_batch([0.3, 0.6], oi)
    assert h.stats().t_plan_ms == 0.0
    g = F.Handle(0)
    g.set_mesh(mesh)
    g.assemble_batch([0.3, 0.6], oi)
    assert g.stats().t_plan_ms > 0.0
    for j in range(2):
        A, B = h.export_batch_matrix(j), g.export_batch_matrix(j)
        assert np.abs(A - B).max() <= 1e-14 * np.abs(B).max()
    h.close()
    g.close()


def test_lower_triangle_on_demand():
    """The assembly writes the tiles on and above the diagonal tiles; the
    rest of the lower triangle is copied when a reader of the whole matrix
    asks (export, the matrix pointer): after two assemblies on one handle
    the whole matrix equals a fresh handle's, bit for bit, and is exactly
    symmetric; the product, which reads only the upper tiles, agrees."""
    mesh = M.disk_for_cells(6000, seed=9)
    od = F.make_opts(deterministic=1, dof_mode="interior")
    h = F.Handle(0)
    h.set_mesh(mesh)
    n = h.assemble(0.3, od)
    h.assemble(0.8, od)  # the lower tiles of the s = 0.3 matrix are left in the buffer
    A = h.export_matrix()
    assert np.array_equal(_bits(A), _bits(A.T))
    assert np.array_equal(_bits(A), _bits(_fresh(mesh, 0.8, od)))
    x = torch.rand(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    h.matvec(x, y)
    yr = A @ x.cpu().numpy()
    assert np.abs(y.cpu().numpy() - yr).max() <= 1e-13 * np.abs(yr).max()
    # the device pointer's view after a further assembly
    h.assemble(0.5, od)
    V = h.matrix_view()
    torch.cuda.synchronize()
    Av = V.cpu().numpy()
    assert np.array_equal(_bits(Av), _bits(Av.T))
    assert np.array_equal(_bits(Av), _bits(_fresh(mesh, 0.5, od)))
    h.close()
