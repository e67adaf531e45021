"""Cluster approximation assembled from the mesh alone (fl_cluster_assemble,
Sec. 6) against the oracle's build_direct: the same tree and blocks and the
same operator, every column to 1e-10, on a disk (both DOF sets, with and
without the boundary term), an interval, an L-shape and a square whose
corner cells have no DOF; CG on it without any dense matrix; and a disk
whose dense FP64 matrix would not fit in device memory."""
import math
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import cluster as H  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_1708_03912_amd import fraclap as F, meshgen as M  # noqa: E402

from test_cluster_oracle import _grid_square  # noqa: E402
from test_gpu_parity import oracle_orders  # noqa: E402


def _direct(mesh, s, opts, m, eta, leaf):
    h = F.Handle(0)
    h.set_mesh(mesh)
    n = h.cluster_assemble(s, opts, m=m, eta=eta, leaf=leaf)
    return h, n


def _columns(h, n):
    """A_H e_j for every j (the operator as a dense array, for checks)."""
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    Y = torch.empty_like(eye)
    for j in range(n):
        h.cluster_matvec(eye[j], Y[j])
    torch.cuda.synchronize()
    return Y.cpu().numpy().T


CASES = {
    "disk_interior": (lambda: M.disk_for_cells(1200, seed=2), 0.75, "paper", True, 5, 2.0, 16),
    "disk_m8": (lambda: M.disk_for_cells(1500, seed=8), 0.4, "interior", True, 8, 2.0, 24),
    "disk_all_nodes": (lambda: M.disk_for_cells(900, seed=5), 0.3, "paper", True, 4, 1.5, 12),
    "disk_regional": (lambda: M.disk_for_cells(900, seed=5), 0.6, "interior", False, 4, 2.0, 16),
    "interval": (lambda: M.interval(256), 0.25, "paper", True, 6, 1.0, 8),
    "lshape": (lambda: M.lshape(h_max=0.8, ratio=16.0), 0.5, "paper", True, 4, 1.5, 24),
    "corner_cells_without_dof": (lambda: _grid_square(10), 0.6, "interior", True, 4, 1.5, 4),
}


@pytest.mark.parametrize("case", list(CASES))
def test_cluster_assemble_parity(case):
    make, s, mode, bnd, m, eta, leaf = CASES[case]
    mesh = make()
    print(f"case {case}: s={s} mode={mode} boundary={bnd} m={m} eta={eta} leaf={leaf}", flush=True)
    o = F.default_opts()
    o.dof_mode = F.FL_DOF_PAPER if mode == "paper" else F.FL_DOF_INTERIOR
    o.with_boundary = 1 if bnd else 0
    h, n = _direct(mesh, s, o, m, eta, leaf)
    nv = np.asarray(mesh["verts"]).size // mesh["dim"]
    dofs = O.dof_nodes(nv, mesh["bfacets"], s, mode)
    assert n == len(dofs) and np.array_equal(h.dofs(), dofs)
    Ho = H.build_direct(mesh, dofs, s, oracle_orders(o), m=m, eta=eta, leaf=leaf, with_boundary=bnd)
    info = h.cluster_info()
    assert info["clusters"] == len(Ho.tree.clusters)
    assert info["leaves"] == len(Ho.tree.leaves())
    assert info["far_pairs"] == len(Ho.far) and info["far_pairs"] > 0
    assert info["near_pairs"] == len(Ho.near)
    Y = _columns(h, n)
    Yo = H.dense(Ho, n)
    err = np.abs(Y - Yo).max() / np.abs(Yo).max()
    print(f"  n={n} max |A_H - oracle| / max |oracle| = {err:.2e}", flush=True)
    assert err <= 1e-10
    h.close()


def test_cluster_assemble_solves_without_dense_matrix():
    """CG on the directly assembled approximation: the iterate solves the
    oracle's operator to the tolerance, and it is within the
    approximation's accuracy of the dense solution; no dense matrix exists
    (the dense-matrix calls report FL_ESTATE)."""
    s = 0.75
    mesh = M.disk_for_cells(3000, seed=7)
    o = F.default_opts()
    h, n = _direct(mesh, s, o, 6, 2.0, 32)
    dofs = h.dofs()
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    h.load_vector_one(b)
    u = torch.zeros_like(b)
    it, rel, rc = h.solve_cluster(b, u, rtol=1e-11)
    assert rc == F.FL_OK and rel <= 1e-11
    with pytest.raises(F.FraclapError) as e:
        h.matvec(u, torch.empty_like(u))
    assert e.value.code == F.FL_ESTATE
    orders = oracle_orders(o)
    Ho = H.build_direct(mesh, dofs, s, orders, m=6, eta=2.0, leaf=32)
    AH = H.dense(Ho, n)
    bo = O.load_vector_one(mesh, dofs)
    uo = np.linalg.solve(AH, bo)
    du = u.cpu().numpy() - uo
    assert math.sqrt(du @ AH @ du) <= 1e-9 * math.sqrt(uo @ AH @ uo)
    A, _, _ = O.assemble(mesh, s, orders)
    ud = O.solve_cholesky(A, bo)
    dd = u.cpu().numpy() - ud
    assert math.sqrt(dd @ A @ dd) <= 1e-4 * math.sqrt(ud @ A @ ud)
    h.close()


def test_cluster_assemble_beyond_dense_memory():
    """Unit disk, ~4e5 triangles, interior DOFs (n ~ 2e5): the dense FP64
    matrix (n^2 x 8 bytes) exceeds the device memory; the cluster
    approximation is assembled and CG converges; the energy error of f = 1
    against the closed form (Sec. 7) is below the one on the ~2e5-triangle
    disk."""
    s = 0.75
    free, total = torch.cuda.mem_get_info()
    errs = {}
    for cells in (200000, 400000):
        mesh = M.disk_for_cells(cells, seed=2)
        o = F.default_opts()
        o.dof_mode = F.FL_DOF_INTERIOR
        t0 = time.perf_counter()
        h, n = _direct(mesh, s, o, 6, 2.0, 32)
        t_asm = time.perf_counter() - t0
        info = h.cluster_info()
        if cells == 400000:
            assert n * n * 8 > total, (n, total)
        assert info["bytes"] < 0.05 * total
        b = torch.empty(n, dtype=torch.float64, device="cuda")
        h.load_vector_one(b)
        u = torch.zeros_like(b)
        t0 = time.perf_counter()
        it, rel, rc = h.solve_cluster(b, u, rtol=1e-9, maxit=5000)
        t_sol = time.perf_counter() - t0
        assert rc == F.FL_OK
        c = 2.0 ** (-2 * s) / (math.gamma(1 + s) ** 2)
        fu = c * math.pi / (s + 1.0)
        e2 = fu - float(torch.dot(b, u))
        errs[cells] = math.sqrt(max(e2, 0.0))
        print(f"cells={len(mesh['cells'])} n={n} dense would be {n * n * 8 / 1e9:.0f} GB, cluster "
              f"{info['bytes'] / 1e9:.2f} GB ({info['near_entries']} near entries); assemble {t_asm:.2f} s, "
              f"CG {it} its {t_sol:.2f} s, energy error {errs[cells]:.4e}", flush=True)
        h.close()
        del h, b, u
        torch.cuda.empty_cache()
    assert 0.0 < errs[400000] < errs[200000] < 0.03
